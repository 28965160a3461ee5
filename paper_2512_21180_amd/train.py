"""Train the learned primal-dual net (any scales) on projector-simulated data.

Training pairs: seeded ellipsoid phantoms in a 300 mm body cylinder (the
clinical-size recipe), Poisson noise at I0 photons per pixel on the library's
forward projection, negative-log normalisation (Sec. 2.2 primary model,
Sec. 2.4 normalisation), all simulated on the GPU by the library.  Units:
attenuation divided by 0.02 /mm (water = 1); data y / 0.02 / L with
L = ||A||_2, so the net sees the normalised operator A / L (Sec. 2.6).
Loss: the squared error over the full field of view (voxels seen in at least
half of the projections), summed over all iterates (the output list I of
Alg. 1).  Adam with linear warm-up and cosine decay.  Augmentation:
left-right and head-foot flips.

Robustness: a step whose loss or any gradient is not finite is skipped
(the run stops after --max-skips in a row); every --checkpoint-every steps
and at the end the weights, the Adam moments and step counts, the next step
and the sampling generator's state go to <out>.ckpt, written to a temporary
file and renamed over the old one, and --resume <out>.ckpt continues the
run where it stopped.

The default training geometry is a 32-layer z-slab of the clinical case with
the panel rows that see it: the same voxel and pixel pitch, angles, offset
and magnification, so the 3x3x3 blocks learn the same local operators at a
quarter of the cost per step.

    python -m paper_2512_21180_amd.train --steps 300 --out weights.pt
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import cbct, learned, simulate, solvers
from . import workloads as W

MU_SCALE = 0.02     # /mm: the attenuation unit of the net (water = 1)


def training_geometry(name: str) -> dict:
    if name == "slab":
        return W.slab(W.C2, nz=32, nv=208)
    if name == "c5":
        return W.C2
    if name == "toy":
        return W.geometry(60, 96, 48, 3.2, 3.2, 48, 48, 16, 6.0, off_u=60.0)
    raise ValueError(name)


def phantom(g: dict, name: str, seed: int) -> np.ndarray:
    if name == "c5":
        return W.phantom_c2(g, seed)[0]
    return W.phantom_c2_slab(g, seed, g_full=W.C2 if name == "slab" else
                             W.geometry(60, 96, 96, 3.2, 3.2, 48, 48, 48, 6.0, off_u=60.0))


def _weights(net: learned.PDNet) -> dict:
    state = {k: v.detach().cpu() for k, v in net.state_dict().items()}
    state["perms"] = torch.tensor(net.perms, dtype=torch.int64)
    state["meta_n_iter"] = torch.tensor(net.n_iter)
    state["meta_scales"] = torch.tensor(net.scales, dtype=torch.int64)
    state["meta_fdk_init"] = torch.tensor(1 if net.init == "fdk" else 0)
    return state


def _write(obj, path: str):
    """torch.save to a temporary file beside path, then rename over it: a
    crash mid-write leaves the previous file intact."""
    tmp = path + ".tmp"
    torch.save(obj, tmp)
    os.replace(tmp, path)


def save(net: learned.PDNet, path: str, meta: dict):
    _write(_weights(net), path)


def _net_from(state: dict) -> learned.PDNet:
    state = dict(state)
    n_iter = int(state.pop("meta_n_iter"))
    scales = state.pop("meta_scales").tolist() if "meta_scales" in state else None
    init = "fdk" if int(state.pop("meta_fdk_init", torch.tensor(0))) else "zero"
    net = learned.PDNet(n_iter=n_iter, scales=scales, init=init)
    net.perms = [list(map(int, r)) for r in state.pop("perms").tolist()]
    net.load_state_dict(state)
    return net


def load(path: str, device="cuda") -> learned.PDNet:
    return _net_from(torch.load(path, map_location="cpu", weights_only=True)).to(device)


def save_checkpoint(path: str, net: learned.PDNet, opt: torch.optim.Optimizer, step: int,
                    rng: np.random.Generator, skipped: int):
    """Everything a resumed run needs to continue as if uninterrupted: the
    weights, the optimiser's moments and step counts, the next step, the
    sampling generator's state and the count of skipped steps."""
    _write({"net": _weights(net), "opt": opt.state_dict(), "step": int(step),
            "rng": json.dumps(rng.bit_generator.state), "skipped": int(skipped)}, path)


def load_checkpoint(path: str, device="cuda"):
    """(net, optimiser state dict, next step, generator, skipped) of a checkpoint."""
    ck = torch.load(path, map_location="cpu", weights_only=True)
    net = _net_from(ck["net"]).to(device)
    rng = np.random.default_rng()
    rng.bit_generator.state = json.loads(ck["rng"])
    return net, ck["opt"], int(ck["step"]), rng, int(ck.get("skipped", 0))


def finite_step(loss: float, params) -> bool:
    """True when the loss and every gradient are finite (a step with a NaN
    or an infinity anywhere is skipped rather than taken)."""
    if not math.isfinite(loss):
        return False
    return all(p.grad is None or bool(torch.isfinite(p.grad).all()) for p in params)


def simulate_pair(geo, x_mu: torch.Tensor, I0: float, seed: int, L: float):
    """(normalised data, normalised truth) for a phantom in /mm."""
    y = simulate.noisy_sinogram(geo, x_mu, I0, seed=seed)
    cbct.axpby(y, 1.0 / (MU_SCALE * L), y, 0.0, y)
    x_n = x_mu.clone()
    cbct.axpby(x_n, 1.0 / MU_SCALE, x_n, 0.0, x_n)
    return y, x_n


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--geometry", default="slab", choices=["slab", "c5", "toy"])
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n-iter", type=int, default=8)
    ap.add_argument("--init", default="zero", choices=["zero", "fdk"])
    ap.add_argument("--scales", default=None,
                    help="comma-separated resolution divisor per iteration, e.g. 4,4,2,2,1,1")
    ap.add_argument("--pool", type=int, default=48, help="distinct training phantoms")
    ap.add_argument("--I0", type=float, default=1e5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--resume", default=None,
                    help="a checkpoint (<out>.ckpt: weights, optimiser, step, generator) "
                         "or a weights file (weights only, fresh optimiser)")
    ap.add_argument("--out", required=True)
    ap.add_argument("--checkpoint-every", type=int, default=50,
                    help="steps between checkpoints written to <out>.ckpt")
    ap.add_argument("--max-skips", type=int, default=20,
                    help="consecutive non-finite steps before giving up")
    ap.add_argument("--time-limit", type=float, default=1e9, help="seconds; stop and save")
    args = ap.parse_args(argv)
    t_start = time.time()
    torch.cuda.set_device(0)
    g = training_geometry(args.geometry)
    geo = cbct.Geometry(g)
    V = torch.tensor(cbct.fov_fraction(g), device="cuda")
    L = solvers.opnorm(geo, iters=50, seed=0)
    fov = (V >= 0.5).float()
    wmask = (fov / fov.sum()).contiguous()
    scales = [int(v) for v in args.scales.split(",")] if args.scales else None
    n_iter = len(scales) if scales else args.n_iter
    start, skipped, opt_state = 0, 0, None
    rng = np.random.default_rng(args.seed + 17)
    if args.resume and args.resume.endswith(".ckpt"):
        net, opt_state, start, rng, skipped = load_checkpoint(args.resume)
    elif args.resume:
        net = load(args.resume)
    else:
        net = learned.PDNet(n_iter, seed=args.seed, scales=scales, init=args.init).cuda()
    model = learned.LearnedPD(net, geo, V, L)
    opt = torch.optim.Adam(net.parameters(), lr=args.lr)
    if opt_state is not None:
        opt.load_state_dict(opt_state)
    ckpt = args.out + ".ckpt"
    print(f"[train] geometry {args.geometry} vol {geo.vol_shape} sino {geo.sino_shape} "
          f"L {L:.5e} params {sum(p.numel() for p in net.parameters())}", flush=True)
    pool = []
    for k in range(args.pool):
        pool.append(torch.tensor(phantom(g, args.geometry, 1000 + k), dtype=torch.float32))
        if (k + 1) % 8 == 0:
            print(f"[train] phantoms {k + 1}/{args.pool} ({time.time() - t_start:.0f} s)",
                  flush=True)
    hist = []
    run_of_skips = 0
    step = start - 1
    for step in range(start, args.steps):
        lr = args.lr * min(1.0, (step + 1) / args.warmup) * \
            0.5 * (1.0 + math.cos(math.pi * step / args.steps))
        for grp in opt.param_groups:
            grp["lr"] = max(lr, 0.02 * args.lr)
        x = pool[int(rng.integers(len(pool)))].cuda()
        if rng.random() < 0.5:
            x = torch.flip(x, dims=[2])       # left-right
        if rng.random() < 0.5:
            x = torch.flip(x, dims=[0])       # head-foot
        x = x.contiguous()
        y, x_n = simulate_pair(geo, x, args.I0, seed=int(rng.integers(1 << 31)), L=L)
        opt.zero_grad(set_to_none=True)
        loss = model.loss_and_grad(y, x_n, wmask)
        if finite_step(loss, net.parameters()):
            torch.nn.utils.clip_grad_norm_(net.parameters(), 1.0)
            opt.step()
            hist.append(loss)
            run_of_skips = 0
        else:
            skipped += 1
            run_of_skips += 1
            print(f"[train] step {step + 1}: non-finite loss or gradient, skipped "
                  f"({skipped} so far)", flush=True)
            if run_of_skips >= args.max_skips:
                print(f"[train] {run_of_skips} non-finite steps in a row: stopping; the "
                      f"last checkpoint is {ckpt}", flush=True)
                return 1
        if (step + 1) % 10 == 0 or step == start:
            print(f"[train] step {step + 1}/{args.steps} loss "
                  f"{np.mean(hist[-10:]) if hist else float('nan'):.5f} "
                  f"lr {lr:.2e} ({time.time() - t_start:.0f} s)", flush=True)
        if (step + 1) % args.checkpoint_every == 0:
            save_checkpoint(ckpt, net, opt, step + 1, rng, skipped)
        if time.time() - t_start > args.time_limit:
            print(f"[train] time limit reached at step {step + 1}", flush=True)
            break
    save_checkpoint(ckpt, net, opt, step + 1, rng, skipped)
    save(net, args.out, {})
    print(f"[train] saved {args.out} and {ckpt} after {time.time() - t_start:.0f} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
