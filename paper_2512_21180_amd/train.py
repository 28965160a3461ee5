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

The default training geometry is a 32-layer z-slab of the clinical case with
the panel rows that see it: the same voxel and pixel pitch, angles, offset
and magnification, so the 3x3x3 blocks learn the same local operators at a
quarter of the cost per step.

    python -m paper_2512_21180_amd.train --steps 300 --out weights.pt
"""
from __future__ import annotations

import argparse
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


def save(net: learned.PDNet, path: str, meta: dict):
    state = {k: v.detach().cpu() for k, v in net.state_dict().items()}
    state["perms"] = torch.tensor(net.perms, dtype=torch.int64)
    state["meta_n_iter"] = torch.tensor(net.n_iter)
    state["meta_scales"] = torch.tensor(net.scales, dtype=torch.int64)
    state["meta_fdk_init"] = torch.tensor(1 if net.init == "fdk" else 0)
    torch.save(state, path)


def load(path: str, device="cuda") -> learned.PDNet:
    state = torch.load(path, map_location="cpu", weights_only=True)
    n_iter = int(state.pop("meta_n_iter"))
    scales = state.pop("meta_scales").tolist() if "meta_scales" in state else None
    init = "fdk" if int(state.pop("meta_fdk_init", torch.tensor(0))) else "zero"
    net = learned.PDNet(n_iter=n_iter, scales=scales, init=init)
    net.perms = [list(map(int, r)) for r in state.pop("perms").tolist()]
    net.load_state_dict(state)
    return net.to(device)


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
    ap.add_argument("--resume", default=None)
    ap.add_argument("--out", required=True)
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
    net = load(args.resume) if args.resume else \
        learned.PDNet(n_iter, seed=args.seed, scales=scales, init=args.init).cuda()
    model = learned.LearnedPD(net, geo, V, L)
    opt = torch.optim.Adam(net.parameters(), lr=args.lr)
    print(f"[train] geometry {args.geometry} vol {geo.vol_shape} sino {geo.sino_shape} "
          f"L {L:.5e} params {sum(p.numel() for p in net.parameters())}", flush=True)
    pool = []
    for k in range(args.pool):
        pool.append(torch.tensor(phantom(g, args.geometry, 1000 + k), dtype=torch.float32))
        if (k + 1) % 8 == 0:
            print(f"[train] phantoms {k + 1}/{args.pool} ({time.time() - t_start:.0f} s)",
                  flush=True)
    rng = np.random.default_rng(args.seed + 17)
    hist = []
    for step in range(args.steps):
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
        torch.nn.utils.clip_grad_norm_(net.parameters(), 1.0)
        opt.step()
        hist.append(loss)
        if (step + 1) % 10 == 0 or step == 0:
            print(f"[train] step {step + 1}/{args.steps} loss {np.mean(hist[-10:]):.5f} "
                  f"lr {lr:.2e} ({time.time() - t_start:.0f} s)", flush=True)
        if time.time() - t_start > args.time_limit:
            print(f"[train] time limit reached at step {step + 1}", flush=True)
            break
    save(net, args.out, {})
    print(f"[train] saved {args.out} after {time.time() - t_start:.0f} s", flush=True)


if __name__ == "__main__":
    sys.exit(main())
