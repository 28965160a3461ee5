"""Time to a fixed PSNR: learned primal-dual net against CGLS, same operators.

Clinical-size case (256^3 at 2 mm, 360 angles, 512^2 panel at 0.8 mm with a
115 mm offset), test phantoms with seeds disjoint from training, Poisson
noise at I0 photons per pixel.  For each phantom:

* CGLS (x_0 = 0, 50 iterations) on the same data, and the learned net's
  8 iterates, each run twice: once timed (HIP events after every iteration,
  no host synchronisation), once with the PSNR of every iterate;
* target PSNR = the best PSNR CGLS reaches in its 50 iterations; reported:
  the time at which each method's iterates first reach it (start: data
  resident in HBM; L and V are per-geometry constants computed once);
* the net with every block zeroed (only the output convolutions act), to
  show what the blocks contribute, and FDK (the classic one-pass method and
  the net's optional starting point).

PSNR over the full field of view (voxels seen in at least half of the
projections): 10 log10(max(x_true)^2 / mean((x - x_true)^2)) in units of
0.02 /mm.

    python -m paper_2512_21180_amd.compare [--weights weights.pt] --json out.json

(default weights: the committed multiscale FDK-start net, `weights/`).
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

from . import cbct, learned, solvers
from . import workloads as W
from .train import MU_SCALE, load, simulate_pair


class PSNR:
    def __init__(self, V: torch.Tensor, ws_n: int):
        self.fov = (V >= 0.5).float().contiguous()
        self.n = float(self.fov.sum())
        self.ws = cbct.dot_workspace(ws_n, V.device)
        self.cell = torch.zeros(2, dtype=torch.float64, device=V.device)
        self.r = torch.empty_like(V)

    def __call__(self, x: torch.Tensor, xt: torch.Tensor, peak: float) -> float:
        cbct.wresid(self.r, self.fov, x, xt)          # fov * (x - xt)
        cbct.dot(self.r, self.r, self.ws, self.cell[0:1])
        mse = float(self.cell[0]) / self.n
        return 10.0 * math.log10(peak * peak / mse)


def timed(run, n_events):
    """Run `run(mark)` where mark(i) records an event after iteration i;
    returns seconds from the start to each mark."""
    ev0 = torch.cuda.Event(enable_timing=True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_events)]
    torch.cuda.synchronize()
    ev0.record()
    run(lambda i: evs[i - 1].record())
    torch.cuda.synchronize()
    return [ev0.elapsed_time(e) * 1e-3 for e in evs]


DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                               "lpd_c5_multiscale_fdk.pt")


class Setup:
    """Geometry, FoV tensor, operator norm, net and PSNR helper of the
    clinical case (per-geometry constants, computed once)."""

    def __init__(self, weights: str):
        self.g = W.C2
        self.geo = cbct.Geometry(self.g)
        self.V = torch.tensor(cbct.fov_fraction(self.g), device="cuda")
        self.L = solvers.opnorm(self.geo, iters=50, seed=0)
        self.net = load(weights)
        self.model = learned.LearnedPD(self.net, self.geo, self.V, self.L)
        n = self.geo.vol_shape[0] * self.geo.vol_shape[1] * self.geo.vol_shape[2]
        self.psnr = PSNR(self.V, n)


def compare_one(S: Setup, seed: int, I0: float = 1e5, K: int = 50, log=print) -> dict:
    """One test phantom: CGLS (K iterations) and the learned net, each timed
    per iteration and scored per iterate; target = CGLS's best PSNR."""
    geo, model, psnr, L, net = S.geo, S.model, S.psnr, S.L, S.net
    t0 = time.time()
    x_mu = torch.tensor(W.phantom_c2(S.g, seed)[0], dtype=torch.float32, device="cuda")
    y, xt = simulate_pair(geo, x_mu, I0, seed=seed, L=L)
    peak = float((xt * psnr.fov).max())
    log(f"[compare] phantom seed {seed} ready in {time.time() - t0:.1f} s")
    # CGLS on the same normalised data: the iterates solve (A / L) x = y
    y_cg = y.clone()
    cbct.axpby(y_cg, L, y_cg, 0.0, y_cg)             # A x = L y
    t_cg = timed(lambda mark: solvers.cgls(geo, y_cg, K, callback=lambda k, x: mark(k)), K)
    ps_cg = []
    solvers.cgls(geo, y_cg, K, callback=lambda k, x: ps_cg.append(psnr(x, xt, peak)))
    log(f"[compare]   CGLS best {max(ps_cg):.2f} dB at iteration "
        f"{int(np.argmax(ps_cg)) + 1} ({t_cg[int(np.argmax(ps_cg))]:.3f} s); "
        f"{K} iterations {t_cg[-1]:.3f} s")
    # FDK (offset-detector weights) on the same data: A x = L y
    t_fdk = timed(lambda mark: (cbct.fdk(geo, y_cg), mark(1)), 1)[0]
    ps_fdk = psnr(cbct.fdk(geo, y_cg), xt, peak)
    ps_fdk_h = psnr(cbct.fdk(geo, y_cg, window="hann"), xt, peak)
    n = net.n_iter
    t_ln = timed(lambda mark: model.reconstruct(y, callback=lambda i, x: mark(i)), n)
    ps_ln = []
    model.reconstruct(y, callback=lambda i, x: ps_ln.append(psnr(x, xt, peak)))
    ps_zero = []
    model.reconstruct(y, zero_blocks=True, callback=lambda i, x: ps_zero.append(psnr(x, xt, peak)))
    target = max(ps_cg)

    def first(ps, ts):
        for v, t in zip(ps, ts):
            if v >= target:
                return t
        return None

    r = {"seed": seed, "target_psnr_db": round(target, 3),
         "cgls_best_iter": int(np.argmax(ps_cg)) + 1,
         "cgls_psnr_db": [round(v, 3) for v in ps_cg],
         "cgls_time_s": [round(v, 4) for v in t_cg],
         "learned_psnr_db": [round(v, 3) for v in ps_ln],
         "learned_time_s": [round(v, 4) for v in t_ln],
         "zero_block_psnr_db": [round(v, 3) for v in ps_zero],
         "fdk_psnr_db": round(ps_fdk, 3), "fdk_hann_psnr_db": round(ps_fdk_h, 3),
         "fdk_time_s": round(t_fdk, 4),
         "cgls_time_to_target_s": first(ps_cg, t_cg),
         "learned_time_to_target_s": first(ps_ln, t_ln)}
    log(f"[compare]   FDK {ps_fdk:.2f} dB, Hann {ps_fdk_h:.2f} dB ({t_fdk:.3f} s)")
    log(f"[compare]   learned {ps_ln[-1]:.2f} dB after {n} iterations ({t_ln[-1]:.3f} s); "
        f"zero-block net {ps_zero[-1]:.2f} dB; time to {target:.2f} dB: CGLS "
        f"{r['cgls_time_to_target_s']} s, learned {r['learned_time_to_target_s']} s")
    return r


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--phantoms", type=int, default=3)
    ap.add_argument("--cgls-iters", type=int, default=50)
    ap.add_argument("--I0", type=float, default=1e5)
    ap.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    S = Setup(args.weights)
    results = [compare_one(S, 50_000 + p, args.I0, args.cgls_iters,
                           log=lambda m: print(m, flush=True)) for p in range(args.phantoms)]
    net = S.net
    summary = {
        "workload": "256^3 @2 mm, 360 angles, 512^2 @0.8 mm, 115 mm offset; Poisson I0 "
                    f"{args.I0:g}; {args.phantoms} test phantoms",
        "cgls_best_psnr_db_mean": round(float(np.mean([r["target_psnr_db"] for r in results])), 3),
        "learned_psnr_db_mean": round(float(np.mean([r["learned_psnr_db"][-1] for r in results])), 3),
        "zero_block_psnr_db_mean": round(float(np.mean([r["zero_block_psnr_db"][-1]
                                                          for r in results])), 3),
        "fdk_psnr_db_mean": round(float(np.mean([r["fdk_psnr_db"] for r in results])), 3),
        "fdk_hann_psnr_db_mean": round(float(np.mean([r["fdk_hann_psnr_db"] for r in results])),
                                       3),
        "net": {"iterations": net.n_iter, "scales": list(net.scales), "init": net.init},
        "results": results,
    }
    print(json.dumps({k: v for k, v in summary.items() if k != "results"}), flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(summary, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
