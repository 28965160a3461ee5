"""GPU least-squares solvers on the projector pair: CGLS and Landweber.

Landweber iterates x <- x - omega A^T (A x - y); its update direction is the
data-consistency (Landweber) term of arXiv 2512.21180, Alg. 1.  CGLS is the
conjugate-gradient method on the normal equations A^T A x = A^T y with the
same operators.  Every vector operation runs in the library's HIP kernels;
the iteration scalars stay on the device, so no iteration synchronises with
the host.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import cbct


def cgls(geom: cbct.Geometry, y: torch.Tensor, iters: int, x0: torch.Tensor | None = None,
         callback=None) -> torch.Tensor:
    """Unregularised CGLS from x0 (default 0).  callback(k, x) runs after
    iteration k (it may synchronise; the solver itself does not)."""
    dev = y.device
    x = torch.zeros(geom.vol_shape, dtype=torch.float32, device=dev) if x0 is None \
        else x0.detach().to(torch.float32).contiguous().clone()
    r = y.detach().to(torch.float32).contiguous().clone()
    q = torch.empty_like(r)
    if x0 is not None:
        cbct.forward(geom, x, out=q)
        cbct.axpby(r, 1.0, r, -1.0, q)
    s = cbct.adjoint(geom, r)
    p = s.clone()
    ws = cbct.dot_workspace(max(r.numel(), s.numel()), dev)
    gam = torch.zeros(2, dtype=torch.float64, device=dev)    # two slots, alternating
    qq = torch.zeros(1, dtype=torch.float64, device=dev)
    cbct.dot(s, s, ws, gam[0:1])
    cur = 0
    for k in range(iters):
        cbct.forward(geom, p, out=q)
        cbct.dot(q, q, ws, qq)
        g = gam[cur:cur + 1]
        cbct.axpy_ratio(x, p, g, qq, 1.0)
        cbct.axpy_ratio(r, q, g, qq, -1.0)
        cbct.adjoint(geom, r, out=s)
        gn = gam[1 - cur:2 - cur]
        cbct.dot(s, s, ws, gn)
        cbct.xpay_ratio(p, s, gn, g)
        cur = 1 - cur
        if callback is not None:
            callback(k + 1, x)
    return x


def opnorm(geom: cbct.Geometry, iters: int = 50, seed: int = 0,
           x0: torch.Tensor | None = None) -> float:
    """||A||_2 by power iteration on A^T A (FP32 operators, FP64 norms),
    from x0 or a seeded Gaussian start."""
    if x0 is None:
        gen = torch.Generator(device="cpu").manual_seed(seed)
        x = torch.randn(geom.vol_shape, generator=gen).to(geom.device)
    else:
        x = x0.detach().to(device=geom.device, dtype=torch.float32).contiguous().clone()
    ws = cbct.dot_workspace(max(x.numel(), int(np.prod(geom.sino_shape))), x.device)
    cells = torch.zeros(2, dtype=torch.float64, device=x.device)
    q = torch.empty(geom.sino_shape, dtype=torch.float32, device=x.device)
    z = torch.empty_like(x)
    lam = 0.0
    for _ in range(iters):
        cbct.dot(x, x, ws, cells[0:1])
        inv = 1.0 / math.sqrt(float(cells[0]))
        cbct.axpby(x, inv, x, 0.0, x)                 # x <- x / |x|
        cbct.forward(geom, x, out=q)
        cbct.adjoint(geom, q, out=z)
        cbct.dot(x, z, ws, cells[1:2])                # Rayleigh quotient of A^T A
        lam = float(cells[1])
        x, z = z, x
    return lam ** 0.5


def landweber(geom: cbct.Geometry, y: torch.Tensor, iters: int, omega: float,
              x0: torch.Tensor | None = None, callback=None) -> torch.Tensor:
    """x <- x - omega A^T(A x - y), omega < 2 / ||A||^2 for convergence."""
    dev = y.device
    x = torch.zeros(geom.vol_shape, dtype=torch.float32, device=dev) if x0 is None \
        else x0.detach().to(torch.float32).contiguous().clone()
    y = y.detach().to(torch.float32).contiguous()
    r = torch.empty_like(y)
    g = torch.empty_like(x)
    for k in range(iters):
        cbct.forward(geom, x, out=r)
        cbct.axpby(r, 1.0, r, -1.0, y)
        cbct.adjoint(geom, r, out=g)
        cbct.axpby(x, 1.0, x, -omega, g)
        if callback is not None:
            callback(k + 1, x)
    return x
