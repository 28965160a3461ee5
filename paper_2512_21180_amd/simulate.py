"""Projection-data simulator on the GPU: seeded phantoms (host), line
integrals by the library's forward projector, and noise by its Philox-based
kernels (arXiv 2512.21180, Sec. 2.2 noisy primary model, monochromatic and
polychromatic water-bone forms; Sec. 2.4 negative-log normalisation)."""
from __future__ import annotations

import torch

from . import cbct


def noisy_sinogram(geom: cbct.Geometry, x: torch.Tensor, I0: float, seed: int,
                   stream_id: int = 0) -> torch.Tensor:
    """-log(min(max(Poisson(I0 exp(-A x)), 1) / I0, 1)) for x on the device."""
    p = cbct.forward(geom, x.contiguous())
    return cbct.sim_poisson_log(p, I0, seed, stream_id, out=p)


def gaussian_sinogram(geom: cbct.Geometry, x: torch.Tensor, sigma: float, seed: int,
                      stream_id: int = 0) -> torch.Tensor:
    """A x + sigma z, z standard normal."""
    p = cbct.forward(geom, x.contiguous())
    return cbct.sim_gaussian(p, sigma, seed, stream_id, out=p)


def poly_primary(geom: cbct.Geometry, hu: torch.Tensor, mu_w, mu_b, resp, I0: torch.Tensor,
                 seed: int, stream_id: int = 0):
    """Polychromatic primary projections of a CT volume in HU (Sec. 2.2):
    water/bone densities, their two line integrals in one two-channel
    forward projection, then per-bin Poisson counts weighted by the detector
    response and the normalised negative log (Sec. 2.4).  Returns
    (y, [P(rho_w), P(rho_b)])."""
    rho = cbct.water_bone(hu.contiguous())
    p = cbct.forward(geom, rho)
    y = cbct.sim_poly(p[0], p[1], mu_w, mu_b, resp, I0, seed, stream_id)
    return y, p
