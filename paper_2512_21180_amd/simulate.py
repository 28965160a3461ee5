"""Projection-data simulator on the GPU: seeded phantoms (host), line
integrals by the library's forward projector, and noise by its Philox-based
kernels (arXiv 2512.21180, Sec. 2.2 noisy primary model, monochromatic form;
Sec. 2.4 negative-log normalisation)."""
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
