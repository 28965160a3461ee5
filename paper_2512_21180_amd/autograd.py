"""Differentiable projector: torch.autograd.Functions whose derivatives are
the library's own kernels.

The forward projector's backward is the adjoint kernel and the adjoint's
backward is the forward kernel, so gradients of data terms such as
0.5 ||A x - y||^2 (whose gradient A^T (A x - y) is the Landweber term of
arXiv 2512.21180, Alg. 1) run entirely on the hand-written HIP path, to any
order.
"""
from __future__ import annotations

import torch

from . import cbct


class ProjectFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, geom):
        ctx.geom = geom
        return cbct.forward(geom, x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return BackprojectFn.apply(g.contiguous(), ctx.geom), None


class BackprojectFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, geom):
        ctx.geom = geom
        return cbct.adjoint(geom, y.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ProjectFn.apply(g.contiguous(), ctx.geom), None


def project(x: torch.Tensor, geom: cbct.Geometry) -> torch.Tensor:
    """A x for x of shape [..., nz, ny, nx] (leading dims are channels)."""
    return ProjectFn.apply(x, geom)


def backproject(y: torch.Tensor, geom: cbct.Geometry) -> torch.Tensor:
    """A^T y for y of shape [..., n_angles, nv, nu]."""
    return BackprojectFn.apply(y, geom)


class Projector(torch.nn.Module):
    """Module wrapper: forward(x) = A x, differentiable through A^T."""

    def __init__(self, geom: cbct.Geometry):
        super().__init__()
        self.geom = geom

    def forward(self, x):
        return project(x, self.geom)

    def adjoint(self, y):
        return backproject(y, self.geom)
