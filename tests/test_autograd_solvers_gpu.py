"""Differentiable projector and GPU least-squares solvers (HIP path) against
the FP64 oracle.

Gradient of f(x) = 0.5 |A x - y|^2 (the Landweber term of Alg. 1): autograd
through the library's kernels vs the oracle's A^T (A x - y); the dot-product
identity through the autograd functions; central differences of f with
h = 1e-3 on 64 seeded voxels; second derivatives; CGLS and Landweber
iterates vs the oracle's FP64 solvers.
"""
import numpy as np
import pytest

from paper_2512_21180_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2512_21180_amd import autograd, cbct, solvers
    return torch, cbct, autograd, solvers


def _say(*a):
    print(*a, flush=True)


C4_BATCH = W.C4                              # 4 x 128^3 @2 mm, 180 angles, 256^2 @1.6 mm
C4_SMALL = W.cropped(W.C4, n_angles=18)      # oracle-sized version of the same geometry


def _phantoms(g, seeds):
    return np.stack([W.phantom_c1(g, s)[0] for s in seeds])


def test_gradient_matches_oracle(dev, oracle):
    torch, cbct, ag, _ = dev
    g = C4_SMALL
    _say("[grad] c4 (18 angles), batch 4")
    geo = cbct.Geometry(g)
    xt = _phantoms(g, range(4000, 4004))
    x0 = xt + 0.003 * W.rng(1).standard_normal(xt.shape)
    y = np.stack([oracle.forward(g, v) for v in xt]) + 1e-3 * W.rng(2).standard_normal(
        (4,) + W.sino_shape(g))
    x = torch.tensor(x0, dtype=torch.float32, device="cuda", requires_grad=True)
    yg = torch.tensor(y, dtype=torch.float32, device="cuda")
    f = 0.5 * ((ag.project(x, geo) - yg).double() ** 2).sum()
    f.backward()
    got = x.grad.double().cpu().numpy()
    ref = np.stack([oracle.adjoint(g, oracle.forward(g, x0[b]) - y[b]) for b in range(4)])
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _say(f"  gradient rel L2 {rel:.2e}")
    assert rel <= 1e-5


def test_gradient_full_c4_sampled_voxels_and_fd(dev, oracle):
    torch, cbct, ag, _ = dev
    g = C4_BATCH
    _say("[grad] c4 full size, batch 4: sampled voxels + central FD")
    geo = cbct.Geometry(g)
    xt = _phantoms(g, range(4000, 4004))
    x0 = (xt + 0.003 * W.rng(1).standard_normal(xt.shape)).astype(np.float32)
    xtg = torch.tensor(xt, dtype=torch.float32, device="cuda")
    yg = ag.project(xtg, geo) + 1e-3 * torch.randn((4,) + geo.sino_shape, device="cuda",
                                                    generator=torch.Generator("cuda").manual_seed(3))
    x = torch.tensor(x0, device="cuda", requires_grad=True)
    f = 0.5 * ((ag.project(x, geo) - yg).double() ** 2).sum()
    f.backward()
    grad = x.grad.detach()

    # oracle gradient at 48 sampled voxels of case 0
    r0 = (cbct.forward(geo, x.detach()[0].contiguous()) - yg[0]).double().cpu().numpy()
    rng = W.rng(4100)
    vox = rng.integers(0, x0[0].size, size=48)
    ref = oracle.adjoint_voxels(g, r0, vox)
    got = grad[0].double().cpu().numpy().ravel()[vox]
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _say(f"  sampled gradient rel L2 {rel:.2e}")
    assert rel <= 1e-5

    # central differences, h = 1e-3, on 64 voxels inside the field of view
    ws = cbct.dot_workspace(yg.numel(), "cuda")
    cell = torch.zeros(1, dtype=torch.float64, device="cuda")

    def fval(xx):
        r = (cbct.forward(geo, xx) - yg).contiguous()
        cbct.dot(r, r, ws, cell)
        return 0.5 * float(cell.item())

    h = 1e-3
    picks = []
    while len(picks) < 64:
        b = int(rng.integers(4))
        v = int(rng.integers(x0[0].size))
        if abs(float(grad[b].view(-1)[v])) > 0:
            picks.append((b, v))
    fd, an = [], []
    xx = x.detach().clone()
    for b, v in picks:
        old = float(xx[b].view(-1)[v])
        xx[b].view(-1)[v] = old + h
        fp = fval(xx)
        xx[b].view(-1)[v] = old - h
        fm = fval(xx)
        xx[b].view(-1)[v] = old
        fd.append((fp - fm) / (2 * h))
        an.append(float(grad[b].view(-1)[v]))
    fd, an = np.array(fd), np.array(an)
    err = np.linalg.norm(fd - an) / np.linalg.norm(an)
    _say(f"  central FD vs autograd rel L2 {err:.2e}")
    assert err <= 2e-3


def test_dot_product_and_second_derivative(dev):
    torch, cbct, ag, _ = dev
    g = C4_SMALL
    _say("[grad] dot product through autograd, double backward")
    geo = cbct.Geometry(g)
    x = torch.tensor(W.random_volume(g, 1), dtype=torch.float32, device="cuda", requires_grad=True)
    y = torch.tensor(W.random_sino(g, 2), dtype=torch.float32, device="cuda", requires_grad=True)
    Ax = ag.project(x, geo)
    ATy = ag.backproject(y, geo)
    lhs = float((Ax.double() * y.double()).sum())
    rhs = float((x.double() * ATy.double()).sum())
    assert abs(lhs - rhs) <= 1e-5 * float(Ax.double().norm() * y.double().norm())
    # d/dy <A^T y, v> = A v, exactly the forward kernel's output
    v = torch.tensor(W.random_volume(g, 3), dtype=torch.float32, device="cuda")
    (gy,) = torch.autograd.grad((ATy * v).sum(), y)
    assert torch.equal(gy, cbct.forward(geo, v))
    # Hessian-vector product of 0.5|Ax|^2 is A^T A v, through two levels
    (gx,) = torch.autograd.grad(0.5 * (ag.project(x, geo) ** 2).sum(), x, create_graph=True)
    (hv,) = torch.autograd.grad((gx * v).sum(), x)
    ref = cbct.adjoint(geo, cbct.forward(geo, v))
    assert torch.allclose(hv, ref, rtol=1e-5, atol=1e-6 * float(ref.abs().max()))


def test_dot_is_deterministic_and_exact(dev):
    torch, cbct, _, _ = dev
    _say("[blas] dot")
    gen = torch.Generator("cuda").manual_seed(5)
    for n in (1, 7, 1000, 3_000_001):
        a = torch.randn(n, device="cuda", generator=gen)
        b = torch.randn(n, device="cuda", generator=gen)
        ws = cbct.dot_workspace(n, "cuda")
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        r1 = float(cbct.dot(a, b, ws, out).item())
        r2 = float(cbct.dot(a, b, ws, out).item())
        ref = float(np.dot(a.double().cpu().numpy(), b.double().cpu().numpy()))
        assert r1 == r2
        assert abs(r1 - ref) <= 1e-12 * max(1.0, float(a.double().norm() * b.double().norm()))


def test_cgls_and_landweber_match_oracle(dev, oracle):
    torch, cbct, _, solvers = dev
    g = W.cropped(W.C1, n_angles=24, n=48)
    _say("[solve] CGLS / Landweber, c1-style, 24 angles, 48^3")
    geo = cbct.Geometry(g)
    xt, _ = W.phantom_c1(g, 7)
    y = oracle.forward(g, xt) + 1e-3 * W.rng(8).standard_normal(W.sino_shape(g))
    yg = torch.tensor(y, dtype=torch.float32, device="cuda")
    its = {}
    xg = solvers.cgls(geo, yg, 8, callback=lambda k, x: its.__setitem__(k, x.double().cpu().numpy()))
    ref_its = {}
    oracle.cgls(g, y, 8, callback=lambda k, x: ref_its.__setitem__(k, x.copy()))
    for k in (1, 4, 8):
        rel = np.linalg.norm(its[k] - ref_its[k]) / np.linalg.norm(ref_its[k])
        _say(f"  CGLS iterate {k}: rel L2 {rel:.2e}")
        assert rel <= 1e-4
    assert xg.shape == tuple(W.vol_shape(g))
    x0 = W.rng(12).standard_normal(W.vol_shape(g))
    L = oracle.opnorm(g, iters=30, x0=x0)
    Lg = solvers.opnorm(geo, iters=30, x0=torch.tensor(x0, dtype=torch.float32, device="cuda"))
    assert abs(Lg - L) <= 1e-5 * L
    omega = 1.0 / L ** 2
    xl = solvers.landweber(geo, yg, 5, omega).double().cpu().numpy()
    xr = oracle.landweber(g, y, 5, omega)
    rel = np.linalg.norm(xl - xr) / np.linalg.norm(xr)
    _say(f"  Landweber(5) rel L2 {rel:.2e}")
    assert rel <= 1e-5
