"""Mixed-precision storage and the batched persistent launch (HIP path).

BF16/FP16 storage with FP32 accumulation: for non-negative data every output
element obeys |out - ref| <= (u_in + u_out + u_in u_out + 2^-20) |ref| + a_out
against the FP64 oracle on the unrounded input, with unit roundoff u = 2^-8
(BF16) or 2^-11 (FP16) for each rounded buffer (u = 0 for FP32) -- rounding
the input moves each term of a non-negative sum by at most u_in relatively,
FP32 sums of a few hundred terms add far less than 2^-20, the final rounding
adds u_out of the rounded-input result, and a_out = 2^-25 covers FP16
subnormal outputs; a further 2e-5 of the largest magnitude is the FP32 path's
own element bound (FP32 ray geometry), which only grazing rays with tiny
values ever approach.
Per-case errors are printed.  The twelve heterogeneous cases run in one
batched call whose results equal the single-case calls bit for bit.
"""
import numpy as np
import pytest

from paper_2512_21180_amd import workloads as W

pytestmark = pytest.mark.gpu

U = {"f32": 0.0, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2512_21180_amd import cbct
    tmap = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
    return torch, cbct, tmap


# FP16 subnormals (below 2^-14) are spaced 2^-24 apart: rounding there adds
# up to 2^-25 absolute, per rounded buffer
ABS = {"f32": 0.0, "bf16": 0.0, "f16": 2.0 ** -25}


# the FP32 path's own element bound against the oracle (test_parity_gpu):
# FP32 ray geometry moves sample positions by ~1e-5 voxel, which matters only
# for grazing rays whose values are tiny
GEO = 2e-5


def _bound(ref, vt, st, scale):
    rel = U[vt] + U[st] + U[vt] * U[st] + 2.0 ** -20
    return rel * np.abs(ref) + ABS[st] + GEO * scale + 1e-30


def _check(got, ref, vt, st, what, scale=None):
    scale = float(np.max(np.abs(ref))) if scale is None else scale
    b = _bound(ref, vt, st, scale)
    ratio = np.abs(got - ref) / b
    k = int(np.argmax(ratio))
    rel = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    print(f"  {what}: rel L2 {rel:.3e}, worst error/bound {ratio.flat[k]:.3f} "
          f"(got {got.flat[k]:.6g}, ref {ref.flat[k]:.6g})", flush=True)
    assert ratio.flat[k] <= 1.0, what


@pytest.mark.parametrize("vt,st", [("bf16", "bf16"), ("f16", "f16"), ("bf16", "f32"),
                                   ("f32", "bf16")])
def test_forward_storage_bounds(dev, oracle, vt, st):
    torch, cbct, tmap = dev
    g = W.cropped(W.C2, n_angles=8, nv=48, n=128)
    print(f"[mixed] forward {vt}->{st}", flush=True)
    geo = cbct.Geometry(g)
    x, _, _ = W.phantom_c2(g, 2025)
    xg = torch.tensor(x, dtype=torch.float32, device="cuda").to(tmap[vt])
    y = cbct.forward(geo, xg, out_dtype=tmap[st]).double().cpu().numpy()
    ref = oracle.forward(g, x)
    _check(y, ref, vt, st, f"forward {vt}->{st}")
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    print(f"  rel L2 {rel:.2e}", flush=True)


@pytest.mark.parametrize("st,vt", [("bf16", "bf16"), ("f16", "f16")])
def test_adjoint_storage_bounds(dev, oracle, st, vt):
    torch, cbct, tmap = dev
    g = W.cropped(W.C2, n_angles=8, nv=48, n=128)
    print(f"[mixed] adjoint {st}->{vt}", flush=True)
    geo = cbct.Geometry(g)
    y = np.abs(W.random_sino(g, 3))
    yg = torch.tensor(y, dtype=torch.float32, device="cuda").to(tmap[st])
    x = cbct.adjoint(geo, yg, out_dtype=tmap[vt]).double().cpu().numpy()
    ref = oracle.adjoint(g, y)
    # the adjoint's input rounding error is bounded on the absolute values:
    # every term is non-negative, so the relative bound applies as is
    _check(x, ref, st, vt, f"adjoint {st}->{vt}")


@pytest.mark.parametrize("st,vt", [("bf16", "bf16"), ("f16", "f16")])
def test_adjoint_storage_bounds_tall_windows(dev, oracle, st, vt):
    """The clinical panel over a 160^3 volume: adjoint windows of at least 96
    rows, which take the gather variant whose staging batches stay inside
    the window's columns, with 16-bit sinogram and volume."""
    torch, cbct, tmap = dev
    g = W.cropped(W.C2, n_angles=3, n=160)
    print(f"[mixed] adjoint {st}->{vt}, tall windows", flush=True)
    geo = cbct.Geometry(g)
    y = np.abs(W.random_sino(g, 7))
    yg = torch.tensor(y, dtype=torch.float32, device="cuda").to(tmap[st])
    x = cbct.adjoint(geo, yg, out_dtype=tmap[vt]).double().cpu().numpy()
    _check(x, oracle.adjoint(g, y), st, vt, f"adjoint {st}->{vt} (tall windows)")


def test_c3_batch_bf16(dev, oracle):
    """Twelve cases (96^3..256^3, 2-4 mm, 90-360 angles, 256^2..512^2 panels)
    in BF16 storage: one batched call each way, bitwise equal to single
    calls, and per case within the BF16 bound on sampled rays and voxels."""
    torch, cbct, tmap = dev
    gs = W.c3_geometries()
    print("[c3] building 12 cases", flush=True)
    geos = [cbct.Geometry(g) for g in gs]
    xs_host = [W.phantom_c3(g, 1000 + i)[0] for i, g in enumerate(gs)]
    xs = [torch.tensor(x, dtype=torch.float32, device="cuda").to(torch.bfloat16) for x in xs_host]
    print("[c3] batch forward", flush=True)
    ys = cbct.batch_forward(geos, xs)
    torch.cuda.synchronize()
    print("[c3] batch adjoint", flush=True)
    bs = cbct.batch_adjoint(geos, ys)
    torch.cuda.synchronize()
    rng = W.rng(31)
    for i, (g, geo, x, y, b) in enumerate(zip(gs, geos, xs, ys, bs)):
        assert torch.equal(y, cbct.forward(geo, x)), i
        assert torch.equal(b, cbct.adjoint(geo, y)), i
        rays = rng.integers(0, y.numel(), size=600)
        ref = oracle.forward_rays(g, xs_host[i], rays)
        got = y.view(-1)[torch.tensor(rays, device="cuda")].double().cpu().numpy()
        _check(got, ref, "bf16", "bf16", f"case {i} forward")
        vox = rng.integers(0, b.numel(), size=40)
        yr = y.double().cpu().numpy()
        refa = oracle.adjoint_voxels(g, yr, vox)
        gota = b.view(-1)[torch.tensor(vox, device="cuda")].double().cpu().numpy()
        _check(gota, refa, "f32", "bf16", f"case {i} adjoint")
        e_f = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        e_a = np.linalg.norm(gota - refa) / max(np.linalg.norm(refa), 1e-30)
        print(f"  case {i}: forward rel L2 {e_f:.2e}, adjoint rel L2 {e_a:.2e}", flush=True)


# one geometry per launch plan: tiled forward and bricked adjoint, the
# one-thread-per-ray forward, the one-thread-per-voxel adjoint
PLANS = {
    "tiled": W.cropped(W.C2, n_angles=6, nv=40, n=96),
    "fallback_fwd": W.geometry(8, 48, 40, 4.0, 4.0, 40, 40, 40, 0.25),
    "fallback_adj": W.geometry(8, 300, 200, 0.5, 0.5, 16, 16, 16, 16.0),
}


@pytest.mark.parametrize("plan", sorted(PLANS))
def test_bf16_f16_pair_on_every_plan(dev, oracle, plan):
    """Every storage pair is accepted whatever kernels a geometry's plan
    selects: BF16 volume -> FP16 sinogram and FP16 sinogram -> BF16 volume
    run on the tiled/bricked and on the one-thread-per-output kernels, each
    within the storage bound against the oracle."""
    torch, cbct, tmap = dev
    g = PLANS[plan]
    print(f"[mixed] bf16<->f16 on the {plan} plan", flush=True)
    geo = cbct.Geometry(g)
    info = geo.plan_info()
    print(f"  forward tiled {info['fwd_tiled']}, adjoint bricked {info['adj_bricked']}",
          flush=True)
    x = W.phantom_c1(g, 3)[0] + 0.01 * np.abs(W.random_volume(g, 4))
    xg = torch.tensor(x, dtype=torch.float32, device="cuda").to(torch.bfloat16)
    y = cbct.forward(geo, xg, out_dtype=torch.float16).double().cpu().numpy()
    _check(y, oracle.forward(g, x), "bf16", "f16", f"{plan} forward bf16->f16")
    s = np.abs(W.random_sino(g, 5))
    sg = torch.tensor(s, dtype=torch.float32, device="cuda").to(torch.float16)
    b = cbct.adjoint(geo, sg, out_dtype=torch.bfloat16).double().cpu().numpy()
    _check(b, oracle.adjoint(g, s), "f16", "bf16", f"{plan} adjoint f16->bf16")
