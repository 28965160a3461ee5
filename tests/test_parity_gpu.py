"""GPU parity of the HIP projector pair against the FP64 oracle (FP32 path).

Bar (FP32 storage and arithmetic): relative L2 error <= 1e-5 against the
oracle, plus an element-wise bound of 2e-5 of the largest oracle magnitude;
bitwise-identical repeats; identical single-case and batched results.
"""
import numpy as np
import pytest

from paper_2512_21180_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_L2 = 1e-5
ELEM = 2e-5


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2512_21180_amd import cbct
    return torch, cbct


def _say(*a):
    print(*a, flush=True)


def _fwd(dev, g, x):
    torch, cbct = dev
    geo = cbct.Geometry(g)
    xg = torch.tensor(x, dtype=torch.float32, device="cuda")
    y = cbct.forward(geo, xg)
    torch.cuda.synchronize()
    return geo, y.double().cpu().numpy()


def _adj(dev, g, y):
    torch, cbct = dev
    geo = cbct.Geometry(g)
    yg = torch.tensor(y, dtype=torch.float32, device="cuda")
    x = cbct.adjoint(geo, yg)
    torch.cuda.synchronize()
    return geo, x.double().cpu().numpy()


def _close(got, ref, what):
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    el = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    _say(f"  {what}: rel L2 {rel:.2e}, max elem {el:.2e}")
    assert rel <= REL_L2, (what, rel)
    assert el <= ELEM, (what, el)


# odd sizes: ragged launch tails, both sampling axes, offsets on both axes
RAGGED = W.geometry(20, 37, 29, 3.3, 2.9, 13, 17, 11, 4.0, vy=3.5, vz=4.5, off_u=31.0,
                    off_v=-7.0, origin=(5.0, -3.0, 2.0))
# plans outside the tiled kernels' LDS limits run the one-thread-per-output kernels:
# fine voxels under coarse pixels overflow the forward box, coarse voxels under
# fine pixels overflow the adjoint window
FINE_VOX = W.geometry(8, 48, 40, 4.0, 4.0, 40, 40, 40, 0.25)
COARSE_VOX = W.geometry(8, 300, 200, 0.5, 0.5, 16, 16, 16, 16.0)
# 4 and 5 mm voxels through 0.8 mm pixels: the adjoint's panel window is too
# tall for 16-voxel bricks (and the volumes too small for two bricks per CU),
# the plan takes 4-voxel bricks; 64^3 (c1) takes 8-voxel bricks (512 of them)
SHORT_BRICKS_2 = W.geometry(10, 150, 170, 0.8, 0.8, 20, 18, 23, 4.0, off_u=20.0)
SHORT_BRICKS_1 = W.geometry(10, 150, 170, 0.8, 0.8, 20, 18, 23, 5.0, off_u=20.0)
# 2 mm pixels over 1 mm voxels: 64 columns of rays spread over more than 64
# voxels, the forward takes 32-column tiles (two row groups per wave)
NARROW_TILES = W.geometry(12, 70, 50, 2.0, 2.0, 40, 36, 30, 1.0, off_u=10.0)
# 300 planes along x: the forward's tiles sweep more planes than one table
# of plane boxes holds (256), so the table is refilled mid-sweep
LONG_SWEEP = W.geometry(6, 48, 24, 1.6, 1.6, 300, 40, 20, 1.0, off_u=5.0)
# a 40000-column panel whose volume projects near column 35000: the
# adjoint's window columns (packed 16 + 16 bits) lie above 32767
WIDE_PANEL = W.geometry(3, 40000, 16, 0.01, 0.01, 16, 16, 8, 0.05, off_u=-150.0)
# a 9 mm slab under a 90 mm panel: most rays pass above or below the volume,
# so the forward's staged boxes reach past both its ends (read as zeros)
THIN_SLAB = W.geometry(10, 60, 90, 1.0, 1.0, 30, 26, 6, 1.5, off_u=4.0, off_v=3.0)
# the clinical panel over a 160^3 volume at 2 mm: adjoint windows of at least
# 96 rows, whose staging batches stay inside the window's columns
TALL_WINDOWS = W.cropped(W.C2, n_angles=3, n=160)
CASES = {
    "tall_windows": TALL_WINDOWS,
    "thin_slab": THIN_SLAB,
    "fallback_fwd": FINE_VOX,
    "fallback_adj": COARSE_VOX,
    "ragged": RAGGED,
    "c1": W.C1,
    "c2_crop": W.cropped(W.C2, n_angles=12, nv=64),
    "c4_crop": W.cropped(W.C4, n_angles=16),
    "short_bricks_8": SHORT_BRICKS_2,
    "short_bricks_4": SHORT_BRICKS_1,
    "narrow_tiles": NARROW_TILES,
    "long_sweep": LONG_SWEEP,
    "wide_panel": WIDE_PANEL,
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_forward_matches_oracle(dev, oracle, name):
    g = CASES[name]
    _say(f"[forward] {name}")
    x = W.phantom_c1(g, 3)[0] + 0.01 * W.random_volume(g, 4)
    geo, got = _fwd(dev, g, x)
    _close(got, oracle.forward(g, x), f"forward {name}")
    assert geo.sample_count() == oracle.sample_count(g)


@pytest.mark.parametrize("name", sorted(CASES))
def test_adjoint_matches_oracle(dev, oracle, name):
    g = CASES[name]
    _say(f"[adjoint] {name}")
    y = np.abs(W.random_sino(g, 5))
    _, got = _adj(dev, g, y)
    _close(got, oracle.adjoint(g, y), f"adjoint {name}")


def test_c2_full_size_sampled(dev, oracle):
    """Full clinical size: sampled rays and voxels computed one by one."""
    g = W.C2
    _say("[c2 full] phantom")
    x, _, _ = W.phantom_c2(g, 2025)
    geo, y = _fwd(dev, g, x)
    r = W.rng(77)
    rays = r.integers(0, y.size, size=4000)
    ref = oracle.forward_rays(g, x, rays)
    got = y.ravel()[rays]
    _close(got, ref, "c2 forward (4000 rays)")
    s = np.abs(W.random_sino(g, 6)).astype(np.float32)
    _, xa = _adj(dev, g, s)
    vox = r.integers(0, xa.size, size=300)
    refa = oracle.adjoint_voxels(g, s.astype(np.float64), vox)
    _close(xa.ravel()[vox], refa, "c2 adjoint (300 voxels)")


def test_dot_product_identity_gpu(dev):
    g = CASES["c2_crop"]
    _say("[dot] c2_crop")
    x = W.random_volume(g, 10)
    y = W.random_sino(g, 11)
    _, Ax = _fwd(dev, g, x)
    _, ATy = _adj(dev, g, y)
    lhs, rhs = float(np.vdot(Ax, y)), float(np.vdot(x, ATy))
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_multichannel_equals_per_channel(dev):
    torch, cbct = dev
    g = RAGGED
    _say("[channels] ragged x3")
    geo = cbct.Geometry(g)
    xs = torch.tensor(np.stack([W.random_volume(g, s) for s in range(3)]), dtype=torch.float32,
                      device="cuda")
    ys = cbct.forward(geo, xs)
    for c in range(3):
        assert torch.equal(ys[c], cbct.forward(geo, xs[c].contiguous()))
    back = cbct.adjoint(geo, ys)
    for c in range(3):
        assert torch.equal(back[c], cbct.adjoint(geo, ys[c].contiguous()))


def test_bitwise_repeatable(dev):
    torch, cbct = dev
    g = CASES["c2_crop"]
    _say("[repeat] c2_crop")
    geo = cbct.Geometry(g)
    x = torch.tensor(W.random_volume(g, 1), dtype=torch.float32, device="cuda")
    y0 = cbct.forward(geo, x)
    a0 = cbct.adjoint(geo, y0)
    for _ in range(2):
        assert torch.equal(cbct.forward(geo, x), y0)
        assert torch.equal(cbct.adjoint(geo, y0), a0)


def test_batch_equals_single(dev):
    torch, cbct = dev
    gs = [RAGGED, CASES["c2_crop"], W.cropped(W.C1, n_angles=7), SHORT_BRICKS_1, SHORT_BRICKS_2,
          NARROW_TILES]
    _say("[batch] 6 cases")
    geos = [cbct.Geometry(g) for g in gs]
    xs = [torch.tensor(W.random_volume(g, i), dtype=torch.float32, device="cuda")
          for i, g in enumerate(gs)]
    ys = cbct.batch_forward(geos, xs)
    for geo, x, y in zip(geos, xs, ys):
        assert torch.equal(y, cbct.forward(geo, x))
    bs = cbct.batch_adjoint(geos, ys)
    for geo, y, b in zip(geos, ys, bs):
        assert torch.equal(b, cbct.adjoint(geo, y))


def test_fallback_cases_take_the_simple_kernels(dev):
    torch, cbct = dev
    assert cbct.Geometry(FINE_VOX).plan_info()["fwd_tiled"] == 0
    assert cbct.Geometry(COARSE_VOX).plan_info()["adj_bricked"] == 0
    assert cbct.Geometry(W.C2).plan_info()["fwd_tiled"] == 1
    assert cbct.Geometry(W.C2).plan_info()["adj_bricked"] == 1
    assert cbct.Geometry(W.C2).plan_info()["adj_kv"] == 4
    assert cbct.Geometry(W.C1).plan_info()["adj_kv"] == 2
    assert cbct.Geometry(SHORT_BRICKS_2).plan_info()["adj_kv"] == 1
    assert cbct.Geometry(SHORT_BRICKS_1).plan_info()["adj_kv"] == 1
    assert cbct.Geometry(W.C2).plan_info()["fwd_tile_cols"] == 64
    assert cbct.Geometry(NARROW_TILES).plan_info()["fwd_tile_cols"] == 32
