"""GPU tests of the multichannel forward (channel stacks that share one
geometry, as Alg. 1 applies the projector to [p2, x]): every channel bitwise
equal to a single-channel call, for stacks through cbct_forward and for
batches whose cases share a geometry handle, on both LDS layouts (41 x 20
boxes, chunks of four channels: small clinical-pitch cases; 65 x 32 boxes,
chunks of two: the 64^3 @4 mm case), 32-column tiles, and stacks cut into
chunks (7 channels: 4 + 2 + 1); one stack against the FP64 oracle."""
import numpy as np
import pytest

from paper_2512_21180_amd import workloads as W

pytestmark = pytest.mark.gpu

RAGGED = W.geometry(20, 37, 29, 3.3, 2.9, 13, 17, 11, 4.0, vy=3.5, vz=4.5, off_u=31.0,
                    off_v=-7.0, origin=(5.0, -3.0, 2.0))
CASES = {
    "crop_c2": W.cropped(W.C2, n_angles=24, nu=160, nv=96, n=64),   # 41 x 20 layout
    "ragged": RAGGED,                                                 # 41 x 20, odd sizes
    "c1": W.C1,                                                       # 65 x 32 layout
    # boxes past both ends of a 6-plane slab
    "thin_slab": W.geometry(10, 60, 90, 1.0, 1.0, 30, 26, 6, 1.5, off_u=4.0, off_v=3.0),
}


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


def _vols(torch, g, C, seed):
    x = np.stack([W.random_volume(g, seed + c) for c in range(C)]).astype(np.float32)
    return torch.tensor(x, device="cuda")


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("C", [2, 3, 4, 5, 7])
def test_stack_equals_single_channels(dev, name, C):
    torch, cbct = dev
    g = CASES[name]
    _say(f"  stack {name} C={C}")
    geo = cbct.Geometry(g)
    x = _vols(torch, g, C, 100 + C)
    y = cbct.forward(geo, x)
    ys = torch.stack([cbct.forward(geo, x[c]) for c in range(C)])
    torch.cuda.synchronize()
    assert torch.equal(y, ys)
    assert float(y.abs().max()) > 0


def test_stack_on_32_column_tiles(dev):
    """1.6 mm pixels over 2 mm voxels at 256^3: 32-column tiles, 65 x 32 boxes."""
    torch, cbct = dev
    g = W.c3_geometries()[7]
    geo = cbct.Geometry(g)
    assert geo.plan_info()["fwd_tile_cols"] == 32
    x = _vols(torch, g, 3, 7)
    y = cbct.forward(geo, x)
    ys = torch.stack([cbct.forward(geo, x[c]) for c in range(3)])
    torch.cuda.synchronize()
    assert torch.equal(y, ys)


def test_batch_groups_equal_single_cases(dev):
    """Cases of two geometries interleaved: each handle's cases run as
    channel groups (five of one: 4 + 1, three of the other: 2 + 1), results
    per case bitwise equal to one call each."""
    torch, cbct = dev
    ga, gb = cbct.Geometry(CASES["crop_c2"]), cbct.Geometry(CASES["c1"])
    order = [ga, ga, gb, ga, gb, ga, gb, ga]
    vols = [_vols(torch, g.params, 1, 300 + i)[0] for i, g in enumerate(order)]
    outs = cbct.batch_forward(order, vols)
    ref = [cbct.forward(g, v) for g, v in zip(order, vols)]
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, ref)):
        assert torch.equal(o, r), i


def test_batch_of_bf16_cases_unchanged(dev):
    """16-bit storage takes the single-channel batch (no channel groups)."""
    torch, cbct = dev
    geo = cbct.Geometry(CASES["crop_c2"])
    vols = [_vols(torch, geo.params, 1, 400 + i)[0].to(torch.bfloat16) for i in range(3)]
    outs = cbct.batch_forward([geo] * 3, vols)
    ref = [cbct.forward(geo, v) for v in vols]
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert torch.equal(o, r)


def test_stack_matches_oracle(dev, oracle):
    torch, cbct = dev
    g = CASES["crop_c2"]
    geo = cbct.Geometry(g)
    x = _vols(torch, g, 5, 500)
    y = cbct.forward(geo, x)
    torch.cuda.synchronize()
    got = y.double().cpu().numpy()
    xh = x.double().cpu().numpy()
    for c in (0, 4):
        ref = oracle.forward(g, xh[c])
        rel = np.linalg.norm(got[c] - ref) / np.linalg.norm(ref)
        el = np.max(np.abs(got[c] - ref)) / np.max(np.abs(ref))
        _say(f"  channel {c}: rel L2 {rel:.2e}, max elem {el:.2e}")
        assert rel <= 1e-5 and el <= 2e-5
