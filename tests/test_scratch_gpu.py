"""GPU tests of the library-owned device buffer and of split launches.

The bricked adjoint (its ray-length pre-pass) and the multichannel forward
(its packed channel volume) stage through one device buffer per device that
the library owns: it grows when a call needs more, and calls on different
streams are ordered on it.  Batches run as several launches (at most 16
single cases, or 8 channel groups, per launch).  Every result here is
compared bitwise with the same operator applied in single calls on the
default stream.
"""
import numpy as np
import pytest

from paper_2512_21180_amd import workloads as W

pytestmark = pytest.mark.gpu

# small clinical-pitch crops (41 x 20 forward boxes: channel groups of four)
SMALL = [W.cropped(W.C2, n_angles=na, nu=nu, nv=nv, n=n)
         for (na, nu, nv, n) in [(6, 96, 40, 32), (9, 128, 48, 40), (5, 160, 64, 48),
                                 (7, 112, 32, 36)]]
FINE_VOX = W.geometry(8, 48, 40, 4.0, 4.0, 40, 40, 40, 0.25)      # one-thread-per-ray forward
COARSE_VOX = W.geometry(8, 300, 200, 0.5, 0.5, 16, 16, 16, 16.0)  # one-thread-per-voxel adjoint


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


def _vol(torch, g, seed, C=None):
    if C is None:
        return torch.tensor(W.random_volume(g, seed), dtype=torch.float32, device="cuda")
    x = np.stack([W.random_volume(g, seed + c) for c in range(C)]).astype(np.float32)
    return torch.tensor(x, device="cuda")


def _sino(torch, g, seed, C=None):
    if C is None:
        return torch.tensor(W.random_sino(g, seed), dtype=torch.float32, device="cuda")
    y = np.stack([W.random_sino(g, seed + c) for c in range(C)]).astype(np.float32)
    return torch.tensor(y, device="cuda")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batch_of_twenty_distinct_cases(dev, dtype):
    """20 cases with their own handles (two launches: 16 + 4), one of them on
    each fallback kernel, both directions."""
    torch, cbct = dev
    t = torch.float32 if dtype == "f32" else torch.bfloat16
    gs = [SMALL[i % len(SMALL)] for i in range(18)]
    gs.insert(5, FINE_VOX)
    gs.insert(13, COARSE_VOX)
    _say(f"[batch] 20 distinct handles, {dtype}")
    geos = [cbct.Geometry(g) for g in gs]
    xs = [_vol(torch, g, 10 + i).to(t) for i, g in enumerate(gs)]
    ys = cbct.batch_forward(geos, xs)
    for i, (geo, x, y) in enumerate(zip(geos, xs, ys)):
        assert torch.equal(y, cbct.forward(geo, x)), i
    bs = cbct.batch_adjoint(geos, ys)
    for i, (geo, y, b) in enumerate(zip(geos, ys, bs)):
        assert torch.equal(b, cbct.adjoint(geo, y)), i
    torch.cuda.synchronize()


def test_batch_of_many_channel_groups(dev):
    """32 FP32 cases: ten handles with two cases each (ten groups of two:
    launches of 8 + 2 groups) and three handles with four cases each (three
    groups of four), interleaved."""
    torch, cbct = dev
    pairs = [cbct.Geometry(SMALL[i % len(SMALL)]) for i in range(10)]
    quads = [cbct.Geometry(SMALL[(i + 1) % len(SMALL)]) for i in range(3)]
    order = []
    for k in range(4):
        order += [pairs[i] for i in range(10) if k < 2] + [quads[i] for i in range(3)]
    assert len(order) == 32
    _say("[batch] 32 cases in 13 channel groups")
    vols = [_vol(torch, g.params, 200 + i) for i, g in enumerate(order)]
    outs = cbct.batch_forward(order, vols)
    ref = [cbct.forward(g, v) for g, v in zip(order, vols)]
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, ref)):
        assert torch.equal(o, r), i


def test_long_stack_in_many_chunks(dev):
    """A 37-channel FP32 stack (nine chunks of four and a single channel)."""
    torch, cbct = dev
    g = SMALL[1]
    geo = cbct.Geometry(g)
    _say("[stack] 37 channels")
    x = _vol(torch, g, 500, C=37)
    y = cbct.forward(geo, x)
    for c in (0, 17, 35, 36):
        assert torch.equal(y[c], cbct.forward(geo, x[c])), c
    torch.cuda.synchronize()


def test_buffer_grows_and_orders_streams(dev):
    """Work on two streams with no host synchronisation between the calls:
    a small adjoint and a four-channel forward on one stream, then on the
    other an eight-channel adjoint at the clinical size (2.9 GB of staged
    projections, more than any other call here: the buffer grows while the
    first stream may still use it), then a small adjoint on the first stream
    again.  Every result bitwise equal to the same call alone on the default
    stream afterwards."""
    torch, cbct = dev
    gS, gB = SMALL[2], W.C2
    geoS, geoB = cbct.Geometry(gS), cbct.Geometry(gB)
    yS = _sino(torch, gS, 600)
    yS2 = _sino(torch, gS, 601)
    xS = _vol(torch, gS, 602, C=4)
    _say("[streams] building the 8-channel clinical sinogram")
    yB = torch.rand((8,) + geoB.sino_shape, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(603))
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    _say("[streams] enqueue on two streams")
    with torch.cuda.stream(s1):
        aS = cbct.adjoint(geoS, yS)
        fS = cbct.forward(geoS, xS)
    with torch.cuda.stream(s2):
        aB = cbct.adjoint(geoB, yB)
    with torch.cuda.stream(s1):
        aS2 = cbct.adjoint(geoS, yS2)
    torch.cuda.synchronize()
    _say("[streams] references on the default stream")
    assert torch.equal(aS, cbct.adjoint(geoS, yS))
    assert torch.equal(fS, cbct.forward(geoS, xS))
    assert torch.equal(aS2, cbct.adjoint(geoS, yS2))
    for c in (0, 7):
        assert torch.equal(aB[c], cbct.adjoint(geoB, yB[c])), c
    torch.cuda.synchronize()
    assert float(aB.abs().max()) > 0
