"""GPU 3x3x3 convolution kernels (BF16 MFMA, FP32 accumulation) against the
oracle's FP64 definitions evaluated on the same BF16-rounded operands.

Bound per element: FP32 accumulation of the 432 products of a tap-channel
sum; |got - ref| <= 1e-5 * (|w| (*) |x|)(s) (the same convolution on absolute
values) + 1e-7; channel-last outputs are additionally rounded to BF16
(relative 2^-8)."""
import numpy as np
import pytest

from paper_2512_21180_amd import workloads as W

pytestmark = pytest.mark.gpu
SLOPE = 0.01


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2512_21180_amd import cbct
    return torch, cbct


def bf(a):
    """Round an FP64 array to bf16 values (nearest even), returned as FP64."""
    import torch
    return torch.tensor(np.asarray(a, np.float32)).to(torch.bfloat16).double().numpy()


# The last grid is deep and thin: the forward kernel's workgroups walk 5 z
# planes each (the rolling halo wraps its ring of four planes), with a
# partial last column of 3 planes; 16 positions per row (half a weight
# gradient chunk).
GRIDS = [(5, 7, 37), (3, 16, 64), (12, 20, 70), (10243, 2, 16)]


def _setup(dev, grid, cin, cout, seed):
    torch, cbct = dev
    r = W.rng(seed)
    x = bf(r.standard_normal((cin,) + grid))
    w = bf(0.2 * r.standard_normal((cout, cin, 3, 3, 3)))
    b = r.standard_normal(cout).astype(np.float32)
    xt = [torch.tensor(x[c], dtype=torch.float32, device="cuda").contiguous() for c in range(cin)]
    x_cl = cbct.pack16(xt)
    wg = cbct.conv3_weights(torch.tensor(w, device="cuda"))
    bg = torch.zeros(16, device="cuda")
    bg[:cout] = torch.tensor(b, device="cuda")
    return x, w, b, x_cl, wg, bg


@pytest.mark.parametrize("grid", GRIDS)
def test_conv3_forward(dev, oracle, grid):
    torch, cbct = dev
    print(f"[conv] forward {grid}", flush=True)
    for cin, cout, act in ((11, 16, True), (16, 16, True), (16, 4, False), (10, 16, True)):
        x, w, b, x_cl, wg, bg = _setup(dev, grid, cin, cout, seed=cin + cout)
        outs = [torch.empty(grid, device="cuda") for _ in range(cout)]
        y_cl = torch.empty((int(np.prod(grid)), 16), dtype=torch.bfloat16, device="cuda")
        cbct.conv3(grid, x_cl, wg, bias=bg, act=act, slope=SLOPE, y_cl=y_cl, y_cf=outs)
        pre = oracle.conv3(x, w, b)
        ref = oracle.leaky_relu(pre, SLOPE) if act else pre
        got = np.stack([o.double().cpu().numpy() for o in outs])
        bound = 1e-5 * (oracle.conv3(np.abs(x), np.abs(w)) + np.abs(b)[:, None, None, None]) + 1e-7
        assert np.all(np.abs(got - ref) <= bound), (cin, cout, np.max(np.abs(got - ref) / bound))
        gcl = y_cl.double().cpu().numpy().T.reshape((16,) + grid)[:cout]
        assert np.all(np.abs(gcl - ref) <= bound + 2.0 ** -8 * np.abs(ref))
        assert np.all(gcl[cout:] == 0) if cout < 16 else True


def test_conv3_residual_accumulate(dev, oracle):
    torch, cbct = dev
    grid = (4, 9, 33)
    print("[conv] residual", flush=True)
    x, w, b, x_cl, wg, bg = _setup(dev, grid, 16, 4, seed=5)
    base = W.rng(6).standard_normal((4,) + grid)
    outs = [torch.tensor(base[c], dtype=torch.float32, device="cuda") for c in range(4)]
    cbct.conv3(grid, x_cl, wg, bias=bg, y_cf=outs, accumulate=True, alpha=-0.5)
    ref = base - 0.5 * oracle.conv3(x, w, b)
    got = np.stack([o.double().cpu().numpy() for o in outs])
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("grid", GRIDS)
def test_conv3_data_gradient_with_mask(dev, oracle, grid):
    torch, cbct = dev
    print(f"[conv] dgrad {grid}", flush=True)
    r = W.rng(7)
    cin, cout = 16, 16
    w = bf(0.2 * r.standard_normal((cout, cin, 3, 3, 3)))
    dy = bf(r.standard_normal((cout,) + grid))
    h = bf(r.standard_normal((cin,) + grid))           # the layer input, post-activation
    dyt = [torch.tensor(dy[c], dtype=torch.float32, device="cuda") for c in range(cout)]
    ht = [torch.tensor(h[c], dtype=torch.float32, device="cuda") for c in range(cin)]
    dy_cl, h_cl = cbct.pack16(dyt), cbct.pack16(ht)
    wg = cbct.conv3_weights(torch.tensor(w, device="cuda"))
    outs = [torch.empty(grid, device="cuda") for _ in range(cin)]
    cbct.conv3(grid, dy_cl, wg, transpose_w=True, mask=h_cl, slope=SLOPE, y_cf=outs)
    ref = oracle.conv3_dgrad(dy, w) * np.where(h > 0, 1.0, SLOPE)
    bound = 1e-5 * oracle.conv3_dgrad(np.abs(dy), np.abs(w)) + 1e-7
    got = np.stack([o.double().cpu().numpy() for o in outs])
    assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)


@pytest.mark.parametrize("grid", GRIDS)
def test_conv3_weight_gradient(dev, oracle, grid):
    torch, cbct = dev
    print(f"[conv] wgrad {grid}", flush=True)
    r = W.rng(8)
    x = bf(r.standard_normal((16,) + grid))
    dy = bf(r.standard_normal((16,) + grid))
    x_cl = cbct.pack16([torch.tensor(x[c], dtype=torch.float32, device="cuda") for c in range(16)])
    dy_cl = cbct.pack16([torch.tensor(dy[c], dtype=torch.float32, device="cuda") for c in range(16)])
    S = int(np.prod(grid))
    dw = torch.empty((27, 16, 16), device="cuda")
    db = torch.empty(16, device="cuda")
    ws = cbct.conv3_wgrad_workspace(S, "cuda")
    cbct.conv3_wgrad(grid, x_cl, dy_cl, dw, db, ws)
    rdw, rdb = oracle.conv3_wgrad(x, dy)
    ref = rdw.transpose(2, 3, 4, 0, 1).reshape(27, 16, 16)
    bound = 1e-5 * oracle.conv3_wgrad(np.abs(x), np.abs(dy))[0].transpose(2, 3, 4, 0, 1).reshape(27, 16, 16) + 1e-6
    got = dw.double().cpu().numpy()
    assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)
    assert np.allclose(db.double().cpu().numpy(), rdb, rtol=1e-5, atol=1e-5)
    # deterministic
    dw2 = torch.empty_like(dw)
    cbct.conv3_wgrad(grid, x_cl, dy_cl, dw2, None, ws)
    assert torch.equal(dw, dw2)
