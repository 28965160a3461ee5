"""Learned primal-dual net on the GPU (library kernels) against the oracle's
FP64 net with the same parameters.

Parameters are rounded to bf16 first, so both sides use the same weights;
the GPU path still rounds each block's packed input and its two hidden
activations to bf16 (unit roundoff u = 2^-9) and accumulates in FP32.  Each
rounding perturbs a block output by about u relative; over the blocks of
the net these add up, so the reconstructions are compared at relative L2
4e-3 (about 8 u) and the parameter gradients at 3e-2 per tensor (the
backward adds the bf16 rounding of the output gradient and the LeakyReLU
mask taken from bf16 activations).  The reversible backward must rebuild
the starting latents (x_0 = 0, A^T y / L, y) to FP32 rounding level."""
import numpy as np
import pytest

from paper_2512_21180_amd import workloads as W

pytestmark = pytest.mark.gpu

TOY = W.geometry(20, 36, 28, 2.6, 2.6, 28, 24, 20, 3.0, off_u=18.0)


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2512_21180_amd import cbct, learned
    return torch, cbct, learned


def _say(*a):
    print(*a, flush=True)


SCALES = [(None, "zero"), ((2, 2, 1), "zero"), ((2, 2, 1), "fdk"), ((4, 2, 1), "zero"),
          ((4, 2, 1), "fdk")]


def _setup(dev, oracle, n_iter=3, seed=0, scales=None, init="zero"):
    torch, cbct, learned = dev
    g = TOY
    geo = cbct.Geometry(g)
    net = learned.PDNet(n_iter=n_iter, seed=seed, scales=scales, init=init).cuda()
    with torch.no_grad():
        for p in net.parameters():
            if p.dim() == 5:
                p.copy_(p.to(torch.bfloat16).float())
    L = oracle.opnorm(g, iters=40)
    x_true = W.phantom_c1(g, 5)[0] / 0.02
    y = oracle.forward(g, x_true) / L + 1e-3 * W.rng(6).standard_normal(W.sino_shape(g))
    y = y.astype(np.float32)
    V = cbct.fov_fraction(g)
    model = learned.LearnedPD(net, geo, torch.tensor(V, device="cuda"), L)
    return g, geo, net, model, L, y, V, x_true


def test_resampling_kernels(dev, oracle):
    torch, cbct, _ = dev
    _say("[learned] pool / projdown / upsample")
    r = W.rng(9)
    for shape, q in (((8, 12, 20), 2), ((16, 8, 24), 4), ((6, 10, 14), 2)):
        a = r.standard_normal(shape).astype(np.float32)
        t = torch.tensor(a, device="cuda")
        got = cbct.pool(t, q).double().cpu().numpy()
        assert np.allclose(got, oracle.downsample(a.astype(np.float64), q), rtol=1e-6, atol=1e-6)
        got = cbct.projdown(t, q).double().cpu().numpy()
        assert np.allclose(got, oracle.projdown(a.astype(np.float64), q), rtol=1e-6, atol=1e-6)
        c = torch.tensor(r.standard_normal(tuple(n // q for n in shape)).astype(np.float32),
                         device="cuda")
        up = cbct.upsample(c, q).double().cpu().numpy()
        assert np.array_equal(up, oracle.upsample(c.double().cpu().numpy(), q))
        acc = t.clone()
        cbct.upsample(c, q, out=acc, scale=0.5, accumulate=True)
        ref = a.astype(np.float64) + 0.5 * oracle.upsample(c.double().cpu().numpy(), q)
        assert np.allclose(acc.double().cpu().numpy(), ref, rtol=1e-6, atol=1e-6)
    with pytest.raises(Exception):
        cbct.pool(torch.zeros((6, 6, 5), device="cuda"), 2)


def test_conv1_and_wresid(dev):
    torch, cbct, _ = dev
    _say("[learned] conv1 / wresid")
    gen = torch.Generator("cuda").manual_seed(1)
    S = 3000
    ch = [torch.randn(S, device="cuda", generator=gen) for _ in range(9)]
    w = torch.randn(10, device="cuda", generator=gen)
    out = torch.empty(S, device="cuda")
    cbct.conv1(ch, w, out)
    ref = w[9].double() + sum(w[c].double() * ch[c].double() for c in range(9))
    assert torch.allclose(out.double(), ref, rtol=1e-6, atol=1e-6)
    base = torch.randn(S, device="cuda", generator=gen)
    acc = base.clone()
    cbct.conv1(ch[:3], w[:4].contiguous(), acc, accumulate=True, alpha=-0.5)
    ref = base.double() - 0.5 * (w[3].double() + sum(w[c].double() * ch[c].double() for c in range(3)))
    assert torch.allclose(acc.double(), ref, rtol=1e-6, atol=1e-6)
    g = torch.empty(S, device="cuda")
    cbct.wresid(g, ch[0], ch[1], ch[2])
    assert torch.equal(g, ch[0] * (ch[1] - ch[2]))


def _x0(oracle, g, y, L, init):
    """The oracle's own starting reconstruction: zero or L * FDK(y)."""
    return None if init == "zero" else L * oracle.fdk(g, y.astype(np.float64), "hann")


@pytest.mark.parametrize("scales,init", SCALES)
def test_forward_matches_oracle(dev, oracle, scales, init):
    torch, cbct, learned = dev
    _say(f"[learned] forward vs oracle (toy, 3 iterations, scales {scales}, init {init})")
    g, geo, net, model, L, y, V, _ = _setup(dev, oracle, scales=scales, init=init)
    x0 = _x0(oracle, g, y, L, init)
    xs = []
    model.reconstruct(torch.tensor(y, device="cuda"),
                      callback=lambda i, x: xs.append(x.double().cpu().numpy()))
    ref = oracle.lpd_forward(g, y.astype(np.float64), V.astype(np.float64),
                             net.oracle_params(), L, scales=scales, x0=x0)
    for i, (a, b) in enumerate(zip(xs, ref)):
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        _say(f"  x_{i + 1}: rel L2 {rel:.2e}")
        assert rel <= 4e-3
    # zero blocks: only the output convolutions act
    xz = model.reconstruct(torch.tensor(y, device="cuda"), zero_blocks=True).double().cpu().numpy()
    ps = net.oracle_params()
    for p in ps:
        for part in ("dual", "primal"):
            p[part] = [np.zeros_like(a) for a in p[part]]
    rz = oracle.lpd_forward(g, y.astype(np.float64), V.astype(np.float64), ps, L,
                            scales=scales, x0=x0)[-1]
    assert np.linalg.norm(xz - rz) <= 1e-5 * np.linalg.norm(rz)


@pytest.mark.parametrize("scales,init", SCALES)
def test_gradient_matches_oracle_and_rebuilds_latents(dev, oracle, scales, init):
    torch, cbct, learned = dev
    _say(f"[learned] reversible gradient vs oracle (toy, 3 iterations, scales {scales}, "
         f"init {init})")
    g, geo, net, model, L, y, V, x_true = _setup(dev, oracle, seed=3, scales=scales, init=init)
    x0 = _x0(oracle, g, y, L, init)
    fov = (V >= 0.5)
    wmask = (fov / fov.sum()).astype(np.float32)
    yt = torch.tensor(y, device="cuda")
    loss = model.loss_and_grad(yt, torch.tensor(x_true, dtype=torch.float32, device="cuda"),
                               torch.tensor(wmask, device="cuda"))
    rloss, rgr = oracle.lpd_loss_grad(g, y.astype(np.float64), V.astype(np.float64),
                                      net.oracle_params(), L, x_true, wmask.astype(np.float64),
                                      scales=scales, x0=x0)
    _say(f"  loss {loss:.6e} oracle {rloss:.6e}")
    assert abs(loss - rloss) <= 4e-3 * rloss
    worst = 0.0
    for i in range(net.n_iter):
        pairs = [(net.dual[i][k], rgr[i]["dual"][k]) for k in range(6)]
        pairs += [(net.primal[i][k], rgr[i]["primal"][k]) for k in range(6)]
        pairs += [(net.out[i], rgr[i]["out"])]
        for p, ref in pairs:
            got = p.grad.double().cpu().numpy()
            rel = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)
            worst = max(worst, rel)
            assert rel <= 3e-2, (i, p.shape, rel)
    _say(f"  worst parameter-gradient rel L2 {worst:.2e}")
    # the backward pass rebuilt the starting latents by inverting the couplings
    f0, h0, _ = model.init_state(yt)
    f, h = model.rebuilt
    for a, b in zip(f + h, f0 + h0):
        err = float((a - b).abs().max())
        scale = float(b.abs().max()) or 1.0
        assert err <= 1e-4 * max(scale, float(yt.abs().max())), err
