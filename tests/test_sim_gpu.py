"""GPU simulator kernels against the oracle's noise model: Philox blocks
bit-exact, Poisson counts exact (the acceptance test runs in FP64 on both
sides), the log-transformed sinogram and the Gaussian variant within FP32
rounding."""
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
    from paper_2512_21180_amd import cbct, simulate
    return torch, cbct, simulate


def test_philox_blocks_bit_exact(dev, oracle):
    torch, cbct, _ = dev
    print("[sim] philox", flush=True)
    out = cbct.philox_blocks(5000, 0x1234_5678_9ABC, 3).cpu().numpy().view(np.uint32)
    for i in list(range(20)) + [4999, 2048, 777]:
        ref = oracle.philox4x32_10([i, 0, 0, 3], [0x56789ABC, 0x1234])
        assert list(out[i]) == ref


def test_poisson_counts_and_log_sinogram(dev, oracle):
    torch, cbct, simulate = dev
    g = W.cropped(W.C1, n_angles=8, nu=64, nv=48, n=48)
    print("[sim] poisson, c1-style", flush=True)
    geo = cbct.Geometry(g)
    x, _ = W.phantom_c1(g, 3)
    p = cbct.forward(geo, torch.tensor(x, dtype=torch.float32, device="cuda"))
    # extend the range: very low counts (p up to 14) and zero attenuation
    p = torch.cat([p.view(-1), torch.linspace(0, 14, 4001, device="cuda")]).contiguous()
    y, c = cbct.sim_poisson_log(p, 1e5, 300001, 5, counts=True)
    yr, cr = oracle.sim_poisson_log(p.double().cpu().numpy(), 1e5, 300001, 5)
    mism = int((c.cpu().numpy() != cr).sum())
    assert mism == 0, mism
    assert np.max(np.abs(y.double().cpu().numpy() - yr)) <= 1e-6 * max(1.0, float(np.max(yr)))


def test_noisy_sinogram_pipeline(dev, oracle):
    torch, cbct, simulate = dev
    g = W.cropped(W.C1, n_angles=6, nu=64, nv=48, n=48)
    print("[sim] pipeline", flush=True)
    geo = cbct.Geometry(g)
    x, _ = W.phantom_c1(g, 9)
    xg = torch.tensor(x, dtype=torch.float32, device="cuda")
    y = simulate.noisy_sinogram(geo, xg, 1e5, 77).double().cpu().numpy()
    p = cbct.forward(geo, xg).double().cpu().numpy()
    yr, _ = oracle.sim_poisson_log(p, 1e5, 77, 0)
    assert np.max(np.abs(y - yr)) <= 1e-6 * max(1.0, float(np.max(yr)))
    z = simulate.gaussian_sinogram(geo, xg, 1e-3, 5).double().cpu().numpy()
    zr = oracle.sim_gaussian(p, 1e-3, 5, 0)
    assert np.max(np.abs(z - zr)) <= 1e-6 * max(1.0, float(np.max(np.abs(zr))))
