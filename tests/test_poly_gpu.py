"""GPU polychromatic primary simulator against the oracle's model (Sec. 2.2,
eq. primarymodel; Sec. 2.4, eq. normprimary): water/bone densities within
FP32 rounding, per-bin Poisson counts bit-exact on the same line integrals
(the means and the acceptance test are FP64 on both sides) and the signal
within its FP32 rounding, the normalised log within FP32 rounding, the one-bin limit equal to
the monochromatic kernel bit for bit, and the whole pipeline (densities, a
two-channel forward projection, noise) against the oracle's."""
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


def test_water_bone_matches_oracle(dev, oracle):
    torch, cbct, _ = dev
    print("[poly] water_bone", flush=True)
    rng = np.random.default_rng(3)
    hu = np.concatenate([rng.uniform(-1500, 3500, 100_001),
                         [-1000.0, 200.0, 600.0, 0.0, -1000.5, 199.99, 600.01]]).astype(np.float32)
    got = cbct.water_bone(torch.tensor(hu, device="cuda")).double().cpu().numpy()
    rw, rb = oracle.water_bone(hu.astype(np.float64))
    assert np.max(np.abs(got[0] - rw)) <= 1e-6 and np.max(np.abs(got[1] - rb)) <= 1e-6


def _tables(oracle):
    c = oracle.energy_bins()
    mw, mb = W.poly_tables(c)
    return c, mw, mb, oracle.detector_response(c)


def test_poly_bins_are_the_papers(dev, oracle):
    _, cbct, _ = dev
    c, r = cbct.poly_bins()
    assert np.array_equal(c, oracle.energy_bins())
    np.testing.assert_allclose(r, oracle.detector_response(c), rtol=0, atol=1e-12)


def test_sim_poly_counts_bit_exact(dev, oracle):
    torch, cbct, _ = dev
    print("[poly] sim_poly counts", flush=True)
    g = W.geometry(7, 40, 24, 3.2, 3.2, 8, 8, 8, 4.0, off_u=30.0)
    c, mw, mb, resp = _tables(oracle)
    I0 = W.intensity_maps(g, c, photons_per_mm2=16000.0)
    rng = np.random.default_rng(8)
    shape = (g["n_angles"], g["nv"], g["nu"])
    # line integrals from transparent to nearly opaque (low counts, zero counts)
    pw = rng.uniform(0.0, 40.0, shape).astype(np.float32)
    pb = rng.uniform(0.0, 6.0, shape).astype(np.float32)
    pw[0, 0, :8] = 0.0          # transparent
    pb[0, 0, :8] = 0.0
    pw[0, 1, :] = 3000.0        # opaque: zero counts in every bin
    pw[0, 2, :] = np.linspace(300.0, 700.0, g["nu"])   # a few photons
    y, sig, cnt = cbct.sim_poly(torch.tensor(pw, device="cuda"), torch.tensor(pb, device="cuda"),
                                mw, mb, resp, torch.tensor(I0, device="cuda"), 424242, 6,
                                signal=True, counts=True)
    yr, sr, cr = oracle.sim_poly(pw.astype(np.float64), pb.astype(np.float64), mw, mb, resp,
                                 I0.astype(np.float64), 424242, 6)
    mism = int((cnt.cpu().numpy() != cr).sum())
    assert mism == 0, mism
    # the signal is an FP64 sum of response-weighted counts on both sides
    # (contracted to fused multiply-adds on the GPU), stored in FP32
    np.testing.assert_allclose(sig.cpu().numpy().astype(np.float64), sr, rtol=2.4e-7, atol=0)
    yg = y.double().cpu().numpy()
    assert np.max(np.abs(yg - yr)) <= 1e-6 * max(1.0, float(np.max(yr)))
    assert np.any(cr.sum(axis=0) == 0)          # the zero-signal floor is exercised


def test_one_bin_is_the_monochromatic_kernel(dev, oracle):
    torch, cbct, _ = dev
    print("[poly] one-bin limit", flush=True)
    nv, nu = 16, 20
    p = torch.linspace(0.0, 13.0, 5 * nv * nu, device="cuda").reshape(5, nv, nu).contiguous()
    pb = torch.full_like(p, 0.5)
    I0 = torch.full((1, nv, nu), 1e5, device="cuda")
    y, cnt = cbct.sim_poly(p, pb, [1.0], [0.0], [1.0], I0, 99, 4, counts=True)
    ym, cm = cbct.sim_poisson_log(p, 1e5, 99, 4, counts=True)
    assert torch.equal(cnt[0], cm)
    assert torch.equal(y, ym)


def test_poly_pipeline_matches_oracle(dev, oracle):
    torch, cbct, simulate = dev
    print("[poly] pipeline", flush=True)
    g = W.geometry(12, 64, 40, 3.2, 3.2, 40, 40, 24, 4.0, off_u=50.0)
    hu = W.hu_phantom(g, 17)
    c, mw, mb, resp = _tables(oracle)
    I0 = W.intensity_maps(g, c)
    geo = cbct.Geometry(g)
    y, p = simulate.poly_primary(geo, torch.tensor(hu, device="cuda"), mw, mb, resp,
                                 torch.tensor(I0, device="cuda"), 7, 1)
    rw, rb = oracle.water_bone(hu.astype(np.float64))
    assert rb.max() > 0 and rw.max() > 0          # both materials present
    pref = np.stack([oracle.forward(g, rw), oracle.forward(g, rb)])
    pg = p.double().cpu().numpy()
    for ch in range(2):
        e = np.linalg.norm(pg[ch] - pref[ch]) / np.linalg.norm(pref[ch])
        assert e <= 1e-5, (ch, e)
    # counts and log from the GPU's own line integrals, against the oracle's model
    yr, _, _ = oracle.sim_poly(pg[0], pg[1], mw, mb, resp, I0.astype(np.float64), 7, 1)
    assert np.max(np.abs(y.double().cpu().numpy() - yr)) <= 1e-6 * max(1.0, float(np.max(yr)))
