"""Pins of the oracle's polychromatic water-bone primary model (Sec. 2.2,
eq. primarymodel; Sec. 2.4, eq. normprimary), CPU only.

* the water/bone densities: spot values worked by hand from the two
  piecewise definitions, continuity at tau_0 = 0, tau_1 and tau_2 (the
  reading that fixes tau_0), and the mixing identity of the transition
  range (rho_w / tau_1 + rho_b / (kappa_b tau_2) = 1: a voxel there is a
  mixture of water at density tau_1 and bone at density tau_2);
* the detector response at its three key points and midway between them;
* linearity of P over the two materials (the reason the model needs only
  two projector channels);
* the one-bin, unit-response limit equals the monochromatic model bit for
  bit;
* the mean and variance of the signal over many elements with the same line
  integrals equal sum_e resp_e lambda_e and sum_e resp_e^2 lambda_e
  (independent Poisson bins with the stated means);
* the zero-signal floor and the clamp of the normalised log.
"""
import math

import numpy as np
import pytest


def test_water_bone_spot_values(oracle):
    hu = np.array([-2000.0, -1000.0, 0.0, 150.0, 400.0, 1000.0, 2000.0])
    rw, rb = oracle.water_bone(hu)
    # rho^ = 0.001 HU + 1: -1, 0, 1, 1.15, 1.4, 2, 3
    np.testing.assert_allclose(rw, [0.0, 0.0, 1.0, 1.15, 0.6, 0.0, 0.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(rb, [0.0, 0.0, 0.0, 0.0, 0.3272, 0.818, 1.227], rtol=0, atol=1e-15)


def test_water_bone_continuity_and_mixing(oracle):
    for tau in (0.0, 1.2, 1.6):
        hu = 1000.0 * (np.array([tau - 1e-9, tau, tau + 1e-9]) - 1.0)
        rw, rb = oracle.water_bone(hu)
        assert np.ptp(rw) < 1e-8 and np.ptp(rb) < 1e-8, (tau, rw, rb)
    r = np.linspace(1.2, 1.6, 41)[:-1]
    rw, rb = oracle.water_bone(1000.0 * (r - 1.0))
    np.testing.assert_allclose(rw / 1.2 + rb / (0.409 * 1.6), 1.0, rtol=0, atol=1e-12)
    assert np.all(np.diff(rb) > 0) and np.all(np.diff(rw) < 0)


def test_detector_response_key_points(oracle):
    e = np.array([20.0, 40.0, 60.0, 90.0, 120.0, 10.0, 150.0])
    np.testing.assert_allclose(oracle.detector_response(e), [5, 12.5, 20, 15, 10, 5, 10],
                               rtol=0, atol=1e-12)
    c = oracle.energy_bins()
    assert c.tolist() == [25.0, 35.0, 45.0, 55.0, 65.0, 75.0, 85.0, 95.0, 105.0, 115.0]


def test_material_linearity_of_projection(oracle):
    from paper_2512_21180_amd import workloads as W
    g = W.geometry(10, 20, 16, 3.0, 3.0, 12, 12, 10, 4.0, off_u=15.0)
    rng = np.random.default_rng(5)
    hu = rng.uniform(-1000.0, 1500.0, size=(g["nz"], g["ny"], g["nx"]))
    rw, rb = oracle.water_bone(hu)
    mw, mb = 0.021, 0.048
    lhs = oracle.forward(g, mw * rw + mb * rb)
    rhs = mw * oracle.forward(g, rw) + mb * oracle.forward(g, rb)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(lhs))


def test_one_bin_unit_response_is_the_monochromatic_model(oracle):
    rng = np.random.default_rng(11)
    nv, nu, na = 6, 7, 5
    p = rng.uniform(0.0, 9.0, size=(na, nv, nu))
    pb = rng.uniform(0.0, 3.0, size=p.shape)          # ignored: mu_b = 0
    I0 = 1e5
    y, sig, c = oracle.sim_poly(p, pb, [1.0], [0.0], [1.0], np.full((1, nv, nu), I0), 77, 3)
    ym, cm = oracle.sim_poisson_log(p, I0, 77, 3)
    assert np.array_equal(c[0], cm)
    assert np.array_equal(y, ym)
    assert np.array_equal(sig, cm.astype(np.float64))


def test_signal_moments_match_independent_poisson_bins(oracle):
    e = oracle.energy_bins()
    resp = oracle.detector_response(e)
    mu_w = 0.02 + 0.6 * (25.0 / e) ** 3          # synthetic tables (decreasing with energy)
    mu_b = 0.04 + 3.0 * (25.0 / e) ** 3
    spec = np.exp(-0.5 * ((e - 60.0) / 25.0) ** 2)
    n = 120_000
    I0 = (50.0 * spec / spec.sum() * 10)[:, None, None] * np.ones((10, 1, 1))
    pw = np.full((n, 1, 1), 2.0)
    pb = np.full((n, 1, 1), 0.7)
    y, sig, c = oracle.sim_poly(pw, pb, mu_w, mu_b, resp, I0, 2025, 9)
    lam = I0[:, 0, 0] * np.exp(-(mu_w * 2.0 + mu_b * 0.7))
    for b in range(10):
        se = math.sqrt(lam[b] / n)
        assert abs(c[b].mean() - lam[b]) < 5 * se + 1e-12, (b, c[b].mean(), lam[b])
    m = float(np.sum(resp * lam))
    v = float(np.sum(resp * resp * lam))
    s = sig.ravel()
    assert abs(s.mean() - m) < 5 * math.sqrt(v / n)
    # the sample variance of a sum of independent Poissons: fourth cumulant sum resp^4 lam
    k4 = float(np.sum(resp ** 4 * lam))
    assert abs(s.var() - v) < 5 * math.sqrt((k4 + 2 * v * v) / n)
    # bins independent: correlation of two bins' counts near zero
    r = np.corrcoef(c[3].ravel(), c[4].ravel())[0, 1]
    assert abs(r) < 5 / math.sqrt(n)


def test_zero_signal_floor_and_clamp(oracle):
    resp = np.array([5.0, 20.0, 10.0])
    I0 = np.array([100.0, 300.0, 50.0])[:, None, None] * np.ones((3, 2, 2))
    air = float(np.sum(resp * I0[:, 0, 0]))
    # opaque: every count is zero, the signal is floored at the smallest response
    y, sig, c = oracle.sim_poly(np.full((3, 2, 2), 1e4), np.zeros((3, 2, 2)), [1.0, 1.0, 1.0],
                                [0.0, 0.0, 0.0], resp, I0, 1, 0)
    assert np.all(c == 0) and np.all(sig == 0)
    np.testing.assert_allclose(y, -math.log(5.0 / air), rtol=1e-15)
    # transparent: the ratio is clamped at one, so y >= 0 everywhere and y = 0 where s >= s_air
    y, sig, c = oracle.sim_poly(np.zeros((400, 2, 2)), np.zeros((400, 2, 2)), [1.0, 1.0, 1.0],
                                [0.0, 0.0, 0.0], resp, I0, 2, 0)
    assert np.all(y >= 0)
    assert np.all(y[sig >= air] == 0) and np.any(sig >= air)
    np.testing.assert_allclose(y[sig < air], -np.log(sig[sig < air] / air), rtol=1e-14)
