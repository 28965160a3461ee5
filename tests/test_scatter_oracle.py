"""Pins of the oracle's scatter model (Sec. 2.3, Alg. 2 SamplePath and Alg. 3
Integrate; appendix eqs. beer, lambdameas, distsample, Compton energy), CPU
only:

* material line integrals through piecewise-constant voxels: a uniform box
  gives density x chord (slab clipping in the test), axis-parallel rays
  through voxel centres give the sum of the voxels times the pitch;
* the Compton energy at 0, 90 and 180 degrees (hand values of the formula),
  the detector response at its key points;
* scattered directions: unit length, cos of the angle to v as asked, the
  azimuth reversing the perpendicular part, also where the frame switches;
* the first interaction distance and weight against the closed form for a
  homogeneous box, l = t_in - log(1 - (1 - exp(-mu L)) u) / mu, w = 1 - exp(-mu L);
* the weight after a scatter, w (1 - mu_p / mu_tot)(1 - p0'), and the
  material fractions of stratified choices;
* rotation: at a quarter turn a z-symmetric volume gives the rotated paths;
* Integrate: in vacuum with isotropic Rayleigh-only tables, the panel total
  equals w (mu_r / mu_tot) resp(e) Omega / (4 pi), Omega the panel's solid
  angle (closed form); one pixel behind a uniform slab is attenuated by
  exp(-mu d).
"""
import math

import numpy as np
import pytest

from paper_2512_21180_amd import workloads as W


def _box(n=8, vox=10.0):
    return W.geometry(4, 16, 12, 12.8, 12.8, n, n, n, vox, off_u=20.0)


def _slab_chord(p, d, lo, hi):
    t0, t1 = 0.0, 1e9
    for q in range(3):
        if d[q] == 0:
            if not (lo[q] < p[q] < hi[q]):
                return 0.0
            continue
        a, b = (lo[q] - p[q]) / d[q], (hi[q] - p[q]) / d[q]
        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
    return max(0.0, t1 - t0)


def test_march_uniform_box_is_the_chord(oracle):
    g = _box()
    n = g["nx"] * g["ny"] * g["nz"]
    rw, rb = np.ones(n), np.full(n, 0.5)
    rng = np.random.default_rng(1)
    half = 40.0
    for _ in range(50):
        p = rng.uniform(-120, 120, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        got = oracle.march(g, rw, rb, p, d, 1e6)
        ch = _slab_chord(p, d, [-half] * 3, [half] * 3)
        assert abs(got[0] - ch) <= 1e-9 and abs(got[1] - 0.5 * ch) <= 1e-9


def test_march_axis_rays_sum_the_voxels(oracle):
    g = _box(n=6, vox=7.0)
    rng = np.random.default_rng(2)
    vol = rng.uniform(0, 2, (6, 6, 6))
    zb = np.zeros_like(vol)
    for k in range(6):
        for j in range(6):
            y = (j - 2.5) * 7.0
            z = (k - 2.5) * 7.0
            got = oracle.march(g, vol.ravel(), zb.ravel(), [-100.0, y, z], [1.0, 0.0, 0.0], 1e6)
            assert abs(got[0] - 7.0 * vol[k, j].sum()) <= 1e-9
            # stopping inside voxel 3: half of it
            got = oracle.march(g, vol.ravel(), zb.ravel(), [-100.0, y, z], [1.0, 0.0, 0.0],
                               100.0 + 3.5)
            assert abs(got[0] - 7.0 * (vol[k, j, :3].sum() + 0.5 * vol[k, j, 3])) <= 1e-9


def test_compton_energy_and_response(oracle):
    for e in (25.0, 60.0, 115.0):
        assert oracle.compton_energy(e, 1.0) == e
        assert abs(oracle.compton_energy(e, 0.0) - e / (1 + e / 510.99895)) <= 1e-12
        assert abs(oracle.compton_energy(e, -1.0) - e / (1 + 2 * e / 510.99895)) <= 1e-12
    assert [oracle.resp(x) for x in (10, 20, 40, 60, 90, 120, 150)] == [5, 5, 12.5, 20, 15, 10, 10]


@pytest.mark.parametrize("v", [[1.0, 0.0, 0.0], [0.3, -0.4, 0.866], [0.0, 0.1, -0.995]])
def test_scatter_direction(oracle, v):
    v = np.asarray(v) / np.linalg.norm(v)
    for cth in (-0.9, 0.0, 0.37, 0.999):
        a = oracle.scatter_direction(v, cth, 0.7)
        b = oracle.scatter_direction(v, cth, 0.7 + math.pi)
        assert abs(np.linalg.norm(a) - 1) <= 1e-12 and abs(a @ v - cth) <= 1e-12
        pa, pb = a - cth * v, b - cth * v
        assert np.allclose(pa, -pb, atol=1e-12)


def _uniform(g, rw=1.0, rb=0.0):
    n = g["nx"] * g["ny"] * g["nz"]
    return np.full(n, rw), np.full(n, rb)


def test_first_interaction_closed_form(oracle):
    g = _box()
    xs = W.scatter_tables()
    rw, rb = _uniform(g, 1.0, 0.0)
    N = 64
    src = np.zeros((N, 4))
    src[:, 0] = -1.0          # along -x from the source at (sid, 0, 0): through the centre
    src[:, 3] = 55.0
    ub = (np.arange(N) + 0.5) / N
    sob = np.zeros((N, 1))
    sob[:, 0] = ub
    rec = oracle.scatter_paths(g, rw, rb, xs, 0, src, sob, 0)
    mu = xs["mu"][0, :, 9].sum()          # 55 keV is grid point 9
    L = 80.0
    t_in = g["sid"] - 40.0
    l = t_in - np.log(1 - (1 - np.exp(-mu * L)) * ub) / mu
    np.testing.assert_allclose(rec[:, 0, 0], g["sid"] - l, rtol=0, atol=1e-9)
    np.testing.assert_allclose(rec[:, 0, 7], 1 - np.exp(-mu * L), rtol=1e-12)
    assert np.all(rec[:, 0, 6] == 55.0)


def test_scatter_weight_and_material_fractions(oracle):
    g = _box()
    xs = W.scatter_tables()
    rw, rb = _uniform(g, 0.7, 0.4)
    N = 200
    src = np.zeros((N, 4))
    src[:, 0] = -1.0
    src[:, 3] = 65.0
    sob = np.full((N, 6), 0.5)
    sob[:, 0] = 0.5
    sob[:, 1] = (np.arange(N) + 0.5) / N      # material choice, stratified
    sob[:, 2] = 0.3
    rec = oracle.scatter_paths(g, rw, rb, xs, 0, src, sob, 1)
    k = 11                                     # 65 keV
    mt = xs["mu"][:, :, k].sum(axis=1)
    fw = 0.7 * mt[0] / (0.7 * mt[0] + 0.4 * mt[1])
    w0 = rec[:, 0, 7]
    # second leg: p0' along the new direction from the first point
    ratio = rec[:, 1, 7] / w0
    e1 = rec[:, 1, 6]
    x1 = rec[:, 0, :3]
    v1 = rec[:, 1, 3:6]
    water = np.zeros(N, dtype=bool)
    for i in range(N):
        P = oracle.march(g, rw, rb, x1[i], v1[i], 1e6)
        surv = []
        for m in (0, 1):
            keep = 1 - xs["mu"][m, 0, k] / mt[m]
            # the distance leg is taken at the energy after the scatter
            f = (e1[i] - 10.0) / 5.0
            kk = min(int(f), 27)
            t = f - kk
            mtw = (1 - t) * xs["mu"][0, :, kk].sum() + t * xs["mu"][0, :, kk + 1].sum()
            mtb = (1 - t) * xs["mu"][1, :, kk].sum() + t * xs["mu"][1, :, kk + 1].sum()
            surv.append(keep * (1 - math.exp(-(mtw * P[0] + mtb * P[1]))))
        assert min(abs(ratio[i] - surv[0]), abs(ratio[i] - surv[1])) <= 1e-12 * max(surv)
        water[i] = abs(ratio[i] - surv[0]) < abs(ratio[i] - surv[1])
    assert water.sum() == int(np.sum(sob[:, 1] < fw))


def test_quarter_turn_rotates_paths(oracle):
    g = W.geometry(4, 16, 12, 12.8, 12.8, 8, 8, 8, 10.0)
    xs = W.scatter_tables()
    rng = np.random.default_rng(4)
    vol = rng.uniform(0, 1, (8, 8, 8))
    vol = vol + np.rot90(vol, 1, axes=(1, 2)) + np.rot90(vol, 2, axes=(1, 2)) + \
        np.rot90(vol, 3, axes=(1, 2))       # invariant under quarter turns about z
    rb = 0.3 * vol
    src = W.scatter_sources(40, g, 3)
    sob = W.sobol_points(40, 11)
    r0 = oracle.scatter_paths(g, vol.ravel(), rb.ravel(), xs, 0, src, sob, 2)
    r1 = oracle.scatter_paths(g, vol.ravel(), rb.ravel(), xs, 1, src, sob, 2)   # angle pi / 2
    rot = lambda a: np.stack([-a[..., 1], a[..., 0], a[..., 2]], axis=-1)
    # the scatter frame turns with v about z, except for nearly vertical
    # directions (|v_z| >= 0.9 takes v x x): photons scattered from such a
    # direction are left out
    ok = np.all(np.abs(r0[:, :-1, 5]) < 0.9, axis=1)
    assert ok.mean() > 0.8
    np.testing.assert_allclose(r1[ok, :, 0:3], rot(r0[ok, :, 0:3]), atol=1e-7)
    np.testing.assert_allclose(r1[ok, :, 3:6], rot(r0[ok, :, 3:6]), atol=1e-9)
    np.testing.assert_allclose(r1[ok, :, 6:], r0[ok, :, 6:], rtol=1e-9)


def _iso_tables():
    xs = W.scatter_tables()
    xs["mu"][:, 1, :] = 0.0                  # no Compton
    xs["icdf"][:] = np.linspace(-1, 1, xs["icdf"].shape[-1])
    xs["dens"][:] = 1.0 / (4 * math.pi)
    return xs


def test_integrate_solid_angle_in_vacuum(oracle):
    # fine panel, a record at the isocentre, nothing attenuates
    g = W.geometry(1, 160, 120, 1.0, 1.0, 4, 4, 4, 5.0)
    xs = _iso_tables()
    n = 64
    rw, rb = np.zeros(n), np.zeros(n)
    rec = np.array([[0.0, 0.0, 0.0, -1.0, 0.0, 0.0, 60.0, 0.8]])
    S = oracle.scatter_integrate(g, rw, rb, xs, 0, rec)
    a, b, d = 80.0, 60.0, g["sdd"] - g["sid"]
    omega = 4 * math.atan(a * b / (d * math.sqrt(a * a + b * b + d * d)))
    k = 10
    fr = xs["mu"][0, 2, k] / xs["mu"][0, :, k].sum()
    want = 0.8 * fr * oracle.resp(60.0) * omega / (4 * math.pi)
    assert abs(S.sum() - want) <= 1e-4 * want


def test_integrate_attenuation_toward_a_pixel(oracle):
    g = W.geometry(1, 3, 3, 2.0, 2.0, 10, 10, 10, 6.0)
    xs = _iso_tables()
    rw, rb = _uniform(g, 1.0, 0.0)
    x = np.array([10.0, 0.0, 0.0])
    rec = np.array([[*x, -1.0, 0.0, 0.0, 60.0, 1.0]])
    S1 = oracle.scatter_integrate(g, rw, rb, xs, 0, rec)
    S0 = oracle.scatter_integrate(g, 0 * rw, rb, xs, 0, rec)
    k = 10
    mu = xs["mu"][0, :, k].sum()
    # the centre pixel lies on -x: the ray leaves the 60 mm box after 40 mm;
    # in vacuum the voxel at x still sets the material mix (water)
    assert abs(S1[1, 1] / S0[1, 1] - math.exp(-mu * 40.0)) <= 1e-12
