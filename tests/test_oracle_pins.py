"""Pins of the FP64 oracle against facts fixed by geometry and mathematics.

The oracle defines the discrete cone-beam transform (paper Sec. 2.2: P is the
line integral from the source to each detector element; P* is its adjoint).
These tests check it against quantities that do not come from the oracle:
geometric invariants of the circular orbit, exact chord lengths of bodies on
which the discretisation is exact, exact line integrals of the trilinear
interpolant, closed-form projections of Gaussians and spheres with their
convergence orders, brute-force path lengths, the transpose identity, the
rotation and reflection symmetries of the orbit, and a dense least-squares
solve.
"""
import math

import numpy as np
import pytest

import analytic
from paper_2512_21180_amd import workloads as W


def tiny(**over):
    g = W.geometry(8, 16, 12, 4.0, 4.0, 8, 8, 8, 4.0, sid=100.0, sdd=160.0, off_u=3.1, off_v=-2.3)
    g.update(over)
    return g


# ---------------------------------------------------------------- geometry ---

def test_orbit_geometry_invariants(oracle):
    g = tiny(n_angles=7)
    ang = oracle.angles_of(g)
    for a in range(g["n_angles"]):
        S, _ = oracle.ray(g, a, 0, 0)
        # source on the orbit circle of radius sid in the z=0 plane, at angle theta
        assert abs(np.linalg.norm(S) - g["sid"]) < 1e-12
        assert abs(math.atan2(S[1], S[0]) % (2 * math.pi) - ang[a] % (2 * math.pi)) < 1e-12
        n = S / np.linalg.norm(S)
        for iu in (0, 5, g["nu"] - 1):
            for iv in (0, 7, g["nv"] - 1):
                S2, d = oracle.ray(g, a, iu, iv)
                assert np.allclose(S2, S, atol=0)
                # every pixel centre lies on the panel plane, sdd from the source
                assert abs(d @ n + g["sdd"]) < 1e-9
        # neighbouring pixels are one pitch apart: columns along the direction
        # of source motion (dS/dtheta), rows along +z
        _, d00 = oracle.ray(g, a, 3, 4)
        _, d10 = oracle.ray(g, a, 4, 4)
        _, d01 = oracle.ray(g, a, 3, 5)
        motion = np.array([-S[1], S[0], 0.0]) / g["sid"]
        assert np.allclose(d10 - d00, g["du"] * motion, atol=1e-12)
        assert np.allclose(d01 - d00, [0, 0, g["dv"]], atol=1e-12)


def test_offset_moves_panel_along_motion_and_centre_ray_hits_isocenter(oracle):
    g0 = tiny(nu=17, nv=13, off_u=0.0, off_v=0.0, n_angles=5)
    g1 = dict(g0, off_u=11.5, off_v=-3.0)
    for a in range(5):
        S, d0 = oracle.ray(g0, a, 8, 6)
        # central ray of an unshifted odd panel passes through the isocenter
        t = -(S @ d0) / (d0 @ d0)
        assert np.linalg.norm(S + t * d0) < 1e-12
        _, d1 = oracle.ray(g1, a, 8, 6)
        motion = np.array([-S[1], S[0], 0.0]) / g0["sid"]
        assert np.allclose(d1 - d0, 11.5 * motion + np.array([0, 0, -3.0]), atol=1e-12)


# ------------------------------------------------- exact bodies (P1, P2) ---

def _qualifying_box_rays(oracle, g, lo, hi, margin):
    """Rays whose major axis is the axis of both the entry and the exit face
    of box [lo,hi], with the other coordinates at both faces >= margin inside."""
    out = []
    for a in range(g["n_angles"]):
        for iv in range(g["nv"]):
            for iu in range(g["nu"]):
                S, d = oracle.ray(g, a, iu, iv)
                m = 0 if abs(d[0]) >= abs(d[1]) else 1
                iv_ = analytic.slab_intervals(S, d, lo, hi)
                t_in = max(x[0] for x in iv_)
                t_out = min(x[1] for x in iv_)
                if not (t_out > t_in):
                    continue
                if iv_[m][0] != t_in or iv_[m][1] != t_out:
                    continue
                ok = True
                for t in (t_in, t_out):
                    p = S + t * d
                    for q in range(3):
                        if q == m:
                            continue
                        if not (lo[q] + margin[q] <= p[q] <= hi[q] - margin[q]):
                            ok = False
                if ok:
                    out.append((a, iv, iu))
    return out


def test_exact_box_chord(oracle):
    """A voxel-aligned box of constant mu: rays through both major-axis faces
    with their lateral crossings at least one voxel inside integrate exactly
    to mu times the chord length."""
    g = W.geometry(12, 48, 40, 1.6, 1.6, 24, 24, 24, 2.0, sid=150.0, sdd=240.0,
                   off_u=3.1, off_v=-2.3, origin=(1.0, -0.5, 0.7))
    cx, cy, cz = W.voxel_centres(g)
    ib, jb, kb = (6, 17), (8, 15), (5, 18)
    vol = np.zeros(W.vol_shape(g))
    mu = 0.37
    vol[kb[0]:kb[1] + 1, jb[0]:jb[1] + 1, ib[0]:ib[1] + 1] = mu
    lo = np.array([cx[ib[0]] - 1.0, cy[jb[0]] - 1.0, cz[kb[0]] - 1.0])
    hi = np.array([cx[ib[1]] + 1.0, cy[jb[1]] + 1.0, cz[kb[1]] + 1.0])
    rays = _qualifying_box_rays(oracle, g, lo, hi, margin=(2.0, 2.0, 2.0))
    assert len(rays) > 200
    y = oracle.forward(g, vol)
    for (a, iv, iu) in rays:
        S, d = oracle.ray(g, a, iu, iv)
        its = analytic.slab_intervals(S, d, lo, hi)
        chord = (min(x[1] for x in its) - max(x[0] for x in its)) * np.linalg.norm(d)
        assert abs(y[a, iv, iu] - mu * chord) <= 1e-12 * mu * chord


def test_all_ones_interior_rays(oracle):
    """A . 1 equals the chord through the volume for rays crossing both
    major-axis faces well inside the lateral faces."""
    g = W.geometry(16, 40, 40, 1.2, 1.2, 20, 20, 20, 2.0, sid=150.0, sdd=240.0, off_u=-4.0)
    cx, cy, cz = W.voxel_centres(g)
    lo = np.array([cx[0] - 1, cy[0] - 1, cz[0] - 1])
    hi = np.array([cx[-1] + 1, cy[-1] + 1, cz[-1] + 1])
    rays = _qualifying_box_rays(oracle, g, lo, hi, margin=(2.0, 2.0, 2.0))
    assert len(rays) > 1000
    y = oracle.forward(g, np.ones(W.vol_shape(g)))
    for (a, iv, iu) in rays:
        chord = oracle.chord_box(g, a, iu, iv, lo, hi)
        assert abs(y[a, iv, iu] - chord) <= 1e-12 * chord


# ------------------------------------------- trilinear interpolant (P3) ---

def test_axis_parallel_rays_equal_interpolant_integral(oracle):
    """Along a ray parallel to a grid axis the trilinear interpolant is
    piecewise linear between voxel-centre planes, so the plane sum is its
    exact integral."""
    g = W.geometry(4, 17, 13, 1.5, 1.5, 10, 12, 9, 2.0, vy=2.5, vz=1.7, sid=150.0, sdd=240.0,
                   angles=np.array([0.0, 0.5 * math.pi, math.pi, 1.5 * math.pi]),
                   origin=(0.3, -0.4, 0.6))
    for seed in range(3):
        vol = W.random_volume(g, seed)
        y = oracle.forward(g, vol)
        for a in range(4):
            S, d = oracle.ray(g, a, 8, 6)
            assert abs(d[2]) == 0 and min(abs(d[0]), abs(d[1])) < 1e-12
            ref = oracle.interp_integral(g, vol, a, 8, 6)
            assert abs(y[a, 6, 8] - ref) <= 1e-12 * abs(ref)


def test_oblique_rays_converge_to_interpolant_integral(oracle):
    """For a smooth body, the plane-sampled sum and the exact interpolant
    integral agree to second order in the voxel pitch."""
    errs = []
    for n, v in ((24, 2.0), (48, 1.0)):
        g = W.geometry(3, 20, 16, 2.4, 2.4, n, n, n, v, sid=150.0, sdd=240.0, off_u=2.0)
        cx, cy, cz = W.voxel_centres(g)
        Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
        vol = np.exp(-((X - 1.5) ** 2 + (Y + 2.0) ** 2 + (Z - 1.0) ** 2) / (2 * 7.0 ** 2))
        y = oracle.forward(g, vol)
        e = []
        for (a, iu, iv) in ((0, 9, 7), (1, 11, 5), (2, 6, 9), (1, 3, 8)):
            ref = oracle.interp_integral(g, vol, a, iu, iv)
            e.append(abs(y[a, iv, iu] - ref) / abs(ref))
        errs.append(max(e))
    assert errs[1] < 5e-4
    assert 3.0 < errs[0] / errs[1] < 5.5


# ------------------------------------------- closed forms (P4, P5, P6) ---

SIG = 5.0


def _gaussian_case(oracle, n, v):
    g = W.geometry(5, 36, 30, 1.6, 1.6, n, n, n, v, sid=200.0, sdd=320.0, off_u=2.5)
    cx, cy, cz = W.voxel_centres(g)
    c0 = np.array([2.3, -3.1, 1.7])
    sig, amp = SIG, 0.02
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    vol = amp * np.exp(-((X - c0[0]) ** 2 + (Y - c0[1]) ** 2 + (Z - c0[2]) ** 2) / (2 * sig * sig))
    rays, ref = [], []
    for a in range(g["n_angles"]):
        for iv in range(0, g["nv"], 3):
            for iu in range(0, g["nu"], 3):
                S, d = oracle.ray(g, a, iu, iv)
                val = analytic.gaussian_line_integral(S, d, c0, sig, amp)
                if val > 0.2 * amp * sig * math.sqrt(2 * math.pi):
                    rays.append((a * g["nv"] + iv) * g["nu"] + iu)
                    ref.append(val)
    got = oracle.forward_rays(g, vol, np.array(rays))
    return np.max(np.abs(got - ref)) / (amp * sig * math.sqrt(2 * math.pi))


def test_gaussian_blob_second_order(oracle):
    """Voxelised Gaussian: the projection error relative to the peak line
    integral stays under the bilinear-interpolation bound h^2/(2 sigma^2) and
    falls by more than 3x when the pitch halves."""
    e_coarse = _gaussian_case(oracle, 32, 2.0)
    e_fine = _gaussian_case(oracle, 64, 1.0)
    assert e_coarse <= 2.0 ** 2 / (2 * SIG ** 2)
    assert e_fine <= 1.0 ** 2 / (2 * SIG ** 2)
    assert e_coarse / e_fine > 3.0


def _sphere_case(oracle, n, v):
    g = W.geometry(6, 40, 40, 1.6, 1.6, n, n, n, v, sid=200.0, sdd=320.0, off_u=-3.0)
    cx, cy, cz = W.voxel_centres(g)
    c0, R, mu = np.array([1.3, -0.7, 2.1]), 14.0, 0.02
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    vol = mu * (((X - c0[0]) ** 2 + (Y - c0[1]) ** 2 + (Z - c0[2]) ** 2) < R * R)
    y = oracle.forward(g, vol)
    rel, worst = [], 0.0
    for a in range(g["n_angles"]):
        for iv in range(g["nv"]):
            for iu in range(g["nu"]):
                S, d = oracle.ray(g, a, iu, iv)
                u = d / np.linalg.norm(d)
                w = c0 - S
                b = math.sqrt(max(w @ w - (w @ u) ** 2, 0.0))
                if b > R / 2:
                    continue
                ref = mu * 2 * math.sqrt(R * R - b * b)
                m = 0 if abs(d[0]) >= abs(d[1]) else 1
                ds = v * np.linalg.norm(d) / abs(d[m])
                worst = max(worst, abs(y[a, iv, iu] - ref) / (mu * ds))
                rel.append((y[a, iv, iu] - ref) / ref)
    return worst, math.sqrt(np.mean(np.square(rel)))


def test_uniform_sphere_chord_first_order(oracle):
    w1, r1 = _sphere_case(oracle, 20, 2.0)
    w2, r2 = _sphere_case(oracle, 40, 1.0)
    assert w1 <= 4.0 and w2 <= 4.0
    assert r1 / r2 > 1.4


def test_ellipsoid_phantom_against_chords(oracle):
    """c1-style phantom: the discrete projection approaches the sum of exact
    ellipsoid chords as the grid is refined (sanity of the phantom path)."""
    errs = []
    for n, v in ((32, 8.0), (64, 4.0)):
        g = W.geometry(8, 64, 64, 6.4, 6.4, n, n, n, v)
        el = W.ellipsoid_list(W.C1, 3)
        vol = W.voxelise(g, el)
        y = oracle.forward(g, vol)
        ref = np.zeros_like(y)
        for a in range(g["n_angles"]):
            for iv in range(g["nv"]):
                for iu in range(g["nu"]):
                    S, d = oracle.ray(g, a, iu, iv)
                    ref[a, iv, iu] = sum(e["mu"] * analytic.chord_ellipsoid(S, d, e["centre"], e["axes"], e["rot"]) for e in el)
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.05
    assert errs[0] / errs[1] > 1.5


# ----------------------------------------------- brute force (P7, P8) ---

def test_siddon_additivity_and_footprint_centroids(oracle):
    g = tiny()
    L = oracle.siddon_dense(g)
    A = oracle.dense_matrix(g)
    cx, cy, cz = W.voxel_centres(g)
    lo = np.array([cx[0] - 2, cy[0] - 2, cz[0] - 2])
    hi = np.array([cx[-1] + 2, cy[-1] + 2, cz[-1] + 2])
    nu, nv = g["nu"], g["nv"]
    for r in range(L.shape[0]):
        iu, iv, a = r % nu, (r // nu) % nv, r // (nu * nv)
        assert abs(L[r].sum() - oracle.chord_box(g, a, iu, iv, lo, hi)) < 1e-12
    U, V = np.meshgrid(np.arange(nu), np.arange(nv))
    checked = 0
    for v in range(A.shape[1]):
        for a in range(g["n_angles"]):
            fa = A[a * nu * nv:(a + 1) * nu * nv, v].reshape(nv, nu)
            fl = L[a * nu * nv:(a + 1) * nu * nv, v].reshape(nv, nu)
            if fa.sum() == 0 or fl.sum() == 0:
                continue
            # only footprints fully inside the panel
            if fl[0].any() or fl[-1].any() or fl[:, 0].any() or fl[:, -1].any():
                continue
            ca = np.array([(fa * U).sum(), (fa * V).sum()]) / fa.sum()
            cl = np.array([(fl * U).sum(), (fl * V).sum()]) / fl.sum()
            assert np.all(np.abs(ca - cl) < 0.5), (v, a, ca, cl)
            checked += 1
    assert checked > 1000


def test_dense_transpose_exact(oracle):
    g = tiny()
    A = oracle.dense_matrix(g)
    nray = A.shape[0]
    e = np.zeros(nray)
    for r in range(nray):
        e[r] = 1.0
        row = oracle.adjoint(g, e.reshape(W.sino_shape(g)), nthreads=1).ravel()
        e[r] = 0.0
        assert np.max(np.abs(row - A[r])) <= 1e-15
    assert np.count_nonzero(A) > 0.02 * A.size


def test_gather_adjoint_equals_scatter_adjoint(oracle):
    g = tiny(n_angles=11, off_u=5.0)
    y = W.random_sino(g, 5)
    full = oracle.adjoint(g, y)
    idx = np.arange(full.size)
    part = oracle.adjoint_voxels(g, y, idx)
    assert np.max(np.abs(part - full.ravel())) <= 1e-13 * np.max(np.abs(full))


def test_sample_count_equals_supported_plane_pairs(oracle):
    """S counts (ray, plane) pairs whose plane carries positive weight."""
    g = tiny()
    A = oracle.dense_matrix(g)
    nx, ny, nz = g["nx"], g["ny"], g["nz"]
    nu, nv = g["nu"], g["nv"]
    count = 0
    for r in range(A.shape[0]):
        iu, iv, a = r % nu, (r // nu) % nv, r // (nu * nv)
        _, d = oracle.ray(g, a, iu, iv)
        Ar = A[r].reshape(nz, ny, nx)
        per_plane = Ar.sum(axis=(0, 1)) if abs(d[0]) >= abs(d[1]) else Ar.sum(axis=(0, 2))
        count += int(np.count_nonzero(per_plane > 0))
    assert oracle.sample_count(g) == count


# ----------------------------------------------- identities (P9, P10) ---

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dot_product_identity(oracle, seed):
    for g in (W.cropped(W.C1, n_angles=16, nu=96, nv=64, n=48),
              W.cropped(W.C2, n_angles=6, nu=160, nv=96, n=64)):
        x = W.random_volume(g, seed)
        y = W.random_sino(g, seed + 100)
        Ax = oracle.forward(g, x)
        ATy = oracle.adjoint(g, y)
        lhs, rhs = float(np.vdot(Ax, y)), float(np.vdot(x, ATy))
        assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_rotation_by_quarter_turn_shifts_angles(oracle):
    n = 12
    g = W.geometry(n, 24, 14, 3.0, 3.0, 12, 12, 7, 3.0, vz=2.5, sid=150.0, sdd=240.0, off_u=4.0)
    x = W.random_volume(g, 11)
    N = g["nx"]
    rot = np.empty_like(x)
    for i in range(N):
        for j in range(N):
            rot[:, j, i] = x[:, N - 1 - i, j]      # x rotated by +90 deg about z
    y = oracle.forward(g, x)
    yr = oracle.forward(g, rot)
    ties = 0
    for a in range(n):
        for iu in range(g["nu"]):
            _, d = oracle.ray(g, a, iu, 0)
            if abs(abs(d[0]) - abs(d[1])) < 1e-9 * abs(d[0]):
                ties += 1
                continue
            ref = y[(a - n // 4) % n, :, iu]
            assert np.max(np.abs(yr[a, :, iu] - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert ties < n


def test_z_flip_and_linearity(oracle):
    g = tiny(off_v=0.0, n_angles=6)
    x1 = W.random_volume(g, 21)
    x2 = W.random_volume(g, 22)
    y1 = oracle.forward(g, x1)
    assert np.allclose(oracle.forward(g, x1[::-1]), y1[:, ::-1], rtol=0, atol=1e-12)
    y2 = oracle.forward(g, x2)
    assert np.allclose(oracle.forward(g, 2.5 * x1 - 0.75 * x2), 2.5 * y1 - 0.75 * y2, rtol=0, atol=1e-12)


# ------------------------------------------------------------ CGLS (P11) ---

def test_cgls_reaches_least_squares_solution(oracle):
    g = tiny(n_angles=24, nu=20, nv=16, nx=6, ny=6, nz=6)
    A = oracle.dense_matrix(g)
    xt = W.random_volume(g, 7)
    y = (A @ xt.ravel() + 0.01 * W.rng(8).standard_normal(A.shape[0])).reshape(W.sino_shape(g))
    ref = np.linalg.lstsq(A, y.ravel(), rcond=None)[0]
    x = oracle.cgls(g, y, 120)
    assert np.linalg.norm(x.ravel() - ref) <= 1e-10 * np.linalg.norm(ref)


def test_cgls_iterates_minimise_over_krylov_subspaces(oracle):
    """The k-th CGLS iterate (x0 = 0) minimises |Ax - y| over the Krylov
    space span{b, Mb, ..., M^(k-1) b}, b = A^T y, M = A^T A."""
    g = tiny(n_angles=10, nu=14, nv=10)
    A = oracle.dense_matrix(g)
    y = W.random_sino(g, 12)
    b = A.T @ y.ravel()
    its = {}
    oracle.cgls(g, y, 8, callback=lambda k, x: its.__setitem__(k, x.ravel().copy()))
    V = np.zeros((b.size, 0))
    v = b.copy()
    for k in range(1, 9):
        for _ in range(2):                       # Gram-Schmidt, twice
            v = v - V @ (V.T @ v)
        V = np.column_stack([V, v / np.linalg.norm(v)])
        coef = np.linalg.lstsq(A @ V, y.ravel(), rcond=None)[0]
        ref = V @ coef
        assert np.linalg.norm(its[k] - ref) <= 1e-9 * np.linalg.norm(ref)
        v = A.T @ (A @ V[:, -1])


def test_landweber_step_is_gradient_of_least_squares(oracle):
    """The Landweber term A^T(Ax - y) is the gradient of 0.5|Ax - y|^2."""
    g = tiny(n_angles=5)
    x = W.random_volume(g, 3)
    y = W.random_sino(g, 4)
    grad = oracle.adjoint(g, oracle.forward(g, x) - y)
    f = lambda z: 0.5 * float(np.sum((oracle.forward(g, z) - y) ** 2))
    r = W.rng(9)
    for _ in range(5):
        v = r.integers(0, x.size)
        e = np.zeros(x.size)
        e[v] = 1e-3
        e = e.reshape(x.shape)
        fd = (f(x + e) - f(x - e)) / 2e-3
        assert abs(fd - grad.ravel()[v]) <= 1e-7 * max(1.0, abs(fd))


def test_samples_stop_at_the_pixel(oracle):
    """Only crossings strictly between source and pixel are sampled: with the
    panel cutting through a constant volume, the ray value is the clipped
    chord to within one plane spacing."""
    g = W.geometry(6, 12, 10, 3.0, 3.0, 20, 20, 20, 3.0, sid=100.0, sdd=115.0)
    cx, cy, cz = W.voxel_centres(g)
    lo = np.array([cx[0] - 1.5, cy[0] - 1.5, cz[0] - 1.5])
    hi = np.array([cx[-1] + 1.5, cy[-1] + 1.5, cz[-1] + 1.5])
    y = oracle.forward(g, np.ones(W.vol_shape(g)))
    for a in range(g["n_angles"]):
        for iv in range(2, g["nv"] - 2):
            for iu in range(2, g["nu"] - 2):
                S, d = oracle.ray(g, a, iu, iv)
                m = 0 if abs(d[0]) >= abs(d[1]) else 1
                ds = 3.0 * np.linalg.norm(d) / abs(d[m])
                chord = oracle.chord_box(g, a, iu, iv, lo, hi)
                assert abs(y[a, iv, iu] - chord) <= 1.01 * ds


def test_opnorm_equals_largest_singular_value(oracle):
    """The power iteration's ||A||_2 (the normalisation constant of the
    learned net's operators) equals the largest singular value of the dense
    matrix, computed by LAPACK's SVD: a missing square root, a wrong Rayleigh
    quotient or a missing normalisation would all miss it by far."""
    g = tiny()
    smax = np.linalg.norm(oracle.dense_matrix(g), 2)
    L = oracle.opnorm(g, iters=200)
    assert abs(L - smax) <= 1e-10 * smax
    # a second geometry with an offset panel and another seed for the start
    g2 = tiny(n_angles=6, off_u=-2.0)
    smax2 = np.linalg.norm(oracle.dense_matrix(g2), 2)
    assert abs(oracle.opnorm(g2, iters=300, seed=3) - smax2) <= 1e-10 * smax2
