"""FP64 CPU oracle for the cone-beam projector pair -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path (the HIP library and its
Python binding) never imports it and shares no code with it.

Contents, each written from the paper (arXiv 2512.21180):

* ``forward`` / ``adjoint`` / ``forward_rays`` / ``adjoint_voxels`` /
  ``sample_count``: the discretised cone-beam transform P and its transpose
  (Sec. 2.2, definition of the projection operator and of the backprojection
  as its adjoint), implemented in plain C (``cbct_oracle.c``) in FP64.
* ``ray``, ``weight``, ``chord_box``, ``siddon_dense``, ``interp_integral``:
  independent references used by the pins (exact chord lengths, brute-force
  path lengths, exact line integrals of the trilinear interpolant).
* ``dense_matrix``: A built column by column from unit volumes.
* ``cgls`` / ``landweber``: FP64 least-squares solvers on top of the oracle
  operators; Landweber uses the gradient term P*(P x - y) of Alg. 1.
* ``water_bone`` / ``detector_response`` / ``sim_poly``: the polychromatic
  water-bone primary model (Sec. 2.2, eq. primarymodel) and the normalised
  negative log (Sec. 2.4, eq. normprimary).
* ``march`` / ``scatter_paths`` / ``scatter_integrate``: the quasi-Monte
  Carlo scatter model (Sec. 2.3, Alg. 2 and Alg. 3).

Geometry is passed as a plain dict with keys sid, sdd, n_angles, angles
(optional, radians), nu, nv, du, dv, off_u, off_v, nx, ny, nz, vx, vy, vz,
origin (3-tuple, mm).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cbct_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle's C source into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _OGeom(ctypes.Structure):
    _fields_ = [
        ("sid", ctypes.c_double), ("sdd", ctypes.c_double),
        ("n_angles", ctypes.c_int), ("angles", ctypes.POINTER(ctypes.c_double)),
        ("nu", ctypes.c_int), ("nv", ctypes.c_int),
        ("du", ctypes.c_double), ("dv", ctypes.c_double),
        ("off_u", ctypes.c_double), ("off_v", ctypes.c_double),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("vx", ctypes.c_double), ("vy", ctypes.c_double), ("vz", ctypes.c_double),
        ("ox", ctypes.c_double), ("oy", ctypes.c_double), ("oz", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i64 = ctypes.c_double, ctypes.c_int64
        G = P(_OGeom)
        lib.orc_ray.argtypes = [G, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(d), P(d)]
        lib.orc_forward.argtypes = [G, P(d), P(d), ctypes.c_int]
        lib.orc_adjoint.argtypes = [G, P(d), P(d), ctypes.c_int]
        lib.orc_forward_rays.argtypes = [G, P(d), P(i64), i64, P(d), ctypes.c_int]
        lib.orc_adjoint_voxels.argtypes = [G, P(d), P(i64), i64, P(d), ctypes.c_int]
        lib.orc_sample_count.argtypes = [G, ctypes.c_int]
        lib.orc_sample_count.restype = i64
        lib.orc_weight.argtypes = [G] + [ctypes.c_int] * 6
        lib.orc_weight.restype = d
        lib.orc_chord_box.argtypes = [G, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(d), P(d)]
        lib.orc_chord_box.restype = d
        lib.orc_siddon_dense.argtypes = [G, P(d)]
        lib.orc_interp_integral.argtypes = [G, P(d), ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.orc_interp_integral.restype = d
        u32 = ctypes.c_uint32
        lib.orc_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
        lib.orc_poisson.argtypes = [d, ctypes.c_uint64, u32, ctypes.c_uint64]
        lib.orc_poisson.restype = i64
        lib.orc_sim_poisson_log.argtypes = [i64, P(d), d, ctypes.c_uint64, u32, P(i64), P(d)]
        lib.orc_sim_gaussian.argtypes = [i64, P(d), d, ctypes.c_uint64, u32, P(d)]
        lib.orc_sim_poly.argtypes = [i64, i64, P(d), P(d), ctypes.c_int, P(d), P(d), P(d), P(d),
                                     ctypes.c_uint64, u32, P(i64), P(d), P(d)]
        X = P(_OXs)
        lib.orc_march.argtypes = [G, P(d), P(d), P(d), P(d), d, P(d)]
        lib.orc_compton_energy.argtypes = [d, d]
        lib.orc_compton_energy.restype = d
        lib.orc_resp.argtypes = [d]
        lib.orc_resp.restype = d
        lib.orc_scatter_direction.argtypes = [P(d), d, d, P(d)]
        lib.orc_scatter_paths.argtypes = [G, P(d), P(d), X, ctypes.c_int, i64, P(d), P(d),
                                          ctypes.c_int, P(d)]
        lib.orc_scatter_integrate.argtypes = [G, P(d), P(d), X, ctypes.c_int, i64, P(d), P(d)]
        _lib = lib
    return _lib


class _OXs(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int), ("e0", ctypes.c_double), ("de", ctypes.c_double),
        ("mu", ctypes.POINTER(ctypes.c_double)),
        ("J", ctypes.c_int), ("icdf", ctypes.POINTER(ctypes.c_double)),
        ("I", ctypes.c_int), ("dens", ctypes.POINTER(ctypes.c_double)),
    ]


def angles_of(g: dict) -> np.ndarray:
    """Source angles: the explicit list if given, else 2*pi*a/n (a = 0..n-1)."""
    if g.get("angles") is not None:
        a = np.asarray(g["angles"], dtype=np.float64)
        assert a.shape == (g["n_angles"],)
        return a
    n = g["n_angles"]
    return 2.0 * np.pi * np.arange(n, dtype=np.float64) / n


class _Geom:
    """ctypes view of a geometry dict; keeps the angle array alive."""

    def __init__(self, g: dict):
        self.angles = np.ascontiguousarray(angles_of(g))
        o = g.get("origin", (0.0, 0.0, 0.0))
        self.s = _OGeom(
            float(g["sid"]), float(g["sdd"]), int(g["n_angles"]),
            self.angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            int(g["nu"]), int(g["nv"]), float(g["du"]), float(g["dv"]),
            float(g.get("off_u", 0.0)), float(g.get("off_v", 0.0)),
            int(g["nx"]), int(g["ny"]), int(g["nz"]),
            float(g["vx"]), float(g["vy"]), float(g["vz"]),
            float(o[0]), float(o[1]), float(o[2]),
        )

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def vol_shape(g: dict):
    return (g["nz"], g["ny"], g["nx"])


def sino_shape(g: dict):
    return (g["n_angles"], g["nv"], g["nu"])


def forward(g: dict, vol: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """Sinogram [n_angles][nv][nu] = A vol (vol is [nz][ny][nx])."""
    lib = _load()
    G = _Geom(g)
    x = np.ascontiguousarray(vol, dtype=np.float64)
    assert x.shape == vol_shape(g)
    y = np.zeros(sino_shape(g), dtype=np.float64)
    lib.orc_forward(G.ref, _dp(x), _dp(y), nthreads)
    return y


def adjoint(g: dict, sino: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """Volume [nz][ny][nx] = A^T sino (scatter form)."""
    lib = _load()
    G = _Geom(g)
    y = np.ascontiguousarray(sino, dtype=np.float64)
    assert y.shape == sino_shape(g)
    x = np.zeros(vol_shape(g), dtype=np.float64)
    rc = lib.orc_adjoint(G.ref, _dp(y), _dp(x), nthreads)
    if rc != 0:
        raise MemoryError("oracle adjoint could not allocate its accumulators")
    return x


def forward_rays(g: dict, vol: np.ndarray, rays: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """A vol at flat ray indices (a*nv + iv)*nu + iu."""
    lib = _load()
    G = _Geom(g)
    x = np.ascontiguousarray(vol, dtype=np.float64)
    r = np.ascontiguousarray(rays, dtype=np.int64)
    out = np.zeros(r.shape[0], dtype=np.float64)
    lib.orc_forward_rays(G.ref, _dp(x), _ip(r), r.shape[0], _dp(out), nthreads)
    return out


def adjoint_voxels(g: dict, sino: np.ndarray, voxels: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """A^T sino at flat voxel indices (k*ny + j)*nx + i (gather form)."""
    lib = _load()
    G = _Geom(g)
    y = np.ascontiguousarray(sino, dtype=np.float64)
    v = np.ascontiguousarray(voxels, dtype=np.int64)
    out = np.zeros(v.shape[0], dtype=np.float64)
    rc = lib.orc_adjoint_voxels(G.ref, _dp(y), _ip(v), v.shape[0], _dp(out), nthreads)
    if rc != 0:
        raise RuntimeError("oracle adjoint_voxels: footprint window too small")
    return out


def sample_count(g: dict, nthreads: int = 0) -> int:
    """Number of (ray, plane) samples with non-empty support."""
    lib = _load()
    G = _Geom(g)
    return int(lib.orc_sample_count(G.ref, nthreads))


def ray(g: dict, a: int, iu: int, iv: int):
    """Source S and direction d = P - S of ray (a, iu, iv)."""
    lib = _load()
    G = _Geom(g)
    S = np.zeros(3)
    d = np.zeros(3)
    lib.orc_ray(G.ref, a, iu, iv, _dp(S), _dp(d))
    return S, d


def weight(g: dict, a: int, iu: int, iv: int, i: int, j: int, k: int) -> float:
    lib = _load()
    G = _Geom(g)
    return float(lib.orc_weight(G.ref, a, iu, iv, i, j, k))


def chord_box(g: dict, a: int, iu: int, iv: int, lo, hi) -> float:
    """Exact length of ray (a, iu, iv) inside the box [lo, hi] (slab clipping)."""
    lib = _load()
    G = _Geom(g)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    return float(lib.orc_chord_box(G.ref, a, iu, iv, _dp(lo), _dp(hi)))


def siddon_dense(g: dict) -> np.ndarray:
    """Dense [n_rays, n_voxels] matrix of exact ray-in-voxel-cube lengths."""
    lib = _load()
    G = _Geom(g)
    nray = g["n_angles"] * g["nv"] * g["nu"]
    nvox = g["nx"] * g["ny"] * g["nz"]
    L = np.zeros((nray, nvox), dtype=np.float64)
    lib.orc_siddon_dense(G.ref, _dp(L))
    return L


def interp_integral(g: dict, vol: np.ndarray, a: int, iu: int, iv: int) -> float:
    """Exact line integral of the zero-padded trilinear interpolant of vol."""
    lib = _load()
    G = _Geom(g)
    x = np.ascontiguousarray(vol, dtype=np.float64)
    return float(lib.orc_interp_integral(G.ref, _dp(x), a, iu, iv))


def dense_matrix(g: dict) -> np.ndarray:
    """A as a dense [n_rays, n_voxels] matrix: column v = A e_v."""
    nvox = g["nx"] * g["ny"] * g["nz"]
    nray = g["n_angles"] * g["nv"] * g["nu"]
    A = np.zeros((nray, nvox))
    e = np.zeros(nvox)
    for v in range(nvox):
        e[v] = 1.0
        A[:, v] = forward(g, e.reshape(vol_shape(g)), nthreads=1).ravel()
        e[v] = 0.0
    return A


def cgls(g: dict, y: np.ndarray, iters: int, x0=None, callback=None) -> np.ndarray:
    """Conjugate gradients on the normal equations A^T A x = A^T y (FP64).

    Unregularised least squares started at x0 (default 0), the classical
    CGLS recursion (Hestenes-Stiefel): q = A p, alpha = |s|^2/|q|^2,
    x += alpha p, r -= alpha q, s = A^T r, beta = |s_new|^2/|s|^2,
    p = s_new + beta p.
    """
    x = np.zeros(vol_shape(g)) if x0 is None else np.array(x0, dtype=np.float64)
    r = np.asarray(y, dtype=np.float64) - forward(g, x)
    s = adjoint(g, r)
    p = s.copy()
    gamma = float(np.vdot(s, s))
    for it in range(iters):
        if gamma == 0.0:
            break
        q = forward(g, p)
        qq = float(np.vdot(q, q))
        if qq == 0.0:
            break
        alpha = gamma / qq
        x += alpha * p
        r -= alpha * q
        s = adjoint(g, r)
        gamma_new = float(np.vdot(s, s))
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        if callback is not None:
            callback(it + 1, x)
    return x


def opnorm(g: dict, iters: int = 50, seed: int = 0, x0=None) -> float:
    """||A||_2 by power iteration on A^T A (FP64), from x0 or a seeded start."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal(vol_shape(g)) if x0 is None else np.array(x0, dtype=np.float64)
    lam = 0.0
    for _ in range(iters):
        x /= np.linalg.norm(x)
        z = adjoint(g, forward(g, x))
        lam = float(np.vdot(x, z))
        x = z
    return float(np.sqrt(lam))


def landweber(g: dict, y: np.ndarray, iters: int, omega: float, x0=None) -> np.ndarray:
    """x <- x - omega * A^T (A x - y): the Landweber term of Alg. 1 as a solver."""
    x = np.zeros(vol_shape(g)) if x0 is None else np.array(x0, dtype=np.float64)
    for _ in range(iters):
        x -= omega * adjoint(g, forward(g, x) - y)
    return x


# ---- noise model (Sec. 2.2 noisy primary counts, Sec. 2.4 log transform) ----

def philox4x32_10(counter, key):
    """One Philox4x32-10 block (Salmon et al. 2011) as four Python ints."""
    lib = _load()
    U = ctypes.c_uint32 * 4
    K = ctypes.c_uint32 * 2
    out = U()
    lib.orc_philox4x32_10(U(*[int(c) & 0xffffffff for c in counter]),
                          K(*[int(k) & 0xffffffff for k in key]), out)
    return [int(v) for v in out]


def poisson(lam: float, seed: int, stream: int, i: int) -> int:
    """Poisson variate of element i (inversion below 10, PTRS from 10)."""
    return int(_load().orc_poisson(float(lam), seed, stream, i))


def sim_poisson_log(p: np.ndarray, I0: float, seed: int, stream: int = 0):
    """(y, counts): counts ~ Poisson(I0 exp(-p)), y = -log(min(max(counts,1)/I0, 1))."""
    lib = _load()
    pp = np.ascontiguousarray(p, dtype=np.float64).ravel()
    y = np.zeros_like(pp)
    c = np.zeros(pp.shape, dtype=np.int64)
    lib.orc_sim_poisson_log(pp.size, _dp(pp), float(I0), seed, stream, _ip(c), _dp(y))
    return y.reshape(np.shape(p)), c.reshape(np.shape(p))


def sim_gaussian(clean: np.ndarray, sigma: float, seed: int, stream: int = 0) -> np.ndarray:
    lib = _load()
    cc = np.ascontiguousarray(clean, dtype=np.float64).ravel()
    out = np.zeros_like(cc)
    lib.orc_sim_gaussian(cc.size, _dp(cc), float(sigma), seed, stream, _dp(out))
    return out.reshape(np.shape(clean))


# ---- polychromatic water-bone primary model (Sec. 2.2) ----

# Water-bone decomposition constants of Sec. 2.2.  tau_0 is not given; the
# decomposition is stated to be continuous in the modified CT number, and
# rho_w jumps from 0 to tau_0 at tau_0, so continuity fixes tau_0 = 0.
TAU0, TAU1, TAU2, KAPPA_B = 0.0, 1.2, 1.6, 0.409


def water_bone(hu: np.ndarray):
    """(rho_w, rho_b): water and bone relative densities of a CT volume in
    Hounsfield units, from the modified CT number rho^ = 0.001 HU + 1 by the
    two piecewise definitions of Sec. 2.2 (FP64)."""
    r = 0.001 * np.asarray(hu, dtype=np.float64) + 1.0
    rw = np.zeros_like(r)
    rb = np.zeros_like(r)
    m1 = (r >= TAU0) & (r < TAU1)
    m2 = (r >= TAU1) & (r < TAU2)
    m3 = r >= TAU2
    rw[m1] = r[m1]
    rw[m2] = TAU1 * (TAU2 - r[m2]) / (TAU2 - TAU1)
    rb[m2] = KAPPA_B * TAU2 * (r[m2] - TAU1) / (TAU2 - TAU1)
    rb[m3] = KAPPA_B * r[m3]
    return rw, rb


def energy_bins() -> np.ndarray:
    """Centres (keV) of the ten energy bins [10 i, 10 (i + 1)) keV, i = 2..11."""
    return np.array([10.0 * i + 5.0 for i in range(2, 12)])


def detector_response(e_kev) -> np.ndarray:
    """resp(e): piecewise linear through (20, 5), (60, 20), (120, 10) keV
    (Sec. 2.2); outside [20, 120] keV it keeps the end values."""
    e = np.asarray(e_kev, dtype=np.float64)
    out = np.empty_like(e)
    lo = e <= 20.0
    a = (e > 20.0) & (e <= 60.0)
    b = (e > 60.0) & (e < 120.0)
    hi = e >= 120.0
    out[lo] = 5.0
    out[a] = 5.0 + (e[a] - 20.0) * (20.0 - 5.0) / (60.0 - 20.0)
    out[b] = 20.0 + (e[b] - 60.0) * (10.0 - 20.0) / (120.0 - 60.0)
    out[hi] = 10.0
    return out


def sim_poly(pw: np.ndarray, pb: np.ndarray, mu_w, mu_b, resp, I0: np.ndarray, seed: int,
             stream: int = 0):
    """Noisy polychromatic primary projections (eq. primarymodel) and their
    normalised negative log (eq. normprimary), given the material line
    integrals pw = P(rho_w), pb = P(rho_b) of shape [..., nv, nu]; I0 is
    [n_bins, nv, nu] (photons per pixel and bin, every projection alike),
    mu_w, mu_b (mm^-1 at unit density) and resp per bin.  Returns
    (y, signal, counts[n_bins, ...]); see orc_sim_poly for the reading of
    zero signal and of the air scan."""
    lib = _load()
    shape = np.shape(pw)
    a = np.ascontiguousarray(pw, dtype=np.float64).ravel()
    b = np.ascontiguousarray(pb, dtype=np.float64).ravel()
    i0 = np.ascontiguousarray(I0, dtype=np.float64)
    nb = i0.shape[0]
    npix = i0[0].size
    assert a.size == b.size and a.size % npix == 0
    mw = np.ascontiguousarray(mu_w, dtype=np.float64)
    mb = np.ascontiguousarray(mu_b, dtype=np.float64)
    rs = np.ascontiguousarray(resp, dtype=np.float64)
    assert mw.size == mb.size == rs.size == nb
    y = np.zeros_like(a)
    sig = np.zeros_like(a)
    c = np.zeros((nb, a.size), dtype=np.int64)
    lib.orc_sim_poly(a.size, npix, _dp(a), _dp(b), nb, _dp(mw), _dp(mb), _dp(rs), _dp(i0.ravel()),
                     seed, stream, _ip(c), _dp(sig), _dp(y))
    return y.reshape(shape), sig.reshape(shape), c.reshape((nb,) + tuple(shape))


# ---- scatter simulator (Sec. 2.3, Alg. 2 and Alg. 3; appendix eqs. beer,
# lambdameas, distsample and the Compton energy) ----
#
# Cross sections are a dict: e0, de (keV grid), mu [2 materials (water, bone)]
# [3 kinds (photoelectric, Compton, Rayleigh)][K] (mm^-1 at unit density),
# icdf [2][2 types (Compton, Rayleigh)][K][J] (cos theta at u = j / (J - 1)),
# dens [2][2][K][I] (scatter directions per steradian at
# cos theta = -1 + 2 i / (I - 1)).  See cbct_oracle.c for the readings.

def _xs_struct(xs: dict):
    mu = np.ascontiguousarray(xs["mu"], dtype=np.float64)
    ic = np.ascontiguousarray(xs["icdf"], dtype=np.float64)
    dn = np.ascontiguousarray(xs["dens"], dtype=np.float64)
    K = mu.shape[-1]
    assert mu.shape == (2, 3, K) and ic.shape[:3] == (2, 2, K) and dn.shape[:3] == (2, 2, K)
    st = _OXs(K, float(xs["e0"]), float(xs["de"]), _dp(mu), ic.shape[3], _dp(ic),
              dn.shape[3], _dp(dn))
    return st, (mu, ic, dn)


def march(g: dict, rw, rb, p, d, tmax: float):
    """(int rho_w, int rho_b) along p + t d, 0 <= t <= tmax (d a unit vector),
    voxels as cubes of constant density."""
    lib = _load()
    G = _Geom(g)
    a = np.ascontiguousarray(rw, dtype=np.float64)
    b = np.ascontiguousarray(rb, dtype=np.float64)
    out = np.zeros(2)
    lib.orc_march(G.ref, _dp(a), _dp(b), _dp(np.asarray(p, dtype=np.float64)),
                  _dp(np.asarray(d, dtype=np.float64)), float(tmax), _dp(out))
    return out


def compton_energy(e: float, cos_theta: float) -> float:
    return float(_load().orc_compton_energy(float(e), float(cos_theta)))


def resp(e: float) -> float:
    return float(_load().orc_resp(float(e)))


def scatter_direction(v, cos_theta: float, phi: float) -> np.ndarray:
    out = np.zeros(3)
    _load().orc_scatter_direction(_dp(np.asarray(v, dtype=np.float64)), float(cos_theta),
                                  float(phi), _dp(out))
    return out


def scatter_paths(g: dict, rw, rb, xs: dict, a: int, src, sob, n: int) -> np.ndarray:
    """SamplePath (Alg. 2) at projection a: [N, n + 1, 8] records (interaction
    point, arriving direction, arriving energy, weight).  src [N, 4]: unit
    direction for the source at angle 0 and energy (keV); sob [N, 5 n + 1]."""
    lib = _load()
    G = _Geom(g)
    st, keep = _xs_struct(xs)
    a_ = np.ascontiguousarray(rw, dtype=np.float64)
    b_ = np.ascontiguousarray(rb, dtype=np.float64)
    sp = np.ascontiguousarray(src, dtype=np.float64)
    so = np.ascontiguousarray(sob, dtype=np.float64)
    N = sp.shape[0]
    assert sp.shape == (N, 4) and so.shape == (N, 5 * n + 1)
    rec = np.zeros((N, n + 1, 8))
    lib.orc_scatter_paths(G.ref, _dp(a_), _dp(b_), ctypes.byref(st), int(a), N, _dp(sp),
                          _dp(so), int(n), _dp(rec))
    return rec


def scatter_integrate(g: dict, rw, rb, xs: dict, a: int, rec) -> np.ndarray:
    """Integrate (Alg. 3) at projection a over records [..., 8]: the expected
    scatter [nv, nu] on the panel of g (before the I_Sigma / |Src| scale)."""
    lib = _load()
    G = _Geom(g)
    st, keep = _xs_struct(xs)
    a_ = np.ascontiguousarray(rw, dtype=np.float64)
    b_ = np.ascontiguousarray(rb, dtype=np.float64)
    r = np.ascontiguousarray(rec, dtype=np.float64).reshape(-1, 8)
    out = np.zeros((g["nv"], g["nu"]))
    lib.orc_scatter_integrate(G.ref, _dp(a_), _dp(b_), ctypes.byref(st), int(a), r.shape[0],
                              _dp(r), _dp(out))
    return out


# ---- 3x3x3 convolutions of the learned blocks (Alg. 1, dual/primal blocks) ----
#
# Plain FP64 definitions, zero padding ("same" size), cross-correlation with
# weight w[co][ci][kz][ky][kx] applied to x[ci][z + kz - 1][y + ky - 1][x + kx - 1].

def _shift_views(D, H, W):
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                yield kz, ky, kx


def conv3(x: np.ndarray, w: np.ndarray, b=None) -> np.ndarray:
    """y[co] = b[co] + sum_{ci,k} w[co,ci,k] x[ci, . + k - 1]  (FP64)."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    C, D, H, W = x.shape
    xp = np.zeros((C, D + 2, H + 2, W + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    y = np.zeros((w.shape[0], D, H, W))
    for kz, ky, kx in _shift_views(D, H, W):
        patch = xp[:, kz:kz + D, ky:ky + H, kx:kx + W].reshape(C, -1)
        y += (w[:, :, kz, ky, kx] @ patch).reshape(y.shape)
    if b is not None:
        y += np.asarray(b, np.float64)[:, None, None, None]
    return y


def conv3_dgrad(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """dx[ci] = sum_{co,k} w[co,ci,k] dy[co, . - k + 1]: the transpose of conv3."""
    dy = np.asarray(dy, np.float64)
    w = np.asarray(w, np.float64)
    Co, D, H, W = dy.shape
    dxp = np.zeros((w.shape[1], D + 2, H + 2, W + 2))
    for kz, ky, kx in _shift_views(D, H, W):
        contrib = (w[:, :, kz, ky, kx].T @ dy.reshape(Co, -1)).reshape(-1, D, H, W)
        dxp[:, kz:kz + D, ky:ky + H, kx:kx + W] += contrib
    return dxp[:, 1:-1, 1:-1, 1:-1]


def conv3_wgrad(x: np.ndarray, dy: np.ndarray):
    """dw[co,ci,k] = sum_s dy[co,s] x[ci, s + k - 1];  db[co] = sum_s dy[co,s]."""
    x = np.asarray(x, np.float64)
    dy = np.asarray(dy, np.float64)
    C, D, H, W = x.shape
    Co = dy.shape[0]
    xp = np.zeros((C, D + 2, H + 2, W + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    dw = np.zeros((Co, C, 3, 3, 3))
    g = dy.reshape(Co, -1)
    for kz, ky, kx in _shift_views(D, H, W):
        patch = xp[:, kz:kz + D, ky:ky + H, kx:kx + W].reshape(C, -1)
        dw[:, :, kz, ky, kx] = g @ patch.T
    return dw, g.sum(axis=1)


def leaky_relu(v, slope):
    return np.where(v > 0, v, slope * v)


# ---- field-of-view tensor V (Alg. 1 input; Sec. 2.6) -------------------------

def fov_fraction(g: dict) -> np.ndarray:
    """V[z][y][x]: fraction of the projections in which the ray from the
    source through the voxel centre meets the panel's sensitive area
    (|u - off_u| <= nu du / 2 and |v - off_v| <= nv dv / 2, u and v the
    central projection of the centre onto the panel plane).  Brute force over
    voxels and angles, FP64."""
    nx, ny, nz = g["nx"], g["ny"], g["nz"]
    o = g.get("origin", (0.0, 0.0, 0.0))
    cx = o[0] + (np.arange(nx) - 0.5 * (nx - 1)) * g["vx"]
    cy = o[1] + (np.arange(ny) - 0.5 * (ny - 1)) * g["vy"]
    cz = o[2] + (np.arange(nz) - 0.5 * (nz - 1)) * g["vz"]
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    count = np.zeros(X.shape)
    for th in angles_of(g):
        c, s = np.cos(th), np.sin(th)
        D = g["sid"] - (X * c + Y * s)            # depth along the central ray
        u = g["sdd"] * (Y * c - X * s) / D
        v = g["sdd"] * Z / D
        vis = ((D > 0) & (np.abs(u - g["off_u"]) <= 0.5 * g["nu"] * g["du"])
               & (np.abs(v - g["off_v"]) <= 0.5 * g["nv"] * g["dv"]))
        count += vis
    return count / g["n_angles"]


# ---- learned primal-dual net (Alg. 1) ----------------------------------------
#
# Per iteration i at resolution 1/r_i (r_i in {1, 2, 4}, non-increasing), with
# primal latent f (8 volumes), dual latent h (8 sinograms) at that resolution,
# the full-resolution reconstruction x, normalised operators A_r / L of the
# scaled geometry (every r-th projection, voxels and pixels r times larger)
# and normalised data y:
#   xb = Downsample_r(x) (average pooling);  yb = ProjDown_r(y);  Vb = Downsample_r(V)
#   d1, d2 = halves of h;  p1, p2 = halves of f
#   d2 <- d2 + Gamma_i([A_r p2 / L, A_r xb / L, d1, yb])       (10 -> 4 channels)
#   p2 <- p2 + Lambda_i([A_r^T d2 / L, p1, xb, LW, Vb])       (11 -> 4 channels)
#        with LW = A_r^T (A_r xb / L - yb) / L, the Landweber term
#   x  <- x + Upsample_r(o_i . [p1, p2] + o_i,bias)             (1x1x1 conv 8 -> 1)
#   h, f <- Perm(h, rho_i), Perm(f, rho_i)    (new channel k = old channel rho_i[k])
#   then, if r_{i+1} < r_i, h and f are upsampled (nearest) by r_i / r_{i+1}.
# Blocks: conv3 -> LeakyReLU -> conv3 -> LeakyReLU -> conv3.  Start: x = x0
# (zero unless given), f = [Downsample(x0), Downsample(A^T y / L)] x 4,
# h = [ProjDown(y)] x 8 at resolution 1/r_1.  One constant L for every scale
# (so that A_r Downsample(x) / L is close to ProjDown(A x / L)).
# params[i] = {"dual": [w1, b1, w2, b2, w3, b3], "primal": [...],
#              "out": array of 9 (8 weights, bias), "perm": 8 indices}.

def scaled_geometry(g: dict, r: int) -> dict:
    """The geometry of P_alpha, r = 1/alpha: every r-th projection, voxels
    and pixels r times larger over the same volume and panel."""
    if r == 1:
        return g
    h = dict(g)
    h["angles"] = angles_of(g)[::r]
    h["n_angles"] = len(h["angles"])
    for n, d in (("nx", "vx"), ("ny", "vy"), ("nz", "vz"), ("nu", "du"), ("nv", "dv")):
        h[n] = g[n] // r
        h[d] = g[d] * r
    return h


def downsample(x: np.ndarray, r: int) -> np.ndarray:
    """Average over r x r x r blocks."""
    a, b, c = x.shape
    return x.reshape(a // r, r, b // r, r, c // r, r).mean(axis=(1, 3, 5))


def projdown(y: np.ndarray, r: int) -> np.ndarray:
    """Every r-th projection, averaged over r x r pixel blocks."""
    a, b, c = y.shape
    return y[::r].reshape(a // r, b // r, r, c // r, r).mean(axis=(2, 4))


def upsample(z: np.ndarray, r: int) -> np.ndarray:
    """Nearest upsampling by r along all three axes."""
    return np.repeat(np.repeat(np.repeat(z, r, axis=0), r, axis=1), r, axis=2)


def _block_fwd(z, p, slope):
    w1, b1, w2, b2, w3, b3 = p
    a1 = conv3(z, w1, b1)
    h1 = leaky_relu(a1, slope)
    a2 = conv3(h1, w2, b2)
    h2 = leaky_relu(a2, slope)
    return conv3(h2, w3, b3), (z, a1, h1, a2, h2)


def _block_bwd(g_out, cache, p, slope):
    w1, b1, w2, b2, w3, b3 = p
    z, a1, h1, a2, h2 = cache
    dw3, db3 = conv3_wgrad(h2, g_out)
    g_a2 = conv3_dgrad(g_out, w3) * np.where(a2 > 0, 1.0, slope)
    dw2, db2 = conv3_wgrad(h1, g_a2)
    g_a1 = conv3_dgrad(g_a2, w2) * np.where(a1 > 0, 1.0, slope)
    dw1, db1 = conv3_wgrad(z, g_a1)
    return conv3_dgrad(g_a1, w1), [dw1, db1, dw2, db2, dw3, db3]


def _lpd_iter(g, f, h, xb, yb, Vb, p, L, slope):
    """One coupling step at one resolution; returns the permuted latents,
    the output convolution's value (at that resolution) and a cache."""
    d1, d2 = h[:4], h[4:]
    p1, p2 = f[:4], f[4:]
    Ax = forward(g, xb) / L
    gin = np.stack([forward(g, c) / L for c in p2] + [Ax] + d1 + [yb])
    gout, cg = _block_fwd(gin, p["dual"], slope)
    d2n = [d2[k] + gout[k] for k in range(4)]
    LW = adjoint(g, Ax - yb) / L
    pin = np.stack([adjoint(g, c) / L for c in d2n] + p1 + [xb, LW, Vb])
    pout, cp = _block_fwd(pin, p["primal"], slope)
    p2n = [p2[k] + pout[k] for k in range(4)]
    fn, hn = p1 + p2n, d1 + d2n
    o = np.asarray(p["out"], np.float64)
    c = sum(o[k] * fn[k] for k in range(8)) + o[8]
    rho = list(p["perm"])
    return [fn[k] for k in rho], [hn[k] for k in rho], c, (cg, cp, fn, hn)


def _scales(params, scales):
    sc = [1] * len(params) if scales is None else [int(r) for r in scales]
    if len(sc) != len(params) or any(b > a for a, b in zip(sc, sc[1:])):
        raise ValueError("one non-increasing scale per iteration")
    return sc


def lpd_init(g, y, L, x0=None, r=1):
    x = np.zeros(vol_shape(g)) if x0 is None else np.asarray(x0, np.float64)
    xbp = downsample(adjoint(g, y) / L, r)
    xb = downsample(x, r)
    yb = projdown(np.asarray(y, np.float64), r)
    return [xb, xbp] * 4, [yb] * 8, x


def _lpd_run(g, y, V, params, L, slope, x0, scales):
    sc = _scales(params, scales)
    f, h, x = lpd_init(g, y, L, x0, sc[0])
    xs, caches = [], []
    for i, p in enumerate(params):
        r = sc[i]
        gr = scaled_geometry(g, r)
        f, h, c, cache = _lpd_iter(gr, f, h, downsample(x, r), projdown(y, r), downsample(V, r),
                                   p, L, slope)
        caches.append(cache)
        x = x + upsample(c, r)
        xs.append(x)
        if i + 1 < len(params) and sc[i + 1] < r:
            f = [upsample(z, r // sc[i + 1]) for z in f]
            h = [upsample(z, r // sc[i + 1]) for z in h]
    return xs, caches, sc


def lpd_forward(g: dict, y, V, params, L: float, slope: float = 0.01, x0=None, scales=None):
    """Reconstructions [x_1, ..., x_n] (full resolution) of the net."""
    return _lpd_run(g, np.asarray(y, np.float64), np.asarray(V, np.float64), params, L, slope,
                    x0, scales)[0]


def lpd_loss_grad(g: dict, y, V, params, L: float, x_true, wmask, slope: float = 0.01, x0=None,
                  scales=None):
    """loss = sum_i 0.5 sum_p wmask_p (x_i,p - x_true,p)^2 over all iterates,
    and its gradient with respect to every parameter (reverse mode with
    stored activations, FP64).  Returns (loss, grads) with grads[i] =
    {"dual": [...6], "primal": [...6], "out": array of 9}."""
    y = np.asarray(y, np.float64)
    V = np.asarray(V, np.float64)
    xs, caches, sc = _lpd_run(g, y, V, params, L, slope, x0, scales)
    loss = sum(0.5 * float(np.sum(wmask * (xi - x_true) ** 2)) for xi in xs)
    n = len(params)
    gf = gh = None
    gx = np.zeros(vol_shape(g))
    grads = [None] * n
    for i in reversed(range(n)):
        p, r = params[i], sc[i]
        gr = scaled_geometry(g, r)
        cg, cp, fn, hn = caches[i]
        if gf is None:
            gf = [np.zeros(vol_shape(gr))] * 8
            gh = [np.zeros(sino_shape(gr))] * 8
        elif sc[i + 1] < r:       # adjoint of the nearest upsampling: block sums
            q = r // sc[i + 1]
            gf = [downsample(z, q) * q ** 3 for z in gf]
            gh = [downsample(z, q) * q ** 3 for z in gh]
        gx = gx + wmask * (xs[i] - x_true)
        rho = list(p["perm"])
        gfn = [np.zeros(vol_shape(gr)) for _ in range(8)]
        ghn = [np.zeros(sino_shape(gr)) for _ in range(8)]
        for k, rr in enumerate(rho):
            gfn[rr] = gfn[rr] + gf[k]
            ghn[rr] = ghn[rr] + gh[k]
        gc = downsample(gx, r) * r ** 3                      # adjoint of Upsample_r
        o = np.asarray(p["out"], np.float64)
        go = np.array([float(np.sum(fn[k] * gc)) for k in range(8)] + [float(np.sum(gc))])
        for k in range(8):
            gfn[k] = gfn[k] + o[k] * gc
        g_p1, g_p2 = gfn[:4], gfn[4:]
        g_d1, g_d2 = ghn[:4], ghn[4:]
        g_pin, gprim = _block_bwd(np.stack(g_p2), cp, p["primal"], slope)
        g_p1 = [g_p1[k] + g_pin[4 + k] for k in range(4)]
        gxb = g_pin[8].copy()
        g_d2 = [g_d2[k] + forward(gr, g_pin[k]) / L for k in range(4)]
        gxb = gxb + adjoint(gr, forward(gr, g_pin[9]) / L) / L
        g_gin, gdual = _block_bwd(np.stack(g_d2), cg, p["dual"], slope)
        g_p2 = [g_p2[k] + adjoint(gr, g_gin[k]) / L for k in range(4)]
        gxb = gxb + adjoint(gr, g_gin[4]) / L
        g_d1 = [g_d1[k] + g_gin[5 + k] for k in range(4)]
        gx = gx + upsample(gxb, r) / r ** 3                  # adjoint of Downsample_r
        gf, gh = g_p1 + g_p2, g_d1 + g_d2
        grads[i] = {"dual": gdual, "primal": gprim, "out": go}
    return loss, grads


# ---- FDK with offset-detector redundancy weights (Alg. 1 initialisation) ----
#
# Feldkamp-Davis-Kress for a circular orbit and a flat panel (Feldkamp et al.,
# JOSA A 1984), in coordinates scaled to the isocentre (R = sid, D = sdd,
# u_i = u R / D, v_i = v R / D for panel coordinates u, v measured from the
# foot of the central ray):
#   1. p_w = w(u) * R / sqrt(R^2 + u_i^2 + v_i^2) * p
#   2. q = p_w (*) h along u, h the band-limited ramp (Ram-Lak) at pitch
#      du_i: h(0) = 1 / (4 du_i^2), h(n du_i) = -1 / (pi^2 n^2 du_i^2) for odd
#      n, 0 for even n; the convolution sum is multiplied by du_i
#   3. f(r) = sum over angles of dbeta * R^2 / U^2 * q(beta, u_i(r), v_i(r)),
#      U = R - (x cos beta + y sin beta), u_i(r) = R (y cos - x sin) / U,
#      v_i(r) = R z / U, q interpolated bilinearly between pixel centres
#      (zero outside the panel); dbeta = 2 pi / n (a full uniform orbit).
# Redundancy weight w: the conjugate of a ray at u is the ray at -u, so the
# weights of a conjugate pair must add to one.  Centred panel: w = 1/2.
# Offset panel covering [off - W/2, off + W/2] with off > 0: overlap
# |u| <= Delta = W/2 - off gets w = sin^2(pi/4 (1 + u / Delta)) (smooth,
# w(u) + w(-u) = 1; Wang, Med. Phys. 2002), w = 1 for u > Delta (measured
# once per orbit), and no measured ray has u < -Delta.

def fdk_weight_u(g: dict, u) -> np.ndarray:
    """Redundancy weight w at panel coordinate u (mm from the central ray)."""
    u = np.asarray(u, np.float64)
    if g["off_u"] == 0.0:
        return np.full(u.shape, 0.5)
    delta = 0.5 * g["nu"] * g["du"] - abs(g["off_u"])
    s = np.sign(g["off_u"])
    t = np.clip(s * u / delta, -1.0, 1.0)
    return np.where(s * u > delta, 1.0, np.sin(0.25 * np.pi * (1.0 + t)) ** 2)


def fdk_weights(g: dict) -> np.ndarray:
    """Redundancy weight w(u) of each panel column."""
    return fdk_weight_u(g, g["off_u"] + (np.arange(g["nu"]) - 0.5 * (g["nu"] - 1)) * g["du"])


def ramp_kernel(n: np.ndarray, pitch: float) -> np.ndarray:
    """Ram-Lak kernel h(n pitch): 1 / (4 pitch^2) at 0, -1 / (pi^2 n^2 pitch^2)
    at odd n, 0 at even n."""
    n = np.asarray(n)
    h = np.zeros(n.shape)
    h[n == 0] = 0.25
    odd = (n % 2) != 0
    h[odd] = -1.0 / (np.pi ** 2 * n[odd].astype(float) ** 2)
    return h / pitch ** 2


def hann_ramp_kernel(n: np.ndarray, pitch: float) -> np.ndarray:
    """Ram-Lak kernel times the Hann window 1/2 + 1/2 cos(2 pi omega pitch)
    in frequency: h(n)/2 + (h(n-1) + h(n+1))/4 in space."""
    n = np.asarray(n)
    return 0.5 * ramp_kernel(n, pitch) + 0.25 * (ramp_kernel(n - 1, pitch) +
                                                 ramp_kernel(n + 1, pitch))


def fdk_filter(g: dict, p: np.ndarray, window: str = "ramlak") -> np.ndarray:
    """Steps 1-2: weighted, ramp-filtered projections q[angle][v][u]
    (window "ramlak" or "hann")."""
    R, D = g["sid"], g["sdd"]
    u = g["off_u"] + (np.arange(g["nu"]) - 0.5 * (g["nu"] - 1)) * g["du"]
    v = g["off_v"] + (np.arange(g["nv"]) - 0.5 * (g["nv"] - 1)) * g["dv"]
    ui, vi = u * R / D, v * R / D
    dui = g["du"] * R / D
    pre = fdk_weights(g)[None, :] * R / np.sqrt(R * R + ui[None, :] ** 2 + vi[:, None] ** 2)
    pw = np.asarray(p, np.float64) * pre[None, :, :]
    kern = {"ramlak": ramp_kernel, "hann": hann_ramp_kernel}[window]
    h = kern(np.arange(-(g["nu"] - 1), g["nu"]), dui)
    q = np.empty_like(pw)
    nu = g["nu"]
    for a in range(pw.shape[0]):
        for iv in range(pw.shape[1]):
            q[a, iv] = np.convolve(pw[a, iv], h)[nu - 1:2 * nu - 1] * dui
    return q


def fdk_backproject(g: dict, q: np.ndarray) -> np.ndarray:
    """Step 3: voxel-driven weighted backprojection of filtered projections."""
    R, D = g["sid"], g["sdd"]
    nx, ny, nz = g["nx"], g["ny"], g["nz"]
    o = g.get("origin", (0.0, 0.0, 0.0))
    cx = o[0] + (np.arange(nx) - 0.5 * (nx - 1)) * g["vx"]
    cy = o[1] + (np.arange(ny) - 0.5 * (ny - 1)) * g["vy"]
    cz = o[2] + (np.arange(nz) - 0.5 * (nz - 1)) * g["vz"]
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    f = np.zeros(X.shape)
    ang = angles_of(g)
    dbeta = 2.0 * np.pi / len(ang)
    nu, nv = g["nu"], g["nv"]
    for a, th in enumerate(ang):
        c, s = np.cos(th), np.sin(th)
        U = R - (X * c + Y * s)
        u = D * (Y * c - X * s) / U            # panel coordinates (mm)
        v = D * Z / U
        fu = (u - g["off_u"]) / g["du"] + 0.5 * (nu - 1)
        fv = (v - g["off_v"]) / g["dv"] + 0.5 * (nv - 1)
        iu0, iv0 = np.floor(fu).astype(int), np.floor(fv).astype(int)
        au, av = fu - iu0, fv - iv0
        val = np.zeros(X.shape)
        for du_, wu in ((0, 1.0 - au), (1, au)):
            for dv_, wv in ((0, 1.0 - av), (1, av)):
                iu, iv = iu0 + du_, iv0 + dv_
                ok = (iu >= 0) & (iu < nu) & (iv >= 0) & (iv < nv)
                val += np.where(ok, wu * wv * q[a, np.clip(iv, 0, nv - 1), np.clip(iu, 0, nu - 1)],
                                0.0)
        f += dbeta * (R * R) / (U * U) * val
    return f


def fdk(g: dict, p: np.ndarray, window: str = "ramlak") -> np.ndarray:
    """FDK reconstruction [nz][ny][nx] from line integrals p[angle][v][u]."""
    return fdk_backproject(g, fdk_filter(g, p, window))
