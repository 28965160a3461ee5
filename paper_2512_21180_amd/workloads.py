"""Seeded synthetic inputs: acquisition geometries and phantoms.

This module generates inputs only.  It holds none of the projector's
arithmetic and is shared, unchanged, by the HIP path's tests and benchmark and
by the oracle's tests.

Geometries follow the clinical set-up of the paper (Sec. 2.2): circular orbit,
source-isocenter 1000 mm, isocenter-detector 536 mm (source-detector 1536 mm),
a 409.6 mm square panel, and a 115 mm lateral detector offset for the
half-fan acquisitions.  The paper trains and evaluates on CT scans that are
not available here; seeded ellipsoid phantoms with tissue-like attenuation
(mm^-1) stand in for them.

A geometry is a plain dict: sid, sdd, n_angles, angles (None = 2*pi*a/n),
nu, nv, du, dv, off_u, off_v, nx, ny, nz, vx, vy, vz, origin.
"""
from __future__ import annotations

import math

import numpy as np


def geometry(n_angles, nu, nv, du, dv, nx, ny, nz, vx, vy=None, vz=None, off_u=0.0,
             off_v=0.0, sid=1000.0, sdd=1536.0, origin=(0.0, 0.0, 0.0), angles=None):
    vy = vx if vy is None else vy
    vz = vx if vz is None else vz
    return dict(sid=float(sid), sdd=float(sdd), n_angles=int(n_angles), angles=angles,
                nu=int(nu), nv=int(nv), du=float(du), dv=float(dv),
                off_u=float(off_u), off_v=float(off_v),
                nx=int(nx), ny=int(ny), nz=int(nz),
                vx=float(vx), vy=float(vy), vz=float(vz), origin=tuple(float(o) for o in origin))


# Small case: 64^3 at 4 mm, 64 angles, 128^2 panel at 3.2 mm, no offset.
C1 = geometry(64, 128, 128, 3.2, 3.2, 64, 64, 64, 4.0)
# Clinical size: 256^3 at 2 mm, 360 angles, 512^2 panel at 0.8 mm, 115 mm offset.
C2 = geometry(360, 512, 512, 0.8, 0.8, 256, 256, 256, 2.0, off_u=115.0)
# Differentiable-projector case: 128^3 at 2 mm, 180 angles, 256^2 at 1.6 mm, offset.
C4 = geometry(180, 256, 256, 1.6, 1.6, 128, 128, 128, 2.0, off_u=115.0)

# Twelve heterogeneous cases (N, voxel mm, angles, detector pixels, offset mm);
# the panel is always 409.6 mm wide, so pitch = 409.6 / det.
C3_CASES = [
    (96, 4.0, 90, 256, 0.0), (128, 4.0, 120, 256, 115.0), (192, 3.0, 180, 384, 0.0),
    (256, 2.0, 360, 512, 115.0), (96, 3.0, 360, 512, 0.0), (128, 2.0, 240, 384, 115.0),
    (192, 2.0, 90, 256, 0.0), (256, 2.0, 180, 256, 115.0), (96, 2.0, 180, 384, 115.0),
    (128, 3.0, 360, 512, 0.0), (192, 3.0, 270, 512, 115.0), (256, 2.0, 90, 384, 0.0),
]


def c3_geometries():
    return [geometry(na, det, det, 409.6 / det, 409.6 / det, n, n, n, v, off_u=off)
            for (n, v, na, det, off) in C3_CASES]


def scaled(g: dict, **over) -> dict:
    """Copy of g with some fields replaced."""
    h = dict(g)
    h.update(over)
    return h


def cropped(g: dict, n_angles=None, nu=None, nv=None, n=None) -> dict:
    """A smaller case with the same magnification, pitch and offset: fewer
    angles (spread over the full orbit), a centred detector window and a
    centred sub-volume."""
    h = dict(g)
    if n_angles is not None:
        h["n_angles"] = int(n_angles)
        h["angles"] = None
    if nu is not None:
        h["nu"] = int(nu)
    if nv is not None:
        h["nv"] = int(nv)
    if n is not None:
        h["nx"] = h["ny"] = h["nz"] = int(n)
    return h


def vol_shape(g):
    return (g["nz"], g["ny"], g["nx"])


def sino_shape(g):
    return (g["n_angles"], g["nv"], g["nu"])


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_volume(g: dict, seed: int, low=0.0, high=1.0) -> np.ndarray:
    return rng(seed).uniform(low, high, size=vol_shape(g))


def random_sino(g: dict, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(size=sino_shape(g))


def random_rotation(r: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation matrix (QR of a Gaussian matrix)."""
    q, rr = np.linalg.qr(r.standard_normal((3, 3)))
    q = q * np.sign(np.diag(rr))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def voxel_centres(g: dict):
    """World coordinates (mm) of voxel centres along x, y, z."""
    o = g.get("origin", (0.0, 0.0, 0.0))
    cx = o[0] + (np.arange(g["nx"]) - 0.5 * (g["nx"] - 1)) * g["vx"]
    cy = o[1] + (np.arange(g["ny"]) - 0.5 * (g["ny"] - 1)) * g["vy"]
    cz = o[2] + (np.arange(g["nz"]) - 0.5 * (g["nz"] - 1)) * g["vz"]
    return cx, cy, cz


def ellipsoid_list(g: dict, seed: int, count=(1, 10), semi=(5.0, 50.0), mu=(0.01, 0.03),
                   body_radius=None):
    """Random ellipsoids (centre, semi-axes, rotation, mu).

    Centres are uniform in the region that keeps each ellipsoid's bounding
    sphere inside the volume, or inside the body cylinder (radius body_radius,
    full height) when one is given.
    """
    r = rng(seed)
    n = int(r.integers(count[0], count[1] + 1))
    o = np.asarray(g.get("origin", (0.0, 0.0, 0.0)))
    half = 0.5 * np.array([g["nx"] * g["vx"], g["ny"] * g["vy"], g["nz"] * g["vz"]])
    out = []
    for _ in range(n):
        ax = r.uniform(semi[0], semi[1], size=3)
        R = random_rotation(r)
        m = float(r.uniform(mu[0], mu[1]))
        rad = float(ax.max())
        if body_radius is None:
            lim = np.maximum(half - rad, 0.0)
            c = o + r.uniform(-lim, lim)
        else:
            rr = max(body_radius - rad, 0.0) * math.sqrt(r.uniform())
            ph = r.uniform(0, 2 * math.pi)
            zl = max(half[2] - rad, 0.0)
            c = o + np.array([rr * math.cos(ph), rr * math.sin(ph), r.uniform(-zl, zl)])
        out.append(dict(centre=c, axes=ax, rot=R, mu=m))
    return out


def voxelise(g: dict, ellipsoids, body=None) -> np.ndarray:
    """Point-sample additive ellipsoids (and an optional z-axis cylinder body
    dict(radius, mu)) at voxel centres; FP64 volume [nz][ny][nx]."""
    cx, cy, cz = voxel_centres(g)
    vol = np.zeros(vol_shape(g))
    if body is not None:
        o = g.get("origin", (0.0, 0.0, 0.0))
        inside = ((cx[None, :] - o[0]) ** 2 + (cy[:, None] - o[1]) ** 2) < body["radius"] ** 2
        vol += body["mu"] * inside[None, :, :]
    for e in ellipsoids:
        c, ax, R, m = e["centre"], e["axes"], e["rot"], e["mu"]
        rad = ax.max()
        sel = [np.nonzero(np.abs(cc - c[q]) <= rad)[0] for q, cc in enumerate((cx, cy, cz))]
        if any(s.size == 0 for s in sel):
            continue
        ix, iy, iz = sel
        P = np.stack(np.meshgrid(cz[iz], cy[iy], cx[ix], indexing="ij")[::-1], axis=-1) - c
        loc = P @ R          # coordinates in the ellipsoid frame (columns of R are its axes)
        inside = ((loc / ax) ** 2).sum(-1) < 1.0
        vol[np.ix_(iz, iy, ix)] += m * inside
    return vol


def phantom_c1(g: dict, seed: int):
    """1-10 ellipsoids, semi-axes 5-50 mm, mu 0.01-0.03 /mm."""
    el = ellipsoid_list(g, seed)
    return voxelise(g, el), el


def phantom_c2(g: dict, seed: int, n=50, body_diameter=300.0):
    """Body cylinder (300 mm, mu 0.02) plus n ellipsoids with mu 0-0.04 /mm."""
    el = ellipsoid_list(g, seed, count=(n, n), mu=(0.0, 0.04), body_radius=0.5 * body_diameter)
    body = dict(radius=0.5 * body_diameter, mu=0.02)
    return voxelise(g, el, body=body), el, body


def phantom_c3(g: dict, seed: int):
    """10-50 ellipsoids inside a body cylinder 0.6x the volume width."""
    w = 0.6 * g["nx"] * g["vx"]
    el = ellipsoid_list(g, seed, count=(10, 50), semi=(5.0, 0.15 * w), mu=(0.0, 0.04),
                        body_radius=0.5 * w)
    body = dict(radius=0.5 * w, mu=0.02)
    return voxelise(g, el, body=body), el, body


def slab(g: dict, nz: int, nv: int) -> dict:
    """The central z-slab of nz voxel layers of g, with the nv panel rows
    centred on it (same pitches, angles and offsets)."""
    return dict(g, nz=int(nz), nv=int(nv))


def phantom_c2_slab(g_slab: dict, seed: int, g_full: dict = None, n=50, body_diameter=300.0):
    """A random z-section of a clinical-size phantom (body cylinder plus n
    ellipsoids, as phantom_c2 on g_full), voxelised on the slab grid."""
    g_full = C2 if g_full is None else g_full
    el = ellipsoid_list(g_full, seed, count=(n, n), mu=(0.0, 0.04),
                        body_radius=0.5 * body_diameter)
    zr = 0.5 * (g_full["nz"] * g_full["vz"] - g_slab["nz"] * g_slab["vz"])
    z0 = rng(seed + 1_000_003).uniform(-zr, zr)
    for e in el:
        e["centre"] = e["centre"] - np.array([0.0, 0.0, z0])
    body = dict(radius=0.5 * body_diameter, mu=0.02)
    return voxelise(g_slab, el, body=body)


# ---- inputs of the polychromatic primary model (Sec. 2.2) ----
#
# The paper derives its intensity maps from a phase file of the scanner's
# source and its material attenuation from published cross-section tables;
# neither is available here.  The stand-ins below are synthetic: smooth
# tables of the right magnitude and trend, not physical data.

def hu_phantom(g: dict, seed: int, mu_water: float = 0.02) -> np.ndarray:
    """A clinical-style phantom in Hounsfield units: the body cylinder
    (300 mm, or 0.9 of the volume's width if smaller) at 0 HU (mu_water),
    air at -1000 HU, and 50 additive ellipsoids of up to 2 mu_water each
    (overlaps reach the bone range of the water-bone split)."""
    rad = min(150.0, 0.45 * g["nx"] * g["vx"])
    el = ellipsoid_list(g, seed, count=(50, 50), semi=(5.0, min(50.0, 0.4 * rad)),
                        mu=(0.0, 2.0 * mu_water), body_radius=rad)
    x = voxelise(g, el, body=dict(radius=rad, mu=mu_water))
    return (1000.0 * (x / mu_water - 1.0)).astype(np.float32)


def poly_tables(centres_kev) -> tuple:
    """Synthetic attenuation per unit density (mm^-1) of water and bone at
    the bin centres: a constant plus a photoelectric-like (25 keV / e)^3
    term, larger for bone."""
    e = np.asarray(centres_kev, dtype=np.float64)
    pe = (25.0 / e) ** 3
    return 0.017 + 0.033 * pe, 0.035 + 0.35 * pe


def intensity_maps(g: dict, centres_kev, photons_per_mm2: float = 66000.0) -> np.ndarray:
    """[n_bins, nv, nu] unattenuated photons per pixel and bin: photons per
    mm^2 times the pixel area, split over the bins by a smooth spectrum
    (peak near 55 keV) and shaped across the panel by a bow-tie-like fall-off
    in the lateral (u) position."""
    e = np.asarray(centres_kev, dtype=np.float64)
    spec = np.exp(-0.5 * ((e - 55.0) / 22.0) ** 2)
    spec /= spec.sum()
    u = (np.arange(g["nu"]) - 0.5 * (g["nu"] - 1)) * g["du"] + g["off_u"]
    bow = np.exp(-(u / 260.0) ** 2)
    per_pix = photons_per_mm2 * g["du"] * g["dv"]
    return (per_pix * spec[:, None, None] * bow[None, None, :] *
            np.ones((1, g["nv"], 1))).astype(np.float32)


# ---- inputs of the scatter model (Sec. 2.3) ----
#
# The paper takes cross sections from a database that is not available here;
# the stand-ins below are smooth synthetic tables of the right form: per
# material (water, bone) the photoelectric, Compton and Rayleigh attenuation
# at unit density on an energy grid, and per material and scatter type the
# distribution of the scattering angle as an inverse CDF of cos(theta) and a
# density of directions per steradian.  Compton angles follow the
# Klein-Nishina shape for free electrons; Rayleigh angles a forward-peaked
# (1 + cos^2) shape narrowing with energy.

ME_C2_KEV = 510.99895


def _angle_tables(pdf, J, I):
    """(icdf [J] at u = j / (J - 1), dens [I] per steradian at
    cos = -1 + 2 i / (I - 1)) of a density pdf(cos) on [-1, 1]."""
    c = np.linspace(-1.0, 1.0, 20001)
    p = pdf(c)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (p[1:] + p[:-1]) * np.diff(c))])
    Z = cdf[-1]
    icdf = np.interp(np.linspace(0.0, 1.0, J), cdf / Z, c)
    ci = np.linspace(-1.0, 1.0, I)
    dens = pdf(ci) / Z / (2.0 * math.pi)
    return icdf, dens


def scatter_tables(e0=10.0, de=5.0, K=29, J=129, I=129) -> dict:
    """Synthetic cross-section tables (see above) for the scatter model:
    dict(e0, de, mu [2, 3, K], icdf [2, 2, K, J], dens [2, 2, K, I])."""
    e = e0 + de * np.arange(K)
    pe = (25.0 / e) ** 3
    mu = np.zeros((2, 3, K))
    mu[0, 0], mu[0, 1], mu[0, 2] = 0.030 * pe, 0.018 * (1.0 - 0.002 * (e - 10.0)), 0.002 * (25.0 / e)
    mu[1, 0], mu[1, 1], mu[1, 2] = 0.300 * pe, 0.030 * (1.0 - 0.002 * (e - 10.0)), 0.006 * (25.0 / e)
    icdf = np.zeros((2, 2, K, J))
    dens = np.zeros((2, 2, K, I))
    for k, ek in enumerate(e):
        a = ek / ME_C2_KEV

        def kn(c, a=a):
            P = 1.0 / (1.0 + a * (1.0 - c))
            return P * P * (P + 1.0 / P - (1.0 - c * c))

        for m, width in ((0, 12.0), (1, 16.0)):
            def ray(c, ek=ek, width=width):
                return (1.0 + c * c) * np.exp(-(1.0 - c) * ek / width)

            icdf[m, 0, k], dens[m, 0, k] = _angle_tables(kn, J, I)
            icdf[m, 1, k], dens[m, 1, k] = _angle_tables(ray, J, I)
    return dict(e0=e0, de=de, mu=mu, icdf=icdf, dens=dens)


def scatter_sources(N: int, g: dict, seed: int, spectrum_kev=None) -> np.ndarray:
    """[N, 4] source photons for the source at angle 0: unit directions
    toward uniformly random points of the panel and energies drawn from the
    ten bin centres with the intensity maps' spectrum."""
    r = rng(seed)
    e = np.array([10.0 * i + 5.0 for i in range(2, 12)]) if spectrum_kev is None \
        else np.asarray(spectrum_kev, dtype=np.float64)
    w = np.exp(-0.5 * ((e - 55.0) / 22.0) ** 2)
    w /= w.sum()
    S = np.array([g["sid"], 0.0, 0.0])
    u = (r.uniform(-0.5, 0.5, N) * g["nu"]) * g["du"] + g["off_u"]
    v = (r.uniform(-0.5, 0.5, N) * g["nv"]) * g["dv"] + g["off_v"]
    P = np.stack([np.full(N, -(g["sdd"] - g["sid"])), u, v], axis=1)
    d = P - S
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.concatenate([d, r.choice(e, size=N, p=w)[:, None]], axis=1)


def sobol_points(N: int, dims: int) -> np.ndarray:
    """[N, dims] points of the unscrambled Sobol sequence (scipy's
    implementation), skipping the first point (all zeros)."""
    import warnings
    from scipy.stats import qmc
    s = qmc.Sobol(d=dims, scramble=False)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")     # balance holds for powers of two only
        return s.random(N + 1)[1:]
