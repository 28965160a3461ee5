"""Host logic of libcbct.so, checked on the CPU through host-only handles.

* the FP32 ray tables agree with the oracle's FP64 ray geometry;
* the library's FP64 sample count equals the oracle's;
* an FP32 emulation of the forward kernel's LDS box arithmetic shows every
  bilinear read inside the staged box, for every tile and plane (sampled
  tiles at clinical size);
* an FP32 emulation of the adjoint kernel's panel windows shows every
  non-zero weight (as the forward kernel computes it) inside the window the
  adjoint scans, and every window inside the staged LDS region.
"""
import ctypes

import numpy as np
import pytest

from paper_2512_21180_amd import workloads as W

RAGGED = W.geometry(20, 37, 29, 3.3, 2.9, 13, 17, 11, 4.0, vy=3.5, vz=4.5, off_u=31.0,
                    off_v=-7.0, origin=(5.0, -3.0, 2.0))
GEOMS = {
    "ragged": RAGGED,
    "c1": W.C1,
    "c4": W.C4,
    "c2": W.C2,
    "c3_8": W.c3_geometries()[8],
    # 3 mm voxels through 0.8 mm pixels: windows too tall for 16-voxel bricks
    "c3_10": W.c3_geometries()[10],
    # 1.6 mm pixels over 2 mm voxels at the clinical size: 64 columns of rays
    # spread over more than 64 voxels near 45 degrees, tiles are 32 columns
    "c3_7": W.c3_geometries()[7],
    "steep_angles": W.geometry(7, 90, 70, 2.0, 2.0, 40, 36, 30, 3.0, off_u=60.0,
                               angles=np.array([0.1, 0.785398, 0.80, 2.3, 3.9, 5.5, 6.0])),
}

f32 = np.float32


def fma32(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)
            ).astype(np.float32)


class Host:
    def __init__(self, g):
        from paper_2512_21180_amd import cbct
        self.cb = cbct
        lib = cbct.lib()
        lib.cbct_geom_create_host.argtypes = [ctypes.POINTER(cbct.Desc), ctypes.POINTER(ctypes.c_void_p)]
        lib.cbct_geom_create_host.restype = ctypes.c_int
        lib.cbct_geom_table.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        lib.cbct_geom_table.restype = ctypes.c_int
        lib.cbct_geom_plan_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        lib.cbct_geom_plan_info.restype = ctypes.c_int
        desc, keep = cbct.make_desc(g)
        h = ctypes.c_void_p()
        assert lib.cbct_geom_create_host(ctypes.byref(desc), ctypes.byref(h)) == 0
        self.h, self.lib, self.g = h, lib, g
        self.cols = self.table(0, np.float32).reshape(g["n_angles"], g["nu"], 8)
        angs = self.table(1, np.uint8)
        self.ang_cs = angs.view(np.float32).reshape(-1, 4)[:, :2]
        self.ang_x = angs.view(np.int32).reshape(-1, 4)[:, 2:]
        self.rows = self.table(2, np.float32).reshape(g["nv"], 2)
        self.tiles = self.table(3, np.int32).reshape(-1, 8)
        wins = self.table(5, np.uint8)
        info = (ctypes.c_int * 14)()
        lib.cbct_geom_plan_info(h, info, 14)
        self.info = list(info)
        nbx, nby = -(-g["nx"] // self.info[12]), -(-g["ny"] // self.info[13])
        self.win_l = wins.view(np.float32).reshape(g["n_angles"], nby, nbx, 4)[..., :2] \
            if wins.size else None
        self.win_i = wins.view(np.uint32).reshape(g["n_angles"], nby, nbx, 4)[..., 2:] \
            if wins.size else None
        sc = self.table(4, np.uint8)
        self.ints = sc[:24].view(np.int32)
        fl = sc[24:].view(np.float32)
        names = ["Kb", "vx", "vy", "vz", "ox", "oy", "oz", "sid", "sdd", "du", "dv", "off_u",
                 "off_v", "cu", "cv", "rv0", "rvs"]
        self.s = dict(zip(names, fl[:len(names)]))

    def table(self, which, dtype):
        n = ctypes.c_size_t()
        assert self.lib.cbct_geom_table(self.h, which, None, 0, ctypes.byref(n)) == 0
        buf = np.zeros(n.value, dtype=np.uint8)
        assert self.lib.cbct_geom_table(self.h, which, buf.ctypes.data, n.value, ctypes.byref(n)) == 0
        return buf.view(dtype)

    def sample_count(self):
        s = ctypes.c_uint64()
        assert self.lib.cbct_sample_count(self.h, ctypes.byref(s)) == 0
        return s.value

    def close(self):
        self.lib.cbct_geom_destroy(self.h)


@pytest.fixture(scope="module")
def hosts():
    out = {k: Host(g) for k, g in GEOMS.items()}
    yield out
    for h in out.values():
        h.close()


def test_compute_on_host_handle_is_rejected(hosts):
    h = hosts["ragged"]
    assert h.lib.cbct_forward(h.h, ctypes.c_void_p(8), 0, ctypes.c_void_p(8), 0, 1, None) == -7


@pytest.mark.parametrize("name", ["ragged", "c1", "c4", "steep_angles"])
def test_ray_tables_match_oracle_geometry(oracle, hosts, name):
    g, h = GEOMS[name], hosts[name]
    o = g["origin"]
    rng = W.rng(3)
    for _ in range(200):
        a, u = int(rng.integers(g["n_angles"])), int(rng.integers(g["nu"]))
        S, d = oracle.ray(g, a, u, 0)
        xm = abs(d[0]) >= abs(d[1])
        assert (h.ang_x[a, 0] <= u < h.ang_x[a, 1]) == xm
        m, q = (0, 1) if xm else (1, 0)
        nm, nq = (g["nx"], g["ny"]) if xm else (g["ny"], g["nx"])
        pm, pq = (g["vx"], g["vy"]) if xm else (g["vy"], g["vx"])
        rec = h.cols[a, u].astype(np.float64)
        for p in (0, nm - 1):
            c_m = o[m] + (p - 0.5 * (nm - 1)) * pm
            t = (c_m - S[m]) / d[m]
            qf = (S[q] + t * d[q] - o[q]) / pq + 0.5 * (nq - 1)
            assert abs(rec[0] + p * rec[1] - qf) <= 2e-6 * max(1.0, abs(qf))
            assert abs(rec[2] + p * rec[3] - t) <= 2e-6 * abs(t)
        ds_true = pm * np.linalg.norm(d) / abs(d[m])
        ds = rec[4] * np.sqrt(rec[5] + h.rows[0, 1])
        assert abs(ds - ds_true) <= 1e-6 * ds_true


@pytest.mark.parametrize("name", ["ragged", "c1", "steep_angles", "c3_8"])
def test_sample_count_matches_oracle(oracle, hosts, name):
    assert hosts[name].sample_count() == oracle.sample_count(GEOMS[name])


def _fwd_tile_check(h, T, q_lim=64, k_lim=32):
    """Emulate the forward kernel's per-plane box (FP32): staged columns
    [qlo, qlo + qw), rows [klo, klo + kw), qw <= q_lim, kw <= k_lim (64 x 32,
    or 40 x 20 for the multichannel kernel's small layout); every bilinear
    read (q0, q0 + 1) x (k0, k0 + 1) of every ray must fall inside."""
    a, cls, u0, nu_t, v0, nv_t, p_lo, p_hi = [int(x) for x in T]
    if nu_t == 0 or p_lo > p_hi:
        return 0
    Kb = h.s["Kb"]
    C = h.cols[a, u0:u0 + nu_t]
    Vz = h.rows[v0:v0 + nv_t, 0]
    p = np.arange(p_lo, p_hi + 1, dtype=np.float32)[:, None, None]
    cA, cB = C[0], C[-1]
    qa, qb = fma32(p, cA[1], cA[0]), fma32(p, cB[1], cB[0])
    ks = [fma32(p, f32(c[3] * z), fma32(c[2], z, Kb)) for c in (cA, cB) for z in (Vz[0], Vz[-1])]
    qlo = np.floor(np.minimum(qa, qb)) - 1
    qw = np.floor(np.maximum(qa, qb)) + 3 - qlo
    kmin = np.minimum(np.minimum(ks[0], ks[1]), np.minimum(ks[2], ks[3]))
    kmax = np.maximum(np.maximum(ks[0], ks[1]), np.maximum(ks[2], ks[3]))
    klo = np.floor(kmin) - 1
    kw = np.floor(kmax) + 3 - klo
    assert qw.max() <= q_lim and kw.max() <= k_lim, (T, qw.max(), kw.max())
    q = fma32(p, C[None, :, 1, None], C[None, :, 0, None])                 # [P, U, 1]
    kb = fma32(C[:, 2, None], Vz[None, :], Kb)                              # [U, V]
    kss = (C[:, 3, None] * Vz[None, :]).astype(np.float32)
    k = (fma32(p, kss[None], kb[None]) - klo.astype(np.float32)).astype(np.float32)
    qi = np.floor(q) - qlo
    ki = np.floor(k)
    assert qi.min() >= 0 and np.all(qi + 1 <= qw - 1), (T, qi.min(), qi.max())
    assert ki.min() >= 0 and np.all(ki + 1 <= kw - 1), (T, ki.min(), ki.max())
    return q.size * nv_t


@pytest.mark.parametrize("name", sorted(GEOMS))
def test_forward_box_indices_stay_in_lds(hosts, name):
    _check_boxes(hosts[name], 64, 32)


def _check_boxes(h, q_lim, k_lim):
    assert h.info[0] == 1, "tiled forward expected"
    assert h.info[2] <= q_lim and h.info[3] <= k_lim
    tiles = h.tiles
    if len(tiles) > 1500:
        rng = W.rng(11)
        pick = rng.choice(len(tiles), 1200, replace=False)
        # always include every tile of the angles nearest 45 degrees (widest boxes)
        ang = np.arctan2(h.ang_cs[:, 1], h.ang_cs[:, 0])
        diag = np.argsort(np.abs(np.abs(np.sin(2 * ang)) - 1))[:2]
        pick = np.union1d(pick, np.nonzero(np.isin(tiles[:, 0], diag))[0])
        tiles = tiles[pick]
    n = sum(_fwd_tile_check(h, T, q_lim, k_lim) for T in tiles)
    assert n > 0


def test_multichannel_small_layout_boxes():
    """The multichannel forward stages boxes in 41 x 20 LDS rows where the
    plan's box extents are at most 39 x 19 voxels (one voxel of FP32
    rounding in reserve per axis): on every such geometry here (the clinical
    case, its half- and quarter-resolution levels, a 3 mm case and the GPU
    tests' small cases), every FP32 box fits 40 x 20 and every read falls
    inside it."""
    from paper_2512_21180_amd.learned import scaled_geometry
    cases = [W.C2, scaled_geometry(W.C2, 2), scaled_geometry(W.C2, 4), W.c3_geometries()[10],
             RAGGED, W.cropped(W.C2, n_angles=24, nu=160, nv=96, n=64)]
    n_small = 0
    for g in cases:
        h = Host(g)
        try:
            if h.info[2] <= 39 and h.info[3] <= 19:
                n_small += 1
                _check_boxes(h, 40, 20)
        finally:
            h.close()
    assert n_small == len(cases)


def taps_rounded(nt):
    """Tap counts the adjoint kernel is instantiated for."""
    for c in (4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 18, 20, 24, 28):
        if nt <= c:
            return c
    return 32


def _brick_depth(h):
    """Voxels per brick along z of the plan (4 per thread along z, KV)."""
    return 4 * h.info[10]


def _adj_plan(h, bk):
    """(W, H, WS, NTmax) of the plan for bricks bk voxels deep."""
    assert bk == _brick_depth(h)
    return h.info[6], h.info[7], h.info[8], h.info[9]


def _adj_brick_check(h, bx, by, bz, angles, bk):
    g = h.g
    s = h.s
    nx, ny, nz, nu, nv = g["nx"], g["ny"], g["nz"], g["nu"], g["nv"]
    W_, H_, WS, NTmax = _adj_plan(h, bk)
    Kb, rvs, rv0, cv = s["Kb"], s["rvs"], s["rv0"], s["cv"]
    BI, BJ = h.info[12], h.info[13]
    i0, i1 = bx * BI, min(bx * BI + BI, nx) - 1
    j0, j1 = by * BJ, min(by * BJ + BJ, ny) - 1
    k0, k1 = bz * bk, min(bz * bk + bk, nz) - 1

    def cx(i):
        return f32(s["ox"] + f32(f32(i) - f32(0.5) * f32(nx - 1)) * s["vx"])

    def cy(j):
        return f32(s["oy"] + f32(f32(j) - f32(0.5) * f32(ny - 1)) * s["vy"])

    def cz(k):
        return f32(s["oz"] + f32(f32(k) - f32(0.5) * f32(nz - 1)) * s["vz"])

    inv_du, inv_dv = f32(f32(1.0) / s["du"]), f32(f32(1.0) / s["dv"])

    def proj(c_, s_, x, y):
        den = fma32(c_, x, fma32(s_, y, -s["sid"]))
        lam = f32(-s["sdd"] * f32(f32(1.0) / den))
        u = fma32(fma32(lam, fma32(-s_, x, f32(c_ * y)), -s["off_u"]), inv_du, s["cu"])
        return f32(u), lam

    checked = skipped = 0
    for a in angles:
        c_, s_ = h.ang_cs[a]
        x_lo, x_hi = h.ang_x[a]
        # the brick column's window as the kernel reads it from the table
        u01, NT = (int(x) for x in h.win_i[a, by, bx])
        lmin, lmax = h.win_l[a, by, bx]
        zs0, zs1 = f32(cz(k0) - s["vz"]), f32(cz(k1) + s["vz"])
        vmin = fma32(f32(min(f32(lmin * zs0), f32(lmax * zs0)) - s["off_v"]), inv_dv, s["cv"])
        vmax = fma32(f32(max(f32(lmin * zs1), f32(lmax * zs1)) - s["off_v"]), inv_dv, s["cv"])
        U0 = u01 & 0xFFFF
        U1 = min(u01 >> 16, U0 + W_ - 1)
        assert NT <= NTmax and NT == taps_rounded(NT)
        V0 = max(int(np.floor(vmin)) - 2, 0)
        V1u = min(int(np.ceil(vmax)) + 2, nv - 1)
        V1 = min(V1u, V0 + H_ - 1)
        if U0 > U1 or V0 > V1:
            # nothing of this brick may be visible at this angle
            continue
        # the plan's window holds the brick's rows (the clamp never cuts) and
        # one run; a run never leaves it
        assert V1 == V1u
        Hs = max(V1 - V0 + 1, NT)
        VS1 = max(V1 - NT + 1, V0)
        assert U1 - U0 + 1 <= W_ and Hs <= H_ and H_ < WS and WS % 4 == 2
        # lane roles: on x planes, plane i and in-plane segment [s, s + 1) of y
        # for s = j0 - 1 .. j0 + BJ - 1; on y planes, plane j and segment of x
        # for s = i0 - 1 .. i0 + BI - 1
        roles = []
        if x_lo < x_hi:
            for i in range(i0, min(i0 + BI, nx)):
                for sg in range(j0 - 1, min(j0 + BJ, ny)):
                    roles.append((0, i, sg))
        if not (x_lo == 0 and x_hi == nu):
            for j in range(j0, min(j0 + BJ, ny)):
                for sg in range(i0 - 1, min(i0 + BI, nx)):
                    roles.append((1, j, sg))
        for cls, pl, sg in roles:
            fp, sf = f32(pl), f32(sg)
            if cls == 0:
                lo_c, hi_c = x_lo, x_hi - 1
                u1, _ = proj(c_, s_, cx(pl), cy(sg))
                u2, _ = proj(c_, s_, cx(pl), f32(cy(sg) + s["vy"]))
                cols_ok = np.arange(x_lo, x_hi)
            else:
                lo_c, hi_c = 0, nu - 1
                u1, _ = proj(c_, s_, cx(sg), cy(pl))
                u2, _ = proj(c_, s_, f32(cx(sg) + s["vx"]), cy(pl))
                cols_ok = np.setdiff1d(np.arange(nu), np.arange(x_lo, x_hi))
            ul = max(max(int(np.floor(min(u1, u2))), lo_c), U0)
            uh = min(min(int(np.ceil(max(u1, u2))), hi_c), U1)
            # the segment's members, as the forward floors the in-plane index
            C = h.cols[a, cols_ok]
            q = fma32(fp, C[:, 1], C[:, 0])
            f = (q - sf).astype(np.float32)
            mem = cols_ok[(f >= 0) & (f < 1)]
            assert np.all((mem >= ul) & (mem <= uh)), (a, cls, pl, sg, mem, ul, uh)
            # the candidates between two members are members too (the kernel
            # trims only the ends; a column inside is tested again anyway)
            for u in mem:
                Cu = h.cols[a, u]
                t = fma32(fp, Cu[3], Cu[2])
                rt = f32(1.0) / t
                Vz = h.rows[:, 0]
                kf = fma32(fp, (Cu[3] * Vz).astype(np.float32), fma32(Cu[2], Vz, Kb))
                for kk in range(k0, k1 + 1):
                    rows_sup = np.nonzero(np.abs(kf.astype(np.float64) - kk) < 1.0)[0]
                    inv_rvs = f32(f32(1.0) / rvs)
                    Bk = f32(f32(f32(f32(kk) - f32(1.0)) - Kb) * inv_rvs)
                    delta = max(nv / 1048576.0, 1.0 / 4096)
                    A0 = fma32(-rv0, inv_rvs, f32(cv + f32(1.0 - delta)))
                    vf = fma32(rt, Bk, A0)
                    vstart = min(max(int(np.floor(vf)), V0), VS1)
                    inrun = (rows_sup >= vstart) & (rows_sup < vstart + NT) & (rows_sup <= V1)
                    # a row may be left out only where its weight is below
                    # 2 delta beta, plus FP32 rounding
                    wgt = 1.0 - np.abs(kf[rows_sup].astype(np.float64) - kk)
                    beta = float(t) * float(rvs)
                    assert np.all(inrun | (wgt <= 2 * delta * beta + 1e-5)), \
                        (a, cls, pl, sg, kk, u, rows_sup, wgt, vstart, NT, V1)
                    skipped += int(np.sum(~inrun))
                    checked += len(rows_sup)
        # every non-zero in-plane weight of an output voxel comes from one of
        # the lanes' segments (the voxel's own or the one below)
        for i in range(i0, i1 + 1):
            for j in range(j0, j1 + 1):
                for cls, fp, qv, ok in ((0, i, j, x_lo < x_hi),
                                        (1, j, i, not (x_lo == 0 and x_hi == nu))):
                    if not ok:
                        continue
                    cols_ok = np.arange(x_lo, x_hi) if cls == 0 else \
                        np.setdiff1d(np.arange(nu), np.arange(x_lo, x_hi))
                    C = h.cols[a, cols_ok]
                    q = fma32(f32(fp), C[:, 1], C[:, 0])
                    segs = np.floor(q[np.abs(q.astype(np.float64) - qv) < 1.0]).astype(int)
                    lane_segs = {r[2] for r in roles if r[0] == cls and r[1] == fp}
                    assert set(segs.tolist()) <= lane_segs, (a, cls, i, j, set(segs), lane_segs)
    # left-out rows need two coincidences and stay rare
    assert skipped <= 1e-4 * max(checked, 1) + 2, (skipped, checked)
    return checked


@pytest.mark.parametrize("name", ["ragged", "c1", "c4", "c2", "steep_angles", "c3_10"])
def test_adjoint_windows_cover_every_weight(hosts, name):
    h = hosts[name]
    g = GEOMS[name]
    assert h.info[5] == 1, "bricked adjoint expected"
    assert (h.info[12], h.info[13]) == (8, 7)
    nbx, nby = -(-g["nx"] // h.info[12]), -(-g["ny"] // h.info[13])
    rng = W.rng(5)
    n_b = 3 if name in ("c2", "c4") else 6
    na = g["n_angles"]
    angs = np.unique(np.concatenate([rng.choice(na, min(na, 6), replace=False),
                                     [0, na // 8, na // 4 + 1]]))
    total = 0
    for bk in (_brick_depth(h),):
        nbz = -(-g["nz"] // bk)
        for _ in range(n_b):
            b = (int(rng.integers(nbx)), int(rng.integers(nby)), int(rng.integers(nbz)))
            total += _adj_brick_check(h, *b, angles=[int(x) % na for x in angs], bk=bk)
        # the central brick is always seen
        total += _adj_brick_check(h, nbx // 2, nby // 2, nbz // 2,
                                  angles=[int(x) % na for x in angs], bk=bk)
    assert total > 0


@pytest.mark.parametrize("name", ["ragged", "c1", "c4", "c2", "steep_angles", "c3_10"])
def test_adjoint_window_bound_holds_for_every_brick(hosts, name):
    """The planned window height bounds the clipped window of every brick
    (all layers, FP32 as in the kernel) at a dozen angles: the kernel's row
    clamp V0 + H - 1 never cuts a brick's rows."""
    h = hosts[name]
    g, s = h.g, h.s
    nx, ny, nz, nv = g["nx"], g["ny"], g["nz"], g["nv"]
    na = g["n_angles"]
    inv_dv = f32(f32(1.0) / s["dv"])
    for bk in (_brick_depth(h),):
        W_, H_, _, _ = _adj_plan(h, bk)
        for a in np.linspace(0, na - 1, 12).astype(int):
            u01 = h.win_i[a, ..., 0]
            seen = (u01 & 0xFFFF) <= (u01 >> 16)
            assert np.all((u01 >> 16) - (u01 & 0xFFFF) + 1 <= np.where(seen, W_, 1 << 20))
            lmin, lmax = h.win_l[a, ..., 0], h.win_l[a, ..., 1]
            for bz in range(-(-nz // bk)):
                k0, k1 = bz * bk, min(bz * bk + bk, nz) - 1
                zl = f32(f32(s["oz"] + f32(f32(k0) - f32(0.5) * f32(nz - 1)) * s["vz"]) - s["vz"])
                zh = f32(f32(s["oz"] + f32(f32(k1) - f32(0.5) * f32(nz - 1)) * s["vz"]) + s["vz"])
                vmin = fma32(np.minimum(lmin * zl, lmax * zl).astype(f32) - s["off_v"], inv_dv,
                             s["cv"])
                vmax = fma32(np.maximum(lmin * zh, lmax * zh).astype(f32) - s["off_v"], inv_dv,
                             s["cv"])
                V0 = np.maximum(np.floor(vmin).astype(int) - 2, 0)
                V1u = np.minimum(np.ceil(vmax).astype(int) + 2, nv - 1)
                bad = seen & (V1u >= V0) & (V1u - V0 + 1 > H_)
                assert not bad.any(), (name, bk, a, bz, np.argwhere(bad)[:3])


def test_brick_depth_follows_the_window():
    """Bricks are 16 voxels deep where the window fits four workgroups per
    CU and there are at least two bricks per CU, shallower where large voxels
    meet fine pixels (all twelve mixed cases stay bricked) or the volume is
    small (64^3: 8 voxels deep, 512 bricks); the window always fits the 64 KB
    budget."""
    for name, kv in (("c2", 4), ("c4", 4), ("c1", 2)):
        assert Host(GEOMS[name]).info[10] == kv, name
    for i, g in enumerate(W.c3_geometries()):
        h = Host(g)
        try:
            assert h.info[5] == 1, i
            assert h.info[10] in (1, 2, 4)
            lds = (h.info[6] * h.info[8] + 4 * h.info[6]) * 4
            assert lds <= 64 * 1024
            if h.info[10] < 4:
                assert lds <= 40 * 1024 or h.info[10] == 1
        finally:
            h.close()


def test_tiled_forward_needs_32bit_offsets():
    """The tiled forward addresses a volume channel with 32-bit byte offsets,
    those below the volume wrapping past its end: volumes that reach 4 GiB
    (FP32) with 64 more z planes take the one-thread-per-ray kernel."""
    small = W.geometry(4, 64, 16, 0.1, 0.1, 1024, 1024, 1024 - 64 - 1, 0.2)
    big = W.geometry(4, 64, 16, 0.1, 0.1, 1024, 1024, 1024 - 64, 0.2)
    hs, hb = Host(small), Host(big)
    try:
        assert hs.info[0] == 1
        assert hb.info[0] == 0
    finally:
        hs.close()
        hb.close()


def test_window_columns_pack_above_32767():
    """The adjoint's window table packs the column range into 16 + 16 bits,
    read unsigned: a 40000-column panel keeps its right half."""
    g = W.geometry(3, 40000, 16, 0.01, 0.01, 16, 16, 8, 0.05, off_u=-150.0)
    h = Host(g)
    try:
        assert h.info[5] == 1
        u01 = h.win_i[..., 0].astype(np.int64)
        seen = (u01 & 0xFFFF) <= (u01 >> 16)
        assert seen.any()
        u1 = (u01 >> 16)[seen]
        assert u1.max() >= 32768 and u1.max() < 40000
        # every seen window is inside the panel and no wider than planned
        assert np.all((u01 & 0xFFFF)[seen] <= u1)
        assert np.all(u1 - (u01 & 0xFFFF)[seen] + 1 <= h.info[6])
    finally:
        h.close()


def _staged_rows(HS, Hs, w, sb=24):
    """Rows of one window column that wave w stores in the adjoint's staging
    of tall columns (HS >= 4 sb): batches of sb rows at stride 4 from row w,
    a batch that would pass the column moved down to the last start of the
    wave's residue class that keeps it inside."""
    top = HS - 1 - 4 * (sb - 1)
    vtop = top - ((top - w) & 3)
    rows = []
    for vv0 in range(w, Hs, 4 * sb):
        vb = min(vv0, vtop)
        rows += [vb + 4 * j for j in range(sb)]
    return rows


def _tall_batch_rows(Hs):
    """Rows per wave and batch of the tall-column staging for Hs staged rows."""
    return 16 if Hs <= 64 else 20 if Hs <= 80 else 24


@pytest.mark.parametrize("HS", [96, 97, 98, 99, 114, 118, 150, 190, 191, 192, 193, 250])
def test_tall_window_staging_stays_in_the_column(HS):
    """Every row the waves of a tall column store lies in [0, HS), each wave
    stores only rows of its own residue class, and the rows below Hs (every
    row a tap may read) are all stored, for every staged height Hs < HS and
    the batch length the kernel takes for it."""
    for Hs in range(1, HS):
        seen = set()
        for w in range(4):
            rows = _staged_rows(HS, Hs, w, _tall_batch_rows(Hs))
            assert all(0 <= r <= HS - 1 for r in rows), (HS, Hs, w)
            assert all(r % 4 == w for r in rows), (HS, Hs, w)
            seen.update(rows)
        assert set(range(Hs)) <= seen, (HS, Hs)


def test_tall_windows_at_clinical_size():
    """The clinical plan's window column (118 rows) takes the tall-column
    staging; the small cases' columns (34 and 54 rows) do not."""
    for name, tall in (("c2", True), ("c1", False), ("c4", False)):
        h = Host(GEOMS[name])
        try:
            assert (h.info[10] == 4 and h.info[8] >= 96) == tall, name
        finally:
            h.close()
