// Host-side launch plans of libcbct.so, computed once per geometry in FP64.
//
// Forward: the panel of every angle is cut into tiles of up to TU columns x
// TV rows that share a sampling axis.  A tile sweeps the voxel-centre planes
// of that axis; on each plane every ray of the tile lands inside a box that
// the kernel stages in LDS, at most 64 x 32 voxels.  BQ and BK are the
// largest box extents over all tiles and planes (the extent of the box is a
// convex function of the plane index, so its maximum is reached on the first
// or the last plane), widened by the rounding margins the kernel relies on.
// TU is 64 columns, or 32 where 64 columns of rays spread wider than 64
// voxels (pixels coarser than the voxels); TV is the largest of 256 / TU
// times 8, 4, 2, 1 rows whose boxes fit.
//
// Adjoint: the volume is cut into 8 x 8 x 4 KV bricks (KV = 4, 2 or 1 voxels
// per thread along z).  For every angle a brick's support (voxel centres +-
// one pitch) projects onto the panel inside a W x H window that is staged in
// LDS; W and H are the largest windows over all bricks and angles.  The
// tallest bricks whose window lets four workgroups share a CU's 160 KB of LDS
// are taken, else the tallest that fit 64 KB (large voxels seen through fine
// pixels make tall windows).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "cbct_internal.h"

namespace cbct {

namespace {

constexpr int kMaxBoxQ = 64;      // staged box: one 64-lane row per z index
constexpr int kMaxBoxK = 32;      // and at most 32 rows
constexpr int kBI = 8, kBJ = 8;
constexpr size_t kAdjLdsShare = 40 * 1024;    // four workgroups per CU
constexpr size_t kAdjLdsBudget = 64 * 1024;
constexpr int kMaxTaps = 32;      // row taps per voxel and column in the adjoint

struct TileBuild {
    std::vector<TileRec> tiles;
    int BQ = 0, BK = 0;
};

double row_vz(const cbct_geom_desc &d, int iv)
{
    return (d.off_v_mm + (iv - 0.5 * (d.nv - 1)) * d.dv_mm) / d.vz_mm;
}

TileBuild make_tiles(const cbct_geom *g, int TU, int TV)
{
    const cbct_geom_desc &d = g->desc;
    const double Kb = 0.5 * (d.nz - 1) - d.origin_mm[2] / d.vz_mm;
    TileBuild tb;
    int maxq = 0, maxk = 0;
    for (int a = 0; a < d.n_angles; ++a) {
        const double c = std::cos(g->angles[a]), s = std::sin(g->angles[a]);
        const AngRec &ar = g->angs[a];
        // column ranges of one sampling axis: x planes [x_lo, x_hi), y planes elsewhere
        int ranges[3][3] = {{0, ar.x_lo, 1}, {ar.x_lo, ar.x_hi, 0}, {ar.x_hi, d.nu, 1}};
        for (auto &rg : ranges) {
            for (int u0 = rg[0]; u0 < rg[1]; u0 += TU) {
                const int nu_t = std::min(TU, rg[1] - u0);
                const Col64 cA = col_consts64(d, c, s, u0);
                const Col64 cB = col_consts64(d, c, s, u0 + nu_t - 1);
                const int cls = rg[2];
                const int nm = cls ? d.ny : d.nx, nq = cls ? d.nx : d.ny;
                for (int v0 = 0; v0 < d.nv; v0 += TV) {
                    const int nv_t = std::min(TV, d.nv - v0);
                    const double zA = row_vz(d, v0), zB = row_vz(d, v0 + nv_t - 1);
                    auto box = [&](double p, double *q0, double *q1, double *k0, double *k1) {
                        double qa = cA.pb + p * cA.ps, qb = cB.pb + p * cB.ps;
                        double ta = cA.t0 + p * cA.tau, tb = cB.t0 + p * cB.tau;
                        double ks[4] = {Kb + ta * zA, Kb + ta * zB, Kb + tb * zA, Kb + tb * zB};
                        *q0 = std::min(qa, qb);
                        *q1 = std::max(qa, qb);
                        *k0 = *std::min_element(ks, ks + 4);
                        *k1 = *std::max_element(ks, ks + 4);
                    };
                    for (double p : {0.0, (double)(nm - 1)}) {
                        double q0, q1, k0, k1;
                        box(p, &q0, &q1, &k0, &k1);
                        maxq = std::max(maxq, (int)(std::floor(q1) - std::floor(q0)));
                        maxk = std::max(maxk, (int)(std::floor(k1) - std::floor(k0)));
                    }
                    auto meets = [&](int p) {
                        double q0, q1, k0, k1;
                        box((double)p, &q0, &q1, &k0, &k1);
                        return q1 > -3.0 && q0 < nq + 2.0 && k1 > -3.0 && k0 < d.nz + 2.0;
                    };
                    int lo = 0, hi = nm - 1;
                    while (lo <= hi && !meets(lo))
                        ++lo;
                    while (hi >= lo && !meets(hi))
                        --hi;
                    TileRec t;
                    t.a = a;
                    t.cls = cls;
                    t.u0 = u0;
                    t.nu_t = nu_t;
                    t.v0 = v0;
                    t.nv_t = nv_t;
                    t.p_lo = lo;
                    t.p_hi = hi;
                    tb.tiles.push_back(t);
                }
            }
        }
    }
    // The kernel stages [floor(min) - 1, floor(max) + 2] on each axis (reads
    // reach floor(q) + 1); one more voxel covers FP32 rounding of the corners.
    tb.BQ = maxq + 4;
    tb.BK = maxk + 4;
    return tb;
}

// Window bounds of bricks 8 x 8 x bk staging `channels` channels per
// element; ok when the window fits the LDS budget.  Every brick and angle
// is evaluated: per (angle, brick column) the corner projections give the
// column range and the extreme source-panel scales, and per brick layer the
// row range follows from them (rows are linear in z for a fixed scale).
// Both ranges are clipped to the panel as the kernel clips them, with the
// kernel's margins plus one for FP32 rounding on each side.
AdjPlan adjoint_plan(const cbct_geom *g, int bk, int channels, int NT, size_t budget)
{
    const cbct_geom_desc &d = g->desc;
    AdjPlan p{};
    int W = 0, H = 0;
    const int nbx = (d.nx + kBI - 1) / kBI, nby = (d.ny + kBJ - 1) / kBJ;
    const int nbz = (d.nz + bk - 1) / bk;
    auto cx = [&](double i) { return d.origin_mm[0] + (i - 0.5 * (d.nx - 1)) * d.vx_mm; };
    auto cy = [&](double j) { return d.origin_mm[1] + (j - 0.5 * (d.ny - 1)) * d.vy_mm; };
    auto cz = [&](double k) { return d.origin_mm[2] + (k - 0.5 * (d.nz - 1)) * d.vz_mm; };
    for (int a = 0; a < d.n_angles; ++a) {
        const double c = std::cos(g->angles[a]), s = std::sin(g->angles[a]);
        for (int by = 0; by < nby; ++by)
            for (int bx = 0; bx < nbx; ++bx) {
                const int i0 = bx * kBI, i1 = std::min(i0 + kBI, d.nx) - 1;
                const int j0 = by * kBJ, j1 = std::min(j0 + kBJ, d.ny) - 1;
                const double xs[2] = {cx(i0) - d.vx_mm, cx(i1) + d.vx_mm};
                const double ys[2] = {cy(j0) - d.vy_mm, cy(j1) + d.vy_mm};
                double umin = 1e300, umax = -1e300, lmin = 1e300, lmax = -1e300;
                for (double x : xs)
                    for (double y : ys) {
                        const double lam = -d.sdd_mm / (c * x + s * y - d.sid_mm);
                        const double u =
                            (lam * (-s * x + c * y) - d.off_u_mm) / d.du_mm + 0.5 * (d.nu - 1);
                        umin = std::min(umin, u);
                        umax = std::max(umax, u);
                        lmin = std::min(lmin, lam);
                        lmax = std::max(lmax, lam);
                    }
                const double u0 = std::max(std::floor(umin) - 2.0, 0.0);
                const double u1 = std::min(std::ceil(umax) + 2.0, (double)(d.nu - 1));
                if (u1 < u0)
                    continue;
                W = std::max(W, (int)(u1 - u0) + 1);
                for (int bz = 0; bz < nbz; ++bz) {
                    const int k0 = bz * bk, k1 = std::min(k0 + bk, d.nz) - 1;
                    const double zl = cz(k0) - d.vz_mm, zh = cz(k1) + d.vz_mm;
                    const double vmin =
                        (std::min(lmin * zl, lmax * zl) - d.off_v_mm) / d.dv_mm + 0.5 * (d.nv - 1);
                    const double vmax =
                        (std::max(lmin * zh, lmax * zh) - d.off_v_mm) / d.dv_mm + 0.5 * (d.nv - 1);
                    const double v0 = std::max(std::floor(vmin) - 3.0, 0.0);
                    const double v1 = std::min(std::ceil(vmax) + 3.0, (double)(d.nv - 1));
                    if (v1 >= v0)
                        H = std::max(H, (int)(v1 - v0) + 1);
                }
            }
    }
    // a tap run never leaves the window (its start is clamped), so the
    // window needs the brick's rows, or one run when that is taller
    H = std::max(H, NT);
    // the window is stored column-major with an odd column stride, so a row
    // of lanes writing consecutive columns hits distinct LDS banks
    int WS = H | 1;
    size_t lds = (size_t)W * WS * channels * sizeof(float) + (size_t)W * 4 * sizeof(float);
    if (W > 0 && lds <= budget && NT <= kMaxTaps) {
        p.ok = true;
        p.W = W;
        p.H = H;
        p.WS = WS;
        p.NTmax = NT;
    }
    return p;
}

}  // namespace

void plan_host(cbct_geom *g)
{
    const cbct_geom_desc &d = g->desc;

    // ---- forward tiles: the largest tiles whose box fits 64 x 32 voxels
    g->fwd = FwdPlan{};
    g->tiles.clear();
    TileBuild tb;
    int R = 0, TU = 64;
    for (int tu : {64, 32}) {
        for (int r : {8, 4, 2, 1}) {
            tb = make_tiles(g, tu, (256 / tu) * r);
            if (tb.BQ <= kMaxBoxQ && tb.BK <= kMaxBoxK) {
                R = r;
                TU = tu;
                break;
            }
        }
        if (R > 0)
            break;
    }
    if (R > 0) {
        while (tb.tiles.size() % 8) {
            TileRec pad{};
            pad.nu_t = 0;
            pad.p_lo = 1;
            pad.p_hi = 0;
            tb.tiles.push_back(pad);
        }
        g->fwd.ok = true;
        g->fwd.R = R;
        g->fwd.TU = TU;
        g->fwd.BQ = tb.BQ;
        g->fwd.BK = tb.BK;
        g->fwd.n_tiles = (int)tb.tiles.size();
        g->tiles = std::move(tb.tiles);
    }

    // ---- adjoint bricks
    g->adj = AdjPlan{};
    double hx = 0.5 * (d.nx + 1) * d.vx_mm, hy = 0.5 * (d.ny + 1) * d.vy_mm;
    double R_sup = 0.0;
    for (int q = 0; q < 4; ++q) {
        double x = d.origin_mm[0] + ((q & 1) ? hx : -hx);
        double y = d.origin_mm[1] + ((q & 2) ? hy : -hy);
        R_sup = std::max(R_sup, std::sqrt(x * x + y * y));
    }
    const double t_min = (d.sid_mm - R_sup) / d.sdd_mm;
    const double rvs = d.dv_mm / d.vz_mm;
    const int NT = adj_taps_rounded((int)std::floor(2.0 / (t_min * rvs)) + 3);
    for (size_t budget : {kAdjLdsShare, kAdjLdsBudget})
        for (int kv : {4, 2, 1}) {
            AdjPlan p = adjoint_plan(g, 4 * kv, 1, NT, budget);
            if (p.ok) {
                p.KV = kv;
                g->adj = p;
                return;
            }
        }
}

}  // namespace cbct
