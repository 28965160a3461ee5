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
// times 8, 4, 2, 1 rows whose boxes fit.  Volumes that reach 4 GiB with 64
// more z planes (the kernel's offsets are 32-bit, and offsets below the
// volume must wrap past its end) take the one-thread-per-ray kernel.
//
// Adjoint: the volume is cut into 8 x 7 x 4 KV bricks (KV = 4, 2 or 1 voxels
// per thread along z).  For every angle a brick's support (voxel centres +-
// one pitch) projects onto the panel inside a W x H window that is staged in
// LDS; W and H are the largest windows over all bricks and angles.  Each
// brick column's window (columns, source-panel scales, row taps) is
// tabulated per angle for the kernel.  The
// tallest bricks whose window lets four workgroups share a CU's 160 KB of LDS
// and that still give two bricks per CU are taken (small volumes take
// shorter bricks to fill the chip), else the tallest that fit 64 KB (large
// voxels seen through fine pixels make tall windows).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "cbct_internal.h"

namespace cbct {

namespace {

constexpr int kMaxBoxQ = 64;      // staged box: one 64-lane row per z index
constexpr int kMaxBoxK = 32;      // and at most 32 rows
constexpr int kBI = kAdjBI, kBJ = kAdjBJ;
constexpr size_t kAdjLdsShare = 40 * 1024;    // four workgroups per CU
constexpr size_t kAdjLdsBudget = 64 * 1024;
constexpr long kMinBricks = 2 * 256;          // two bricks per CU
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

// Panel windows of every brick column (8 x 7 voxels, all z) at every angle,
// in FP64: the projections of the support box corners (voxel centres +- one
// pitch) give the column range (one column of margin on each side, clipped
// to the panel), the extreme source-panel scales and the smallest ray
// parameter t, from which the row taps follow (a voxel's non-zero rows in
// one column span less than 2 / (t dv / vz) rows: at most floor of that
// plus one, counted from the first of them, where the run starts).  The
// kernel reads these instead of computing them.
struct WinTable {
    std::vector<BrickWin> w;         // [n_angles][nby][nbx]
    std::vector<double> lmin, lmax;  // the scales in FP64
    int W = 0;                       // widest column range
};

WinTable brick_windows(const cbct_geom *g, int NTmax)
{
    const cbct_geom_desc &d = g->desc;
    const int nbx = (d.nx + kBI - 1) / kBI, nby = (d.ny + kBJ - 1) / kBJ;
    const size_t n = (size_t)d.n_angles * nby * nbx;
    WinTable t;
    t.w.resize(n);
    t.lmin.resize(n);
    t.lmax.resize(n);
    const double rvs = d.dv_mm / d.vz_mm;
    auto cx = [&](double i) { return d.origin_mm[0] + (i - 0.5 * (d.nx - 1)) * d.vx_mm; };
    auto cy = [&](double j) { return d.origin_mm[1] + (j - 0.5 * (d.ny - 1)) * d.vy_mm; };
    for (int a = 0; a < d.n_angles; ++a) {
        const double c = std::cos(g->angles[a]), s = std::sin(g->angles[a]);
        for (int by = 0; by < nby; ++by)
            for (int bx = 0; bx < nbx; ++bx) {
                const int i0 = bx * kBI, i1 = std::min(i0 + kBI, d.nx) - 1;
                const int j0 = by * kBJ, j1 = std::min(j0 + kBJ, d.ny) - 1;
                const double xs[2] = {cx(i0) - d.vx_mm, cx(i1) + d.vx_mm};
                const double ys[2] = {cy(j0) - d.vy_mm, cy(j1) + d.vy_mm};
                double umin = 1e300, umax = -1e300, lmin = 1e300, lmax = -1e300, tmin = 1e300;
                for (double x : xs)
                    for (double y : ys) {
                        const double den = c * x + s * y - d.sid_mm;
                        const double lam = -d.sdd_mm / den;
                        const double u =
                            (lam * (-s * x + c * y) - d.off_u_mm) / d.du_mm + 0.5 * (d.nu - 1);
                        umin = std::min(umin, u);
                        umax = std::max(umax, u);
                        lmin = std::min(lmin, lam);
                        lmax = std::max(lmax, lam);
                        tmin = std::min(tmin, -den / d.sdd_mm);
                    }
                const int u0 = (int)std::max(std::floor(umin) - 1.0, 0.0);
                const int u1 = (int)std::min(std::ceil(umax) + 1.0, (double)(d.nu - 1));
                const size_t e = ((size_t)a * nby + by) * nbx + bx;
                BrickWin &bw = t.w[e];
                bw.lmin = (float)lmin;
                bw.lmax = (float)lmax;
                if (u0 <= u1) {
                    bw.u01 = (uint32_t)u0 | ((uint32_t)u1 << 16);
                    t.W = std::max(t.W, u1 - u0 + 1);
                } else {
                    bw.u01 = 1u;   // u0 = 1 > u1 = 0: not seen
                }
                const int nt = (int)std::floor(2.0 / (tmin * rvs)) + 1;
                bw.nt = adj_taps_rounded(std::min(nt, NTmax));
                t.lmin[e] = lmin;
                t.lmax[e] = lmax;
            }
    }
    return t;
}

// Window bounds of bricks 8 x 7 x bk staging `channels` channels per
// element; ok when the window fits the LDS budget.  Per brick layer the row
// range follows from the brick column's scales (rows are linear in z for a
// fixed scale), clipped to the panel as the kernel clips it, with the
// kernel's margins plus one for its FP32 rounding on each side.
AdjPlan adjoint_plan(const cbct_geom *g, const WinTable &t, int bk, int channels, int NT,
                     size_t budget)
{
    const cbct_geom_desc &d = g->desc;
    AdjPlan p{};
    int H = 0;
    const int nbz = (d.nz + bk - 1) / bk;
    auto cz = [&](double k) { return d.origin_mm[2] + (k - 0.5 * (d.nz - 1)) * d.vz_mm; };
    for (size_t e = 0; e < t.w.size(); ++e) {
        if ((t.w[e].u01 & 0xffffu) > (t.w[e].u01 >> 16))
            continue;
        const double lmin = t.lmin[e], lmax = t.lmax[e];
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
    const int W = t.W;
    // a tap run never leaves the window (its start is clamped), so the
    // window needs the brick's rows, or one run when that is taller
    H = std::max(H, NT);
    // the window is stored column-major; a column stride of 2 mod 4 words
    // spreads the gather's reads (lanes of a wave read different columns)
    // over the LDS banks best: at the clinical size 23.0 ms for the adjoint
    // against 24.0 ms with odd strides, which would instead spare the
    // staging's row writes a two-way conflict.  The stride exceeds H: the
    // staging writes the rows of a batch past the window to the rows above
    // it (tall columns) or to the spare row (short ones), never past the
    // column.
    int WS = H + 1 + (5 - H % 4) % 4;
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
    // the tiled kernel addresses one volume channel with 32-bit byte offsets,
    // those of slots below the volume wrapping past its end (64 planes of
    // margin)
    const bool off32 = (uint64_t)d.nx * d.ny * (d.nz + 64) * sizeof(float) < (1ull << 32);
    for (int tu : {64, 32}) {
        if (!off32)
            break;
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
    const int NT = adj_taps_rounded((int)std::floor(2.0 / (t_min * rvs)) + 1);
    const long bricks_xy = (long)((d.nx + kBI - 1) / kBI) * ((d.ny + kBJ - 1) / kBJ);
    WinTable wt = brick_windows(g, NT);
    g->wins = wt.w;
    for (size_t budget : {kAdjLdsShare, kAdjLdsBudget}) {
        AdjPlan shortest{};
        for (int kv : {4, 2, 1}) {
            AdjPlan p = adjoint_plan(g, wt, 4 * kv, 1, NT, budget);
            if (!p.ok)
                continue;
            p.KV = kv;
            shortest = p;
            if (bricks_xy * ((d.nz + 4 * kv - 1) / (4 * kv)) >= kMinBricks) {
                g->adj = p;
                return;
            }
        }
        if (shortest.ok) {   // no height gives kMinBricks: the shortest bricks
            g->adj = shortest;
            return;
        }
    }
    g->wins.clear();   // the one-thread-per-voxel kernel needs no windows
}

}  // namespace cbct
