// Adjoint A^T for gfx950: atomic-free gather over LDS-staged panel windows.
//
// Operator: the transpose of the plane-sampled cone-beam projector
// (arXiv 2512.21180, Sec. 2.2, backprojection P* as the adjoint of P).  The
// weight of voxel (i,j,k) in ray (a,u,v) is
//   ds(u,v) * hat(q_u(p) - q_vox) * hat(k(u,v,p) - k),   hat(s) = max(0, 1-|s|),
// where p is the voxel's index along the ray's sampling axis and q_vox its
// in-plane index; these are the weights the forward kernel applies.
//
// A workgroup owns a brick of 8 x 7 x 4 KV output voxels (KV = 4, 2 or 1,
// chosen by the plan so that the window fits in LDS); wave w owns the KV
// voxel layers k0 + KV w .. k0 + KV w + KV - 1.  The in-plane weight of a
// sample is shared by two voxels: a ray crossing the plane p at in-plane
// index q lies in the segment [s, s + 1), s = floor(q), and weighs 1 - f on
// voxel s and f on voxel s + 1 (f = q - s) with the same z weights.  So the
// lanes own (plane, segment) pairs rather than voxels: on x planes lane l
// takes plane i0 + l % 8 and segment j0 - 1 + l / 8 (eight segments feed
// the seven output rows), on y planes lane l < 63 takes plane j0 + l / 9
// and segment i0 - 1 + l % 9 (nine segments, eight output columns).  Each
// column whose ray crosses the lane's plane in its segment (the test is the
// forward's floor, so every column falls in exactly one segment) gets its
// z run computed once and added with weight 1 - f and f to two register
// sums; after the last angle the four shares of every output voxel (own and
// lower segment, both axes) are added in a fixed order through LDS and
// written once -- no atomics, and the order does not depend on timing.
// Against one voxel per lane this halves the z runs per voxel.
// For each angle the brick's panel window is staged in LDS, pre-multiplied
// by the ray length per plane ds, together with the column constants; the
// window's columns, the source-panel scales that give its rows and the row
// taps NT come from a table the host computes in FP64 per angle and brick
// column.  Per voxel and column, the rows with non-zero weight lie above
// the row v_c where the ray crosses z = k - 1 and span less than 2 / beta
// rows (beta: rows to z index, at least that of the brick's nearest point
// to the source); the run of NT = floor(2 / beta) + 1 rows that starts at
// floor(v_c) + 1, the first row above v_c, holds them all.  The start is
// taken as floor(v_c + 1 - delta), delta a few times the FP32 rounding of v_c
// (adj_start_delta): it is the first row above v_c, or one row lower when
// v_c lies within 2 delta above an integer -- a row of zero weight, and then
// the run still reaches the last non-zero row unless 2 / beta also lies
// within 2 delta below an integer (a row of weight below 2 delta beta is
// then left out, about once in 10^6 runs).
// The taps use the clamped hat, so rows outside the support add exact
// zeros (a run that would leave the window starts lower instead).  The
// window is stored column-major, so a run is consecutive LDS words read two
// at a time with immediate offsets in a fully unrolled sequence.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "cbct_internal.h"
#include "cbct_lds.h"
#include "cbct_storage.h"

namespace cbct {
namespace {

constexpr int kThreads = 256;
// Window rows per wave and staging batch (loads in flight per lane).
constexpr int kStageRows = 24;
// Columns of at least 4 kStageRows rows take the staging whose batches stay
// inside the column (bricks of KV = 4, the clinical windows).
constexpr bool adj_tall(int KV, int HS) { return KV == 4 && HS >= 4 * kStageRows; }

struct BrickArgs {
    DevGeom g;
    const BrickWin *wins;  // [n_angles][nby][nbx] panel windows
    int W, H, HS;          // window columns and rows, LDS column stride
    int nbx, nby, nbz;
    int KV;                // voxels per lane along z (bricks 8 x 7 x 4 KV)
    float rbias;           // 1 - adj_start_delta(nv)
};

__device__ inline float sat(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }

// A run's LDS address is a plain 32-bit number (lds_addr, lds_ptr): it comes
// out of one float-to-integer conversion with no base to add.

// Fractional panel column of the ray through (x, y, .) and its source-panel
// scale lambda (a point at height z lands at V = lambda z).  Used only for a
// voxel's column range, which is widened to whole columns and trimmed by the
// exact weights, so approximate reciprocals are enough.
__device__ inline void project_xy(const DevGeom &g, float inv_du, float c, float s, float x,
                                  float y, float &u, float &lam)
{
    const float den = fmaf(c, x, fmaf(s, y, -g.sid));
    lam = -g.sdd * __builtin_amdgcn_rcpf(den);
    u = fmaf(fmaf(lam, fmaf(-s, x, c * y), -g.off_u), inv_du, g.cu);
}

// Inputs of one angle's gather for one lane.
struct GatherIn {
    const DevGeom &g;
    const AngRec &ar;
    const float *yt;
    const float4 *cr;
    int HS, U0, U1, V0;
    int VS1;   // largest run start: max(V1 - NT + 1, V0), so a run ends in the window
    int k0;
    int pl[2], sg[2];   // per sampling axis (0: x planes, 1: y planes): this lane's
                        // plane and in-plane segment; pl < 0: no work on that axis
    float inv_du, inv_rvs;
    float rbias;        // 1 - delta: run start floor(v_c + 1 - delta)
};

__device__ inline float centre_x(const DevGeom &g, float i)
{
    return g.ox + (i - 0.5f * (float)(g.nx - 1)) * g.vx;
}

__device__ inline float centre_y(const DevGeom &g, float j)
{
    return g.oy + (j - 0.5f * (float)(g.ny - 1)) * g.vy;
}

// Accumulate one angle's contributions of the columns whose rays cross this
// lane's plane inside its segment [s, s + 1) of the in-plane index (the
// forward's floor(q) = s): such a sample weighs 1 - f on in-plane voxel s and
// f on voxel s + 1 (f = q - s), and the same z weights on both, so each
// column's z run is computed once for the two voxels: lo[ax][n] collects the
// 1 - f share (voxel s), hi[ax][n] the f share (voxel s + 1) for the KV
// voxels k0 + n.  NT taps per voxel and column (rows past the non-zero run
// have zero weight).  Forced inline: a call would impose the calling
// convention's register budget and stack on the kernel.
template <int NT, int KV>
__device__ __forceinline__ void gather_angle(const GatherIn &in, float (&lo)[2][KV],
                                             float (&hi)[2][KV])
{
    const DevGeom &g = in.g;
    const AngRec &ar = in.ar;
    const int HS = in.HS, U0 = in.U0, V0 = in.V0, VS1 = in.VS1;
    const int k0 = in.k0;
    const float inv_du = in.inv_du, inv_rvs = in.inv_rvs;
    const float *yt = in.yt;
    const float4 *cr = in.cr;
    // Per voxel n: the row v_c where a ray with parameter t crosses z index
    // k0 + n - 1 is Bk / t + A0 - (1 - delta); the hat argument at row r is
    // t ((r - cv) rvs + rv0) + Kb - k.
    float Bk[KV], KbK[KV];
#pragma unroll
    for (int n = 0; n < KV; ++n) {
        const float kk = (float)(k0 + n);
        Bk[n] = (kk - 1.0f - g.Kb) * inv_rvs;
        KbK[n] = g.Kb - kk;
    }
    const float A0 = fmaf(-g.rv0, inv_rvs, g.cv + in.rbias);

    const float V0f = (float)V0, VS1f = (float)VS1;
#pragma unroll
    for (int cls = 0; cls < 2; ++cls) {
        // this axis has columns at this angle (uniform) and this lane a segment
        if (cls == 0 ? ar.x_lo >= ar.x_hi : (ar.x_lo == 0 && ar.x_hi == g.nu))
            continue;
        if (in.pl[cls] < 0)
            continue;
        const float fp = (float)in.pl[cls], sf = (float)in.sg[cls];
        int c_lo, c_hi;   // this axis' columns
        float u1, u2, lam;
        if (cls == 0) {   // x planes: plane i, segment [s, s + 1) in y
            c_lo = ar.x_lo;
            c_hi = ar.x_hi - 1;
            const float xp = centre_x(g, fp), ya = centre_y(g, sf);
            project_xy(g, inv_du, ar.c, ar.s, xp, ya, u1, lam);
            project_xy(g, inv_du, ar.c, ar.s, xp, ya + g.vy, u2, lam);
        } else {          // y planes: plane j, segment [s, s + 1) in x
            c_lo = 0;
            c_hi = g.nu - 1;
            const float yp = centre_y(g, fp), xa = centre_x(g, sf);
            project_xy(g, inv_du, ar.c, ar.s, xa, yp, u1, lam);
            project_xy(g, inv_du, ar.c, ar.s, xa + g.vx, yp, u2, lam);
        }
        // The segment's columns lie between the projections of its two
        // edges (within rounding, far below a column): trim the candidate
        // range's ends to columns that are members by the exact test (the
        // membership test below keeps the partition exact in any case).
        int ul = max(max((int)floorf(fminf(u1, u2)), c_lo), U0);
        int uh = min(min((int)ceilf(fmaxf(u1, u2)), c_hi), in.U1);
        auto member = [&](int u) {
            if (cls == 1 && u >= ar.x_lo && u < ar.x_hi)
                return false;
            const float4 cq = cr[u - U0];
            const float f = fmaf(fp, cq.y, cq.x) - sf;
            return f >= 0.0f && f < 1.0f;
        };
        while (ul <= uh && !member(ul))
            ++ul;
        while (uh > ul && !member(uh))
            --uh;
        for (int u = ul; u <= uh; ++u) {
            if (cls == 1 && u >= ar.x_lo && u < ar.x_hi)
                continue;   // those columns are sampled on x planes
            const float4 cq = cr[u - U0];
            const float f = fmaf(fp, cq.y, cq.x) - sf;
            if (!(f >= 0.0f && f < 1.0f))
                continue;   // the ray crosses this plane in another segment
            const float wl = 1.0f - f;
            const float t = fmaf(fp, cq.w, cq.z);
            const float beta = t * g.rvs;
            const float rt = __builtin_amdgcn_rcpf(t);
            // LDS byte address of row 0 of this column in the window, signed
            // (row 0 lies below the window when V0 > 0; every row read,
            // vsf >= V0, has a non-negative address); exact in FP32: LDS
            // addresses are far below 2^24
            const float colb = (float)((int)lds_addr(yt) + 4 * ((u - U0) * HS - V0));
#pragma unroll
            for (int n = 0; n < KV; ++n) {
                // run start: the first row above v_c (floor(v_c) + 1), or one
                // row lower, of zero weight (see the file comment); clamped
                // into [V0, VS1] (a start moved down to VS1 only adds rows
                // below the run, of zero weight)
                const float vsf =
                    __builtin_amdgcn_fmed3f(floorf(fmaf(rt, Bk[n], A0)), V0f, VS1f);
                // hat argument at the run start; (vsf - cv) is exact, which keeps
                // the rounding of this difference of two large z indices small
                float s = fmaf(t, fmaf(vsf - g.cv, g.rvs, g.rv0), KbK[n]);
                const lds_float *py = lds_ptr((uint32_t)fmaf(vsf, 4.0f, colb));
                float yv[NT];
#pragma unroll
                for (int m = 0; m < NT; ++m)
                    yv[m] = py[m];
                float csum = 0.0f;
#pragma unroll
                for (int m = 0; m < NT; ++m) {
                    csum = fmaf(sat(1.0f - fabsf(s)), yv[m], csum);
                    s += beta;
                }
                lo[cls][n] = fmaf(wl, csum, lo[cls][n]);
                hi[cls][n] = fmaf(f, csum, hi[cls][n]);
            }
        }
    }
}

// Stage one angle's panel window into a tall column layout (HS >= 4 SB):
// Wc columns (from U0) x Hs rows of the ds-weighted projection, whose rows
// V0 .. V1 the buffer resource `rows` holds, into yt, column-major with
// stride HS, and the columns' records into cr.  Columns on lanes, rows on
// waves (stride 4), SB rows per wave and batch.  A batch that would run past
// the column starts lower instead, at the last row of the wave's residue
// class that keeps it inside (it then stores some rows of the wave's
// previous batch again, with the same values), so its stores take immediate
// offsets from one address.
template <int SB>
__device__ __forceinline__ void stage_tall(const DevGeom &g, int a, __amdgpu_buffer_rsrc_t rows,
                                           int U0, int Wc, int Hs, int HS, int w, int lane,
                                           float *yt, float4 *cr)
{
    const int row_bytes = 4 * g.nu;
    const int top = HS - 1 - 4 * (SB - 1);   // >= 3 in tall columns
    const int vtop = top - ((top - w) & 3);  // largest start = w mod 4
    for (int uu = lane; uu < Wc; uu += 64) {
        float4 ctab;   // one wave writes the column table (see gather_brick)
        if (w == 0) {
            const ColRec col = g.cols[(size_t)a * g.nu + U0 + uu];
            ctab = make_float4(col.pb, col.ps, col.t0, col.tau);
        }
        const int cb = 4 * (U0 + uu);   // byte offset of the column in a row
        float *dst = yt + (size_t)uu * HS;
        for (int vv0 = w; vv0 < Hs; vv0 += 4 * SB) {
            const int vb = min(vv0, vtop);
            int off = cb + vb * row_bytes;   // kept in one register (see gather_brick)
            asm volatile("" : "+v"(off));
            float val[SB];
#pragma unroll
            for (int jj = 0; jj < SB; ++jj)
                val[jj] = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(rows, off + 4 * jj * row_bytes, 0, 0));
            float *d = dst + vb;
#pragma unroll
            for (int jj = 0; jj < SB; ++jj)
                d[4 * jj] = val[jj];
        }
        if (w == 0)
            cr[uu] = ctab;
    }
}

// Gather one brick (index b): bricks hold kAdjBI x kAdjBJ x 4 KV output
// voxels.  Lane roles (wave w owns the KV voxel layers from 4 KV (brick z) +
// KV w up): on x planes lane l takes plane i0 + l % 8 and in-plane segment
// j0 - 1 + l / 8 (eight segments serve the seven output rows j0 .. j0 + 6);
// on y planes lane l < 63 takes plane j0 + l / 9 and segment i0 - 1 + l % 9
// (nine segments serve the eight output columns).  After the last angle the
// four shares each output voxel receives (lo of its own segment and hi of
// the one below, on each axis) are added in a fixed order through LDS.
// `lds` holds the panel window, column-major ([W][HS], HS = 2 mod 4, which
// suits the gather's reads), and the column table; then the exchange.
template <class VS, int KV, bool TALL>
__device__ __forceinline__ void gather_brick(const BrickArgs &A, int b, const float *ws,
                                             typename VS::T *vol, float *lds)
{
    constexpr int kBK = 4 * KV;
    constexpr int kSB = kStageRows;
    const DevGeom &g = A.g;
    const int HS = A.HS;
    float *yt = lds;                                    // ds-weighted panel window
    float4 *cr = (float4 *)(lds + (size_t)A.W * HS);    // [W] (pb, ps, t0, tau)

    const int bx = b % A.nbx, by = (b / A.nbx) % A.nby, bz = b / (A.nbx * A.nby);

    // the wave index is uniform (scalar registers for its row and layer indices)
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i0 = bx * kAdjBI, j0 = by * kAdjBJ;
    const int k0 = bz * kBK + w * KV;
    int pl0 = i0 + (lane & 7), sg0 = j0 - 1 + (lane >> 3);
    int pl1 = j0 + lane / 9, sg1 = i0 - 1 + lane % 9;
    if (pl0 >= g.nx || sg0 >= g.ny)
        pl0 = -1;
    if (lane >= 63 || pl1 >= g.ny || sg1 >= g.nx)
        pl1 = -1;

    // z extent of the brick's support (voxel centres +- one pitch), uniform
    const int kz0 = bz * kBK, kz1 = min(kz0 + kBK, g.nz) - 1;
    const float zs0 = g.oz + ((float)kz0 - 0.5f * (float)(g.nz - 1)) * g.vz - g.vz;
    const float zs1 = g.oz + ((float)kz1 - 0.5f * (float)(g.nz - 1)) * g.vz + g.vz;
    // the brick column's panel windows, one per angle (host FP64)
    const BrickWin *wcol = A.wins + (size_t)by * A.nbx + bx;
    const size_t wstep = (size_t)A.nbx * A.nby;

    const float inv_du = 1.0f / g.du, inv_dv = 1.0f / g.dv;
    // z of this wave's first voxel layer (wave-uniform)
    const float zc_w0 = g.oz + ((float)k0 - 0.5f * (float)(g.nz - 1)) * g.vz;
    const float inv_rvs = 1.0f / g.rvs;
    float lo[2][KV], hi[2][KV];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int n = 0; n < KV; ++n) {
            lo[c][n] = 0.0f;
            hi[c][n] = 0.0f;
        }

    __syncthreads();   // the previous work item's readers of lds are done
    for (int a = 0; a < g.n_angles; ++a) {
        // ---- panel window of the brick (uniform): columns and row taps from
        // the table, rows from the extreme source-panel scales (positive) at
        // the support's lowest and highest z
        const BrickWin bw = wcol[(size_t)a * wstep];
        const int U0 = (int)(bw.u01 & 0xffffu);
        const int U1 = min((int)(bw.u01 >> 16), U0 + A.W - 1);
        if (U0 > U1)
            continue;
        const float lmin = bw.lmin, lmax = bw.lmax;
        const float vmin = fmaf(fminf(lmin * zs0, lmax * zs0) - g.off_v, inv_dv, g.cv);
        const float vmax = fmaf(fmaxf(lmin * zs1, lmax * zs1) - g.off_v, inv_dv, g.cv);
        const int V0 = max((int)floorf(vmin) - 2, 0);
        const int V1 = min(min((int)ceilf(vmax) + 2, g.nv - 1), V0 + A.H - 1);
        if (V0 > V1)
            continue;
        const int NT = bw.nt;
        const AngRec ar = g.angs[a];
        const int Wc = U1 - U0 + 1;
        // staged rows; rows past V1 (only when the window is shorter than a
        // run) are zero
        const int Hs = max(V1 - V0 + 1, NT);
        const int VS1 = max(V1 - NT + 1, V0);

        __syncthreads();   // previous angle's readers are done
        // Columns on lanes, rows on waves (stride 4).  The loads of a batch
        // of rows are issued before any of them is used, so their latencies
        // overlap instead of adding up row after row.  They go through a
        // buffer resource holding exactly rows V0 .. V1 of this projection:
        // the range check returns zero for every row past V1 (the window's
        // zero rows and a batch's rows past Hs) without touching memory, so
        // no load needs a test of its own.  Byte offsets within the rows are
        // 32-bit (nv nu < 2^24).  Every store is unconditional, so no load
        // can be moved behind the wait for the others; one wave also writes
        // the column table, its load issued with the rows' and stored after
        // them, so that wave does not wait for it before issuing its row
        // loads.  The batch's first row offset for a lane is kept in one
        // register (the empty asm stops the compiler from hoisting a lane
        // offset per row out of the loop, which costs a register per row);
        // each load adds a wave-uniform row offset.
        const float *proj = ws + ((size_t)a * g.nv + V0) * g.nu;   // row V0, ds-weighted
        const __amdgpu_buffer_rsrc_t rows =
            __builtin_amdgcn_make_buffer_rsrc((void *)proj, (short)0, (V1 - V0 + 1) * g.nu * 4,
                                              kBufferWord3);
        if constexpr (TALL) {
            // Batches no longer than the window needs: SB rows per wave
            // cover 4 SB rows, SB = 16 up to 64 rows, 20 up to 80, else 24
            // (and more batches past 96 rows), so fewer rows past the window
            // are loaded and stored.  (Seven lengths from 8 to 24 saved a
            // further tenth of the staged rows but cost registers and were
            // slower.)
            if (Hs <= 64)
                stage_tall<16>(g, a, rows, U0, Wc, Hs, HS, w, lane, yt, cr);
            else if (Hs <= 80)
                stage_tall<20>(g, a, rows, U0, Wc, Hs, HS, w, lane, yt, cr);
            else
                stage_tall<kSB>(g, a, rows, U0, Wc, Hs, HS, w, lane, yt, cr);
        } else {
            // Short columns: batches of kSB rows per wave whose rows past Hs
            // (zeros) all go to row HS - 1, a spare row no tap reads (HS > H
            // >= Hs).  Written out here rather than in a function like
            // stage_tall, so these kernels compile as they did before the
            // tall variant existed (the call changed their register
            // allocation).
            const int row_bytes = 4 * g.nu;
            for (int uu = lane; uu < Wc; uu += 64) {
                float4 ctab;
                if (w == 0) {
                    const ColRec col = g.cols[(size_t)a * g.nu + U0 + uu];
                    ctab = make_float4(col.pb, col.ps, col.t0, col.tau);
                }
                const int cb = 4 * (U0 + uu);
                float *dst = yt + (size_t)uu * HS;
                for (int vv0 = w; vv0 < Hs; vv0 += 4 * kSB) {
                    int off = cb + vv0 * row_bytes;
                    asm volatile("" : "+v"(off));
                    float val[kSB];
#pragma unroll
                    for (int jj = 0; jj < kSB; ++jj)
                        val[jj] = __builtin_bit_cast(
                            float, __builtin_amdgcn_raw_buffer_load_b32(
                                       rows, off + 4 * jj * row_bytes, 0, 0));
#pragma unroll
                    for (int jj = 0; jj < kSB; ++jj)
                        dst[min(vv0 + 4 * jj, HS - 1)] = val[jj];
                }
                if (w == 0)
                    cr[uu] = ctab;
            }
        }
        __syncthreads();

        // ---- this wave's KV voxel layers (z of the voxel centres +- one
        // pitch) land on rows [wv0, wv1] for every ray through the brick's
        // box (lambda is extreme at the box corners); a wave whose rows miss
        // the staged rows entirely has only zero weights and skips the angle
        // (wave-uniform branch; one row of margin for rounding).
        {
            const float zl = zc_w0 - g.vz, zh = zc_w0 + (float)(KV - 1) * g.vz + g.vz;
            const float wv0 = fmaf(fminf(lmin * zl, lmax * zl) - g.off_v, inv_dv, g.cv);
            const float wv1 = fmaf(fmaxf(lmin * zh, lmax * zh) - g.off_v, inv_dv, g.cv);
            if (wv1 < (float)V0 - 1.0f || wv0 > (float)V1 + 1.0f)
                continue;
        }
        // ---- gather with a compile-time tap count (NT rounded up to a
        // supported count; extra taps read zero weight)
        const GatherIn in{g, ar, yt, cr, HS, U0, U1, V0, VS1, k0, {pl0, pl1}, {sg0, sg1},
                          inv_du, inv_rvs, A.rbias};
        switch (NT) {
        case 4: gather_angle<4, KV>(in, lo, hi); break;
        case 5: gather_angle<5, KV>(in, lo, hi); break;
        case 6: gather_angle<6, KV>(in, lo, hi); break;
        case 7: gather_angle<7, KV>(in, lo, hi); break;
        case 8: gather_angle<8, KV>(in, lo, hi); break;
        case 9: gather_angle<9, KV>(in, lo, hi); break;
        case 10: gather_angle<10, KV>(in, lo, hi); break;
        case 11: gather_angle<11, KV>(in, lo, hi); break;
        case 12: gather_angle<12, KV>(in, lo, hi); break;
        case 13: gather_angle<13, KV>(in, lo, hi); break;
        case 14: gather_angle<14, KV>(in, lo, hi); break;
        case 15: gather_angle<15, KV>(in, lo, hi); break;
        case 16: gather_angle<16, KV>(in, lo, hi); break;
        case 18: gather_angle<18, KV>(in, lo, hi); break;
        case 20: gather_angle<20, KV>(in, lo, hi); break;
        case 24: gather_angle<24, KV>(in, lo, hi); break;
        case 28: gather_angle<28, KV>(in, lo, hi); break;
        default: gather_angle<32, KV>(in, lo, hi); break;
        }
    }

    // ---- each output voxel's four shares, added in a fixed order: x planes
    // (lo of its own segment, hi of the segment below), then y planes (same)
    __syncthreads();   // every wave is done with the window
    float *xch = lds + (size_t)w * (4 * 64 * KV);
#pragma unroll
    for (int n = 0; n < KV; ++n) {
        xch[(0 * KV + n) * 64 + lane] = lo[0][n];
        xch[(1 * KV + n) * 64 + lane] = hi[0][n];
        xch[(2 * KV + n) * 64 + lane] = lo[1][n];
        xch[(3 * KV + n) * 64 + lane] = hi[1][n];
    }
    __syncthreads();
    const int io = lane & 7, jo = lane >> 3;
    const int i = i0 + io, j = j0 + jo;
    if (jo < kAdjBJ && i < g.nx && j < g.ny) {
        const int xl = ((jo + 1) << 3) | io, xh = (jo << 3) | io;   // x-plane lanes
        const int yl = jo * 9 + io + 1, yh = jo * 9 + io;           // y-plane lanes
#pragma unroll
        for (int n = 0; n < KV; ++n) {
            const int k = k0 + n;
            if (k < g.nz) {
                float v = xch[(0 * KV + n) * 64 + xl] + xch[(1 * KV + n) * 64 + xh];
                v += xch[(2 * KV + n) * 64 + yl];
                v += xch[(3 * KV + n) * 64 + yh];
                VS::st(vol, ((size_t)k * g.ny + j) * g.nx + i, v);
            }
        }
    }
}

// Workgroups are dealt to the 8 XCDs round robin (XCD = id % 8).  XCD xc
// takes the brick rows by = xc, xc + 8, ... (every z layer of them, so each
// XCD holds an even share of cheap and costly bricks), in the order bx, bz,
// row: workgroups resident together on one XCD are neighbouring bricks whose
// panel windows overlap in its L2 (adjoint 33 -> 27 ms for the clinical
// case; a contiguous brick range per XCD unbalances the XCDs, 71 ms).
// Slot li of XCD xc -> brick index, or -1 for the padding slots.
__device__ inline int brick_of_slot(const BrickArgs &A, int xc, int li)
{
    const int plane = A.nbx * A.nbz;
    const int by = xc + 8 * (li / plane);
    if (by >= A.nby)
        return -1;
    const int bz = (li % plane) / A.nbx, bx = li % A.nbx;
    return (bz * A.nby + by) * A.nbx + bx;
}

// Slots per XCD of one case (padded so that every XCD has the same count).
__host__ __device__ inline int slots_per_xcd(const BrickArgs &A)
{
    return A.nbx * A.nbz * ((A.nby + 7) / 8);
}

template <class VS, int KV, bool TALL>
__global__ void __launch_bounds__(kThreads)
adjoint_brick(BrickArgs A, const float *__restrict__ ws, typename VS::T *__restrict__ vol)
{
    extern __shared__ float lds[];
    const int b = brick_of_slot(A, blockIdx.x & 7, blockIdx.x >> 3);
    if (b < 0)
        return;
    const int ch = blockIdx.y;
    const size_t nvox = (size_t)A.g.nx * A.g.ny * A.g.nz;
    const size_t nsino = (size_t)A.g.n_angles * A.g.nv * A.g.nu;
    gather_brick<VS, KV, TALL>(A, b, ws + ch * nsino, vol + ch * nvox, lds);
}

// The ds-weighted copy of a sinogram that the bricks stage from:
// out = y ds(a, u, v) in FP32 (ds by ray_ds, the forward's ray length per
// plane), so that the ray length is computed once per element instead of
// once per brick that stages it.  One workgroup per panel row of one angle
// and channel.
template <class SS>
__global__ void __launch_bounds__(kThreads)
ds_weight(DevGeom g, const typename SS::T *__restrict__ y, float *__restrict__ out)
{
    const int row = blockIdx.x;   // a * nv + v
    const int a = row / g.nv, v = row - a * g.nv;
    const size_t base = ((size_t)blockIdx.y * g.n_angles * g.nv + row) * g.nu;
    const float v2 = g.rows[v].y;
    const ColRec *cols = g.cols + (size_t)a * g.nu;
    for (int u = threadIdx.x; u < g.nu; u += kThreads) {
        const ColRec c = cols[u];
        out[base + u] = SS::wide(SS::raw(y, base + u)) * ray_ds(c.dsf, c.n2, v2);
    }
}

// ---- batched adjoint: one launch over all (case, brick) items ---------------

struct AdjCase {
    BrickArgs A;
    const float *ws;   // the case's ds-weighted sinogram
    void *vol;
};

struct BatchAdjArgs {
    int n_cases, n_items;
    int first[kMaxBatch + 1];   // first slot (per XCD) of each case
    AdjCase c[kMaxBatch];
};

template <class VS>
__global__ void __launch_bounds__(kThreads)
adjoint_batch(BatchAdjArgs B)
{
    extern __shared__ float lds[];
    // one item per workgroup; per XCD the slots of case 0, then case 1, ...,
    // each case's slots mapped to bricks as in adjoint_brick
    const int xc = blockIdx.x & 7, li = blockIdx.x >> 3;
    int cs = 0;
    while (cs + 1 < B.n_cases && li >= B.first[cs + 1])
        ++cs;
    const AdjCase &C = B.c[cs];
    const int b = brick_of_slot(C.A, xc, li - B.first[cs]);
    if (b < 0)
        return;
    auto *vs = (typename VS::T *)C.vol;
    switch (C.A.KV) {   // uniform over the workgroup
    case 4: gather_brick<VS, 4, false>(C.A, b, C.ws, vs, lds); break;
    case 2: gather_brick<VS, 2, false>(C.A, b, C.ws, vs, lds); break;
    default: gather_brick<VS, 1, false>(C.A, b, C.ws, vs, lds); break;
    }
}

}  // namespace

static BrickArgs brick_args(const DevGeom &g, const AdjPlan &p)
{
    const int bk = 4 * p.KV;
    return BrickArgs{g, p.wins, p.W, p.H, p.WS, (g.nx + kAdjBI - 1) / kAdjBI,
                     (g.ny + kAdjBJ - 1) / kAdjBJ, (g.nz + bk - 1) / bk, p.KV,   // WS: column stride
                     1.0f - adj_start_delta(g.nv)};
}

// The window and column table, or the final exchange (four shares per lane
// and voxel layer, four waves) if that is larger.
static size_t brick_lds(const AdjPlan &p)
{
    const size_t window = (size_t)p.W * p.WS + (size_t)p.W * 4;
    const size_t exchange = (size_t)4 * 4 * 64 * p.KV;
    return std::max(window, exchange) * sizeof(float);
}

static hipError_t launch_ds_weight(const DevGeom &g, const void *sino, cbct_dtype st, float *ws,
                                   int channels, hipStream_t s)
{
    dim3 grid((unsigned)(g.n_angles * g.nv), channels), block(kThreads);
    // the volume type plays no part here: dispatch on (F32, st)
    return dispatch_storage(CBCT_F32, st, [&](auto, auto ss) -> hipError_t {
        using SS = decltype(ss);
        hipLaunchKernelGGL((ds_weight<SS>), grid, block, 0, s, g, (const typename SS::T *)sino, ws);
        return hipGetLastError();
    });
}

hipError_t launch_adjoint_brick(const DevGeom &g, const AdjPlan &p, const void *sino,
                                cbct_dtype st, void *vol, cbct_dtype vt, int channels,
                                hipStream_t s)
{
    BrickArgs A = brick_args(g, p);
    dim3 grid(8 * slots_per_xcd(A), channels), block(kThreads);
    const size_t nsino = (size_t)g.n_angles * g.nv * g.nu;
    ScratchLease lease;
    hipError_t e = scratch_acquire(nsino * channels * sizeof(float), s, lease);
    if (e == hipSuccess)
        e = launch_ds_weight(g, sino, st, (float *)lease.ptr, channels, s);
    if (e == hipSuccess)
        e = dispatch_storage(vt, st, [&](auto vs, auto) -> hipError_t {
            using VS = decltype(vs);
            const size_t lds = brick_lds(p);
            const float *w = (const float *)lease.ptr;
            auto *x = (typename VS::T *)vol;
            if (adj_tall(p.KV, p.WS))
                hipLaunchKernelGGL((adjoint_brick<VS, 4, true>), grid, block, lds, s, A, w, x);
            else if (p.KV == 4)
                hipLaunchKernelGGL((adjoint_brick<VS, 4, false>), grid, block, lds, s, A, w, x);
            else if (p.KV == 2)
                hipLaunchKernelGGL((adjoint_brick<VS, 2, false>), grid, block, lds, s, A, w, x);
            else
                hipLaunchKernelGGL((adjoint_brick<VS, 1, false>), grid, block, lds, s, A, w, x);
            return hipGetLastError();
        });
    const hipError_t r = scratch_release(s, lease);
    return e != hipSuccess ? e : r;
}

hipError_t launch_adjoint_batch(int n, const cbct_geom *const *gs, const void *const *sinos,
                                void *const *vols, cbct_dtype st, cbct_dtype vt, hipStream_t s)
{
    BatchAdjArgs B{};
    B.n_cases = n;
    size_t lds = 0, total = 0;
    int items = 0;
    size_t off[kMaxBatch];
    for (int i = 0; i < n; ++i) {
        const cbct_geom *g = gs[i];
        B.first[i] = items;
        B.c[i] = AdjCase{brick_args(g->dev, g->adj), nullptr, vols[i]};
        items += slots_per_xcd(B.c[i].A);
        lds = std::max(lds, brick_lds(g->adj));
        off[i] = total;
        total += (size_t)g->dev.n_angles * g->dev.nv * g->dev.nu;
    }
    B.first[n] = items;
    B.n_items = items;
    const int grid = 8 * items;
    ScratchLease lease;
    hipError_t e = scratch_acquire(total * sizeof(float), s, lease);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        B.c[i].ws = (const float *)lease.ptr + off[i];
        e = launch_ds_weight(gs[i]->dev, sinos[i], st, (float *)lease.ptr + off[i], 1, s);
    }
    if (e == hipSuccess)
        e = dispatch_storage(vt, st, [&](auto vs, auto) -> hipError_t {
            using VS = decltype(vs);
            hipLaunchKernelGGL((adjoint_batch<VS>), dim3(grid), dim3(kThreads), lds, s, B);
            return hipGetLastError();
        });
    const hipError_t r = scratch_release(s, lease);
    return e != hipSuccess ? e : r;
}

}  // namespace cbct
