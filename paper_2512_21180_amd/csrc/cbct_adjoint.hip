// Adjoint A^T for gfx950: atomic-free gather over LDS-staged panel windows.
//
// Operator: the transpose of the plane-sampled cone-beam projector
// (arXiv 2512.21180, Sec. 2.2, backprojection P* as the adjoint of P).  The
// weight of voxel (i,j,k) in ray (a,u,v) is
//   ds(u,v) * hat(q_u(p) - q_vox) * hat(k(u,v,p) - k),   hat(s) = max(0, 1-|s|),
// where p is the voxel's index along the ray's sampling axis and q_vox its
// in-plane index; these are the weights the forward kernel applies.
//
// A workgroup owns a brick of 8 x 8 x 16 voxels; lane l of wave w owns the
// voxel column (i0 + l%8, j0 + l/8) and the four voxels k0 + 4w .. k0 + 4w + 3,
// and keeps their sums in registers over all angles (fixed order: angles,
// then columns, then rows), so every voxel is written once and no atomics
// are needed.  For each angle the brick's panel window is staged in LDS,
// pre-multiplied by the ray length per plane ds, together with the column
// constants.  Per voxel and column, the rows with non-zero weight form a run
// that starts below the row where the ray crosses z = k - 1 and holds at
// most NT rows; the taps use the clamped hat, so rows past the run add zero.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cbct_internal.h"
#include "cbct_storage.h"

namespace cbct {
namespace {

constexpr int kThreads = 256;
constexpr int kBI = 8, kBJ = 8, kBK = 16, kV = 4;

struct BrickArgs {
    DevGeom g;
    int W, H, WS, NTmax;
    int nbx, nby, nbz;
};

__device__ inline float sat(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }

// Fractional panel column of the ray through (x, y, .) and its source-panel
// scale lambda (a point at height z lands at V = lambda z).
__device__ inline void project_xy(const DevGeom &g, float c, float s, float x, float y,
                                  float &u, float &lam)
{
    const float den = fmaf(c, x, fmaf(s, y, -g.sid));
    lam = -g.sdd / den;
    u = (lam * fmaf(-s, x, c * y) - g.off_u) / g.du + g.cu;
}

// Gather one brick (index b) of one channel: y is that channel's sinogram,
// vol that channel's volume.  `lds` holds the panel window and column table.
template <class SS, class VS>
__device__ void gather_brick(const BrickArgs &A, int b, const typename SS::T *__restrict__ y,
                             typename VS::T *__restrict__ vol, float *lds)
{
    const DevGeom &g = A.g;
    float *yt = lds;                                    // [H][WS] ds-weighted panel window
    float4 *cr = (float4 *)(lds + (size_t)A.H * A.WS);  // [W] (pb, ps, t0, tau)

    const int bx = b % A.nbx, by = (b / A.nbx) % A.nby, bz = b / (A.nbx * A.nby);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i = bx * kBI + (lane & 7), j = by * kBJ + (lane >> 3);
    const int k0 = bz * kBK + w * kV;
    const int ic = min(i, g.nx - 1), jc = min(j, g.ny - 1);
    const float cxv = g.ox + ((float)ic - 0.5f * (float)(g.nx - 1)) * g.vx;
    const float cyv = g.oy + ((float)jc - 0.5f * (float)(g.ny - 1)) * g.vy;

    // brick support box (voxel centres +- one pitch), uniform
    const int i0 = bx * kBI, i1 = min(i0 + kBI, g.nx) - 1;
    const int j0 = by * kBJ, j1 = min(j0 + kBJ, g.ny) - 1;
    const int kz0 = bz * kBK, kz1 = min(kz0 + kBK, g.nz) - 1;
    const float xs0 = g.ox + ((float)i0 - 0.5f * (float)(g.nx - 1)) * g.vx - g.vx;
    const float xs1 = g.ox + ((float)i1 - 0.5f * (float)(g.nx - 1)) * g.vx + g.vx;
    const float ys0 = g.oy + ((float)j0 - 0.5f * (float)(g.ny - 1)) * g.vy - g.vy;
    const float ys1 = g.oy + ((float)j1 - 0.5f * (float)(g.ny - 1)) * g.vy + g.vy;
    const float zs0 = g.oz + ((float)kz0 - 0.5f * (float)(g.nz - 1)) * g.vz - g.vz;
    const float zs1 = g.oz + ((float)kz1 - 0.5f * (float)(g.nz - 1)) * g.vz + g.vz;

    const float inv_rvs = 1.0f / g.rvs;
    float acc[kV] = {0.0f, 0.0f, 0.0f, 0.0f};

    __syncthreads();   // the previous work item's readers of lds are done
    for (int a = 0; a < g.n_angles; ++a) {
        const AngRec ar = g.angs[a];
        // ---- panel window of the brick (uniform)
        float umin = 1e30f, umax = -1e30f, vmin = 1e30f, vmax = -1e30f, tmin = 1e30f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float x = (q & 1) ? xs1 : xs0, yy = (q & 2) ? ys1 : ys0;
            float u, lam;
            project_xy(g, ar.c, ar.s, x, yy, u, lam);
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
            const float va = (lam * zs0 - g.off_v) / g.dv + g.cv;
            const float vb = (lam * zs1 - g.off_v) / g.dv + g.cv;
            vmin = fminf(vmin, fminf(va, vb));
            vmax = fmaxf(vmax, fmaxf(va, vb));
            tmin = fminf(tmin, (g.sid - fmaf(ar.c, x, ar.s * yy)) / g.sdd);
        }
        const int U0 = max((int)floorf(umin) - 1, 0);
        const int U1 = min(min((int)ceilf(umax) + 1, g.nu - 1), U0 + A.W - 1);
        int NT = (int)floorf(2.0f / (tmin * g.rvs)) + 3;
        NT = __builtin_amdgcn_readfirstlane(min(NT, A.NTmax));
        const int V0 = max((int)floorf(vmin) - 2, 0);
        const int V1 = min(min((int)ceilf(vmax) + 2, g.nv - 1), V0 + A.H - NT - 1);
        if (U0 > U1 || V0 > V1)
            continue;
        const int Wc = U1 - U0 + 1;
        const int Hs = V1 - V0 + 1 + NT;   // staged rows (rows past V1 are zero)

        __syncthreads();   // previous angle's readers are done
        for (int uu = lane; uu < Wc; uu += 64) {
            const ColRec col = g.cols[(size_t)a * g.nu + U0 + uu];
            if (w == 0)
                cr[uu] = make_float4(col.pb, col.ps, col.t0, col.tau);
            for (int vv = w; vv < Hs; vv += 4) {
                const int v = V0 + vv;
                float val = 0.0f;
                if (v <= V1) {
                    const float ds = col.dsf * sqrtf(col.n2 + g.rows[v].y);
                    val = SS::ld(y, ((size_t)a * g.nv + v) * g.nu + U0 + uu) * ds;
                }
                yt[vv * A.WS + uu] = val;
            }
        }
        __syncthreads();

        // ---- gather, once per sampling axis present at this angle
#pragma unroll
        for (int cls = 0; cls < 2; ++cls) {
            int c_lo, c_hi;   // this axis' columns, intersected below
            float fp, qv;
            float u1, u2, lam;
            if (cls == 0) {   // x planes: plane i, in-plane j
                if (ar.x_lo >= ar.x_hi)
                    continue;
                c_lo = ar.x_lo;
                c_hi = ar.x_hi - 1;
                fp = (float)ic;
                qv = (float)jc;
                project_xy(g, ar.c, ar.s, cxv, cyv - g.vy, u1, lam);
                project_xy(g, ar.c, ar.s, cxv, cyv + g.vy, u2, lam);
            } else {          // y planes: plane j, in-plane i
                if (ar.x_lo == 0 && ar.x_hi == g.nu)
                    continue;
                c_lo = 0;
                c_hi = g.nu - 1;
                fp = (float)jc;
                qv = (float)ic;
                project_xy(g, ar.c, ar.s, cxv - g.vx, cyv, u1, lam);
                project_xy(g, ar.c, ar.s, cxv + g.vx, cyv, u2, lam);
            }
            int ul = max(max((int)floorf(fminf(u1, u2)), c_lo), U0);
            int uh = min(min((int)ceilf(fmaxf(u1, u2)), c_hi), U1);
            for (int u = ul; u <= uh; ++u) {
                if (cls == 1 && u >= ar.x_lo && u < ar.x_hi)
                    continue;   // those columns are sampled on x planes
                const float4 C = cr[u - U0];
                const float q = fmaf(fp, C.y, C.x);
                const float wq = sat(1.0f - fabsf(q - qv));
                const float t = fmaf(fp, C.w, C.z);
                const float beta = t * g.rvs;
                const float rt = __builtin_amdgcn_rcpf(t);
                const int colo = u - U0;
#pragma unroll
                for (int n = 0; n < kV; ++n) {
                    const float kk = (float)(k0 + n);
                    // row where the ray crosses z index kk - 1, minus one for rounding
                    const float vf = fmaf(fmaf(kk - 1.0f - g.Kb, rt, -g.rv0), inv_rvs, g.cv);
                    const int vs = min(max((int)floorf(vf) - 1, V0), V1);
                    const float vz = fmaf((float)vs - g.cv, g.rvs, g.rv0);
                    float s = fmaf(t, vz, g.Kb - kk);
                    const float *py = yt + (vs - V0) * A.WS + colo;
                    float csum = 0.0f;
                    for (int m = 0; m < NT; ++m) {
                        csum = fmaf(sat(1.0f - fabsf(s)), py[m * A.WS], csum);
                        s += beta;
                    }
                    acc[n] = fmaf(wq, csum, acc[n]);
                }
            }
        }
    }

    if (i < g.nx && j < g.ny) {
#pragma unroll
        for (int n = 0; n < kV; ++n) {
            const int k = k0 + n;
            if (k < g.nz)
                VS::st(vol, ((size_t)k * g.ny + j) * g.nx + i, acc[n]);
        }
    }
}

template <class SS, class VS>
__global__ void __launch_bounds__(kThreads)
adjoint_brick(BrickArgs A, const typename SS::T *__restrict__ sino,
              typename VS::T *__restrict__ vol)
{
    extern __shared__ float lds[];
    const int ch = blockIdx.y;
    const size_t nvox = (size_t)A.g.nx * A.g.ny * A.g.nz;
    const size_t nsino = (size_t)A.g.n_angles * A.g.nv * A.g.nu;
    gather_brick<SS, VS>(A, blockIdx.x, sino + ch * nsino, vol + ch * nvox, lds);
}

// ---- batched adjoint: one persistent launch over (case, brick) items -------

struct AdjCase {
    BrickArgs A;
    const void *sino;
    void *vol;
};

struct BatchAdjArgs {
    int n_cases, n_items;
    int first[kMaxBatch + 1];
    AdjCase c[kMaxBatch];
};

template <class SS, class VS>
__global__ void __launch_bounds__(kThreads)
adjoint_batch(BatchAdjArgs B)
{
    extern __shared__ float lds[];
    for (int item = blockIdx.x; item < B.n_items; item += gridDim.x) {
        int cs = 0;
        while (cs + 1 < B.n_cases && item >= B.first[cs + 1])
            ++cs;
        const AdjCase &C = B.c[cs];
        gather_brick<SS, VS>(C.A, item - B.first[cs], (const typename SS::T *)C.sino,
                             (typename VS::T *)C.vol, lds);
    }
}

}  // namespace

static BrickArgs brick_args(const DevGeom &g, const AdjPlan &p)
{
    return BrickArgs{g, p.W, p.H, p.WS, p.NTmax, (g.nx + kBI - 1) / kBI, (g.ny + kBJ - 1) / kBJ,
                     (g.nz + kBK - 1) / kBK};
}

static size_t brick_lds(const AdjPlan &p)
{
    return ((size_t)p.H * p.WS + (size_t)p.W * 4) * sizeof(float);
}

hipError_t launch_adjoint_brick(const DevGeom &g, const AdjPlan &p, const void *sino,
                                cbct_dtype st, void *vol, cbct_dtype vt, int channels,
                                hipStream_t s)
{
    BrickArgs A = brick_args(g, p);
    dim3 grid(A.nbx * A.nby * A.nbz, channels), block(kThreads);
    return dispatch_storage(vt, st, [&](auto vs, auto ss) -> hipError_t {
        using VS = decltype(vs);
        using SS = decltype(ss);
        hipLaunchKernelGGL((adjoint_brick<SS, VS>), grid, block, brick_lds(p), s, A,
                           (const typename SS::T *)sino, (typename VS::T *)vol);
        return hipGetLastError();
    });
}

hipError_t launch_adjoint_batch(int n, const cbct_geom *const *gs, const void *const *sinos,
                                void *const *vols, cbct_dtype st, cbct_dtype vt, hipStream_t s)
{
    BatchAdjArgs B{};
    B.n_cases = n;
    size_t lds = 0;
    int items = 0;
    for (int i = 0; i < n; ++i) {
        const cbct_geom *g = gs[i];
        B.first[i] = items;
        B.c[i] = AdjCase{brick_args(g->dev, g->adj), sinos[i], vols[i]};
        items += B.c[i].A.nbx * B.c[i].A.nby * B.c[i].A.nbz;
        lds = std::max(lds, brick_lds(g->adj));
    }
    B.first[n] = items;
    B.n_items = items;
    const int grid = std::min(items, 256 * 4);
    return dispatch_storage(vt, st, [&](auto vs, auto ss) -> hipError_t {
        using VS = decltype(vs);
        using SS = decltype(ss);
        hipLaunchKernelGGL((adjoint_batch<SS, VS>), dim3(grid), dim3(kThreads), lds, s, B);
        return hipGetLastError();
    });
}

}  // namespace cbct
