// Reference-shaped HIP kernels of libcbct.so (gfx950): one thread per ray for
// the forward projector A and one thread per voxel gathering over every
// angle for A^T (arXiv 2512.21180, Sec. 2.2: projection operator P and
// backprojection P*).  They serve geometries whose footprints exceed the
// LDS limits of the tiled kernels.
//
// Both kernels evaluate the same FP32 expressions for every weight:
//   q  = fma(p, ps, pb)                 in-plane fractional index on plane p
//   kb = fma(t0, Vz, Kb), ks = tau*Vz,  k = fma(p, ks, kb)
//   ds = dsf * sqrt(n2 + V*V)   (V*V tabulated per row)
// so A^T applies exactly the weights A applies; only the summation order
// differs.
#include <hip/hip_runtime.h>

#include "cbct_internal.h"
#include "cbct_storage.h"

namespace cbct {
namespace {

// ---- forward: one thread per ray -------------------------------------------

template <class VS, class SS>
__global__ void __launch_bounds__(256)
forward_simple(DevGeom g, const typename VS::T *__restrict__ vol, typename SS::T *__restrict__ sino)
{
    const int iu = blockIdx.x * blockDim.x + threadIdx.x;
    const int iv = blockIdx.y;
    const int a = blockIdx.z % g.n_angles;
    const int ch = blockIdx.z / g.n_angles;
    if (iu >= g.nu)
        return;
    const size_t nvox = (size_t)g.nx * g.ny * g.nz;
    const size_t nsino = (size_t)g.n_angles * g.nv * g.nu;
    const typename VS::T *v = vol + ch * nvox;

    const ColRec c = g.cols[(size_t)a * g.nu + iu];
    const float2 row = g.rows[iv];
    const AngRec ar = g.angs[a];
    const bool xm = iu >= ar.x_lo && iu < ar.x_hi;
    const float kb = fmaf(c.t0, row.x, g.Kb);
    const float ks = c.tau * row.x;
    const int nm = xm ? g.nx : g.ny;
    const int nq = xm ? g.ny : g.nx;
    // strides of (plane, in-plane) in the x-fastest volume
    const size_t sm = xm ? 1 : (size_t)g.nx;
    const size_t sq = xm ? (size_t)g.nx : 1;
    const size_t sk = (size_t)g.nx * g.ny;

    float acc = 0.0f;
    for (int p = 0; p < nm; ++p) {
        const float fp = (float)p;
        const float q = fmaf(fp, c.ps, c.pb);
        const float k = fmaf(fp, ks, kb);
        const float qf = floorf(q), kf = floorf(k);
        const int q0 = (int)qf, k0 = (int)kf;
        const float wq = q - qf, wk = k - kf;
        if (q0 < -1 || q0 >= nq || k0 < -1 || k0 >= g.nz)
            continue;
        const bool q0in = q0 >= 0, q1in = q0 + 1 < nq;
        const bool k0in = k0 >= 0, k1in = k0 + 1 < g.nz;
        const size_t base = (size_t)p * sm;
        float v00 = 0.f, v10 = 0.f, v01 = 0.f, v11 = 0.f;
        if (k0in) {
            const size_t bk = base + (size_t)k0 * sk;
            if (q0in) v00 = VS::ld(v, bk + (size_t)q0 * sq);
            if (q1in) v10 = VS::ld(v, bk + (size_t)(q0 + 1) * sq);
        }
        if (k1in) {
            const size_t bk = base + (size_t)(k0 + 1) * sk;
            if (q0in) v01 = VS::ld(v, bk + (size_t)q0 * sq);
            if (q1in) v11 = VS::ld(v, bk + (size_t)(q0 + 1) * sq);
        }
        const float lo = fmaf(wq, v10 - v00, v00);
        const float hi = fmaf(wq, v11 - v01, v01);
        acc += fmaf(wk, hi - lo, lo);
    }
    const float ds = ray_ds(c.dsf, c.n2, row.y);
    SS::st(sino, ch * nsino + ((size_t)a * g.nv + iv) * g.nu + iu, acc * ds);
}

// ---- adjoint: one thread per voxel, gather over every angle -----------------

__device__ inline float panel_u(const DevGeom &g, float c, float s, float x, float y)
{
    // fractional column where the ray from the source through (x, y, .) meets the panel
    const float den = fmaf(c, x, fmaf(s, y, -g.sid));
    const float num = -g.sdd * fmaf(-s, x, c * y);
    return (num / den - g.off_u) / g.du + g.cu;
}

// Gather the contributions of the columns [u_lo, u_hi] of angle a whose rays
// sample this voxel on plane p (in-plane index qi).
template <class SS>
__device__ inline float gather_columns(const DevGeom &g, int a, int u_lo, int u_hi, int p, int qi,
                                       int k, const typename SS::T *__restrict__ y)
{
    float acc = 0.0f;
    const float fp = (float)p;
    for (int u = u_lo; u <= u_hi; ++u) {
        const ColRec c = g.cols[(size_t)a * g.nu + u];
        const float q = fmaf(fp, c.ps, c.pb);
        const float wq = 1.0f - fabsf(q - (float)qi);
        if (!(wq > 0.0f))
            continue;
        // rows whose z index on this plane is within one voxel of k
        const float t = fmaf(fp, c.tau, c.t0);
        const float za = ((float)k - 1.0f - g.Kb) / t, zb = ((float)k + 1.0f - g.Kb) / t;
        const float va = (za - g.rv0) / g.rvs + g.cv, vb = (zb - g.rv0) / g.rvs + g.cv;
        int v_lo = (int)floorf(fminf(va, vb)) - 1, v_hi = (int)ceilf(fmaxf(va, vb)) + 1;
        v_lo = max(v_lo, 0);
        v_hi = min(v_hi, g.nv - 1);
        float col = 0.0f;
        for (int v = v_lo; v <= v_hi; ++v) {
            const float2 row = g.rows[v];
            const float kb = fmaf(c.t0, row.x, g.Kb);
            const float ks = c.tau * row.x;
            const float kk = fmaf(fp, ks, kb);
            const float wk = 1.0f - fabsf(kk - (float)k);
            if (!(wk > 0.0f))
                continue;
            const float ds = ray_ds(c.dsf, c.n2, row.y);
            col = fmaf(ds * wk, SS::ld(y, ((size_t)a * g.nv + v) * g.nu + u), col);
        }
        acc = fmaf(wq, col, acc);
    }
    return acc;
}

template <class SS, class VS>
__global__ void __launch_bounds__(256)
adjoint_simple(DevGeom g, const typename SS::T *__restrict__ sino, typename VS::T *__restrict__ vol)
{
    const size_t nvox = (size_t)g.nx * g.ny * g.nz;
    const size_t nsino = (size_t)g.n_angles * g.nv * g.nu;
    const size_t vid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ch = blockIdx.y;
    if (vid >= nvox)
        return;
    const int i = (int)(vid % g.nx);
    const int j = (int)((vid / g.nx) % g.ny);
    const int k = (int)(vid / ((size_t)g.nx * g.ny));
    const float cx = g.ox + ((float)i - 0.5f * (float)(g.nx - 1)) * g.vx;
    const float cy = g.oy + ((float)j - 0.5f * (float)(g.ny - 1)) * g.vy;
    const typename SS::T *ys = sino + ch * nsino;

    float acc = 0.0f;
    for (int a = 0; a < g.n_angles; ++a) {
        const AngRec ar = g.angs[a];
        float part = 0.0f;
        if (ar.x_lo < ar.x_hi) {     // columns sampled on x planes: plane i, in-plane j
            const float u1 = panel_u(g, ar.c, ar.s, cx, cy - g.vy);
            const float u2 = panel_u(g, ar.c, ar.s, cx, cy + g.vy);
            const int lo = max((int)floorf(fminf(u1, u2)) - 1, ar.x_lo);
            const int hi = min((int)ceilf(fmaxf(u1, u2)) + 1, ar.x_hi - 1);
            if (lo <= hi)
                part += gather_columns<SS>(g, a, lo, hi, i, j, k, ys);
        }
        if (ar.x_lo > 0 || ar.x_hi < g.nu) {   // columns sampled on y planes: plane j, in-plane i
            const float u1 = panel_u(g, ar.c, ar.s, cx - g.vx, cy);
            const float u2 = panel_u(g, ar.c, ar.s, cx + g.vx, cy);
            int lo = max((int)floorf(fminf(u1, u2)) - 1, 0);
            int hi = min((int)ceilf(fmaxf(u1, u2)) + 1, g.nu - 1);
            // y-sampled columns are [0, x_lo) and [x_hi, nu)
            if (ar.x_lo < ar.x_hi) {
                const int a_hi = min(hi, ar.x_lo - 1);
                if (lo <= a_hi)
                    part += gather_columns<SS>(g, a, lo, a_hi, j, i, k, ys);
                lo = max(lo, ar.x_hi);
            }
            if (lo <= hi)
                part += gather_columns<SS>(g, a, lo, hi, j, i, k, ys);
        }
        acc += part;
    }
    VS::st(vol, ch * nvox + vid, acc);
}

}  // namespace

hipError_t launch_forward_simple(const DevGeom &g, const void *vol, cbct_dtype vt, void *sino,
                                 cbct_dtype st, int channels, hipStream_t s)
{
    dim3 block(256);
    dim3 grid((g.nu + 255) / 256, g.nv, g.n_angles * channels);
    // every storage pair the tiled kernels accept (dispatch_storage)
    return dispatch_storage(vt, st, [&](auto vs, auto ss) -> hipError_t {
        using VS = decltype(vs);
        using SS = decltype(ss);
        hipLaunchKernelGGL((forward_simple<VS, SS>), grid, block, 0, s, g,
                           (const typename VS::T *)vol, (typename SS::T *)sino);
        return hipGetLastError();
    });
}

hipError_t launch_adjoint_simple(const DevGeom &g, const void *sino, cbct_dtype st, void *vol,
                                 cbct_dtype vt, int channels, hipStream_t s)
{
    const size_t nvox = (size_t)g.nx * g.ny * g.nz;
    dim3 block(256);
    dim3 grid((unsigned)((nvox + 255) / 256), channels);
    return dispatch_storage(vt, st, [&](auto vs, auto ss) -> hipError_t {
        using VS = decltype(vs);
        using SS = decltype(ss);
        hipLaunchKernelGGL((adjoint_simple<SS, VS>), grid, block, 0, s, g,
                           (const typename SS::T *)sino, (typename VS::T *)vol);
        return hipGetLastError();
    });
}

}  // namespace cbct
