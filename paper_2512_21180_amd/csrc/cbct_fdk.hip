// FDK reconstruction with offset-detector redundancy weights: the
// initialisation x <- FDK_w(y) of arXiv 2512.21180, Alg. 1 (and the classic
// baseline it is compared with).  Feldkamp-Davis-Kress for a circular orbit
// and a flat panel, in coordinates scaled to the isocentre (R = sid,
// D = sdd, u_i = u R / D, v_i = v R / D):
//   filter:       q = du_i * (p w(u) R / sqrt(R^2 + u_i^2 + v_i^2)) (*) h,
//                 h the Ram-Lak kernel at pitch du_i
//   backproject:  f(r) = (2 pi / n) sum_a R^2 / U^2 q(a, u(r), v(r)),
//                 U = R - (x cos + y sin), bilinear between pixel centres,
//                 zero off the panel.
// Redundancy weight: 1/2 for a centred panel; for a panel offset by off_u,
// sin^2(pi/4 (1 + s u / Delta)) over the overlap |u| <= Delta = W/2 - |off_u|
// (s = sign(off_u)) and 1 beyond it, so conjugate rays' weights add to one
// (Wang, Med. Phys. 2002).
//
// Optional Hann apodisation of the ramp (gain |omega| (1/2 + 1/2 cos(2 pi
// omega du_i)), the spatial kernel h/2 + (h(. - 1) + h(. + 1))/4).
//
// Filter: one workgroup per panel row of one projection; the weighted row
// is staged in LDS between two zero pads of nu + 1 words, so every output
// sums all odd offsets in one fixed order without bounds tests; the ramp
// output is formed at columns -1 .. nu and the Hann window applied to it.  Backprojection:
// one thread per voxel, angles in order, the sum in a register.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cbct_internal.h"
#include "cbct_nn.h"

namespace cbct {
namespace {

constexpr int kT = 256;
constexpr int kMaxNu = 4096;

struct FdkArgs {
    DevGeom g;
    float R, D, dui, delta, sgn;   // sgn = 0: centred panel (w = 1/2)
    float dbeta;
    int hann;                      // 1: Hann-apodised ramp
};

__device__ inline float red_weight(const FdkArgs &A, float u)
{
    if (A.sgn == 0.0f)
        return 0.5f;
    const float t = A.sgn * u;
    if (t > A.delta)
        return 1.0f;
    const float sw = sinf(0.7853981633974483f * (1.0f + fmaxf(t / A.delta, -1.0f)));
    return sw * sw;
}

__global__ void __launch_bounds__(kT) k_fdk_filter(FdkArgs A, const float *p, float *q)
{
    extern __shared__ float lds[];
    const DevGeom &g = A.g;
    const int nu = g.nu;
    const int P = nu + 1;              // zero pads of nu + 1 words on each side
    float *row = lds + P;
    float *coef = lds + 2 * P + nu;    // coef[m] = 1 / (pi^2 (2m+1)^2)
    float *qr = coef + (nu + 1) / 2;   // ramp output at columns -1 .. nu
    const int a = blockIdx.x / g.nv, iv = blockIdx.x % g.nv;
    const size_t base = ((size_t)a * g.nv + iv) * nu;
    const float vi = (g.off_v + ((float)iv - g.cv) * g.dv) * (A.R / A.D);
    for (int k = threadIdx.x; k < nu; k += kT) {
        const float u = g.off_u + ((float)k - g.cu) * g.du;
        const float ui = u * (A.R / A.D);
        const float cw = A.R * rsqrtf(fmaf(A.R, A.R, fmaf(ui, ui, vi * vi)));
        row[k] = p[base + k] * red_weight(A, u) * cw;
    }
    for (int k = threadIdx.x; k < P; k += kT) {
        lds[k] = 0.0f;
        lds[P + nu + k] = 0.0f;
    }
    for (int m = threadIdx.x; m < (nu + 1) / 2; m += kT) {
        const float n = (float)(2 * m + 1);
        coef[m] = 1.0f / (9.869604401089358f * n * n);
    }
    __syncthreads();
    const float scale = 1.0f / A.dui;  // du_i * h, h ~ 1 / du_i^2
    // Ram-Lak output at columns -1 .. nu (the zero-padded row's convolution)
    for (int j = threadIdx.x - 1; j <= nu; j += kT) {
        float acc = 0.0f;
        for (int m = 0; m < (nu + 1) / 2; ++m) {
            const int n = 2 * m + 1;
            acc = fmaf(coef[m], row[j - n] + row[j + n], acc);
        }
        qr[j + 1] = scale * fmaf(0.25f, row[j], -acc);
    }
    __syncthreads();
    // Hann window: the kernel h/2 + (h(. - 1) + h(. + 1))/4
    for (int j = threadIdx.x; j < nu; j += kT)
        q[base + j] = A.hann ? fmaf(0.5f, qr[j + 1], 0.25f * (qr[j] + qr[j + 2])) : qr[j + 1];
}

__global__ void __launch_bounds__(kT) k_fdk_backproject(FdkArgs A, const float *q, float *f)
{
    const DevGeom &g = A.g;
    const size_t nvox = (size_t)g.nx * g.ny * g.nz;
    const size_t s = (size_t)blockIdx.x * kT + threadIdx.x;
    if (s >= nvox)
        return;
    const int ix = (int)(s % g.nx), iy = (int)((s / g.nx) % g.ny);
    const int iz = (int)(s / ((size_t)g.nx * g.ny));
    const float x = g.ox + ((float)ix - 0.5f * (float)(g.nx - 1)) * g.vx;
    const float y = g.oy + ((float)iy - 0.5f * (float)(g.ny - 1)) * g.vy;
    const float z = g.oz + ((float)iz - 0.5f * (float)(g.nz - 1)) * g.vz;
    const float inv_du = 1.0f / g.du, inv_dv = 1.0f / g.dv;
    float acc = 0.0f;
    for (int a = 0; a < g.n_angles; ++a) {
        const AngRec ar = g.angs[a];
        const float U = A.R - fmaf(x, ar.c, y * ar.s);
        const float rU = 1.0f / U;
        const float fu = fmaf(fmaf(A.D * rU, fmaf(y, ar.c, -x * ar.s), -g.off_u), inv_du, g.cu);
        const float fv = fmaf(fmaf(A.D * rU, z, -g.off_v), inv_dv, g.cv);
        const float u0f = floorf(fu), v0f = floorf(fv);
        const int u0 = (int)u0f, v0 = (int)v0f;
        const float au = fu - u0f, av = fv - v0f;
        if (u0 < -1 || u0 >= g.nu || v0 < -1 || v0 >= g.nv)
            continue;
        const float *qa = q + (size_t)a * g.nv * g.nu;
        const bool uin0 = u0 >= 0, uin1 = u0 + 1 < g.nu;
        const bool vin0 = v0 >= 0, vin1 = v0 + 1 < g.nv;
        const float q00 = (uin0 && vin0) ? qa[(size_t)v0 * g.nu + u0] : 0.0f;
        const float q01 = (uin1 && vin0) ? qa[(size_t)v0 * g.nu + u0 + 1] : 0.0f;
        const float q10 = (uin0 && vin1) ? qa[(size_t)(v0 + 1) * g.nu + u0] : 0.0f;
        const float q11 = (uin1 && vin1) ? qa[(size_t)(v0 + 1) * g.nu + u0 + 1] : 0.0f;
        const float r0 = fmaf(au, q01 - q00, q00);
        const float r1 = fmaf(au, q11 - q10, q10);
        const float val = fmaf(av, r1 - r0, r0);
        const float wr = A.R * rU;
        acc = fmaf(wr * wr, val, acc);
    }
    f[s] = A.dbeta * acc;
}

}  // namespace
}  // namespace cbct

using namespace cbct;

extern "C" cbct_status cbct_fdk(const cbct_geom *g, const float *sino, int window, float *work,
                                float *vol, void *stream)
{
    if (!g || !sino || !work || !vol)
        return CBCT_E_NULL;
    if (window != 0 && window != 1)
        return CBCT_E_ARG;
    if (!g->dev_block)
        return CBCT_E_ARG;
    const cbct_geom_desc &d = g->desc;
    if (d.nu > kMaxNu)
        return CBCT_E_SHAPE;
    // a full orbit of equally spaced angles
    const int n = d.n_angles;
    for (int a = 0; a < n; ++a) {
        const double want = g->angles[0] + 2.0 * M_PI * a / n;
        if (std::fabs(g->angles[a] - want) > 1e-9)
            return CBCT_E_ARG;
    }
    FdkArgs A{};
    A.g = g->dev;
    A.R = (float)d.sid_mm;
    A.D = (float)d.sdd_mm;
    A.dui = (float)(d.du_mm * d.sid_mm / d.sdd_mm);
    A.delta = (float)(0.5 * d.nu * d.du_mm - std::fabs(d.off_u_mm));
    A.sgn = d.off_u_mm > 0 ? 1.0f : (d.off_u_mm < 0 ? -1.0f : 0.0f);
    if (A.sgn != 0.0f && !(A.delta > 0))
        return CBCT_E_GEOM;   // no overlap: no redundancy weighting possible
    A.dbeta = (float)(2.0 * M_PI / n);
    A.hann = window;
    hipStream_t s = (hipStream_t)stream;
    const size_t lds = (2 * ((size_t)d.nu + 1) + d.nu + (d.nu + 1) / 2 + d.nu + 2) * sizeof(float);
    hipLaunchKernelGGL(k_fdk_filter, dim3((unsigned)((size_t)n * d.nv)), dim3(kT), lds, s, A,
                       sino, work);
    const size_t nvox = (size_t)d.nx * d.ny * d.nz;
    hipLaunchKernelGGL(k_fdk_backproject, dim3((unsigned)((nvox + kT - 1) / kT)), dim3(kT), 0, s,
                       A, (const float *)work, vol);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_hip_error(e);
        return CBCT_E_HIP;
    }
    return CBCT_OK;
}
