// Quasi-Monte Carlo scatter simulator (arXiv 2512.21180, Sec. 2.3: the
// scatter signal as an integral over photon paths, split into path sampling,
// Alg. 2, and integration toward every detector element, Alg. 3; appendix:
// Beer-Lambert escape probability, the travel-distance measure and its
// inverse-transform sampling, the interaction choices and the Compton
// energy).  See cbct_scatter.h for the readings of the paper this follows.
//
// Paths: one thread per source photon, FP32.  Each leg marches the ray
// through the voxel grid twice (Amanatides-Woo traversal of the voxel cubes):
// once for the optical depth to the volume's exit, which gives the escape
// probability p0 and the weight factor 1 - p0, and once to the depth
// -log(1 - (1 - p0) u), which gives the interaction point.
// Integration: a workgroup holds 64 pixels and 16 record phases, one phase
// per wave (every lane of a wave reads the same record, so its loads are
// uniform); per record a march from the interaction point to the pixel
// centre gives the two material line integrals, from which the escape
// probabilities at the incoming and the Compton energy follow by linearity.
// Each pixel's 16 phase sums are added in phase order: deterministic.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cbct_internal.h"
#include "cbct_scatter.h"

namespace cbct {
namespace {

constexpr int kT = 256;
constexpr float kMeC2 = 510.99895f;   // electron rest energy, keV

struct Xs {
    int K, J, I;
    float e0, inv_de;
    const float *mu;     // [2][3][K]
    const float *icdf;   // [2][2][K][J]
    const float *dens;   // [2][2][K][I]
};

struct Grid {
    int nx, ny, nz;
    float vx, vy, vz;
    float lox, loy, loz;     // lower corner of the volume
    const float *rw, *rb;    // relative densities [nz][ny][nx]
};

__device__ inline void e_pos(const Xs &x, float e, int &k, float &f)
{
    float t = fminf(fmaxf((e - x.e0) * x.inv_de, 0.0f), (float)(x.K - 1));
    k = min((int)floorf(t), x.K - 2);
    f = t - (float)k;
}

__device__ inline float mu_kind(const Xs &x, int m, int kind, int k, float f)
{
    const float *t = x.mu + (m * 3 + kind) * x.K;
    return fmaf(f, t[k + 1] - t[k], t[k]);
}

__device__ inline float mu_tot(const Xs &x, int m, int k, float f)
{
    return mu_kind(x, m, 0, k, f) + mu_kind(x, m, 1, k, f) + mu_kind(x, m, 2, k, f);
}

// bilinear on a [K][n] table at energy (k, f) and abscissa s in [0, n - 1]
__device__ inline float table2(const float *tab, int n, int k, float f, float s)
{
    s = fminf(fmaxf(s, 0.0f), (float)(n - 1));
    const int j = min((int)floorf(s), n - 2);
    const float g = s - (float)j;
    const float *r0 = tab + k * n, *r1 = r0 + n;
    const float a = fmaf(g, r0[j + 1] - r0[j], r0[j]);
    const float b = fmaf(g, r1[j + 1] - r1[j], r1[j]);
    return fmaf(f, b - a, a);
}

__device__ inline float resp(float e)
{
    if (e <= 20.0f)
        return 5.0f;
    if (e <= 60.0f)
        return 5.0f + (e - 20.0f) * (15.0f / 40.0f);
    if (e < 120.0f)
        return 20.0f - (e - 60.0f) * (10.0f / 60.0f);
    return 10.0f;
}

__device__ inline long voxel_at(const Grid &G, float x, float y, float z)
{
    const float fx = (x - G.lox) / G.vx, fy = (y - G.loy) / G.vy, fz = (z - G.loz) / G.vz;
    if (!(fx >= 0.0f && fx < (float)G.nx && fy >= 0.0f && fy < (float)G.ny && fz >= 0.0f &&
          fz < (float)G.nz))
        return -1;
    const int i = min((int)fx, G.nx - 1), j = min((int)fy, G.ny - 1), k = min((int)fz, G.nz - 1);
    return ((long)k * G.ny + j) * G.nx + i;
}

// Walk the voxel cubes along p + t d (|d| = 1) from t = 0 to tmax, calling
// visit(len, voxel) per segment; visit returns false to stop.  Returns the
// parameter where the walk ended (the volume's exit, tmax, or where visit
// stopped it: the end of that segment).
template <class F>
__device__ inline float walk(const Grid &G, const float p[3], const float d[3], float tmax,
                             F &&visit)
{
    const int n[3] = {G.nx, G.ny, G.nz};
    const float v[3] = {G.vx, G.vy, G.vz}, lo[3] = {G.lox, G.loy, G.loz};
    float t0 = 0.0f, t1 = tmax;
    for (int q = 0; q < 3; ++q) {
        const float hi = lo[q] + (float)n[q] * v[q];
        if (d[q] == 0.0f) {
            if (!(p[q] > lo[q] && p[q] < hi))
                return 0.0f;
            continue;
        }
        const float inv = 1.0f / d[q];
        float ta = (lo[q] - p[q]) * inv, tb = (hi - p[q]) * inv;
        t0 = fmaxf(t0, fminf(ta, tb));
        t1 = fminf(t1, fmaxf(ta, tb));
    }
    if (!(t1 > t0))
        return 0.0f;
    // march from the entry point: the crossing parameters are then small
    // numbers measured from it (a source a metre away would otherwise round
    // every crossing to its 1e-4 mm units of the last place)
    const float pe[3] = {fmaf(t0, d[0], p[0]), fmaf(t0, d[1], p[1]), fmaf(t0, d[2], p[2])};
    const float te = t1 - t0;
    int idx[3], step[3];
    float tnext[3], tdelta[3];
    // the first voxel is the one holding a point just past the start (a
    // ten-thousandth of a voxel along the ray): a start on a voxel face or
    // on the volume's boundary then counts the voxel the ray goes into
    const float tm = fminf(1e-4f * fminf(v[0], fminf(v[1], v[2])), 0.5f * te);
    for (int q = 0; q < 3; ++q) {
        const float x = fmaf(tm, d[q], pe[q]);
        idx[q] = min(max((int)floorf((x - lo[q]) / v[q]), 0), n[q] - 1);
        if (d[q] > 0.0f) {
            step[q] = 1;
            tdelta[q] = v[q] / d[q];
            tnext[q] = (lo[q] + (float)(idx[q] + 1) * v[q] - pe[q]) / d[q];
        } else if (d[q] < 0.0f) {
            step[q] = -1;
            tdelta[q] = -v[q] / d[q];
            tnext[q] = (lo[q] + (float)idx[q] * v[q] - pe[q]) / d[q];
        } else {
            step[q] = 0;
            tdelta[q] = 0.0f;
            tnext[q] = INFINITY;
        }
    }
    float t = 0.0f;   // from the entry point
    while (t < te) {
        const int q = tnext[0] <= tnext[1] ? (tnext[0] <= tnext[2] ? 0 : 2)
                                           : (tnext[1] <= tnext[2] ? 1 : 2);
        const float tn = fminf(tnext[q], te);
        const long vi = ((long)idx[2] * G.ny + idx[1]) * G.nx + idx[0];
        if (tn > t && !visit(tn - t, vi, t0 + t))
            return t0 + tn;
        t = tn;
        idx[q] += step[q];
        tnext[q] += tdelta[q];
        if (idx[q] < 0 || idx[q] >= n[q])
            break;
    }
    return t1;
}

__device__ inline void normalise(float v[3])
{
    const float r = rsqrtf(fmaf(v[0], v[0], fmaf(v[1], v[1], v[2] * v[2])));
    v[0] *= r;
    v[1] *= r;
    v[2] *= r;
}

struct PathArgs {
    Grid G;
    Xs X;
    float sx, sy, c, s;      // source position (z = 0) and rotation of the angle
    long N;
    int n;                   // scatters per photon (records: n + 1)
    const float *src;        // [N][4]
    const float *qmc;        // [N][5 n + 1]
    float *rec;              // [N][n + 1][8]
};

__global__ void __launch_bounds__(kT) k_scatter_paths(PathArgs A)
{
    const long i = (long)blockIdx.x * kT + threadIdx.x;
    if (i >= A.N)
        return;
    const Grid &G = A.G;
    const Xs &X = A.X;
    const float *sp = A.src + 4 * i;
    const float *u = A.qmc + (size_t)i * (5 * A.n + 1);
    float x[3] = {A.sx, A.sy, 0.0f};
    float v[3] = {A.c * sp[0] - A.s * sp[1], A.s * sp[0] + A.c * sp[1], sp[2]};
    normalise(v);
    float e = sp[3], w = 1.0f;
    for (int o = 0; o <= A.n; ++o) {
        int k;
        float f;
        e_pos(X, e, k, f);
        const float mw = mu_tot(X, 0, k, f), mb = mu_tot(X, 1, k, f);
        // optical depth to the exit
        float tau = 0.0f;
        walk(G, x, v, 1e7f, [&](float len, long vi, float) {
            tau = fmaf(len, fmaf(G.rw[vi], mw, G.rb[vi] * mb), tau);
            return true;
        });
        // 1 - p0 and the target depth without cancellation where little
        // matter is crossed
        const float q0 = tau > 0.0f ? -expm1f(-tau) : 0.0f;   // 1 - p0
        float l = 0.0f;
        if (tau > 0.0f) {
            const float target = -log1pf(-q0 * u[5 * o]);
            float acc = 0.0f;
            walk(G, x, v, 1e7f, [&](float len, long vi, float t) {
                const float mu = fmaf(G.rw[vi], mw, G.rb[vi] * mb);
                if (mu > 0.0f && fmaf(len, mu, acc) >= target) {
                    l = t + (target - acc) / mu;
                    return false;
                }
                acc = fmaf(len, mu, acc);
                l = t + len;
                return true;
            });
        }
        w *= q0;
        for (int q = 0; q < 3; ++q)
            x[q] = fmaf(l, v[q], x[q]);
        float *r = A.rec + ((size_t)i * (A.n + 1) + o) * 8;
        r[0] = x[0];
        r[1] = x[1];
        r[2] = x[2];
        r[3] = v[0];
        r[4] = v[1];
        r[5] = v[2];
        r[6] = e;
        r[7] = w;
        if (o == A.n)
            break;
        const int kq = 1 + 5 * o;
        const long vi = voxel_at(G, x[0], x[1], x[2]);
        const float aw = vi >= 0 ? G.rw[vi] * mw : 0.0f, ab = vi >= 0 ? G.rb[vi] * mb : 0.0f;
        const float fw = (aw + ab) > 0.0f ? aw / (aw + ab) : 1.0f;
        const int m = u[kq] < fw ? 0 : 1;
        const float mc = mu_kind(X, m, 1, k, f), mr = mu_kind(X, m, 2, k, f);
        const int T = u[kq + 1] < mc / (mc + mr) ? 0 : 1;
        w *= 1.0f - mu_kind(X, m, 0, k, f) / (m == 0 ? mw : mb);
        const float cth = table2(X.icdf + (m * 2 + T) * X.K * X.J, X.J, k, f,
                                 u[kq + 2] * (float)(X.J - 1));
        const float phi = 6.283185307179586f * u[kq + 3];
        // frame around v: a = v x z normalised (v x x when |v_z| >= 0.9), b = v x a
        float a3[3];
        if (fabsf(v[2]) < 0.9f) {
            a3[0] = v[1];
            a3[1] = -v[0];
            a3[2] = 0.0f;
        } else {
            a3[0] = 0.0f;
            a3[1] = v[2];
            a3[2] = -v[1];
        }
        normalise(a3);
        const float b3[3] = {v[1] * a3[2] - v[2] * a3[1], v[2] * a3[0] - v[0] * a3[2],
                             v[0] * a3[1] - v[1] * a3[0]};
        const float sth = sqrtf(fmaxf(0.0f, 1.0f - cth * cth));
        float sn, cs;
        sincosf(phi, &sn, &cs);
        float vn[3];
        for (int q = 0; q < 3; ++q)
            vn[q] = fmaf(cth, v[q], sth * fmaf(cs, a3[q], sn * b3[q]));
        normalise(vn);
        v[0] = vn[0];
        v[1] = vn[1];
        v[2] = vn[2];
        if (T == 0)
            e = e / (1.0f + e * (1.0f - cth) / kMeC2);
    }
}

struct IntArgs {
    Grid G;
    Xs X;
    int nu, nv;
    float Dx, Dy, Dz;        // panel centre
    float eux, euy;          // e_u (z = 0); e_v = z
    float du, dv, cu, cv;
    float nx_, ny_;          // panel normal (z = 0)
    long nrec;
    const float *rec;        // [nrec][8]
    float *out;              // [nv][nu]
};

// One workgroup: 64 pixels x 16 record phases, one phase per wave (wave p
// takes records p, p + 16, ...; all its lanes read the same record); the
// sixteen partial sums of a pixel are added in phase order.
constexpr int kPixTile = 64, kPhases = 16;

__global__ void __launch_bounds__(kPixTile * kPhases) k_scatter_integrate(IntArgs A)
{
    __shared__ float part[kPhases][kPixTile];
    const int lane = threadIdx.x % kPixTile;
    const int ph = __builtin_amdgcn_readfirstlane(threadIdx.x / kPixTile);
    const int pix = blockIdx.x * kPixTile + lane;
    const bool live = pix < A.nu * A.nv;
    const Grid &G = A.G;
    const Xs &X = A.X;
    const int pc = live ? pix : 0;
    const int iu = pc % A.nu, iv = pc / A.nu;
    const float pu = ((float)iu - A.cu) * A.du, pv = ((float)iv - A.cv) * A.dv;
    const float P[3] = {fmaf(pu, A.eux, A.Dx), fmaf(pu, A.euy, A.Dy), A.Dz + pv};
    float acc = 0.0f;
    for (long r = ph; r < A.nrec; r += kPhases) {
        const float *q = A.rec + 8 * r;
        const float w = q[7];
        if (!(w > 0.0f) || !live)
            continue;
        const float x[3] = {q[0], q[1], q[2]};
        const float e = q[6];
        float vs[3] = {P[0] - x[0], P[1] - x[1], P[2] - x[2]};
        const float r2 = fmaf(vs[0], vs[0], fmaf(vs[1], vs[1], vs[2] * vs[2]));
        const float dist = sqrtf(r2);
        const float id = 1.0f / dist;
        vs[0] *= id;
        vs[1] *= id;
        vs[2] *= id;
        const float cth = fmaf(q[3], vs[0], fmaf(q[4], vs[1], q[5] * vs[2]));
        const float ec = e / (1.0f + e * (1.0f - cth) / kMeC2);
        float Pw = 0.0f, Pb = 0.0f;
        walk(G, x, vs, dist, [&](float len, long vi, float) {
            Pw = fmaf(len, G.rw[vi], Pw);
            Pb = fmaf(len, G.rb[vi], Pb);
            return true;
        });
        int k, kc;
        float f, fc;
        e_pos(X, e, k, f);
        e_pos(X, ec, kc, fc);
        const float mw = mu_tot(X, 0, k, f), mb = mu_tot(X, 1, k, f);
        const long vi = voxel_at(G, x[0], x[1], x[2]);
        const float aw = vi >= 0 ? G.rw[vi] * mw : 0.0f, ab = vi >= 0 ? G.rb[vi] * mb : 0.0f;
        const float tot = aw + ab;
        const float fm[2] = {tot > 0.0f ? aw / tot : 1.0f, tot > 0.0f ? ab / tot : 0.0f};
        const float sd = (cth + 1.0f) * 0.5f * (float)(X.I - 1);
        float sc = 0.0f, sr = 0.0f;
        for (int m = 0; m < 2; ++m) {
            const float mt = m == 0 ? mw : mb;
            sc = fmaf(fm[m] * mu_kind(X, m, 1, k, f) / mt,
                      table2(X.dens + (m * 2 + 0) * X.K * X.I, X.I, k, f, sd), sc);
            sr = fmaf(fm[m] * mu_kind(X, m, 2, k, f) / mt,
                      table2(X.dens + (m * 2 + 1) * X.K * X.I, X.I, k, f, sd), sr);
        }
        const float p0c = expf(-fmaf(mu_tot(X, 0, kc, fc), Pw, mu_tot(X, 1, kc, fc) * Pb));
        const float p0r = expf(-fmaf(mw, Pw, mb * Pb));
        const float s = fmaf(sc * p0c, resp(ec), sr * p0r * resp(e));
        const float cn = fabsf(fmaf(A.nx_, vs[0], A.ny_ * vs[1]));
        acc = fmaf(s * w * cn, A.du * A.dv / r2, acc);
    }
    part[ph][lane] = acc;
    __syncthreads();
    if (ph == 0 && live) {
        float v = part[0][lane];
        for (int k = 1; k < kPhases; ++k)
            v += part[k][lane];
        A.out[pix] = v;
    }
}

cbct_status scat_done(hipError_t e)
{
    if (e == hipSuccess)
        return CBCT_OK;
    set_hip_error(e);
    return CBCT_E_HIP;
}

bool xs_ok(const cbct_xs *x)
{
    return x && x->mu && x->icdf && x->dens && x->K >= 2 && x->J >= 2 && x->I >= 2 &&
           x->de > 0.0;
}

Grid grid_of(const cbct_geom *g, const float *rho)
{
    const cbct_geom_desc &d = g->desc;
    Grid G;
    G.nx = d.nx;
    G.ny = d.ny;
    G.nz = d.nz;
    G.vx = (float)d.vx_mm;
    G.vy = (float)d.vy_mm;
    G.vz = (float)d.vz_mm;
    G.lox = (float)(d.origin_mm[0] - 0.5 * d.nx * d.vx_mm);
    G.loy = (float)(d.origin_mm[1] - 0.5 * d.ny * d.vy_mm);
    G.loz = (float)(d.origin_mm[2] - 0.5 * d.nz * d.vz_mm);
    G.rw = rho;
    G.rb = rho + (size_t)d.nx * d.ny * d.nz;
    return G;
}

Xs xs_of(const cbct_xs *x)
{
    return Xs{x->K, x->J, x->I, (float)x->e0, (float)(1.0 / x->de), x->mu, x->icdf, x->dens};
}

}  // namespace
}  // namespace cbct

using namespace cbct;

extern "C" cbct_status cbct_scatter_paths(const cbct_geom *g, const float *rho, const cbct_xs *xs,
                                          int angle, int64_t n_photons, const float *src,
                                          const float *qmc, int n_scatter, float *rec,
                                          void *stream)
{
    if (!g || !rho || !src || !qmc || !rec)
        return CBCT_E_NULL;
    if (!xs_ok(xs))
        return CBCT_E_ARG;
    if (!g->dev_block)
        return CBCT_E_ARG;
    if (angle < 0 || angle >= g->desc.n_angles || n_photons < 0 || n_scatter < 0 ||
        n_scatter > 16 || n_photons / kT >= 0x7fffffff)
        return CBCT_E_SHAPE;
    if (n_photons == 0)
        return CBCT_OK;
    const double th = g->angles[angle];
    PathArgs A;
    A.G = grid_of(g, rho);
    A.X = xs_of(xs);
    A.c = (float)std::cos(th);
    A.s = (float)std::sin(th);
    A.sx = (float)(g->desc.sid_mm * std::cos(th));
    A.sy = (float)(g->desc.sid_mm * std::sin(th));
    A.N = n_photons;
    A.n = n_scatter;
    A.src = src;
    A.qmc = qmc;
    A.rec = rec;
    hipLaunchKernelGGL(k_scatter_paths, dim3((unsigned)((n_photons + kT - 1) / kT)), dim3(kT), 0,
                       (hipStream_t)stream, A);
    return scat_done(hipGetLastError());
}

extern "C" cbct_status cbct_scatter_integrate(const cbct_geom *g, const float *rho,
                                              const cbct_xs *xs, int angle, int64_t n_rec,
                                              const float *rec, float *out, void *stream)
{
    if (!g || !rho || !rec || !out)
        return CBCT_E_NULL;
    if (!xs_ok(xs))
        return CBCT_E_ARG;
    if (!g->dev_block)
        return CBCT_E_ARG;
    const cbct_geom_desc &d = g->desc;
    if (angle < 0 || angle >= d.n_angles || n_rec < 0 || (int64_t)d.nu * d.nv >= 0x7fffffff)
        return CBCT_E_SHAPE;
    const double th = g->angles[angle], c = std::cos(th), s = std::sin(th);
    IntArgs A;
    A.G = grid_of(g, rho);
    A.X = xs_of(xs);
    A.nu = d.nu;
    A.nv = d.nv;
    A.Dx = (float)(-(d.sdd_mm - d.sid_mm) * c - d.off_u_mm * s);
    A.Dy = (float)(-(d.sdd_mm - d.sid_mm) * s + d.off_u_mm * c);
    A.Dz = (float)d.off_v_mm;
    A.eux = (float)-s;
    A.euy = (float)c;
    A.du = (float)d.du_mm;
    A.dv = (float)d.dv_mm;
    A.cu = 0.5f * (float)(d.nu - 1);
    A.cv = 0.5f * (float)(d.nv - 1);
    A.nx_ = (float)c;
    A.ny_ = (float)s;
    A.nrec = n_rec;
    A.rec = rec;
    A.out = out;
    const int npix = d.nu * d.nv;
    hipLaunchKernelGGL(k_scatter_integrate, dim3((unsigned)((npix + kPixTile - 1) / kPixTile)),
                       dim3(kPixTile * kPhases), 0, (hipStream_t)stream, A);
    return scat_done(hipGetLastError());
}
