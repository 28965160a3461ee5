// Projection-data simulator kernels (see cbct_sim.h): Philox4x32-10 counter
// based random numbers, Poisson counts of the attenuated beam and the
// negative-log normalisation (monochromatic, or polychromatic over energy
// bins with the water-bone decomposition), or additive Gaussian noise.  One thread per
// element; the Poisson rejection loop is bounded (64 trials).
#include <hip/hip_runtime.h>

#include "cbct_internal.h"
#include "cbct_sim.h"

namespace cbct {
namespace {

constexpr int kT = 256;

struct Words {
    uint32_t w[4];
};

// Philox4x32-10: ten rounds of (two 32x32 multiplications, xor with the other
// counter words and the key), key advanced by the Weyl increments in between.
__device__ inline Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                               uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words{{c0, c1, c2, c3}};
}

__device__ inline Words draw(uint64_t seed, uint32_t sid, uint64_t i, uint32_t j)
{
    return philox((uint32_t)i, (uint32_t)(i >> 32), j, sid, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ inline double unif53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// Poisson(lam): CDF inversion below 10, Hormann's PTRS from 10 up.  Trial j
// of the variate uses counter word 2 = trial0 + j.
__device__ int64_t poisson(double lam, uint64_t seed, uint32_t sid, uint64_t i,
                           uint32_t trial0 = 0)
{
    if (!(lam > 0.0))
        return 0;
    if (lam < 10.0) {
        const Words d = draw(seed, sid, i, trial0);
        const double u = unif53(d.w[0], d.w[1]);
        double p = exp(-lam), F = p;
        int64_t k = 0;
        while (u > F && k < 1000) {
            ++k;
            p *= lam / (double)k;
            F += p;
        }
        return k;
    }
    const double sl = sqrt(lam), ll = log(lam);
    const double b = 0.931 + 2.53 * sl;
    const double a = -0.059 + 0.02483 * b;
    const double log_inv_alpha = log(1.1239 + 1.1328 / (b - 3.4));
    const double v_r = 0.9277 - 3.6224 / (b - 2.0);
    for (uint32_t j = 0; j < 64; ++j) {
        const Words d = draw(seed, sid, i, trial0 + j);
        const double U = unif53(d.w[0], d.w[1]) - 0.5;
        const double V = unif53(d.w[2], d.w[3]);
        const double us = 0.5 - fabs(U);
        const double kf = floor((2.0 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && V <= v_r)
            return (int64_t)kf;
        if (kf < 0.0 || (us < 0.013 && V > us))
            continue;
        if (log(V) + log_inv_alpha - log(a / (us * us) + b) <= -lam + kf * ll - lgamma(kf + 1.0))
            return (int64_t)kf;
    }
    return (int64_t)floor(lam + 0.5);
}

__global__ void __launch_bounds__(kT) k_philox(size_t n, uint64_t seed, uint32_t sid, uint32_t *out)
{
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n)
        return;
    const Words d = philox((uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0, sid, (uint32_t)seed,
                           (uint32_t)(seed >> 32));
    uint4 v = make_uint4(d.w[0], d.w[1], d.w[2], d.w[3]);
    reinterpret_cast<uint4 *>(out)[i] = v;
}

__global__ void __launch_bounds__(kT) k_poisson_log(size_t n, const float *p, float *y, int64_t *cnt,
                                                    double I0, uint64_t seed, uint32_t sid)
{
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n)
        return;
    const int64_t c = poisson(I0 * exp(-(double)p[i]), seed, sid, i);
    if (cnt)
        cnt[i] = c;
    const double r = (double)(c < 1 ? 1 : c) / I0;
    y[i] = (float)(-log(r < 1.0 ? r : 1.0));
}

// Water-bone decomposition constants (Sec. 2.2); tau_0 = 0 makes rho_w
// continuous at tau_0.
constexpr float kTau0 = 0.0f, kTau1 = 1.2f, kTau2 = 1.6f, kKappaB = 0.409f;

__global__ void __launch_bounds__(kT) k_water_bone(size_t n, const float *hu, float *rw,
                                                   float *rb)
{
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n)
        return;
    const float r = fmaf(0.001f, hu[i], 1.0f);   // modified CT number
    float w = 0.0f, b = 0.0f;
    if (r >= kTau2) {
        b = kKappaB * r;
    } else if (r >= kTau1) {
        const float inv = 1.0f / (kTau2 - kTau1);
        w = kTau1 * (kTau2 - r) * inv;
        b = kKappaB * kTau2 * (r - kTau1) * inv;
    } else if (r >= kTau0) {
        w = r;
    }
    rw[i] = w;
    rb[i] = b;
}

constexpr int kMaxBins = 32;

struct PolyArgs {
    size_t n, npix;
    int nbins;
    double r_min;                  // smallest positive response (zero-signal floor)
    double mu_w[kMaxBins], mu_b[kMaxBins], resp[kMaxBins];
};

// Per element: one Poisson variate per energy bin of the attenuated beam
// (bin e's trials counted from 256 e), the response-weighted signal, and its
// negative log over the noise-free air signal, clamped at one.  The means and
// sums are FP64 in bin order (the Poisson acceptance test runs in FP64), so
// the counts equal those of an FP64 evaluation of the same model.
__global__ void __launch_bounds__(kT) k_sim_poly(PolyArgs A, const float *pw, const float *pb,
                                                 const float *I0, uint64_t seed, uint32_t sid,
                                                 float *y, float *signal, int64_t *counts)
{
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i >= A.n)
        return;
    const size_t pix = i % A.npix;
    const double w = (double)pw[i], b = (double)pb[i];
    double sig = 0.0, air = 0.0;
    for (int e = 0; e < A.nbins; ++e) {
        const double i0 = (double)I0[(size_t)e * A.npix + pix];
        double att;
        {
#pragma clang fp contract(off)
            att = A.mu_w[e] * w + A.mu_b[e] * b;   // the two products rounded, then summed
        }
        const int64_t c = poisson(i0 * exp(-att), seed, sid, i, 256u * (uint32_t)e);
        if (counts)
            counts[(size_t)e * A.n + i] = c;
        sig += A.resp[e] * (double)c;
        air += A.resp[e] * i0;
    }
    if (signal)
        signal[i] = (float)sig;
    if (!(air > 0.0)) {
        y[i] = 0.0f;
        return;
    }
    const double r = (sig < A.r_min ? A.r_min : sig) / air;
    y[i] = (float)(-log(r < 1.0 ? r : 1.0));
}

__global__ void __launch_bounds__(kT) k_gaussian(size_t n, const float *clean, float *out,
                                                 double sigma, uint64_t seed, uint32_t sid)
{
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n)
        return;
    const Words d = draw(seed, sid, i, 0);
    const double u1 = 1.0 - unif53(d.w[0], d.w[1]);
    const double u2 = unif53(d.w[2], d.w[3]);
    const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
    out[i] = (float)((double)clean[i] + sigma * z);
}

cbct_status sim_done(hipError_t e)
{
    if (e == hipSuccess)
        return CBCT_OK;
    set_hip_error(e);
    return CBCT_E_HIP;
}

dim3 grid_for(size_t n) { return dim3((unsigned)((n + kT - 1) / kT)); }

}  // namespace
}  // namespace cbct

using namespace cbct;

extern "C" cbct_status cbct_philox_blocks(size_t n_blocks, uint64_t seed, uint32_t stream_id,
                                          uint32_t *out, void *stream)
{
    if (!out)
        return CBCT_E_NULL;
    if (n_blocks == 0)
        return CBCT_OK;
    if (n_blocks / kT >= 0x7fffffffu)
        return CBCT_E_SHAPE;
    hipLaunchKernelGGL(k_philox, grid_for(n_blocks), dim3(kT), 0, (hipStream_t)stream, n_blocks,
                       seed, stream_id, out);
    return sim_done(hipGetLastError());
}

extern "C" cbct_status cbct_sim_poisson_log(size_t n, const float *p, float *y, int64_t *counts,
                                            double I0, uint64_t seed, uint32_t stream_id,
                                            void *stream)
{
    if (!p || !y)
        return CBCT_E_NULL;
    if (!(I0 > 0.0))
        return CBCT_E_ARG;
    if (n == 0)
        return CBCT_OK;
    if (n / kT >= 0x7fffffffu)
        return CBCT_E_SHAPE;
    hipLaunchKernelGGL(k_poisson_log, grid_for(n), dim3(kT), 0, (hipStream_t)stream, n, p, y,
                       counts, I0, seed, stream_id);
    return sim_done(hipGetLastError());
}

extern "C" cbct_status cbct_water_bone(size_t n, const float *hu, float *rho_w, float *rho_b,
                                       void *stream)
{
    if (!hu || !rho_w || !rho_b)
        return CBCT_E_NULL;
    if (n == 0)
        return CBCT_OK;
    if (n / kT >= 0x7fffffffu)
        return CBCT_E_SHAPE;
    hipLaunchKernelGGL(k_water_bone, grid_for(n), dim3(kT), 0, (hipStream_t)stream, n, hu, rho_w,
                       rho_b);
    return sim_done(hipGetLastError());
}

extern "C" cbct_status cbct_poly_bins(int cap, double *centres_kev, double *resp, int *n_bins)
{
    if (!n_bins)
        return CBCT_E_NULL;
    *n_bins = 10;
    if (cap < 10)
        return centres_kev || resp ? CBCT_E_SHAPE : CBCT_OK;
    for (int k = 0; k < 10; ++k) {
        // bins [10 i, 10 (i + 1)) keV for i = 2..11, centred
        const double e = 10.0 * (k + 2) + 5.0;
        // piecewise linear through (20, 5), (60, 20), (120, 10) keV
        double r;
        if (e <= 20.0)
            r = 5.0;
        else if (e <= 60.0)
            r = 5.0 + (e - 20.0) * (15.0 / 40.0);
        else if (e < 120.0)
            r = 20.0 - (e - 60.0) * (10.0 / 60.0);
        else
            r = 10.0;
        if (centres_kev)
            centres_kev[k] = e;
        if (resp)
            resp[k] = r;
    }
    return CBCT_OK;
}

extern "C" cbct_status cbct_sim_poly(size_t n, size_t npix, const float *pw, const float *pb,
                                     int n_bins, const double *mu_w, const double *mu_b,
                                     const double *resp, const float *I0, uint64_t seed,
                                     uint32_t stream_id, float *y, float *signal,
                                     int64_t *counts, void *stream)
{
    if (!pw || !pb || !mu_w || !mu_b || !resp || !I0 || !y)
        return CBCT_E_NULL;
    if (n_bins < 1 || n_bins > kMaxBins || npix == 0 || n % npix != 0)
        return CBCT_E_SHAPE;
    if (n == 0)
        return CBCT_OK;
    if (n / kT >= 0x7fffffffu)
        return CBCT_E_SHAPE;
    PolyArgs A{};
    A.n = n;
    A.npix = npix;
    A.nbins = n_bins;
    for (int e = 0; e < n_bins; ++e) {
        if (!(resp[e] >= 0.0) || !(mu_w[e] == mu_w[e]) || !(mu_b[e] == mu_b[e]))
            return CBCT_E_ARG;
        A.mu_w[e] = mu_w[e];
        A.mu_b[e] = mu_b[e];
        A.resp[e] = resp[e];
        if (resp[e] > 0.0 && (A.r_min == 0.0 || resp[e] < A.r_min))
            A.r_min = resp[e];
    }
    hipLaunchKernelGGL(k_sim_poly, grid_for(n), dim3(kT), 0, (hipStream_t)stream, A, pw, pb, I0,
                       seed, stream_id, y, signal, counts);
    return sim_done(hipGetLastError());
}

extern "C" cbct_status cbct_sim_gaussian(size_t n, const float *clean, float *out, double sigma,
                                         uint64_t seed, uint32_t stream_id, void *stream)
{
    if (!clean || !out)
        return CBCT_E_NULL;
    if (n == 0)
        return CBCT_OK;
    if (n / kT >= 0x7fffffffu)
        return CBCT_E_SHAPE;
    hipLaunchKernelGGL(k_gaussian, grid_for(n), dim3(kT), 0, (hipStream_t)stream, n, clean, out,
                       sigma, seed, stream_id);
    return sim_done(hipGetLastError());
}
