/*
 * cbct_sim.h -- projection-data simulator kernels of libcbct.so: seeded
 * noise on line integrals computed by cbct_forward.
 *
 * Noise model (arXiv 2512.21180, Sec. 2.2, noisy primary projections as
 * Poisson counts of the attenuated beam; Sec. 2.4, negative log of the counts
 * over the air scan, clamped at one), monochromatic form:
 *   counts ~ Poisson(I0 exp(-p)),  y = -log(min(max(counts, 1) / I0, 1)).
 * An additive Gaussian variant y = p + sigma z serves small test cases.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11), counter-based, so
 * every element's draws depend only on (seed, stream id, element index, trial
 * index): element i, trial j uses counter (i mod 2^32, i div 2^32, j, stream)
 * and key (seed mod 2^32, seed div 2^32).  Uniforms take 53 bits from two
 * words; Poisson variates use CDF inversion below a mean of 10 and Hormann's
 * transformed rejection (PTRS, 1993) above, one counter block per trial, the
 * acceptance test in FP64; Box-Muller for the Gaussian.
 *
 * All arrays are device pointers of n elements owned by the caller; calls
 * enqueue on `stream` (hipStream_t, NULL = null stream).
 */
#ifndef CBCT_SIM_H
#define CBCT_SIM_H

#include "cbct.h"

#ifdef __cplusplus
extern "C" {
#endif

/* out[4 i + w] = word w of Philox4x32-10 at counter (i, 0, 0, stream id) for
 * i < n_blocks (for testing the generator). */
cbct_status cbct_philox_blocks(size_t n_blocks, uint64_t seed, uint32_t stream_id, uint32_t *out,
                               void *stream);

/* y = -log(min(max(counts, 1) / I0, 1)) with counts ~ Poisson(I0 exp(-p));
 * p and y are FP32 (they may alias); counts (optional, may be NULL) receives
 * the integer counts. */
cbct_status cbct_sim_poisson_log(size_t n, const float *p, float *y, int64_t *counts, double I0,
                                 uint64_t seed, uint32_t stream_id, void *stream);

/*
 * Polychromatic primary model (arXiv 2512.21180, Sec. 2.2, water-bone
 * decomposition and eq. primarymodel; Sec. 2.4, eq. normprimary).
 *
 * cbct_water_bone: water and bone relative densities of a CT volume given in
 * Hounsfield units (FP32 device arrays of n elements): with the modified CT
 * number r = 0.001 HU + 1 and tau_1 = 1.2, tau_2 = 1.6, kappa_b = 0.409,
 *   rho_w = r on [0, tau_1), tau_1 (tau_2 - r) / (tau_2 - tau_1) on
 *           [tau_1, tau_2), 0 elsewhere;
 *   rho_b = 0 below tau_1, kappa_b tau_2 (r - tau_1) / (tau_2 - tau_1) on
 *           [tau_1, tau_2), kappa_b r from tau_2 up.
 * (The paper leaves tau_0 unstated; tau_0 = 0 is the value that makes rho_w
 * continuous, as the paper says it is.)  Outputs may not alias the input.
 */
cbct_status cbct_water_bone(size_t n, const float *hu, float *rho_w, float *rho_b,
                            void *stream);

/*
 * The paper's energy bins and detector response: *n_bins = 10 bins
 * [10 i, 10 (i + 1)) keV, i = 2..11, centred at 25, 35, ..., 115 keV, and
 * resp at those centres, piecewise linear through (20 keV, 5), (60 keV, 20),
 * (120 keV, 10).  Host arrays of cap doubles (either may be NULL);
 * CBCT_E_SHAPE if cap < 10 and an array is given.  No device work.
 */
cbct_status cbct_poly_bins(int cap, double *centres_kev, double *resp, int *n_bins);

/*
 * Noisy polychromatic primary projections and their normalised negative log.
 * pw = P(rho_w), pb = P(rho_b): FP32 device arrays of n elements (sinogram
 * order [angle][v][u]; by linearity of P the line integral of the energy-e
 * attenuation mu_w[e] rho_w + mu_b[e] rho_b is mu_w[e] pw + mu_b[e] pb).
 * I0: FP32 device array [n_bins][npix], the unattenuated photon count per
 * detector pixel and bin (the paper's intensity maps I_0,e, the same for
 * every projection; element i sits at pixel i mod npix, n a multiple of
 * npix).  mu_w, mu_b (mm^-1 at unit density) and resp: host arrays of n_bins
 * doubles (1 <= n_bins <= 32), caller-supplied.  Per element, in FP64:
 *   c_e ~ Poisson(I0_e exp(-(mu_w[e] pw + mu_b[e] pb))),
 *   s = sum_e resp[e] c_e,   s_air = sum_e resp[e] I0_e   (noise-free air scan),
 *   y = -log(min(max(s, r_min) / s_air, 1))   (r_min: smallest positive resp),
 * y = 0 where s_air <= 0.  Outputs: y (FP32, required), signal s (FP32,
 * optional), counts (int64 [n_bins][n], optional).  Bin e's variate uses
 * trial counters from 256 e, so bin 0 draws exactly as cbct_sim_poisson_log
 * with the same seed and stream id, and one bin with mu_w = 1, mu_b = 0,
 * resp = 1 reproduces it bit for bit.  CBCT_E_SHAPE for n_bins outside
 * [1, 32] or n not a multiple of npix; CBCT_E_ARG for a negative response
 * or a NaN attenuation.
 */
cbct_status cbct_sim_poly(size_t n, size_t npix, const float *pw, const float *pb, int n_bins,
                          const double *mu_w, const double *mu_b, const double *resp,
                          const float *I0, uint64_t seed, uint32_t stream_id, float *y,
                          float *signal, int64_t *counts, void *stream);

/* out = clean + sigma z, z standard normal (FP32 arrays, may alias). */
cbct_status cbct_sim_gaussian(size_t n, const float *clean, float *out, double sigma,
                              uint64_t seed, uint32_t stream_id, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CBCT_SIM_H */
