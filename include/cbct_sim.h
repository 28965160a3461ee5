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

/* out = clean + sigma z, z standard normal (FP32 arrays, may alias). */
cbct_status cbct_sim_gaussian(size_t n, const float *clean, float *out, double sigma,
                              uint64_t seed, uint32_t stream_id, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CBCT_SIM_H */
