/* Peak probes for the projector's on-chip limits (diagnostics).
 *
 * The projector pair of arXiv 2512.21180 (Sec. 2.2, P and P*) is bound on
 * MI355X by FP32 vector-ALU issue and LDS reads, not by HBM.  These calls
 * launch kernels that measure those two rates; the caller times them on the
 * same stream (e.g. with HIP events) and converts:
 *
 *   FMA lane-operations = n_blocks * cbct_probe_threads() * iters * 8
 *   LDS bytes read      = n_blocks * cbct_probe_threads() * iters * 64
 *
 * out: device buffer of n_blocks * cbct_probe_threads() floats, written once
 * per thread (keeps the work observable); caller-owned.  Launches are
 * asynchronous on `stream` (a hipStream_t, NULL for the default stream).
 * Returns CBCT_E_NULL for a NULL out, CBCT_E_SHAPE for n_blocks or iters
 * below 1, CBCT_E_HIP on a launch error.
 */
#ifndef CBCT_PROBE_H
#define CBCT_PROBE_H

#include "cbct.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Threads per probe workgroup (256). */
int cbct_probe_threads(void);

/* Eight independent dependent-FMA chains per thread, iters steps each. */
cbct_status cbct_probe_valu(int n_blocks, int iters, float *out, void *stream);

/* Four conflict-free 16-byte LDS reads per thread and step, iters steps. */
cbct_status cbct_probe_lds(int n_blocks, int iters, float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif
