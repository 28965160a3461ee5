/*
 * cbct_solve.h -- BLAS-1 kernels of libcbct.so for the least-squares solvers
 * that use the projector pair: CGLS and Landweber iteration (the Landweber
 * gradient term P*(P x - y) is the data-consistency term of arXiv 2512.21180,
 * Alg. 1; CGLS is the conjugate-gradient method on the same normal
 * equations).
 *
 * All vectors are device FP32 arrays of n elements owned by the caller.
 * Scalars that the solvers update every iteration stay on the device (FP64
 * cells), so an iteration needs no host synchronisation.  Reductions are
 * deterministic: fixed per-block partial sums in FP64, then one ordered final
 * sum; the result does not depend on timing.
 *
 * Calls enqueue on `stream` (a hipStream_t; NULL = null stream) and return a
 * cbct_status (see cbct.h).
 */
#ifndef CBCT_SOLVE_H
#define CBCT_SOLVE_H

#include "cbct.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of FP64 workspace cells cbct_dot needs for n elements. */
size_t cbct_dot_workspace(size_t n);

/* *out = sum_i a[i] * b[i], accumulated in FP64.  ws: device FP64 array of
 * cbct_dot_workspace(n) cells; out: one device FP64 cell. */
cbct_status cbct_dot(size_t n, const float *a, const float *b, double *ws, double *out,
                     void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight solver loops, harnesses that forbid hipMalloc): the same
 * dot product as cbct_dot, bitwise equal to it, with its per-block partial
 * sums in a fixed device array of cbct_dot_noalloc_max_cells() FP64 cells
 * (8 KiB) that the library holds on each GPU until the process ends.  No
 * allocation happens in this call; the array's device address is looked up
 * on the first call on each device.  Every call on one GPU shares the
 * array: calls that overlap on one GPU (different streams, or host threads
 * without ordering) race and give undefined results; calls ordered on one
 * stream are safe.  Returns CBCT_E_SHAPE if n would need more partial sums
 * than the array holds (never, for the current fixed block count),
 * CBCT_E_NULL for a NULL pointer, CBCT_E_HIP if the array cannot be found
 * on the current device.  out: one device FP64 cell.
 */
size_t cbct_dot_noalloc_max_cells(void);
cbct_status cbct_dot_noalloc(size_t n, const float *a, const float *b, double *out,
                             void *stream);

/* y[i] += sign * (*num / *den) * x[i], with the ratio of two device FP64
 * cells evaluated on the device (a zero denominator gives a zero step). */
cbct_status cbct_axpy_ratio(size_t n, float *y, const float *x, const double *num,
                            const double *den, double sign, void *stream);

/* y[i] = x[i] + (*num / *den) * y[i] (zero denominator: y = x). */
cbct_status cbct_xpay_ratio(size_t n, float *y, const float *x, const double *num,
                            const double *den, void *stream);

/* z[i] = alpha * x[i] + beta * y[i] (host scalars); z may alias x or y. */
cbct_status cbct_axpby(size_t n, float *z, float alpha, const float *x, float beta,
                       const float *y, void *stream);

/* g[i] = w[i] * (x[i] - t[i]): the gradient of the weighted squared error
 * 0.5 sum_i w[i] (x[i] - t[i])^2 (the training loss of the learned
 * primal-dual net, weights = field-of-view mask / its size). */
cbct_status cbct_wresid(size_t n, float *g, const float *w, const float *x, const float *t,
                        void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CBCT_SOLVE_H */
