/*
 * cbct_nn.h -- convolution kernels of libcbct.so for the learned primal-dual
 * blocks (arXiv 2512.21180, Alg. 1: the dual block Gamma and primal block
 * Lambda are stacks of 3x3x3 convolutions with LeakyReLU between them, their
 * outputs added to half of the dual or primal latent; the output block is a
 * 1x1x1 convolution).
 *
 * Activations inside a block are channel-last BF16 with exactly 16 channels:
 * an array of S = nz*ny*nx positions (x fastest) of 16 bf16 values (unused
 * channels are zero).  Latents and projector I/O stay channel-first FP32
 * ([C][nz][ny][nx]); pack and the convolution epilogues convert.
 *
 * Weights of a 3x3x3 layer: bf16 [27][16 cout][16 cin], tap index
 * t = (dz+1)*9 + (dy+1)*3 + (dx+1) for offsets dz, dy, dx in {-1, 0, 1};
 * zero padding outside the grid ("same" convolution).  Arithmetic: BF16
 * operands on the matrix cores (v_mfma_f32_16x16x32_bf16), FP32 accumulation.
 *
 * Every pointer is a device pointer owned by the caller except the host
 * arrays of channel pointers; calls enqueue on `stream` (hipStream_t, NULL =
 * null stream).  Results are deterministic (fixed reduction orders, no
 * atomics).
 */
#ifndef CBCT_NN_H
#define CBCT_NN_H

#include "cbct.h"

#ifdef __cplusplus
extern "C" {
#endif

/* out[s][c] = bf16(scale[c] * in[c][s]) for c < n_in, 0 for n_in <= c < 16.
 * in: host array of n_in device FP32 channel pointers (S elements each);
 * scale: host array of n_in factors, or NULL for 1. */
cbct_status cbct_pack16(size_t S, int n_in, const float *const *in, const float *scale,
                        uint16_t *out, void *stream);

/*
 * One 3x3x3 convolution over a (nz, ny, nx) grid: acc[s][co] = bias[co] +
 * sum_{t, ci} w[t][co][ci] x[s + offset(t)][ci].
 *   transpose_w = 1 uses w[26 - t][ci][co] instead (the transposed, flipped
 *   kernel: the data gradient of a convolution with w).
 *   act_mask (optional, channel-last bf16 [S][16]): acc[s][co] *= 1 where
 *   act_mask[s][co] > 0, else slope (the LeakyReLU derivative of the layer
 *   whose output act_mask is).
 *   act = 1 applies LeakyReLU(slope) to acc before the stores.
 * Stores (either or both):
 *   y_cl (channel-last bf16 [S][16]) <- acc;
 *   y_cf[co][s] (host array of n_cf device FP32 channel pointers, co < n_cf)
 *     <- acc (accumulate = 0) or += alpha * acc (accumulate = 1).
 * bias may be NULL (zero).
 */
cbct_status cbct_conv3(int nz, int ny, int nx, const uint16_t *x, const uint16_t *w,
                       int transpose_w, const float *bias, const uint16_t *act_mask, int act,
                       float slope, uint16_t *y_cl, int n_cf, float *const *y_cf, int accumulate,
                       float alpha, void *stream);

/* Workspace cells (FP32) cbct_conv3_wgrad needs for a grid of S positions. */
size_t cbct_conv3_wgrad_workspace(size_t S);

/*
 * Weight and bias gradients of a 3x3x3 convolution with input x and output
 * gradient dy (both channel-last bf16 [S][16]):
 *   dw[t][co][ci] = sum_s dy[s][co] x[s + offset(t)][ci],  db[co] = sum_s dy[s][co]
 * (FP32, overwritten; db may be NULL).  Blocked partial sums in a fixed order
 * in ws, then one ordered reduction.
 */
cbct_status cbct_conv3_wgrad(int nz, int ny, int nx, const uint16_t *x, const uint16_t *dy,
                             float *dw, float *db, float *ws, void *stream);

/*
 * 1x1x1 convolution of n_in channel-first FP32 channels (the output
 * convolution of Alg. 1): v[s] = w[n_in] + sum_c w[c] in[c][s], accumulated
 * in channel order with fused multiply-adds; out <- v (accumulate = 0) or
 * out += alpha * v (accumulate = 1).  in: host array of n_in device
 * pointers; w: device array of n_in + 1 floats (weights, then bias).
 * out may not alias an input.  0 <= n_in <= 16.
 */
cbct_status cbct_conv1(size_t S, int n_in, const float *const *in, const float *w, float *out,
                       int accumulate, float alpha, void *stream);

/*
 * Field-of-view tensor V of Alg. 1 (Sec. 2.6): for each voxel, the fraction
 * of the n_angles projections in which it is visible, i.e. in which the ray
 * from the source through the voxel centre meets the panel's sensitive area
 * |u - off_u| <= nu du / 2, |v - off_v| <= nv dv / 2 (u, v: panel coordinates
 * of that point, by central projection onto the panel plane).  Computed on
 * the host in FP64 (works on host-only handles); out is a host array of
 * nx ny nz floats, [nz][ny][nx].
 */
cbct_status cbct_fov_fraction(const cbct_geom *g, float *out);

/*
 * Resolution changes of the multiscale scheme (Alg. 1; r = 1/alpha in
 * {1, 2, 4}; all arrays [n0][n1][n2] FP32, device, n2 fastest; sizes are the
 * fine grid's and must be multiples of r; out may not alias in).
 *   cbct_pool:      out[i][j][k] = scale * sum_{a,b,c<r} in[r i+a][r j+b][r k+c]
 *                   (scale 1/r^3: Downsample, average pooling; scale 1: the
 *                   adjoint of nearest upsampling)
 *   cbct_projdown:  out[a][v][u] = scale * sum_{b,c<r} in[r a][r v+b][r u+c]
 *                   (scale 1/r^2: ProjDown, which keeps every r-th projection
 *                   and averages r x r pixel blocks)
 *   cbct_upsample:  out[i][j][k] (+)= scale * in[i/r][j/r][k/r] over the fine
 *                   grid (scale 1: nearest Upsample; scale 1/r^3: the adjoint
 *                   of average pooling); accumulate = 1 adds to out.
 */
cbct_status cbct_pool(int r, int n0, int n1, int n2, const float *in, float *out, float scale,
                      void *stream);
cbct_status cbct_projdown(int r, int n0, int n1, int n2, const float *in, float *out,
                          float scale, void *stream);
cbct_status cbct_upsample(int r, int n0, int n1, int n2, const float *in, float *out,
                          float scale, int accumulate, void *stream);

/*
 * FDK reconstruction, the initialisation x <- FDK_w(y) of Alg. 1:
 * Feldkamp-Davis-Kress for the circular orbit and flat panel of g, with the
 * offset-detector redundancy weight w (1/2 for a centred panel; for an
 * offset panel sin^2(pi/4 (1 + u/Delta)) over the overlap |u| <= Delta =
 * nu du / 2 - |off_u| and 1 beyond), cosine weighting, Ram-Lak filtering
 * along panel rows (window 0; window 1 applies the Hann window, kernel
 * h/2 + (h(. - 1) + h(. + 1))/4 on the zero-padded row; other values:
 * CBCT_E_ARG), and voxel-driven backprojection with the R^2/U^2 weight
 * and bilinear interpolation between pixel centres (zero off the panel).
 * sino: FP32 line integrals [n_angles][nv][nu]; work: FP32 device buffer of
 * the same size (receives the filtered projections); vol: FP32
 * [nz][ny][nx].  The angles must be a full orbit of equally spaced angles
 * (else CBCT_E_ARG); nu <= 4096 (else CBCT_E_SHAPE); an offset panel must
 * overlap the central ray (else CBCT_E_GEOM).  FP32 arithmetic.
 */
cbct_status cbct_fdk(const cbct_geom *g, const float *sino, int window, float *work,
                     float *vol, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CBCT_NN_H */
