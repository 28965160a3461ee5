// Resolution changes of the multiscale learned primal-dual scheme
// (arXiv 2512.21180, Alg. 1: Downsample by average pooling, ProjDown that
// also keeps every r-th projection, nearest Upsample of the latents and of
// the output convolution).  Streaming kernels, one thread per output
// element; the r^3 (or r^2) inputs of an output are summed in a fixed order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cbct_internal.h"
#include "cbct_nn.h"

namespace cbct {
namespace {

constexpr int kT = 256;

// out[z][y][x] = scale * sum_{a,b,c < r} in[r z + a][r y + b][r x + c]
__global__ void __launch_bounds__(kT) k_pool(int r, int oz, int oy, int ox, const float *in,
                                             float *out, float scale)
{
    const size_t n = (size_t)oz * oy * ox;
    const size_t s = (size_t)blockIdx.x * kT + threadIdx.x;
    if (s >= n)
        return;
    const int x = (int)(s % ox), y = (int)((s / ox) % oy), z = (int)(s / ((size_t)ox * oy));
    const size_t iy_n = (size_t)oy * r, ix_n = (size_t)ox * r;
    float acc = 0.0f;
    for (int a = 0; a < r; ++a)
        for (int b = 0; b < r; ++b) {
            const float *row = in + (((size_t)z * r + a) * iy_n + (size_t)y * r + b) * ix_n +
                               (size_t)x * r;
            for (int c = 0; c < r; ++c)
                acc += row[c];
        }
    out[s] = scale * acc;
}

// out[a][v][u] = scale * sum_{b,c < r} in[r a][r v + b][r u + c]
__global__ void __launch_bounds__(kT) k_projdown(int r, int oa, int ov, int ou, const float *in,
                                                 float *out, float scale)
{
    const size_t n = (size_t)oa * ov * ou;
    const size_t s = (size_t)blockIdx.x * kT + threadIdx.x;
    if (s >= n)
        return;
    const int u = (int)(s % ou), v = (int)((s / ou) % ov), a = (int)(s / ((size_t)ou * ov));
    const size_t iv_n = (size_t)ov * r, iu_n = (size_t)ou * r;
    float acc = 0.0f;
    for (int b = 0; b < r; ++b) {
        const float *row = in + (((size_t)a * r) * iv_n + (size_t)v * r + b) * iu_n + (size_t)u * r;
        for (int c = 0; c < r; ++c)
            acc += row[c];
    }
    out[s] = scale * acc;
}

// out[z][y][x] = scale * in[z / r][y / r][x / r]  (+ out, when accumulating)
__global__ void __launch_bounds__(kT) k_upsample(int r, int nz, int ny, int nx, const float *in,
                                                 float *out, float scale, int accumulate)
{
    const size_t n = (size_t)nz * ny * nx;
    const size_t s = (size_t)blockIdx.x * kT + threadIdx.x;
    if (s >= n)
        return;
    const int x = (int)(s % nx), y = (int)((s / nx) % ny), z = (int)(s / ((size_t)nx * ny));
    const int cy = ny / r, cx = nx / r;
    const float v = scale * in[((size_t)(z / r) * cy + y / r) * cx + x / r];
    out[s] = accumulate ? out[s] + v : v;
}

bool dims_ok(int r, int nz, int ny, int nx)
{
    return (r == 1 || r == 2 || r == 4) && nz > 0 && ny > 0 && nx > 0 && nz % r == 0 &&
           ny % r == 0 && nx % r == 0 && (int64_t)nz * ny * nx < (int64_t(1) << 31);
}

cbct_status finish(hipError_t e)
{
    if (e == hipSuccess)
        return CBCT_OK;
    set_hip_error(e);
    return CBCT_E_HIP;
}

unsigned blocks(size_t n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace
}  // namespace cbct

using namespace cbct;

extern "C" cbct_status cbct_pool(int r, int nz, int ny, int nx, const float *in, float *out,
                                 float scale, void *stream)
{
    if (!in || !out)
        return CBCT_E_NULL;
    if (!dims_ok(r, nz, ny, nx))
        return CBCT_E_SHAPE;
    const int oz = nz / r, oy = ny / r, ox = nx / r;
    hipLaunchKernelGGL(k_pool, dim3(blocks((size_t)oz * oy * ox)), dim3(kT), 0,
                       (hipStream_t)stream, r, oz, oy, ox, in, out, scale);
    return finish(hipGetLastError());
}

extern "C" cbct_status cbct_projdown(int r, int na, int nv, int nu, const float *in, float *out,
                                     float scale, void *stream)
{
    if (!in || !out)
        return CBCT_E_NULL;
    if (!dims_ok(r, na, nv, nu))
        return CBCT_E_SHAPE;
    const int oa = na / r, ov = nv / r, ou = nu / r;
    hipLaunchKernelGGL(k_projdown, dim3(blocks((size_t)oa * ov * ou)), dim3(kT), 0,
                       (hipStream_t)stream, r, oa, ov, ou, in, out, scale);
    return finish(hipGetLastError());
}

extern "C" cbct_status cbct_upsample(int r, int nz, int ny, int nx, const float *in, float *out,
                                     float scale, int accumulate, void *stream)
{
    if (!in || !out)
        return CBCT_E_NULL;
    if (!dims_ok(r, nz, ny, nx))
        return CBCT_E_SHAPE;
    hipLaunchKernelGGL(k_upsample, dim3(blocks((size_t)nz * ny * nx)), dim3(kT), 0,
                       (hipStream_t)stream, r, nz, ny, nx, in, out, scale, accumulate ? 1 : 0);
    return finish(hipGetLastError());
}
