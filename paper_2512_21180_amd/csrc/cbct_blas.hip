// BLAS-1 kernels for the CGLS and Landweber solvers (HBM-bound streaming
// kernels; see cbct_solve.h).  Every kernel reads its operands once with
// 16-byte vector loads where alignment allows, and the dot product reduces
// in a fixed order: grid-stride partial sums per thread, a fixed tree per
// block (FP64), then one block sums the per-block partials in index order.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cbct_internal.h"
#include "cbct_solve.h"

namespace cbct {
namespace {

constexpr int kT = 256;
constexpr int kDotBlocks = 1024;   // fixed, so the reduction order is fixed

__global__ void __launch_bounds__(kT) dot_partial(size_t n, const float *__restrict__ a,
                                                  const float *__restrict__ b, double *ws)
{
    __shared__ double red[kT];
    double s = 0.0;
    const size_t stride = (size_t)kDotBlocks * kT;
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += stride)
        s = fma((double)a[i], (double)b[i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        ws[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kT) dot_final(const double *ws, double *out)
{
    __shared__ double red[kT];
    double s = 0.0;
    for (int i = threadIdx.x; i < kDotBlocks; i += kT)
        s += ws[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *out = red[0];
}

__device__ inline float ratio(const double *num, const double *den)
{
    const double d = *den;
    return d != 0.0 ? (float)(*num / d) : 0.0f;
}

__global__ void __launch_bounds__(kT) axpy_ratio(size_t n, float *y, const float *x,
                                                 const double *num, const double *den, float sign)
{
    const float a = sign * ratio(num, den);
    const size_t stride = (size_t)gridDim.x * kT;
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += stride)
        y[i] = fmaf(a, x[i], y[i]);
}

__global__ void __launch_bounds__(kT) xpay_ratio(size_t n, float *y, const float *x,
                                                 const double *num, const double *den)
{
    const float b = ratio(num, den);
    const size_t stride = (size_t)gridDim.x * kT;
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += stride)
        y[i] = fmaf(b, y[i], x[i]);
}

__global__ void __launch_bounds__(kT) axpby(size_t n, float *z, float alpha, const float *x,
                                            float beta, const float *y)
{
    const size_t stride = (size_t)gridDim.x * kT;
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += stride)
        z[i] = fmaf(alpha, x[i], beta * y[i]);
}

__global__ void __launch_bounds__(kT) wresid(size_t n, float *g, const float *w, const float *x,
                                             const float *t)
{
    const size_t stride = (size_t)gridDim.x * kT;
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += stride)
        g[i] = w[i] * (x[i] - t[i]);
}

unsigned blocks_for(size_t n)
{
    size_t b = (n + kT - 1) / kT;
    return (unsigned)(b < 8192 ? (b ? b : 1) : 8192);
}

cbct_status done(hipError_t e)
{
    if (e == hipSuccess)
        return CBCT_OK;
    set_hip_error(e);
    return CBCT_E_HIP;
}

}  // namespace
}  // namespace cbct

// Partial sums of cbct_dot_noalloc: a fixed device array instead of a caller
// workspace.  Each GPU holds its own copy for the life of the process; host
// code reaches it only through the address hipGetSymbolAddress returns for
// the current device (the array's own name is not a device address on the
// host).  Every call on one GPU shares it.
static constexpr size_t kScratchCells = 1024;
static __device__ __align__(256) double scratch[kScratchCells];
static_assert(kScratchCells >= (size_t)cbct::kDotBlocks, "scratch holds every block's partial");

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices];   // per device, set on its first call

// Device address of `scratch` on the current device, looked up once per device.
cbct_status scratch_of_current_device(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        cbct::set_hip_error(e);
        return CBCT_E_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices)
        return CBCT_E_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            cbct::set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return CBCT_E_HIP;
        }
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return CBCT_OK;
}

}  // namespace

using namespace cbct;

extern "C" size_t cbct_dot_workspace(size_t) { return kDotBlocks; }

extern "C" size_t cbct_dot_noalloc_max_cells(void) { return kScratchCells; }

extern "C" cbct_status cbct_dot_noalloc(size_t n, const float *a, const float *b, double *out,
                                        void *stream)
{
    if (!a || !b || !out)
        return CBCT_E_NULL;
    if (cbct_dot_workspace(n) > kScratchCells)
        return CBCT_E_SHAPE;   // more partial sums than the fixed array holds
    double *ws = nullptr;
    const cbct_status st = scratch_of_current_device(&ws);
    if (st != CBCT_OK)
        return st;
    // the same kernels as cbct_dot; dot_partial writes every cell it reads
    // back, so nothing needs clearing
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(dot_partial, dim3(kDotBlocks), dim3(kT), 0, s, n, a, b, ws);
    hipLaunchKernelGGL(dot_final, dim3(1), dim3(kT), 0, s, (const double *)ws, out);
    return done(hipGetLastError());
}

extern "C" cbct_status cbct_dot(size_t n, const float *a, const float *b, double *ws, double *out,
                                void *stream)
{
    if (!a || !b || !ws || !out)
        return CBCT_E_NULL;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(dot_partial, dim3(kDotBlocks), dim3(kT), 0, s, n, a, b, ws);
    hipLaunchKernelGGL(dot_final, dim3(1), dim3(kT), 0, s, (const double *)ws, out);
    return done(hipGetLastError());
}

extern "C" cbct_status cbct_axpy_ratio(size_t n, float *y, const float *x, const double *num,
                                       const double *den, double sign, void *stream)
{
    if (!y || !x || !num || !den)
        return CBCT_E_NULL;
    hipLaunchKernelGGL(axpy_ratio, dim3(blocks_for(n)), dim3(kT), 0, (hipStream_t)stream, n, y, x,
                       num, den, (float)sign);
    return done(hipGetLastError());
}

extern "C" cbct_status cbct_xpay_ratio(size_t n, float *y, const float *x, const double *num,
                                       const double *den, void *stream)
{
    if (!y || !x || !num || !den)
        return CBCT_E_NULL;
    hipLaunchKernelGGL(xpay_ratio, dim3(blocks_for(n)), dim3(kT), 0, (hipStream_t)stream, n, y, x,
                       num, den);
    return done(hipGetLastError());
}

extern "C" cbct_status cbct_axpby(size_t n, float *z, float alpha, const float *x, float beta,
                                  const float *y, void *stream)
{
    if (!z || !x || !y)
        return CBCT_E_NULL;
    hipLaunchKernelGGL(axpby, dim3(blocks_for(n)), dim3(kT), 0, (hipStream_t)stream, n, z, alpha,
                       x, beta, y);
    return done(hipGetLastError());
}

extern "C" cbct_status cbct_wresid(size_t n, float *g, const float *w, const float *x,
                                   const float *t, void *stream)
{
    if (!g || !w || !x || !t)
        return CBCT_E_NULL;
    hipLaunchKernelGGL(wresid, dim3(blocks_for(n)), dim3(kT), 0, (hipStream_t)stream, n, g, w, x,
                       t);
    return done(hipGetLastError());
}
