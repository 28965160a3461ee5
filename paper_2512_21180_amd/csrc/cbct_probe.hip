// Peak probes of the projector's two on-chip limits on gfx950: vector FP32
// FMA issue and LDS read bandwidth.  The projector kernels are bound by VALU
// issue and on-chip gathers, not by HBM (Sec. 2.2's operators move each
// volume and sinogram element once from HBM); these kernels measure what the
// chip delivers for those two, for comparison with the projector's counts.
#include <hip/hip_runtime.h>

#include "cbct_internal.h"

namespace cbct {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kChains = 8;   // independent FMA chains per thread

// kChains dependent FMA chains per thread, `iters` steps each: every step is
// one 4-byte v_fmac_f32 per chain, a += m k with m and k kernel arguments (so
// no literal constants; packed FP32 is disabled for every unit).
__global__ void __launch_bounds__(kProbeThreads) k_valu_probe(int iters, float m, float k,
                                                              float *out)
{
    float a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        a[c] = (float)(threadIdx.x + c);
    const float kv = __builtin_amdgcn_readfirstlane(0) + k;   // k in a vector register
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c)
            a[c] = fmaf(m, kv, a[c]);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        s += a[c];
    out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// Every thread reads four 16-byte LDS words per step (the whole 16 KB
// buffer per workgroup, lanes on consecutive words: no bank conflicts),
// `iters` steps; a compiler barrier per step keeps the reads in the loop.
__global__ void __launch_bounds__(kProbeThreads) k_lds_probe(int iters, float *out)
{
    __shared__ float4 buf[4 * kProbeThreads];
    for (int i = threadIdx.x; i < 4 * kProbeThreads; i += kProbeThreads)
        buf[i] = make_float4((float)i, 1.0f, 2.0f, 3.0f);
    __syncthreads();
    float4 s = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const int t = threadIdx.x;
    for (int i = 0; i < iters; ++i) {
        asm volatile("" ::: "memory");
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float4 v = buf[t + r * kProbeThreads];
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
    }
    out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = s.x + s.y + s.z + s.w;
}

}  // namespace
}  // namespace cbct

using namespace cbct;

extern "C" int cbct_probe_threads(void) { return kProbeThreads; }

extern "C" cbct_status cbct_probe_valu(int n_blocks, int iters, float *out, void *stream)
{
    if (!out)
        return CBCT_E_NULL;
    if (n_blocks < 1 || iters < 1)
        return CBCT_E_SHAPE;
    hipLaunchKernelGGL(k_valu_probe, dim3(n_blocks), dim3(kProbeThreads), 0,
                       (hipStream_t)stream, iters, 1.0f, 1e-7f, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_hip_error(e);
        return CBCT_E_HIP;
    }
    return CBCT_OK;
}

extern "C" cbct_status cbct_probe_lds(int n_blocks, int iters, float *out, void *stream)
{
    if (!out)
        return CBCT_E_NULL;
    if (n_blocks < 1 || iters < 1)
        return CBCT_E_SHAPE;
    hipLaunchKernelGGL(k_lds_probe, dim3(n_blocks), dim3(kProbeThreads), 0,
                       (hipStream_t)stream, iters, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_hip_error(e);
        return CBCT_E_HIP;
    }
    return CBCT_OK;
}
