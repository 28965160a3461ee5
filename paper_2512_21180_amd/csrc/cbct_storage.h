// Storage conversions for the projector kernels: FP32 arithmetic on FP32,
// BF16 or FP16 buffers (widened on load, rounded to nearest-even on store).
// `raw` loads the stored bits into a 32-bit register (`raw_at`: at a 32-bit
// byte offset from the base; `buf_at`, FP32 only: through a buffer
// resource, zero outside its range) and `wide` widens them:
// a kernel that keeps loads in flight across other work holds raw values and
// widens them where they are used (widening, or packing two 16-bit values
// into one register, right after the load would wait for it).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cbct {

struct F32 {
    using T = float;
    __device__ static float ld(const T *p, size_t i) { return p[i]; }
    using Raw = float;
    __device__ static Raw raw(const T *p, size_t i) { return p[i]; }
    __device__ static Raw raw_at(const T *p, uint32_t byte_off)
    {
        return *(const T *)((const char *)p + byte_off);
    }
    __device__ static Raw buf_at(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
    }
    __device__ static float wide(Raw x) { return x; }
    __device__ static void st(T *p, size_t i, float v) { p[i] = v; }
};

struct BF16 {
    using T = uint16_t;
    using Raw = uint32_t;
    __device__ static float ld(const T *p, size_t i) { return wide(p[i]); }
    __device__ static Raw raw(const T *p, size_t i) { return p[i]; }
    __device__ static Raw raw_at(const T *p, uint32_t byte_off)
    {
        return *(const T *)((const char *)p + byte_off);
    }
    __device__ static float wide(Raw x) { return __uint_as_float(x << 16); }
    __device__ static void st(T *p, size_t i, float v)
    {
        uint32_t b = __float_as_uint(v);
        uint32_t r;
        if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu))
            r = (b >> 16) | 0x0040u;                       // quiet NaN
        else
            r = (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;    // round to nearest even
        p[i] = (uint16_t)r;
    }
};

struct F16 {
    using T = _Float16;
    __device__ static float ld(const T *p, size_t i) { return (float)p[i]; }
    using Raw = uint32_t;
    __device__ static Raw raw(const T *p, size_t i)
    {
        return __builtin_bit_cast(uint16_t, p[i]);
    }
    __device__ static Raw raw_at(const T *p, uint32_t byte_off)
    {
        return __builtin_bit_cast(uint16_t, *(const T *)((const char *)p + byte_off));
    }
    __device__ static float wide(Raw x)
    {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)x);
    }
    __device__ static void st(T *p, size_t i, float v) { p[i] = (_Float16)v; }
};

// Bytes of one stored element.
inline size_t storage_bytes(cbct_dtype t) { return t == CBCT_F32 ? 4 : 2; }

// Dispatch a functor templated on <VolStorage, SinoStorage> by runtime codes.
template <class F>
inline hipError_t dispatch_storage(cbct_dtype vt, cbct_dtype st, F &&f)
{
    if (vt == CBCT_F32 && st == CBCT_F32) return f(F32{}, F32{});
    if (vt == CBCT_BF16 && st == CBCT_BF16) return f(BF16{}, BF16{});
    if (vt == CBCT_F16 && st == CBCT_F16) return f(F16{}, F16{});
    if (vt == CBCT_BF16 && st == CBCT_F32) return f(BF16{}, F32{});
    if (vt == CBCT_F16 && st == CBCT_F32) return f(F16{}, F32{});
    if (vt == CBCT_F32 && st == CBCT_BF16) return f(F32{}, BF16{});
    if (vt == CBCT_F32 && st == CBCT_F16) return f(F32{}, F16{});
    if (vt == CBCT_BF16 && st == CBCT_F16) return f(BF16{}, F16{});
    if (vt == CBCT_F16 && st == CBCT_BF16) return f(F16{}, BF16{});
    return hipErrorInvalidValue;
}

// Ray length per plane, ds = dsf * sqrt(n2 + V^2), for a column with
// constants (dsf, n2) and a row with V^2 = v2.  Every kernel computes ds with
// this one function (the hardware square root, within 1 ulp), so the forward
// and the adjoint apply the same weights.
__device__ inline float ray_ds(float dsf, float n2, float v2)
{
    return dsf * __builtin_amdgcn_sqrtf(n2 + v2);
}

}  // namespace cbct
