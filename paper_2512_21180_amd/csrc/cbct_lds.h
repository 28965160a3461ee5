// Small device helpers shared by the projector kernels: LDS addresses as
// 32-bit numbers (so a row address is one integer multiply-add), a
// one-instruction floor-to-integer conversion, a 24-bit multiply-add and the
// buffer-resource word the staging loads use.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cbct {

typedef __attribute__((address_space(3))) const float lds_float;

__device__ inline uint32_t lds_addr(const float *p)
{
    return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const float *)p;
}

__device__ inline lds_float *lds_ptr(uint32_t a) { return (lds_float *)(uintptr_t)a; }

// floor(x) as int32 in one VALU instruction (x finite, |x| < 2^31): the
// compiler otherwise emits a floor and a truncating conversion.
__device__ inline int floor_i32(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// a * b + c with a, b signed 24-bit (b wave-uniform) in one VALU
// instruction: written plainly, an LDS address made this way becomes a
// sign extension and a 64-bit multiply-add.
__device__ inline int mad_i24(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// Fourth word of a buffer resource on the gfx9 family (gfx950 included):
// 32-bit data format, no swizzle; raw loads use only the base, the size (for
// the range check: offsets at or past it read zero) and this word.
constexpr int kBufferWord3 = 0x00020000;

}  // namespace cbct
