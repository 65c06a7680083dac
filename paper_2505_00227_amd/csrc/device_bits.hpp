// Device bit helpers shared by the encoder and the decoder kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mdr {

// Pointers taken from job tables are generic; casting them to the global
// address space lets the compiler use global (not flat) loads and stores, which
// do not share a wait counter with LDS traffic.
// 16-byte vectors for global loads / stores through such pointers (the HIP
// vector classes cannot be copied out of another address space)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

// In-register transpose of a 32x32 bit matrix: afterwards bit r of a[c] is the
// former bit c of a[r].  Five butterfly stages swap the off-diagonal blocks of
// size 16, 8, 4, 2, 1.  The two byte-granular stages are one byte permute per
// output word; the bit-granular ones a shift and a bit-field insert.
__device__ __forceinline__ void transpose32(uint32_t (&a)[32])
{
    // __builtin_amdgcn_perm(hi, lo, sel): byte i of the result is byte sel.i of
    // the 8-byte value hi:lo (lo = bytes 0..3)
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t x = a[k], y = a[k + 16];
        a[k] = __builtin_amdgcn_perm(y, x, 0x05040100u);       // x.lo16 | y.lo16 << 16
        a[k + 16] = __builtin_amdgcn_perm(y, x, 0x07060302u);  // x.hi16 | y.hi16 << 16
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (k & 8) continue;
        const uint32_t x = a[k], y = a[k + 8];
        a[k] = __builtin_amdgcn_perm(y, x, 0x06020400u);      // x0 y0 x2 y2
        a[k + 8] = __builtin_amdgcn_perm(y, x, 0x07030501u);  // x1 y1 x3 y3
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (k & 4) continue;
        const uint32_t x = a[k], y = a[k + 4];
        a[k] = (x & 0x0F0F0F0Fu) | ((y << 4) & 0xF0F0F0F0u);
        a[k + 4] = ((x >> 4) & 0x0F0F0F0Fu) | (y & 0xF0F0F0F0u);
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (k & 2) continue;
        const uint32_t x = a[k], y = a[k + 2];
        a[k] = (x & 0x33333333u) | ((y << 2) & 0xCCCCCCCCu);
        a[k + 2] = ((x >> 2) & 0x33333333u) | (y & 0xCCCCCCCCu);
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (k & 1) continue;
        const uint32_t x = a[k], y = a[k + 1];
        a[k] = (x & 0x55555555u) | ((y << 1) & 0xAAAAAAAAu);
        a[k + 1] = ((x >> 1) & 0x55555555u) | (y & 0xAAAAAAAAu);
    }
}

}  // namespace mdr
