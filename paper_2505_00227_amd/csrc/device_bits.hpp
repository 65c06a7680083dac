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
// size 16, 8, 4, 2, 1 (each output word is one bit-field insert).
__device__ __forceinline__ void transpose32(uint32_t (&a)[32])
{
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        uint32_t x = a[k], y = a[k + 16];
        a[k] = (x & 0x0000FFFFu) | (y << 16);
        a[k + 16] = (x >> 16) | (y & 0xFFFF0000u);
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (k & 8) continue;
        uint32_t x = a[k], y = a[k + 8];
        a[k] = (x & 0x00FF00FFu) | ((y << 8) & 0xFF00FF00u);
        a[k + 8] = ((x >> 8) & 0x00FF00FFu) | (y & 0xFF00FF00u);
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (k & 4) continue;
        uint32_t x = a[k], y = a[k + 4];
        a[k] = (x & 0x0F0F0F0Fu) | ((y << 4) & 0xF0F0F0F0u);
        a[k + 4] = ((x >> 4) & 0x0F0F0F0Fu) | (y & 0xF0F0F0F0u);
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (k & 2) continue;
        uint32_t x = a[k], y = a[k + 2];
        a[k] = (x & 0x33333333u) | ((y << 2) & 0xCCCCCCCCu);
        a[k + 2] = ((x >> 2) & 0x33333333u) | (y & 0xCCCCCCCCu);
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (k & 1) continue;
        uint32_t x = a[k], y = a[k + 1];
        a[k] = (x & 0x55555555u) | ((y << 1) & 0xAAAAAAAAu);
        a[k + 1] = ((x >> 1) & 0x55555555u) | (y & 0xAAAAAAAAu);
    }
}

}  // namespace mdr
