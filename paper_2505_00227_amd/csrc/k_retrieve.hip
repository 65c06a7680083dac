// Retrieve kernels for gfx950: bitplane decoding (inverse of Alg. 1) and the
// exact reconstruction of each value from the sign plane and its first k
// magnitude planes.
#include <type_traits>

#include "device_bits.hpp"
#include "mdr_internal.hpp"

namespace mdr {
namespace {

// One thread per block of 32 values: load the sign word and the words of the
// first k planes (plane p holds bit B-1-p), transpose back to magnitudes, and
// write x = (-1)^s * mag * 2^(e-B).  The magnitude keeps at most the input
// type's significand bits, so the integer-to-float conversion and the ldexp
// are exact (subnormal results included).
template <bool F64, bool VEC>
__global__ __launch_bounds__(kThreads) void k_reconstruct(ReconJob j)
{
    using T = std::conditional_t<F64, double, float>;
    const uint32_t blk = blockIdx.x * kThreads + threadIdx.x;
    if (blk >= j.nbd) return;
    const uint64_t base = (uint64_t)blk * 32;
    if (base >= j.n) return;
    const uint32_t cnt = (uint32_t)min<uint64_t>(32, j.n - base);
    T* out = static_cast<T*>(j.out) + base;
    T v[32];
    if (j.k == 0) {
#pragma unroll
        for (int t = 0; t < 32; ++t) v[t] = T(0);
    } else {
        const uint32_t B = j.B, k = j.k;
        const uint32_t sgn = j.rows[0][blk];
        uint32_t lo[32];
        uint32_t hi[F64 ? 32 : 1];
        // bit c lives in plane p = B-1-c, present when p < k, i.e. c >= B-k
#pragma unroll
        for (int c = 0; c < 32; ++c)
            lo[c] = (c < (int)B && c >= (int)(B - k)) ? j.rows[B - c][blk] : 0u;
        transpose32(lo);
        if constexpr (F64) {
#pragma unroll
            for (int c = 0; c < 32; ++c)
                hi[c] = (32 + c < (int)B && 32 + c >= (int)(B - k)) ? j.rows[B - 32 - c][blk] : 0u;
            transpose32(hi);
        }
        const int sh = j.e - (int)B;
#pragma unroll
        for (int t = 0; t < 32; ++t) {
            T mag;
            if constexpr (F64)
                mag = (double)hi[t] * 0x1p32 + (double)lo[t];
            else
                mag = (float)lo[t];
            T a = F64 ? (T)__builtin_amdgcn_ldexp((double)mag, sh)
                      : (T)__builtin_amdgcn_ldexpf((float)mag, sh);
            v[t] = ((sgn >> t) & 1u) ? -a : a;
        }
    }
    if (VEC && cnt == 32) {
        if constexpr (F64) {
            double2* p = reinterpret_cast<double2*>(out);
#pragma unroll
            for (int q = 0; q < 16; ++q) p[q] = make_double2(v[2 * q], v[2 * q + 1]);
        } else {
            float4* p = reinterpret_cast<float4*>(out);
#pragma unroll
            for (int q = 0; q < 8; ++q) p[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        }
    } else {
#pragma unroll
        for (int t = 0; t < 32; ++t)
            if ((uint32_t)t < cnt) out[t] = v[t];
    }
}

// V_total error estimate (Sec. 5.2): with |v - vhat| <= eps_c per component,
// |v^2 - vhat^2| <= eps_c (2|vhat| + eps_c); the estimate is the maximum over
// points of the sum over x, y, z, evaluated in double in that order (no
// contraction: the library is built with -ffp-contract=off).
template <bool F64>
__global__ __launch_bounds__(kThreads) void k_qoi_vtotal(const void* px, const void* py,
                                                         const void* pz, uint64_t n, double ex,
                                                         double ey, double ez,
                                                         unsigned long long* out)
{
    using T = std::conditional_t<F64, double, float>;
    const T* x = static_cast<const T*>(px);
    const T* y = static_cast<const T*>(py);
    const T* z = static_cast<const T*>(pz);
    double worst = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double ax = fabs((double)x[i]), ay = fabs((double)y[i]), az = fabs((double)z[i]);
        double tx = ex * ((2.0 * ax) + ex);
        double ty = ey * ((2.0 * ay) + ey);
        double tz = ez * ((2.0 * az) + ez);
        double s = 0.0;
        s = s + tx;
        s = s + ty;
        s = s + tz;
        worst = s > worst ? s : worst;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double o = __shfl_xor(worst, off, 64);
        worst = o > worst ? o : worst;
    }
    __shared__ double s_w[kThreads / 64];
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = worst;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / 64; ++w) worst = s_w[w] > worst ? s_w[w] : worst;
        atomicMax(out, (unsigned long long)__double_as_longlong(worst));
    }
}

}  // namespace

hipError_t launch_qoi_vtotal(const void* x, const void* y, const void* z, uint64_t n, bool f64,
                             const double eps[3], unsigned long long* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint64_t g = (n + kThreads * 8 - 1) / (kThreads * 8);
    if (g > 1024) g = 1024;
    if (f64)
        hipLaunchKernelGGL((k_qoi_vtotal<true>), dim3((unsigned)g), dim3(kThreads), 0, s, x, y, z, n,
                           eps[0], eps[1], eps[2], out);
    else
        hipLaunchKernelGGL((k_qoi_vtotal<false>), dim3((unsigned)g), dim3(kThreads), 0, s, x, y, z, n,
                           eps[0], eps[1], eps[2], out);
    return hipGetLastError();
}

hipError_t launch_reconstruct(const ReconJob& job, bool f64, hipStream_t s)
{
    if (job.n == 0) return hipSuccess;
    dim3 g((job.nbd + kThreads - 1) / kThreads), b(kThreads);
    bool vec = ((uintptr_t)job.out % 16) == 0;
    if (f64) {
        if (vec)
            hipLaunchKernelGGL((k_reconstruct<true, true>), g, b, 0, s, job);
        else
            hipLaunchKernelGGL((k_reconstruct<true, false>), g, b, 0, s, job);
    } else {
        if (vec)
            hipLaunchKernelGGL((k_reconstruct<false, true>), g, b, 0, s, job);
        else
            hipLaunchKernelGGL((k_reconstruct<false, false>), g, b, 0, s, job);
    }
    return hipGetLastError();
}

}  // namespace mdr
