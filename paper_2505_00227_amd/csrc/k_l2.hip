// Squared L2 error of a level after k planes, k = 0..B: the L2 error table
// that MDR offers beside the L-infinity one (the paper controls L-infinity
// error throughout).  E2[k] = sum_i (|x_i| - xhat_k(|x_i|))^2 with
// xhat_k(a) = floor(a 2^(k-e)) 2^(e-k), the magnitude the retrieval rebuilds
// from k planes of the level aligned to exponent e.  Every residual is exact
// in fp64 (it is a run of the value's own significand bits); each square is
// rounded once and the sums run in fp64 in a fixed order (per thread, then a
// fixed tree per workgroup, then workgroups in index order), so the table is
// the same on every run.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "mdr_internal.hpp"

namespace mdr {
namespace {

constexpr uint32_t kL2 = 256;  // threads per workgroup

// table entries KLO..KHI (and <= B) of every workgroup's partial row (B + 2
// entries: E2[0..B], then the largest |x| the workgroup read, written by the
// KLO = 0 launch); f64 tables run as two launches so that a thread holds at
// most 33 accumulators
template <typename T, int KLO, int KHI>
__global__ __launch_bounds__(kL2) void k_l2_partial(const T* __restrict__ x, uint64_t n, int e, uint32_t B,
                                                    double* __restrict__ part)
{
#pragma clang fp contract(off)
    constexpr int KN = KHI - KLO + 1;
    __shared__ double red[kL2 / 64][KN];
    __shared__ double s_amax[kL2 / 64];
    double acc[KN];
#pragma unroll
    for (int j = 0; j < KN; ++j) acc[j] = 0.0;
    double amax = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kL2;
    for (uint64_t i = (uint64_t)blockIdx.x * kL2 + threadIdx.x; i < n; i += stride) {
        const double a = std::fabs((double)x[i]);
        if (KLO == 0) amax = a > amax ? a : amax;
#pragma unroll
        for (int j = 0; j < KN; ++j) {
            const int k = KLO + j;
            if (k <= (int)B) {
                // exact power-of-two scalings (a scaled value below 1 may round, its floor is 0 either way)
                const double r = a - std::ldexp(std::floor(std::ldexp(a, k - e)), e - k);
                acc[j] += r * r;
            }
        }
    }
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < KN; ++j) {
        double v = acc[j];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wave][j] = v;
    }
    if (KLO == 0) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double v = __shfl_xor(amax, o, 64);
            amax = v > amax ? v : amax;
        }
        if (lane == 0) s_amax[wave] = amax;
    }
    __syncthreads();
    const uint32_t k = KLO + threadIdx.x;
    if (threadIdx.x < (uint32_t)KN && k <= B) {
        double v = 0.0;
#pragma unroll
        for (uint32_t w = 0; w < kL2 / 64; ++w) v += red[w][threadIdx.x];
        part[(uint64_t)blockIdx.x * (B + 2) + k] = v;
    }
    if (KLO == 0 && threadIdx.x == 0) {
        double m = 0.0;
        for (uint32_t w = 0; w < kL2 / 64; ++w) m = s_amax[w] > m ? s_amax[w] : m;
        part[(uint64_t)blockIdx.x * (B + 2) + B + 1] = m;
    }
}

// out[0..B]: the table (workgroup rows summed in index order); out[B + 1]: the
// largest |x| read, which the caller checks against the refactored level's
__global__ void k_l2_final(const double* __restrict__ part, uint32_t nwg, uint32_t B, double* __restrict__ out)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > B + 1) return;
    double v = 0.0;
    for (uint32_t w = 0; w < nwg; ++w) {
        const double p = part[(uint64_t)w * (B + 2) + k];
        v = k <= B ? v + p : (p > v ? p : v);
    }
    out[k] = v;
}

// Fixed scratch of mdr_l2_table_noalloc: the partial rows of at most 1024
// workgroups, then the rows of at most kL2NoAllocLevels levels, kL2RowMax
// entries (B + 2 for B <= 64) each: 574,464 bytes per device, held until the
// process ends.  Host code never passes this name to a kernel: it is a
// host-side stand-in; the device address comes from hipGetSymbolAddress, per
// device.
constexpr uint64_t kL2PartDoubles = 1024ull * kL2RowMax;
constexpr uint64_t kL2ScratchDoubles = kL2PartDoubles + (uint64_t)kL2NoAllocLevels * kL2RowMax;
__device__ __align__(256) double scratch[kL2ScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t l2_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) {
        e = hipSetDevice(device);
        if (e != hipSuccess) return e;
    }
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
    return hipSuccess;
}

hipError_t l2_scratch(int device, double** part, double** out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    double* p;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_ptr[device];
    }
    if (!p) return hipErrorNotInitialized;
    *part = p;
    *out = p + kL2PartDoubles;
    return hipSuccess;
}

uint32_t l2_table_workgroups(uint64_t n)
{
    const uint64_t w = (n + kL2 * 8 - 1) / (kL2 * 8);
    return (uint32_t)(w < 1 ? 1 : (w > 1024 ? 1024 : w));
}

hipError_t launch_l2_table(bool f64, const void* x, uint64_t n, int e, uint32_t B, double* part, double* out,
                           hipStream_t s)
{
    const uint32_t nwg = l2_table_workgroups(n);
    if (f64) {
        hipLaunchKernelGGL((k_l2_partial<double, 0, 32>), dim3(nwg), dim3(kL2), 0, s, static_cast<const double*>(x),
                           n, e, B, part);
        if (B > 32)
            hipLaunchKernelGGL((k_l2_partial<double, 33, 64>), dim3(nwg), dim3(kL2), 0, s,
                               static_cast<const double*>(x), n, e, B, part);
    } else {
        hipLaunchKernelGGL((k_l2_partial<float, 0, 32>), dim3(nwg), dim3(kL2), 0, s, static_cast<const float*>(x), n,
                           e, B, part);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_l2_final, dim3(1), dim3(128), 0, s, part, nwg, B, out);  // B + 2 <= 66 entries
    return hipGetLastError();
}

}  // namespace mdr
