// Encoder-design ablation (Sec. 3, Sec. 6 encoding experiments): 32-bit words
// into 32 bitplanes and back, by each parallelisation the paper compares,
// written for gfx950's 64-wide wavefronts.  Plane p holds bit 31 - p (MSB
// first).  Block layout (every design but the register block): word j of a
// plane holds bit t of value 32j + t.  Register-block layout: regions of 2048
// values; word 64r + l holds, at bit k, value 2048r + l + 64k (a lane's
// interleaved elements, so that its loads coalesce).  Values past n are 0.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_bits.hpp"
#include "mdr_internal.hpp"

namespace mdr {
namespace {

constexpr uint32_t kAbl = 256;  // threads per workgroup

__device__ __forceinline__ uint32_t word_or_zero(const uint32_t* p, uint64_t n, uint64_t i)
{
    return i < n ? p[i] : 0u;
}

// ---- locality block: one thread per block of 32 contiguous values (16-byte
// loads of its own 128 bytes), an in-register transpose, coalesced plane stores
__global__ __launch_bounds__(kAbl) void k_abl_locality_enc(const uint32_t* __restrict__ in, uint64_t n,
                                                           uint32_t* __restrict__ planes, uint64_t nb)
{
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    const uint64_t base = j * 32;
    uint32_t a[32];
    if (base + 32 <= n) {
        const auto p = gmem(reinterpret_cast<const u32x4*>(in + base));
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const u32x4 v = p[q];
            a[4 * q] = v.x;
            a[4 * q + 1] = v.y;
            a[4 * q + 2] = v.z;
            a[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int t = 0; t < 32; ++t) a[t] = word_or_zero(in, n, base + t);
    }
    transpose32(a);  // a[c] bit t = bit c of value base + t
#pragma unroll
    for (int p = 0; p < 32; ++p) planes[(uint64_t)p * nb + j] = a[31 - p];
}

__global__ __launch_bounds__(kAbl) void k_abl_locality_dec(const uint32_t* __restrict__ planes, uint64_t n,
                                                           uint64_t nb, uint32_t* __restrict__ out)
{
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    const uint64_t base = j * 32;
    uint32_t a[32];
#pragma unroll
    for (int p = 0; p < 32; ++p) a[31 - p] = planes[(uint64_t)p * nb + j];
    transpose32(a);  // a[t] = value base + t
    if (base + 32 <= n) {
        const auto p = gmem(reinterpret_cast<u32x4*>(out + base));
#pragma unroll
        for (int q = 0; q < 8; ++q) p[q] = u32x4{a[4 * q], a[4 * q + 1], a[4 * q + 2], a[4 * q + 3]};
    } else {
#pragma unroll
        for (int t = 0; t < 32; ++t)
            if (base + t < n) out[base + t] = a[t];
    }
}

// ---- register shuffling: one value per lane (coalesced loads); a wavefront's
// 64 values are two blocks, lanes 0-31 and 32-63.  Afterwards lane l holds the
// word of plane 31 - (l mod 32) of its half's block and stores it.
__device__ __forceinline__ void store_lane_word(uint32_t* planes, uint64_t nb, uint64_t wave, uint32_t lane,
                                                uint32_t w)
{
    const uint64_t blk = wave * 2 + (lane >> 5);
    if (blk < nb) planes[(uint64_t)(31 - (lane & 31)) * nb + blk] = w;
}

// ballot: one wave-wide vote per bit; only the lane that stores a plane keeps
// its half of the vote
__global__ __launch_bounds__(kAbl) void k_abl_ballot_enc(const uint32_t* __restrict__ in, uint64_t n,
                                                         uint32_t* __restrict__ planes, uint64_t nb)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t v = word_or_zero(in, n, i);
    uint32_t mine = 0;
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        const uint64_t m = __ballot((v >> b) & 1u);
        const uint32_t w = lane < 32 ? (uint32_t)m : (uint32_t)(m >> 32);
        mine = (int)(lane & 31) == b ? w : mine;
    }
    store_lane_word(planes, nb, i / 64, lane, mine);
}

// shift: per bit, a five-round OR tree over the half-wavefront
__global__ __launch_bounds__(kAbl) void k_abl_shift_enc(const uint32_t* __restrict__ in, uint64_t n,
                                                        uint32_t* __restrict__ planes, uint64_t nb)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t v = word_or_zero(in, n, i);
    uint32_t mine = 0;
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        uint32_t x = ((v >> b) & 1u) << (lane & 31);
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) x |= (uint32_t)__shfl_xor((int)x, off, 64);
        mine = (int)(lane & 31) == b ? x : mine;
    }
    store_lane_word(planes, nb, i / 64, lane, mine);
}

// butterfly: the 32x32 transpose across the half-wavefront in five exchange
// rounds (lanes l and l ^ s swap their off-diagonal s-bit blocks); afterwards
// bit r of lane l's word is bit l of lane r's value.  The same rounds undo it.
__device__ __forceinline__ uint32_t lane_transpose(uint32_t x, uint32_t lane)
{
    constexpr uint32_t kMask[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        const int s = 16 >> r;
        const uint32_t m = kMask[r];
        const uint32_t y = (uint32_t)__shfl_xor((int)x, s, 64);
        x = (lane & s) ? ((x & ~m) | ((y >> s) & m)) : ((x & m) | ((y & m) << s));
    }
    return x;
}

__global__ __launch_bounds__(kAbl) void k_abl_butterfly_enc(const uint32_t* __restrict__ in, uint64_t n,
                                                            uint32_t* __restrict__ planes, uint64_t nb)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63;
    store_lane_word(planes, nb, i / 64, lane, lane_transpose(word_or_zero(in, n, i), lane));
}

// decode of the one-value-per-lane designs: lane l loads the word of plane
// 31 - (l mod 32); butterfly: the same rounds; ballot / shift: 32 lane reads
__device__ __forceinline__ uint32_t load_lane_word(const uint32_t* planes, uint64_t nb, uint64_t wave,
                                                   uint32_t lane)
{
    const uint64_t blk = wave * 2 + (lane >> 5);
    return blk < nb ? planes[(uint64_t)(31 - (lane & 31)) * nb + blk] : 0u;
}

__global__ __launch_bounds__(kAbl) void k_abl_butterfly_dec(const uint32_t* __restrict__ planes, uint64_t n,
                                                            uint64_t nb, uint32_t* __restrict__ out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t v = lane_transpose(load_lane_word(planes, nb, i / 64, lane), lane);
    if (i < n) out[i] = v;
}

__global__ __launch_bounds__(kAbl) void k_abl_gather_dec(const uint32_t* __restrict__ planes, uint64_t n,
                                                         uint64_t nb, uint32_t* __restrict__ out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = load_lane_word(planes, nb, i / 64, lane);
    uint32_t v = 0;
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        const uint32_t x = (uint32_t)__shfl((int)w, (int)((lane & 32) | (uint32_t)b), 64);
        v |= ((x >> (lane & 31)) & 1u) << b;
    }
    if (i < n) out[i] = v;
}

// ---- register block: lane l of region r loads values 2048r + l + 64k
// (k = 0..31, each load coalesced across the wavefront), transposes in
// registers, and stores word 64r + l of every plane (coalesced)
__global__ __launch_bounds__(kAbl) void k_abl_regblock_enc(const uint32_t* __restrict__ in, uint64_t n,
                                                           uint32_t* __restrict__ planes, uint64_t nw)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;  // = 64 r + l
    if (g >= nw) return;
    const uint64_t base = (g >> 6) * 2048 + (g & 63);
    uint32_t a[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) a[k] = word_or_zero(in, n, base + 64ull * k);
    transpose32(a);
#pragma unroll
    for (int p = 0; p < 32; ++p) planes[(uint64_t)p * nw + g] = a[31 - p];
}

__global__ __launch_bounds__(kAbl) void k_abl_regblock_dec(const uint32_t* __restrict__ planes, uint64_t n,
                                                           uint64_t nw, uint32_t* __restrict__ out)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nw) return;
    const uint64_t base = (g >> 6) * 2048 + (g & 63);
    uint32_t a[32];
#pragma unroll
    for (int p = 0; p < 32; ++p) a[31 - p] = planes[(uint64_t)p * nw + g];
    transpose32(a);
#pragma unroll
    for (int k = 0; k < 32; ++k)
        if (base + 64ull * k < n) out[base + 64ull * k] = a[k];
}

unsigned blocks(uint64_t threads)
{
    return (unsigned)((threads + kAbl - 1) / kAbl);
}

}  // namespace

uint64_t ablation_plane_words(int design, uint64_t n)
{
    if (design == kAblRegBlock) return (n + 2047) / 2048 * 64;
    return (n + 31) / 32;
}

hipError_t launch_ablation(int design, bool encode, const uint32_t* in, uint64_t n, uint32_t* planes,
                           uint32_t* out, hipStream_t s)
{
    const uint64_t w = ablation_plane_words(design, n);
    if (w == 0) return hipSuccess;
    // one-value-per-lane designs: a wavefront per pair of blocks
    const uint64_t lanes = (w + 1) / 2 * 64;
    switch (design) {
    case kAblLocality:
        if (encode)
            hipLaunchKernelGGL(k_abl_locality_enc, dim3(blocks(w)), dim3(kAbl), 0, s, in, n, planes, w);
        else
            hipLaunchKernelGGL(k_abl_locality_dec, dim3(blocks(w)), dim3(kAbl), 0, s, planes, n, w, out);
        break;
    case kAblBallot:
    case kAblShift:
        if (!encode)
            hipLaunchKernelGGL(k_abl_gather_dec, dim3(blocks(lanes)), dim3(kAbl), 0, s, planes, n, w, out);
        else if (design == kAblBallot)
            hipLaunchKernelGGL(k_abl_ballot_enc, dim3(blocks(lanes)), dim3(kAbl), 0, s, in, n, planes, w);
        else
            hipLaunchKernelGGL(k_abl_shift_enc, dim3(blocks(lanes)), dim3(kAbl), 0, s, in, n, planes, w);
        break;
    case kAblButterfly:
        if (encode)
            hipLaunchKernelGGL(k_abl_butterfly_enc, dim3(blocks(lanes)), dim3(kAbl), 0, s, in, n, planes, w);
        else
            hipLaunchKernelGGL(k_abl_butterfly_dec, dim3(blocks(lanes)), dim3(kAbl), 0, s, planes, n, w, out);
        break;
    case kAblRegBlock:
        if (encode)
            hipLaunchKernelGGL(k_abl_regblock_enc, dim3(blocks(w)), dim3(kAbl), 0, s, in, n, planes, w);
        else
            hipLaunchKernelGGL(k_abl_regblock_dec, dim3(blocks(w)), dim3(kAbl), 0, s, planes, n, w, out);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mdr
