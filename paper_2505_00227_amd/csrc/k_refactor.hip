// Refactor kernels for gfx950: level statistics, bitplane encoding with the
// per-plane error table and per-group lossless statistics, and the device-side
// hybrid selection of Alg. 2 (Sec. 4.2) with its Huffman codebook.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "device_bits.hpp"
#include "mdr_internal.hpp"

namespace mdr {
namespace {

// rows a general-path encoder workgroup stages in LDS at once
constexpr uint32_t kPassRows = 33;

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int frexp_exp_f32(uint32_t absbits)
{
    uint32_t eb = absbits >> 23;
    if (eb) return (int)eb - 126;
    return -117 - (int)__clz(absbits & 0x7FFFFFu);
}

__device__ __forceinline__ int frexp_exp_f64(uint64_t absbits)
{
    uint32_t eb = (uint32_t)(absbits >> 52);
    if (eb) return (int)eb - 1022;
    return -1010 - (int)__clzll(absbits & 0xFFFFFFFFFFFFFull);
}

__device__ __forceinline__ uint64_t order_key_f32(uint32_t bits)
{
    return (bits >> 31) ? (uint64_t)(~bits) : (uint64_t)(bits | 0x80000000u);
}

__device__ __forceinline__ uint64_t order_key_f64(uint64_t bits)
{
    return (bits >> 63) ? ~bits : (bits | 0x8000000000000000ull);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

// ------------------------------------------------------------------ fills
__global__ void k_fill_u32(uint32_t* p, uint64_t count, uint32_t value)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        p[i] = value;
}

// Copy from pinned host memory, read through its device address, into device
// memory on the stream's own queue.  System-scope loads go past any cache the
// host's writes could miss.
__global__ void k_copy_in(const uint64_t* src, uint64_t* __restrict__ dst, uint64_t count)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Start of a refactor pass: the level statistics to their neutral values and
// two regions of accumulators to zero, in one launch.
__global__ void k_init_pass(LevelStats* st, uint32_t count, uint32_t* z0, uint64_t n0, uint32_t* z1,
                            uint64_t n1)
{
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    if (i0 < count) {
        st[i0].minkey = ~0ull;
        st[i0].maxkey = 0;
        st[i0].maxabs_bits = 0;
    }
    for (uint64_t i = i0; i < n0; i += stride) z0[i] = 0;
    for (uint64_t i = i0; i < n1; i += stride) z1[i] = 0;
}

// ------------------------------------------------------------------ level statistics
// One streaming pass: min / max / max|x| (max |x| gives Alg. 1's alignment
// exponent and the non-finite check).  Each thread folds 16-byte vectors, the
// workgroup reduces in LDS, and one lane per workgroup publishes with three
// device atomics.  Atomics on one address serialize in the memory system, so
// a level gets few large workgroups (kStatsThreads threads, at most
// kStatsMaxWg of them).  Per thread: the largest |x| bit pattern and the float
// minimum / maximum (zeros of either sign are reported as +0.0, so their order
// does not matter).
template <bool F64>
struct StatAcc {
    using U = std::conditional_t<F64, uint64_t, uint32_t>;
    using T = std::conditional_t<F64, double, float>;
    U amax = 0;
    T vmin = __builtin_huge_val(), vmax = -__builtin_huge_val();
    __device__ __forceinline__ void add(U b)
    {
        const U ab = b & (F64 ? 0x7FFFFFFFFFFFFFFFull : 0x7FFFFFFFu);
        amax = ab > amax ? ab : amax;
        T v;
        __builtin_memcpy(&v, &b, sizeof(T));
        vmin = __builtin_fmin(vmin, v);
        vmax = __builtin_fmax(vmax, v);
    }
};

// One launch covers every level of a batch: workgroup -> job through wg_job,
// then a grid-stride loop over that level with the job's own workgroup count.
template <bool F64, bool VEC>
__global__ __launch_bounds__(kStatsThreads) void k_stats(const StatsJob* __restrict__ jobs,
                                                    const uint32_t* __restrict__ wg_job)
{
    using U = typename StatAcc<F64>::U;
    using T = typename StatAcc<F64>::T;
    constexpr int PER = 16 / sizeof(U);  // values per 16-byte vector
    const StatsJob& job = jobs[wg_job[blockIdx.x]];
    const auto x = gmem(static_cast<const U*>(job.x));
    const uint64_t n = job.n;
    LevelStats* st = job.stats;
    StatAcc<F64> acc;
    const uint64_t stride = (uint64_t)job.grid * blockDim.x;
    const uint64_t tid0 = (uint64_t)(blockIdx.x - job.wg_base) * blockDim.x + threadIdx.x;
    uint64_t done = 0;
    if (VEC) {
        const uint64_t nvec = n / PER;
        const auto xv4 = gmem(reinterpret_cast<const u32x4*>(job.x));
#pragma unroll 4
        for (uint64_t i = tid0; i < nvec; i += stride) {
            const u32x4 q = __builtin_nontemporal_load(&xv4[i]);
            if constexpr (F64) {
                acc.add(((uint64_t)q.y << 32) | q.x);
                acc.add(((uint64_t)q.w << 32) | q.z);
            } else {
                acc.add(q.x);
                acc.add(q.y);
                acc.add(q.z);
                acc.add(q.w);
            }
        }
        done = nvec * PER;
    }
    for (uint64_t i = done + tid0; i < n; i += stride) acc.add(x[i]);

    __shared__ unsigned long long s_amax[kStatsThreads / 64];
    __shared__ T s_min[kStatsThreads / 64], s_max[kStatsThreads / 64];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t amax = wave_max((uint64_t)acc.amax);
    T vmin = wave_min(acc.vmin), vmax = wave_max(acc.vmax);
    if (lane == 0) {
        s_amax[wave] = amax;
        s_min[wave] = vmin;
        s_max[wave] = vmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kStatsThreads / 64; ++w) {
            amax = s_amax[w] > amax ? s_amax[w] : amax;
            vmin = s_min[w] < vmin ? s_min[w] : vmin;
            vmax = s_max[w] > vmax ? s_max[w] : vmax;
        }
        U bmin, bmax;
        __builtin_memcpy(&bmin, &vmin, sizeof(T));
        __builtin_memcpy(&bmax, &vmax, sizeof(T));
        const uint64_t kmin = F64 ? order_key_f64(bmin) : order_key_f32((uint32_t)bmin);
        const uint64_t kmax = F64 ? order_key_f64(bmax) : order_key_f32((uint32_t)bmax);
        atomicMin((unsigned long long*)&st->minkey, (unsigned long long)kmin);
        atomicMax((unsigned long long*)&st->maxkey, (unsigned long long)kmax);
        if (amax) atomicMax((unsigned long long*)&st->maxabs_bits, (unsigned long long)amax);
    }
}

// ------------------------------------------------------------------ bitplane encoder
// One thread owns one block of 32 consecutive values (one u32 word of every
// plane); a workgroup covers a tile of 256 blocks and walks a contiguous range
// of tiles.  Per block:
//   y = |x| * 2^(B-e) (exact), mag = floor(y), sign bit;
//   error keys: key_k = fract(y * 2^(k-B)) = (|x| mod 2^(e-k)) / 2^(e-k); the
//     workgroup keeps max_k key_k in LDS.  Values with mag = 0 lie below every
//     cut: their error is |x| for every k (tracked as `small`);
//   32x32 in-register bit transpose (two for f64) -> plane words;
//   coalesced stores of each plane row, per-unit byte histograms (LDS), and
//   counts of W-bit word transitions for the run-length estimate.
//
// Exact pruning of the f32 error keys.  Let K_k be the workgroup's running
// maximum.  When K_k >= 1 - 2^-t (its binary fraction starts with t ones), a
// value can exceed it only if the t bits just below the cut, in y's binary
// expansion, are all ones.  With Y = (mag << 32) | top 32 fraction bits, bit p
// of r_t = AND_{i<t} (Y << i) says "bits p..p-t+1 of Y are ones"; r_1, r_2,
// r_4, r_8, r_12 come from four shift-ANDs, and each cut c = B-k (bit c-1 of
// the high word) is tested with the longest of them its K_k allows, so one
// pass flags every candidate cut of a value.  Only flagged cuts are evaluated
// and folded in with an LDS max; the others cannot change the result.  Cuts
// with K_k < 1/2 take the direct per-block maximum; k = 0 is max |x|, known from
// the statistics.  Stale maxima only add candidates, so the result is exact.
// FAST: 32 planes of f32 or 64 planes of f64, in groups of 4 (every row, its
// unit and its histogram offset known at compile time): rows go from registers
// straight to memory, neighbours come by lane shuffle, runs are counted per
// thread (f32) or per wavefront (f64) and unit.
template <bool F64, bool VEC, bool FAST>
__device__ __forceinline__ void encode_body(const EncodeJob& job, const uint32_t wg)
{
    using T = std::conditional_t<F64, double, float>;
    constexpr int G = F64 ? 2 : 1;  // u32 words per W-bit word
    constexpr int NROW = F64 ? 65 : 33;
    // dynamic LDS (general path only): [nunits][256] byte histograms, then the
    // tile's plane words [rows][256]
    extern __shared__ uint32_t s_dyn[];
    __shared__ uint32_t s_prev[kMaxRows][G];  // last word(s) of the previous tile, per row
    __shared__ uint32_t s_trans[kMaxRows];
    __shared__ uint32_t s_key32[F64 ? 1 : kKeyStride];
    __shared__ unsigned long long s_key64[F64 ? kKeyStride : 1];
    __shared__ uint32_t s_zero[FAST && !F64 ? 1 : kThreads];  // sink for zero bytes (one slot per thread)
    // FAST: the byte histograms at fixed LDS addresses, so each unit's offset is
    // an instruction immediate
    constexpr int FUNITS = F64 ? 17 : 9;  // FAST: units (sign + 16 or 8 groups)
    // f64 FAST: each unit's 256 bins are followed by one sink slot per lane for
    // zero bytes (counted by difference), at the same offset from every unit
    constexpr int HSTRIDE = F64 ? 320 : 256;
    __shared__ uint32_t s_hist_fast[FAST ? FUNITS * HSTRIDE : 1];

    __shared__ uint32_t s_hoff[kMaxRows];  // row -> its unit's histogram offset
    // FAST: each wave's last words of every row for the next wave's first lanes
    // (f32: lane 63's; f64: lanes 62 and 63, the two halves of its last W-bit word)
    __shared__ uint32_t s_edge[FAST && !F64 ? 4 : 1][kThreads / 64][FAST && !F64 ? 33 : 1];
    // f64: every wave's first (lanes 0, 1) and last (lanes 62, 63) words per row
    __shared__ uint32_t s_first64[FAST && F64 ? 4 : 1][kThreads / 64][2][FAST && F64 ? 65 : 1];
    __shared__ uint32_t s_last64[FAST && F64 ? 4 : 1][kThreads / 64][2][FAST && F64 ? 65 : 1];
    uint32_t edge_trc[2] = {0, 0};  // f64 FAST: transitions at the wave's left edge, rows lane and lane + 64
    uint32_t trc[FAST && !F64 ? 9 : 1];  // f32 FAST: this thread's word transitions per unit
#pragma unroll
    for (int i = 0; i < (FAST && !F64 ? 9 : 1); ++i) trc[i] = 0;
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    // every field the tile loop needs, in registers: stores through the row
    // pointer could otherwise alias the job table and force reloads
    const uint32_t B = job.B, nbd = job.nbd, m = job.m, nunits = job.nunits;
    const uint32_t ntiles = job.ntiles, tpw = job.tiles_per_wg;
    const uint64_t n = job.n;
    const uint64_t amax = job.stats->maxabs_bits;  // 0: every value is zero
    const int e = amax == 0 ? 0 : (F64 ? frexp_exp_f64(amax) : frexp_exp_f32((uint32_t)amax));
    const T* xg = static_cast<const T*>(job.x);
    const auto x = gmem(xg);
    const auto rows = gmem(job.rows);
    const auto recs = gmem(job.recs);
    if (tid < kMaxRows) s_hoff[tid] = job.hist_off[tid];
    (void)m;
    uint32_t* s_hist = FAST ? s_hist_fast : s_dyn;
    uint32_t* s_pl = FAST ? s_dyn : s_dyn + nunits * 256;  // [rows of one pass][256]

    for (uint32_t i = tid; i < nunits * (FAST ? HSTRIDE : 256); i += kThreads) s_hist[i] = 0;
    if (tid < kMaxRows) s_trans[tid] = 0;
    if (tid < kKeyStride) {
        if constexpr (F64)
            s_key64[tid] = 0;
        else
            s_key32[tid] = 0;
    }

    uint32_t frac_max = 0;  // f32: bits of max fract(y) = the k = B key (nonnegative: bits order as values)
    uint64_t frac_max64 = 0;  // the same for f64
    T small = 0;

    const uint32_t t0 = wg * tpw;
    const uint32_t t1 = min(ntiles, t0 + tpw);
    const uint32_t last_blk = min(nbd, t1 * kTileBlocks) - 1;
    // the zeroed histograms and key maxima must be visible to every wave
    // before any reads or updates them (the fast path has no barrier at the
    // top of a tile)
    __syncthreads();

    // ---- 32 consecutive values of tile tt (zeros past the level's end)
    // the u32 word of the tile this thread encodes: its own index, except on
    // the f64 fast path, where lane l of a wave takes half l / 32 (low half
    // first) of the wave's W-bit word l % 32, so that the same half of the
    // previous word is one lane down
    const uint32_t slot = (FAST && F64) ? ((tid & ~63u) | ((lane & 31u) << 1) | (lane >> 5)) : tid;
    auto load_tile = [&](uint32_t tt, T (&vv)[32]) {
        const uint32_t b = tt * kTileBlocks + slot;
        const uint64_t bs = (uint64_t)b * 32;
        if (VEC && b < nbd && bs + 32 <= n) {
            if constexpr (F64) {
                const auto p = gmem(reinterpret_cast<const f64x2*>(xg + bs));
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const f64x2 q = p[j];
                    vv[2 * j] = q.x;
                    vv[2 * j + 1] = q.y;
                }
            } else {
                const auto p = gmem(reinterpret_cast<const f32x4*>(xg + bs));
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const f32x4 q = p[j];
                    vv[4 * j] = q.x;
                    vv[4 * j + 1] = q.y;
                    vv[4 * j + 2] = q.z;
                    vv[4 * j + 3] = q.w;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < 32; ++j) vv[j] = (b < nbd && bs + j < n) ? x[bs + j] : T(0);
        }
    };
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t blk = t * kTileBlocks + slot;
        const bool valid = blk < nbd;
        // the fast path shares nothing between tiles but the edge buffers (four
        // of them), so its waves need no barrier here
        if constexpr (!FAST) __syncthreads();  // the previous tile's rows have been consumed
        T v[32];
        load_tile(t, v);

        // ---- align to the level exponent: y = |x| 2^(B-e), mag = floor(y)
        uint32_t sgn = 0;
        uint32_t lo[32];
        uint32_t hi[F64 ? 32 : 1];
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            if constexpr (F64) {
                uint64_t bits = (uint64_t)__double_as_longlong(v[j]);
                sgn |= (uint32_t)(bits >> 63) << j;
                double a = __longlong_as_double((long long)(bits & 0x7FFFFFFFFFFFFFFFull));
                double y = __builtin_amdgcn_ldexp(a, (int)B - e);
                bool tiny = y < 1.0;  // mag = floor(y) = 0
                small = (tiny && a > small) ? a : small;
                v[j] = tiny ? 0.0 : y;
            } else {
                uint32_t bits = __float_as_uint(v[j]);
                sgn |= (bits >> 31) << j;
                float a = __uint_as_float(bits & 0x7FFFFFFFu);
                float y = __builtin_amdgcn_ldexpf(a, (int)B - e);
                bool tiny = y < 1.0f;  // mag = floor(y) = 0
                small = (tiny && a > small) ? a : small;
                v[j] = tiny ? 0.0f : y;
            }
        }

        // materialise y and the running `small` here, so the raw values die
        // before the key loop instead of being carried through it
#pragma unroll
        for (int j = 0; j < 32; ++j) asm volatile("" : "+v"(v[j]));
        asm volatile("" : "+v"(small));
        // ---- exact error keys, k = 0..B
        if constexpr (F64) {
            // The f32 pruning below on the 128-bit fixed point of y: words
            // X3:X2 = magnitude (hi[j]:lo[j]), X1 = the top 32 fraction bits.
            // Cut c (1..B-1) is bit 64+c-1; a tested run is at most 12 bits
            // long, so it never reaches below bit 53 and the word below X1 is
            // not needed (the runs computed for X1's low bits, which take
            // zeros from below, are never used).  Lane l decides cut l+1.
            uint64_t S1, S2, S4, S8, S12;
            if (t == t0 && B > 1) {
                const int c = (int)(lane % (B - 1)) + 1;  // seeds, as for f32
                double km = 0.0;
#pragma unroll
                for (int j = 0; j < 32; ++j) {
                    const double key = __builtin_amdgcn_fract(__builtin_amdgcn_ldexp(v[j], -c));
                    km = key > km ? key : km;
                }
                atomicMax(&s_key64[B - c], (unsigned long long)__double_as_longlong(km));
                __syncthreads();
            }
            {
                const uint32_t c = lane + 1;
                uint32_t tl = 0;
                if (c < B) {
                    const double M = __longlong_as_double((long long)s_key64[B - c]);
                    if (M >= 0.5) tl = __clz(~(uint32_t)(M * 0x1p32));
                }
                const bool live = c < B;
                S12 = __ballot(live && tl >= 12);
                S8 = __ballot(live && tl >= 8 && tl < 12);
                S4 = __ballot(live && tl >= 4 && tl < 8);
                S2 = __ballot(live && tl >= 2 && tl < 4);
                S1 = __ballot(live && tl == 1);
            }
            const uint64_t strong = S1 | S2 | S4 | S8 | S12;
            const uint32_t S1l = (uint32_t)S1, S2l = (uint32_t)S2, S4l = (uint32_t)S4, S8l = (uint32_t)S8,
                           S12l = (uint32_t)S12;
            const uint32_t S1h = (uint32_t)(S1 >> 32), S2h = (uint32_t)(S2 >> 32), S4h = (uint32_t)(S4 >> 32),
                           S8h = (uint32_t)(S8 >> 32), S12h = (uint32_t)(S12 >> 32);
            // ALL12: every cut's maximum already starts with 12 ones (the usual
            // case past a workgroup's first tile), so the 12-bit runs alone flag
            // the candidates and the shorter runs' masks drop out
            auto key_pass = [&](auto all12_t) {
                constexpr bool ALL12 = decltype(all12_t)::value;
#pragma unroll
                for (int j = 0; j < 32; ++j) {
                    const double y = v[j];
                    const double f = __builtin_amdgcn_fract(y);
                    frac_max64 = max(frac_max64, (uint64_t)__double_as_longlong(f));
                    asm volatile("" : "+v"(frac_max64));  // fold in now, not at the end
                    const double yh = __builtin_trunc(y * 0x1p-32);
                    const uint32_t X3 = (uint32_t)yh, X2 = (uint32_t)(y - yh * 0x1p32), X1 = (uint32_t)(f * 0x1p32);
                    // (word << k) = alignbit(word, word below, 32 - k)
                    const uint32_t r2_3 = X3 & __builtin_amdgcn_alignbit(X3, X2, 31);
                    const uint32_t r2_2 = X2 & __builtin_amdgcn_alignbit(X2, X1, 31);
                    const uint32_t r2_1 = X1 & (X1 << 1);
                    const uint32_t r4_3 = r2_3 & __builtin_amdgcn_alignbit(r2_3, r2_2, 30);
                    const uint32_t r4_2 = r2_2 & __builtin_amdgcn_alignbit(r2_2, r2_1, 30);
                    const uint32_t r4_1 = r2_1 & (r2_1 << 2);
                    const uint32_t r8_3 = r4_3 & __builtin_amdgcn_alignbit(r4_3, r4_2, 28);
                    const uint32_t r8_2 = r4_2 & __builtin_amdgcn_alignbit(r4_2, r4_1, 28);
                    const uint32_t r8_1 = r4_1 & (r4_1 << 4);
                    const uint32_t r12_3 = r8_3 & __builtin_amdgcn_alignbit(r8_3, r8_2, 28);
                    const uint32_t r12_2 = r8_2 & __builtin_amdgcn_alignbit(r8_2, r8_1, 28);
                    uint32_t ca, cb;
                    if constexpr (ALL12) {
                        ca = r12_2 & S12l;
                        cb = r12_3 & S12h;
                    } else {
                        ca = (X2 & S1l) | (r2_2 & S2l) | (r4_2 & S4l) | (r8_2 & S8l) | (r12_2 & S12l);
                        cb = (X3 & S1h) | (r2_3 & S2h) | (r4_3 & S4h) | (r8_3 & S8h) | (r12_3 & S12h);
                    }
                    uint64_t cand = ((uint64_t)cb << 32) | ca;  // bit c-1: cut c
                    while (cand) {
                        const int c = __ffsll((unsigned long long)cand);
                        cand &= cand - 1;
                        const double key = __builtin_amdgcn_fract(__builtin_amdgcn_ldexp(y, -c));
                        atomicMax(&s_key64[B - c], (unsigned long long)__double_as_longlong(key));
                    }
                }
            };
            if (S12 == (B > 1 ? (1ull << (B - 1)) - 1ull : 0ull)) {
                key_pass(std::true_type{});
            } else {
                key_pass(std::false_type{});
                const uint64_t all = B > 1 ? (1ull << (B - 1)) - 1ull : 0ull;  // cuts 1 .. B-1
                uint64_t weak = all & ~strong;
                while (weak) {
                    const int c = __ffsll((unsigned long long)weak);
                    weak &= weak - 1;
                    double km = 0.0;
#pragma unroll
                    for (int j = 0; j < 32; ++j) {
                        const double key = __builtin_amdgcn_fract(__builtin_amdgcn_ldexp(v[j], -c));
                        km = key > km ? key : km;
                    }
                    km = wave_max(km);
                    if (lane == 0) atomicMax(&s_key64[B - c], (unsigned long long)__double_as_longlong(km));
                }
            }
            // mag = hi:lo (0 when tiny), converted afresh: reusing the key
            // pass's conversions would keep 64 more registers alive through it
#pragma unroll
            for (int j = 0; j < 32; ++j) {
                asm volatile("" : "+v"(v[j]));
                const double yh = __builtin_trunc(v[j] * 0x1p-32);
                hi[j] = (uint32_t)yh;
                lo[j] = (uint32_t)(v[j] - yh * 0x1p32);
            }
        } else {
            // Cut c = B - k (k = 1..B-1) is bit c-1 of y; k = B is the fraction
            // itself (frac_max).  A value can raise the running maximum M_c only
            // if its key exceeds M_c; when M_c has t leading ones (M_c >= 1 - 2^-t)
            // that needs bits c-1 .. c-t of y to be ones.  Each cut is tested with
            // the longest run in {12, 8, 4, 2, 1} that its M_c allows; cuts with
            // M_c < 1/2 take the direct maximum.  Lane l decides cut l+1.
            uint32_t S1, S2, S4, S8, S12;
            if (t == t0 && B > 1) {
                // Seed the workgroup's running maxima before its first tile:
                // lane l takes the exact maximum over its own 32 values for
                // one cut, so every cut starts from the largest of about 256
                // actual keys.  Without it every cut would take the direct
                // maximum below (about three times the work of a pruned tile);
                // seeds are keys of actual values, so the pruning stays exact.
                const int c = (int)(lane % (B - 1)) + 1;
                float km = 0.0f;
#pragma unroll
                for (int j = 0; j < 32; ++j)
                    km = fmaxf(km, __builtin_amdgcn_fractf(__builtin_amdgcn_ldexpf(v[j], -c)));
                atomicMax(&s_key32[B - c], __float_as_uint(km));
                __syncthreads();
            }
            {
                const uint32_t c = lane + 1;
                uint32_t tl = 0;
                if (c < B) {
                    const float M = __uint_as_float(s_key32[B - c]);
                    if (M >= 0.5f) tl = __clz(~(uint32_t)(M * 0x1p32f));
                }
                const bool live = c < B;
                S12 = (uint32_t)__ballot(live && tl >= 12);
                S8 = (uint32_t)__ballot(live && tl >= 8 && tl < 12);
                S4 = (uint32_t)__ballot(live && tl >= 4 && tl < 8);
                S2 = (uint32_t)__ballot(live && tl >= 2 && tl < 4);
                S1 = (uint32_t)__ballot(live && tl == 1);
            }
            const uint32_t strong = S1 | S2 | S4 | S8 | S12;
            auto one = [&](float y) {
                const float f = __builtin_amdgcn_fractf(y);
                frac_max = max(frac_max, __float_as_uint(f));
                asm volatile("" : "+v"(frac_max));  // fold in now, not at the end
                const uint64_t Y = ((uint64_t)(uint32_t)y << 32) | (uint32_t)(f * 0x1p32f);
                const uint64_t r2 = Y & (Y << 1);    // bit p: bits p, p-1 are ones
                const uint64_t r4 = r2 & (r2 << 2);  // p .. p-3
                const uint64_t r8 = r4 & (r4 << 4);  // p .. p-7
                const uint64_t r12 = r8 & (r8 << 4); // p .. p-11
                uint32_t cand = ((uint32_t)(Y >> 32) & S1) | ((uint32_t)(r2 >> 32) & S2) |
                                ((uint32_t)(r4 >> 32) & S4) | ((uint32_t)(r8 >> 32) & S8) |
                                ((uint32_t)(r12 >> 32) & S12);
                while (cand) {
                    const int c = __ffs(cand);  // 1-based bit index == cut
                    cand &= cand - 1;
                    const float key = __builtin_amdgcn_fractf(__builtin_amdgcn_ldexpf(y, -c));
                    atomicMax(&s_key32[B - c], __float_as_uint(key));
                }
            };
#pragma unroll
            for (int j = 0; j < 32; ++j) one(v[j]);
            const uint32_t all = (1u << (B - 1)) - 1u;  // cuts 1 .. B-1
            uint32_t weak = all & ~strong;
            while (weak) {
                const int c = __ffs(weak);
                weak &= weak - 1;
                float km = 0.0f;
#pragma unroll
                for (int j = 0; j < 32; ++j)
                    km = fmaxf(km, __builtin_amdgcn_fractf(__builtin_amdgcn_ldexpf(v[j], -c)));
                km = wave_max(km);
                if (lane == 0) atomicMax(&s_key32[B - c], __float_as_uint(km));
            }
        }

        if constexpr (!F64) {
            // mag = floor(y) (0 when tiny), converted afresh: reusing the key
            // loop's conversions would keep 32 more registers alive through it
#pragma unroll
            for (int j = 0; j < 32; ++j) {
                asm volatile("" : "+v"(v[j]));
                lo[j] = (uint32_t)v[j];
            }
        }
        // ---- bit transpose: lo[c] (and hi[c]) become the plane words of bit c (32 + c);
        // row 0 = sign, row r >= 1 = plane r-1 = bit B-r
        transpose32(lo);
        if constexpr (F64) transpose32(hi);
        if constexpr (FAST && F64) {
            // row r (0..64) is sgn, hi[32 - r] (r <= 32) or lo[64 - r]; unit
            // of row r is (r + 3) / 4.  Lanes l and l + 32 hold the halves of
            // the wave's W-bit word l (l < 32), so the same half of the
            // previous word comes by one wave shift.  At the wave's left edge:
            // lanes 0 and 32 (its first word) and 31 and 63 (its last) leave
            // their words in LDS, and after the tile's barrier lane r of each
            // wave compares row r of its first word with the left wave's last
            // (wave 0: wave 3 of the previous tile), so the row loop reads no LDS.
            const uint32_t wave = tid >> 6, h = lane >> 5, lw32 = lane & 31u;
            const uint32_t par = (t - t0) & 3;  // edge buffers in use, as for f32
#define MDR_ROW64(r) ((r) == 0 ? sgn : ((r) <= 32 ? hi[32 - (r)] : lo[64 - (r)]))
            if (lw32 == 0 || lw32 == 31) {
                uint32_t* dst = lw32 == 0 ? &s_first64[par][wave][h][0] : &s_last64[par][wave][h][0];
#pragma unroll
                for (int r = 0; r <= 64; ++r) dst[r] = MDR_ROW64(r);
            }
            if (t == t0 && wave == 0 && lw32 == 0) {
#pragma unroll
                for (int r = 0; r <= 64; ++r) recs[((uint64_t)wg * kMaxRows + r) * 4 + h] = MDR_ROW64(r);
            }
            if (valid && blk + 2 > last_blk) {
#pragma unroll
                for (int r = 0; r <= 64; ++r)
                    recs[((uint64_t)wg * kMaxRows + r) * 4 + 2 + (blk + 1 - last_blk)] = MDR_ROW64(r);
            }
            __syncthreads();  // edges written; every thread is done with its y values
            {
                // the wave's first word against its left neighbour; the range's
                // first word (wave 0 of its first tile) has none
                const uint32_t first_blk = t * kTileBlocks + wave * 64;
                if (first_blk < nbd && (wave > 0 || t > t0)) {
                    const uint32_t lp = wave ? par : ((par + 3) & 3), lwv = wave ? wave - 1 : 3;
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh) {
                        const uint32_t r = lane + 64u * hh;
                        if (r <= 64) {
                            const bool ne = s_first64[par][wave][0][r] != s_last64[lp][lwv][0][r] ||
                                            s_first64[par][wave][1][r] != s_last64[lp][lwv][1][r];
                            edge_trc[hh] += ne ? 1u : 0u;
                        }
                    }
                }
            }
            const uint32_t zsink = (256u + lane) * 4u;  // this lane's sink, bytes past a unit's bins
            auto rows_out = [&](auto full_tile) {
                constexpr bool FULL = decltype(full_tile)::value;
                uint64_t rb = reinterpret_cast<uint64_t>(job.rows);
                asm volatile("" : "+s"(rb));
                const uint32_t boff = blk * 4u;
                // lanes whose word has a left neighbour in the wave
                const unsigned long long keep = __ballot((FULL || valid) && lw32 != 0);
                uint32_t ucnt = 0;  // the current unit's transitions (wave-wide)
#pragma unroll
                for (int r = 0; r <= 64; ++r) {
                    const uint32_t w = MDR_ROW64(r);
                    const int unit = (r + 3) / 4;
                    if (FULL || valid) {
                        *gmem(reinterpret_cast<uint32_t*>(rb + boff)) = w;
                        // nonzero bytes into the unit's bins, zero bytes into this
                        // lane's sink slot after them (no branches)
                        uint8_t* hb = reinterpret_cast<uint8_t*>(&s_hist_fast[unit * HSTRIDE]);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const uint32_t byte = (w >> (8 * q)) & 0xFFu;
                            atomicAdd(reinterpret_cast<uint32_t*>(hb + (byte ? byte * 4u : zsink)), 1u);
                        }
                    }
                    // the same half of the previous word: one wave_shr:1 (lanes 0
                    // and 32 compare at the edge above instead)
                    const int p1 = __builtin_amdgcn_update_dpp((int)w, (int)w, 0x138, 0xF, 0xF, false);
                    const unsigned long long ne = __ballot((int)w != p1) & keep;
                    // a word differs if either half does; a unit's count goes to
                    // its first row's slot (the selection sums a unit's rows)
                    ucnt += (uint32_t)__popc((uint32_t)ne | (uint32_t)(ne >> 32));
                    if (r == 0 || r % 4 == 0) {
                        if (lane == 0 && ucnt) atomicAdd(&s_trans[r == 0 ? 0 : r - 3], ucnt);
                        ucnt = 0;
                    }
                    rb += 4ull * nbd;
                }
            };
            if ((t + 1) * kTileBlocks <= nbd)
                rows_out(std::true_type{});
            else
                rows_out(std::false_type{});
#undef MDR_ROW64
            continue;
        } else if constexpr (FAST) {
            // row r (0..32) is sgn or lo[32 - r]; unit of row r is (r + 3) / 4
            const uint32_t wave = tid >> 6;
            // four buffers: without a barrier at the top of the tile, a wave can
            // be one tile ahead of another, never two (the edge barrier below)
            const uint32_t par = (t - t0) & 3;
            if (lane == 63) {
                s_edge[par][wave][0] = sgn;
#pragma unroll
                for (int r = 1; r <= 32; ++r) s_edge[par][wave][r] = lo[32 - r];
            }
            if (t == t0 && tid == 0) {
                // the first block of the range has no left neighbour: it sees its
                // own words there (no transition).  Slot 3 of wave 3 is next
                // written three tiles later, after this tile's barrier.
                s_edge[3][3][0] = sgn;
#pragma unroll
                for (int r = 1; r <= 32; ++r) s_edge[3][3][r] = lo[32 - r];
                recs[((uint64_t)wg * kMaxRows) * 2] = sgn;
#pragma unroll
                for (int r = 1; r <= 32; ++r) recs[((uint64_t)wg * kMaxRows + r) * 2] = lo[32 - r];
            }
            __syncthreads();  // edges written; every thread is done with its y values
            const uint32_t* edge = wave ? &s_edge[par][wave - 1][0] : &s_edge[(par + 3) & 3][3][0];
            if (valid && blk == last_blk) {
                recs[((uint64_t)wg * kMaxRows) * 2 + 1] = sgn;
#pragma unroll
                for (int r = 1; r <= 32; ++r) recs[((uint64_t)wg * kMaxRows + r) * 2 + 1] = lo[32 - r];
            }
            // per row: coalesced store, nonzero bytes into the unit's histogram
            // (zero bytes are counted by difference later), and a transition
            // against the left neighbour's word, which the wave shift brings
            // from lane l-1 (lane 0: the previous wave's last word)
            auto rows_out = [&](auto full_tile) {
                constexpr bool FULL = decltype(full_tile)::value;
                // row base in scalar registers, advanced per row (kept out of the
                // tile loop's invariants, which would not fit), plus a 32-bit
                // byte offset: a level holds < 2^32 values, so blk * 4 < 2^29
                uint64_t rb = reinterpret_cast<uint64_t>(job.rows);
                asm volatile("" : "+s"(rb));
                const uint32_t boff = blk * 4u;
#pragma unroll
                for (int r = 0; r <= 32; ++r) {
                    const uint32_t w = r == 0 ? sgn : lo[32 - r];
                    const int unit = (r + 3) / 4;
                    if (FULL || valid) {
                        *gmem(reinterpret_cast<uint32_t*>(rb + boff)) = w;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const uint32_t byte = (w >> (8 * q)) & 0xFFu;
                            if (byte) atomicAdd(&s_hist_fast[unit * 256 + byte], 1u);
                        }
                    }
                    // wave_shr:1 (lane l <- lane l-1); lane 0 keeps `old`
                    const uint32_t nb = (uint32_t)__builtin_amdgcn_update_dpp((int)edge[r], (int)w, 0x138, 0xF, 0xF, false);
                    trc[unit] += ((FULL || valid) && w != nb) ? 1u : 0u;
                    rb += 4ull * nbd;
                }
            };
            if ((t + 1) * kTileBlocks <= nbd)
                rows_out(std::true_type{});
            else
                rows_out(std::false_type{});
            continue;
        }
        // Rows go through LDS in passes of at most kPassRows (f64's 65 rows in
        // two), so that two f64 workgroups fit a CU.
        const uint32_t nrows = B + 1;
        const uint32_t npass = nrows > kPassRows ? 2u : 1u;
        const uint32_t per = (nrows + npass - 1) / npass;
        const bool have_prev = t > t0;
        const bool lead = valid && (tid % G) == 0 && (tid >= G || have_prev);
        for (uint32_t pass = 0; pass < npass; ++pass) {
            const uint32_t rlo = pass * per, rhi = min(nrows, rlo + per);
            __syncthreads();  // every thread is done with its y values / the previous pass's rows
            if (rlo == 0) s_pl[tid] = sgn;
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                const uint32_t r = B - (uint32_t)c;  // row of bit c (when c < B)
                if (c < (int)B && r >= rlo && r < rhi) s_pl[(r - rlo) * kTileBlocks + tid] = lo[c];
            }
            if constexpr (F64) {
#pragma unroll
                for (int c = 0; c < 32; ++c) {
                    const uint32_t r = B - 32u - (uint32_t)c;  // row of bit 32 + c
                    if (32 + c < (int)B && r >= rlo && r < rhi) s_pl[(r - rlo) * kTileBlocks + tid] = hi[c];
                }
            }
            __syncthreads();

            // ---- per row: coalesced store, byte histogram, word transitions.
            // Rows go four at a time so their LDS reads overlap; zero bytes are
            // counted by difference later and go to this thread's sink slot here.
            for (uint32_t r0 = rlo; r0 < rhi; r0 += 4) {
                uint32_t w[4], pv[4], pv1[4], nx[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t r = min(r0 + i, rhi - 1);
                    const uint32_t* row = s_pl + (r - rlo) * kTileBlocks;
                    w[i] = row[tid];
                    pv[i] = tid >= G ? row[tid - G] : s_prev[r][tid];
                    if constexpr (G == 2) {
                        nx[i] = row[tid + 1 < kTileBlocks ? tid + 1 : tid];
                        pv1[i] = tid >= G ? row[tid - 1] : s_prev[r][1];
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t r = r0 + i;
                    if (r >= rhi) break;
                    if (valid) {
                        rows[(uint64_t)r * nbd + blk] = w[i];
                        uint32_t* h = s_hist + s_hoff[r];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const uint32_t byte = (w[i] >> (8 * q)) & 0xFFu;
                            atomicAdd(byte ? &h[byte] : &s_zero[tid], 1u);
                        }
                    }
                    bool flag = w[i] != pv[i];
                    if constexpr (G == 2) flag = flag || nx[i] != pv1[i];
                    unsigned long long bal = __ballot(lead && flag);
                    if (lane == 0 && bal) atomicAdd(&s_trans[r], (uint32_t)__popcll(bal));
                }
            }
            // first / last words of this workgroup's range, for the boundaries
            if (t == t0 && tid < G)
                for (uint32_t r = rlo; r < rhi; ++r)
                    recs[((uint64_t)wg * kMaxRows + r) * 2 * G + tid] = s_pl[(r - rlo) * kTileBlocks + tid];
            if (valid && blk + G > last_blk)
                for (uint32_t r = rlo; r < rhi; ++r)
                    recs[((uint64_t)wg * kMaxRows + r) * 2 * G + G + (blk - (last_blk + 1 - G))] =
                        s_pl[(r - rlo) * kTileBlocks + tid];
            __syncthreads();
            if (tid >= kTileBlocks - G)
                for (uint32_t r = rlo; r < rhi; ++r)
                    s_prev[r][tid - (kTileBlocks - G)] = s_pl[(r - rlo) * kTileBlocks + tid];
        }
        (void)NROW;
    }

    // ---- flush: per-workgroup partials (reduced by the selection kernel)
    if constexpr (FAST && F64) {
        // the rows' counts are in their slots already; the edge counts go to their row's
        if (edge_trc[0]) atomicAdd(&s_trans[lane], edge_trc[0]);
        if (lane == 0 && edge_trc[1]) atomicAdd(&s_trans[64], edge_trc[1]);
    } else if constexpr (FAST) {
        // a unit's transitions go to its first row's slot (the selection sums a unit's rows)
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            uint32_t v = trc[i];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0 && v) atomicAdd(&s_trans[i == 0 ? 0 : 1 + (i - 1) * 4], v);
        }
    }
    small = wave_max(small);
    if constexpr (F64) {
        frac_max64 = wave_max(frac_max64);
        if (lane == 0) {
            atomicMax(&s_key64[B], (unsigned long long)frac_max64);
            atomicMax(&s_key64[kKeyStride - 1], (unsigned long long)__double_as_longlong(small));
        }
    } else {
        frac_max = wave_max(frac_max);
        if (lane == 0) {
            atomicMax(&s_key32[B], frac_max);
            atomicMax(&s_key32[kKeyStride - 1], __float_as_uint(small));
        }
    }
    __syncthreads();
    // fold this workgroup's results into the level totals (zeroed before the
    // pass): key maxima (nonnegative float bits order as integers), nonzero
    // byte counts and transitions
    if (tid < kKeyStride) {
        const unsigned long long kv = F64 ? s_key64[tid] : (unsigned long long)s_key32[tid];
        if (kv) atomicMax(&job.keys[tid], kv);
    }
    for (uint32_t i = tid; i < nunits * 256; i += kThreads) {
        const uint32_t hv = s_hist[FAST ? (i >> 8) * HSTRIDE + (i & 255u) : i];
        if (hv) atomicAdd(&job.hist[i], hv);
    }
    if (tid < kMaxRows && s_trans[tid]) atomicAdd(&job.trans[tid], s_trans[tid]);
}

// f32 fits five waves per SIMD (96 registers) with LDS to spare; f64 two
// (256 registers, without spills: left alone the compiler takes 259 and one)
template <bool VEC, bool FAST>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_encode_f32(
    const EncodeJob* __restrict__ jobs, const uint32_t* __restrict__ wg_job)
{
    const EncodeJob& job = jobs[wg_job[blockIdx.x]];
    encode_body<false, VEC, FAST>(job, blockIdx.x - job.wg_base);
}

template <bool VEC, bool FAST>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_encode_f64(
    const EncodeJob* __restrict__ jobs, const uint32_t* __restrict__ wg_job)
{
    const EncodeJob& job = jobs[wg_job[blockIdx.x]];
    encode_body<true, VEC, FAST>(job, blockIdx.x - job.wg_base);
}

// the f64 fast path: two waves per SIMD (up to 256 registers); at four (128
// registers) it spilled and ran 12% slower, at three (168) within 4% of two
template <bool VEC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_encode_f64_fast(
    const EncodeJob* __restrict__ jobs, const uint32_t* __restrict__ wg_job)
{
    const EncodeJob& job = jobs[wg_job[blockIdx.x]];
    encode_body<true, VEC, true>(job, blockIdx.x - job.wg_base);
}

// ------------------------------------------------------------------ hybrid selection
// One workgroup of NT threads per (unit, level) (Alg. 2): gather the byte
// histogram and the run count, build length-limited Huffman code lengths with
// the two-queue construction, canonical codes, both size estimates, and the
// method decision.  Units that Alg. 2 can only copy (S <= T_s) skip the codebook.
// NT = 256, 512 or 1024 threads (a launch knob): the tree is built on one
// lane, so smaller workgroups let more units build theirs at once (a batch of
// many variables has thousands; 1024 threads made such a batch's selection 3x
// slower than 512), while the histogram and rank steps of a few large units
// go faster with more threads (256 made a single field's 20 % slower).
template <int NT>
__global__ __launch_bounds__(NT) void k_select(const SelectParams job,
                                                         const SelectLevel* __restrict__ levels)
{
    __shared__ unsigned long long s_f[256];     // working counts (halved when limiting)
    __shared__ unsigned long long s_f0[256];    // original counts
    __shared__ unsigned long long s_w[512];
    __shared__ int s_parent[512];
    __shared__ int s_sorted[256];
    __shared__ int s_dp[1024];  // depths and parents while measuring the tree
    __shared__ uint8_t s_len[256];
    __shared__ unsigned long long s_red[NT / 64];
    __shared__ int s_nl, s_maxlen;
    __shared__ uint32_t s_count[33], s_first[33];

    const SelectLevel& lv = levels[blockIdx.y];
    const uint32_t u = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t B = job.B, m = job.m, G = job.G, grid = lv.grid;
    const uint32_t r0 = u == 0 ? 0 : 1 + (u - 1) * m;
    const uint32_t r1 = u == 0 ? 1 : min(B + 1, r0 + m);
    const uint64_t S = (uint64_t)(r1 - r0) * lv.nbd * 4;
    if (lv.nbd == 0) {
        // empty level: no planes; every unit is an empty stream of the forced
        // method (direct copy under Alg. 2)
        if (tid < 256) {
            lv.lens[u * 256 + tid] = 0;
            lv.codes[u * 256 + tid] = 0;
        }
        if (tid == 0) {
            UnitInfo ui;
            ui.S = 0;
            ui.est_huf = 8 + 256 + 4;
            ui.est_rle = 8;
            ui.nruns = 0;
            ui.method = job.force_method >= 0 ? (uint32_t)job.force_method : 0u;
            ui.nchunks = 0;
            ui.maxlen = 0;
            ui.pad = 0;
            lv.units[u] = ui;
        }
        return;
    }

    auto block_sum = [&](unsigned long long v) -> unsigned long long {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) s_red[wave] = v;
        __syncthreads();
        unsigned long long t = 0;
        for (int w = 0; w < NT / 64; ++w) t += s_red[w];
        __syncthreads();
        return t;
    };

    // ---- byte histogram (level totals from the encoder)
    unsigned long long f = tid < 256 ? lv.hist[(uint64_t)u * 256 + tid] : 0;
    unsigned long long nz = block_sum((tid > 0 && tid < 256) ? f : 0);
    if (tid == 0) f = S - nz;  // zero bytes are not counted by the encoder
    if (tid < 256) {
        s_f[tid] = f;
        s_f0[tid] = f;
    }

    // ---- runs of equal W-bit words: transitions inside workgroup ranges (level
    // totals from the encoder), at range boundaries, and between consecutive
    // planes of the group
    const uint32_t nrow = r1 - r0;
    unsigned long long tr = tid < nrow ? lv.trans[r0 + tid] : 0;
    {
        // boundary i: first word(s) of range w = 1 + i / nrow against the last
        // of range w - 1, row r0 + i % nrow; four boundaries per thread in flight
        const auto recs = gmem(lv.recs);
        const uint32_t nbnd = (grid - 1) * nrow;
        for (uint32_t i0 = tid; i0 < nbnd; i0 += 4 * NT) {
            uint32_t cw[4][2], pw[4][2];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t i = min(i0 + k * NT, nbnd - 1);
                const uint32_t w = 1 + i / nrow, r = r0 + i % nrow;
                const uint64_t cur = ((uint64_t)w * kMaxRows + r) * 2 * G;
                const uint64_t prv = ((uint64_t)(w - 1) * kMaxRows + r) * 2 * G;
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    cw[k][g] = g < (int)G ? recs[cur + g] : 0u;
                    pw[k][g] = g < (int)G ? recs[prv + G + g] : 0u;
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (i0 + k * NT < nbnd) tr += (cw[k][0] != pw[k][0] || cw[k][1] != pw[k][1]) ? 1 : 0;
        }
    }
    for (uint32_t r = r0 + 1 + tid; r < r1; r += NT) {
        const uint32_t* cur = lv.recs + ((uint64_t)0 * kMaxRows + r) * 2 * G;
        const uint32_t* prv = lv.recs + ((uint64_t)(grid - 1) * kMaxRows + (r - 1)) * 2 * G;
        bool ne = false;
        for (uint32_t g = 0; g < G; ++g) ne = ne || cur[g] != prv[G + g];
        tr += ne ? 1 : 0;
    }
    const unsigned long long trans = block_sum(tr);
    const unsigned long long nruns = S ? 1 + trans : 0;

    const bool need_code = job.force_method == 2 || (job.force_method < 0 && S > job.t_s);
    if (tid < 256) s_len[tid] = 0;
    if (tid == 0) s_maxlen = 0;
    __syncthreads();

    // ---- Huffman code lengths: two-queue tree, depths by pointer jumping, and
    // the per-length count adjustment when the tree is deeper than huf_lmax
    if (need_code) {
        // rank of each present symbol in (count, symbol) order: kRankParts
        // threads per symbol, 256 / kRankParts comparisons each
        {
            constexpr uint32_t kRankParts = NT / 256;
            constexpr int kSpan = 256 / kRankParts;
            const uint32_t sym = tid & 255, part = tid >> 8;
            const unsigned long long fsym = s_f[sym];
            if (tid < 256) s_dp[tid] = 0;
            if (tid == 0) s_nl = 0;
            __syncthreads();
            if (fsym) {
                int r = 0;
#pragma unroll 16
                for (int q = (int)part * kSpan; q < (int)part * kSpan + kSpan; ++q) {
                    const unsigned long long fs = s_f[q];
                    r += (fs && (fs < fsym || (fs == fsym && q < (int)sym))) ? 1 : 0;
                }
                if (r) atomicAdd(&s_dp[sym], r);
            }
            __syncthreads();
        }
        const unsigned long long ft = tid < 256 ? s_f[tid] : 0;
        const int rank = tid < 256 ? s_dp[tid] : 0;
        __syncthreads();
        if (tid < 256 && ft) {
            s_sorted[rank] = (int)tid;
            atomicAdd(&s_nl, 1);
        }
        __syncthreads();
        const int nl = s_nl;
        if (tid < nl) s_w[tid] = s_f[s_sorted[tid]];
        __syncthreads();
        if (tid == 0 && nl > 1) {
            // leaves s_w[0, nl) ascending, merged nodes appended from nl; the
            // two heads of each queue live in registers (an empty slot holds
            // ~0, above any weight) and are refilled from LDS one pick ahead.
            // A tie takes the leaf.
            constexpr unsigned long long kNone = ~0ull;
            int q1 = 0, q2 = nl, next = nl;
            unsigned long long l0 = s_w[0], l1 = s_w[1], i0 = kNone, i1 = kNone;
            auto pick = [&](unsigned long long& wt) -> int {
                int at;
                if (l0 <= i0) {
                    at = q1++;
                    wt = l0;
                    l0 = l1;
                    l1 = q1 + 1 < nl ? s_w[q1 + 1] : kNone;
                } else {
                    at = q2++;
                    wt = i0;
                    i0 = i1;
                    i1 = q2 + 1 < next ? s_w[q2 + 1] : kNone;
                }
                return at;
            };
            while ((nl - q1) + (next - q2) > 1) {
                unsigned long long wa, wb;
                const int a = pick(wa);
                const int b = pick(wb);
                const unsigned long long sum = wa + wb;
                s_w[next] = sum;
                s_parent[a] = next;
                s_parent[b] = next;
                if (q2 == next)
                    i0 = sum;
                else if (q2 + 1 == next)
                    i1 = sum;
                ++next;
            }
            s_parent[next - 1] = next - 1;  // the root points to itself
        }
        __syncthreads();
        // depth of every node: d <- d + d[parent], parent <- parent[parent] (9 rounds for 511 nodes)
        const int nnodes = nl > 1 ? 2 * nl - 1 : 0;
        int* s_d = s_dp;
        int* s_p = s_dp + 512;
        constexpr int kNodesPer = (512 + NT - 1) / NT;  // nodes per thread
#pragma unroll
        for (int h = 0; h < kNodesPer; ++h) {
            const int v = (int)tid + h * NT;
            if (v < nnodes) {
                s_p[v] = s_parent[v];
                s_d[v] = (v == nnodes - 1) ? 0 : 1;
            }
        }
        __syncthreads();
        for (int round = 0; round < 9; ++round) {
            int nd[kNodesPer], np[kNodesPer];
#pragma unroll
            for (int h = 0; h < kNodesPer; ++h) {
                const int v = (int)tid + h * NT;
                nd[h] = 0, np[h] = 0;
                if (v < nnodes) {
                    const int p = s_p[v];
                    nd[h] = s_d[v] + s_d[p];
                    np[h] = s_p[p];
                }
            }
            __syncthreads();
#pragma unroll
            for (int h = 0; h < kNodesPer; ++h) {
                const int v = (int)tid + h * NT;
                if (v < nnodes) {
                    s_d[v] = nd[h];
                    s_p[v] = np[h];
                }
            }
            __syncthreads();
        }
        if (tid == 0 && nl == 1) {
            int s0 = s_sorted[0];
            s_len[s0] = 1;
            s_len[s0 == 0 ? 1 : 0] = 1;
            s_maxlen = 1;
        }
        if (nl > 1 && tid < nl) atomicMax(&s_maxlen, s_d[tid]);  // leaves are nodes 0 .. nl-1
        __syncthreads();
        if (nl > 1 && s_maxlen <= (int)job.huf_lmax) {
            if (tid < nl) s_len[s_sorted[tid]] = (uint8_t)s_d[tid];
        } else if (nl > 1) {
            // ITU-T T.81 Annex K count adjustment on one lane, then hand the
            // lengths out again: heaviest leaf (last in sorted order) shortest
            uint32_t* s_bits = reinterpret_cast<uint32_t*>(s_parent);  // 256+1 entries
            for (uint32_t i = tid; i <= 256; i += NT) s_bits[i] = 0;
            __syncthreads();
            if (tid < nl) atomicAdd(&s_bits[s_d[tid]], 1u);
            __syncthreads();
            const int maxlen = s_maxlen;
            if (maxlen < 64) {
                // one wavefront, lane l holding the count of length l; j is the
                // longest length below i - 1 with a code
                if (wave == 0) {
                    int b = (int)s_bits[lane];
                    for (int i = maxlen; i > (int)job.huf_lmax; --i) {
                        while (__builtin_amdgcn_readlane(b, i) > 0) {
                            const unsigned long long nzm = __ballot(b != 0) & ((1ull << (i - 1)) - 1);
                            if (!nzm) break;  // cannot happen for a full tree
                            const int j = 63 - __clzll((long long)nzm);
                            const int l = (int)lane;
                            b += (l == i ? -2 : 0) + (l == i - 1 ? 1 : 0) + (l == j + 1 ? 2 : 0) + (l == j ? -1 : 0);
                        }
                    }
                    s_bits[lane] = (uint32_t)b;
                }
            } else if (tid == 0) {
                for (int i = maxlen; i > (int)job.huf_lmax; --i) {
                    while (s_bits[i] > 0) {
                        int j = i - 2;
                        while (s_bits[j] == 0) --j;
                        s_bits[i] -= 2;
                        s_bits[i - 1] += 1;
                        s_bits[j + 1] += 2;
                        s_bits[j] -= 1;
                    }
                }
            }
            __syncthreads();
            if (tid == 0) s_maxlen = (int)job.huf_lmax;
            if (tid < nl) {
                const uint32_t pos = (uint32_t)(nl - 1) - tid;  // 0 = heaviest
                uint32_t cum = 0, Lh = 1;
                for (; Lh <= job.huf_lmax; ++Lh) {
                    cum += s_bits[Lh];
                    if (pos < cum) break;
                }
                s_len[s_sorted[tid]] = (uint8_t)Lh;
            }
        }
        __syncthreads();
    }

    // ---- canonical codes: (length, symbol) order
    if (tid < 33) s_count[tid] = 0;
    __syncthreads();
    const uint32_t L = tid < 256 ? s_len[tid] : 0;
    if (L) atomicAdd(&s_count[L], 1u);
    __syncthreads();
    if (tid == 0) {
        uint32_t c = 0;
        for (int l = 1; l <= 32; ++l) {
            s_first[l] = c;
            c = (c + s_count[l]) << 1;
        }
    }
    __syncthreads();
    if (tid < 256) {
        uint32_t code = 0;
        if (L) {
            uint32_t before = 0;
#pragma unroll 16
            for (uint32_t q = 0; q < tid; ++q) before += s_len[q] == L ? 1u : 0u;
            code = s_first[L] + before;
        }
        lv.lens[u * 256 + tid] = (uint8_t)L;
        lv.codes[u * 256 + tid] = code;
    }

    // ---- estimates and the decision
    unsigned long long bits = block_sum(tid < 256 ? s_f0[tid] * (unsigned long long)L : 0);
    if (tid == 0) {
        const uint64_t nchunks = (S + job.huf_chunk - 1) / job.huf_chunk;
        const uint64_t est_huf = need_code ? (bits + 7) / 8 + 8 + 256 + 4 * (nchunks + 1) : 0;
        const uint64_t est_rle = 8 + nruns * (4ull * G + 4);
        uint32_t method;
        if (job.force_method >= 0) {
            method = (uint32_t)job.force_method;
        } else if (S > job.t_s) {
            if (1000ull * S > (uint64_t)job.t_cr_milli * est_huf)
                method = 2;  // MDR_HUF
            else if (1000ull * S > (uint64_t)job.t_cr_milli * est_rle)
                method = 1;  // MDR_RLE
            else
                method = 0;  // MDR_DC
        } else {
            method = 0;
        }
        UnitInfo ui;
        ui.S = S;
        ui.est_huf = est_huf;
        ui.est_rle = est_rle;
        ui.nruns = nruns;
        ui.method = method;
        ui.nchunks = (uint32_t)nchunks;
        ui.maxlen = (uint32_t)s_maxlen;
        ui.pad = 0;
        lv.units[u] = ui;
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers
static unsigned grid_for(uint64_t items, unsigned per_block, unsigned cap)
{
    uint64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, kThreads, 4096)), dim3(kThreads), 0, s, p,
                       count, value);
    return hipGetLastError();
}

hipError_t launch_copy_in(void* dst, const void* host, uint64_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    if (bytes % 8) return hipErrorInvalidValue;
    void* src = nullptr;
    hipError_t e = hipHostGetDevicePointer(&src, const_cast<void*>(host), 0);
    if (e != hipSuccess) return e;
    const uint64_t count = bytes / 8;
    hipLaunchKernelGGL(k_copy_in, dim3(grid_for(count, kThreads, 1024)), dim3(kThreads), 0, s,
                       static_cast<const uint64_t*>(src), static_cast<uint64_t*>(dst), count);
    return hipGetLastError();
}

hipError_t launch_init_pass(LevelStats* st, uint32_t count, uint32_t* z0, uint64_t n0, uint32_t* z1,
                            uint64_t n1, hipStream_t s)
{
    const uint64_t most = std::max<uint64_t>(count, std::max(n0, n1));
    if (most == 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_pass, dim3(grid_for(most, kThreads, 4096)), dim3(kThreads), 0, s, st, count, z0,
                       n0, z1, n1);
    return hipGetLastError();
}

hipError_t launch_stats_batch(const StatsJob* jobs, const uint32_t* wg_job, uint32_t grid, bool f64,
                              bool vec, hipStream_t s)
{
    if (grid == 0) return hipSuccess;
    if (f64) {
        if (vec)
            hipLaunchKernelGGL((k_stats<true, true>), dim3(grid), dim3(kStatsThreads), 0, s, jobs, wg_job);
        else
            hipLaunchKernelGGL((k_stats<true, false>), dim3(grid), dim3(kStatsThreads), 0, s, jobs, wg_job);
    } else {
        if (vec)
            hipLaunchKernelGGL((k_stats<false, true>), dim3(grid), dim3(kStatsThreads), 0, s, jobs, wg_job);
        else
            hipLaunchKernelGGL((k_stats<false, false>), dim3(grid), dim3(kStatsThreads), 0, s, jobs, wg_job);
    }
    return hipGetLastError();
}

size_t encode_lds_bytes(uint32_t nunits, uint32_t B, uint32_t m, bool f64)
{
    if ((!f64 && B == 32 && m == 4) || (f64 && B == 64 && m == 4)) return 0;  // the fast paths: static LDS only
    const uint32_t npass = B + 1 > kPassRows ? 2u : 1u;  // as the kernel stages its rows
    const size_t planes = (size_t)((B + 1 + npass - 1) / npass) * kTileBlocks * sizeof(uint32_t);
    return (size_t)nunits * 256 * sizeof(uint32_t) + planes;
}

hipError_t encode_set_lds(uint32_t nunits, uint32_t B, uint32_t m, bool f64)
{
    const size_t shmem = encode_lds_bytes(nunits, B, m, f64);
    if (shmem <= 64 * 1024) return hipSuccess;  // the fast path always fits
    const void* fns[2] = {f64 ? (const void*)k_encode_f64<true, false> : (const void*)k_encode_f32<true, false>,
                          f64 ? (const void*)k_encode_f64<false, false> : (const void*)k_encode_f32<false, false>};
    for (const void* fn : fns) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_encode_batch(const EncodeJob* jobs, const uint32_t* wg_job, uint32_t grid,
                               uint32_t nunits, uint32_t B, uint32_t m, bool f64, bool vec, hipStream_t s)
{
    const bool fast = (!f64 && B == 32 && m == 4) || (f64 && B == 64 && m == 4);
    if (grid == 0) return hipSuccess;
    const size_t shmem = encode_lds_bytes(nunits, B, m, f64);
    dim3 g(grid), b(kThreads);
    if (f64) {
        if (fast) {
            if (vec)
                hipLaunchKernelGGL((k_encode_f64_fast<true>), g, b, shmem, s, jobs, wg_job);
            else
                hipLaunchKernelGGL((k_encode_f64_fast<false>), g, b, shmem, s, jobs, wg_job);
        } else {
            if (vec)
                hipLaunchKernelGGL((k_encode_f64<true, false>), g, b, shmem, s, jobs, wg_job);
            else
                hipLaunchKernelGGL((k_encode_f64<false, false>), g, b, shmem, s, jobs, wg_job);
        }
    } else {
        if (fast) {
            if (vec)
                hipLaunchKernelGGL((k_encode_f32<true, true>), g, b, shmem, s, jobs, wg_job);
            else
                hipLaunchKernelGGL((k_encode_f32<false, true>), g, b, shmem, s, jobs, wg_job);
        } else {
            if (vec)
                hipLaunchKernelGGL((k_encode_f32<true, false>), g, b, shmem, s, jobs, wg_job);
            else
                hipLaunchKernelGGL((k_encode_f32<false, false>), g, b, shmem, s, jobs, wg_job);
        }
    }
    return hipGetLastError();
}

hipError_t launch_select_batch(const SelectParams& p, const SelectLevel* lv, uint32_t nlev,
                               hipStream_t s)
{
    if (nlev == 0) return hipSuccess;
    const dim3 g(p.nunits, nlev);
    if (p.threads == 256)
        hipLaunchKernelGGL(k_select<256>, g, dim3(256), 0, s, p, lv);
    else if (p.threads == 1024)
        hipLaunchKernelGGL(k_select<1024>, g, dim3(1024), 0, s, p, lv);
    else
        hipLaunchKernelGGL(k_select<512>, g, dim3(512), 0, s, p, lv);
    return hipGetLastError();
}

}  // namespace mdr
