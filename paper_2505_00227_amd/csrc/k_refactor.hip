// Refactor kernels for gfx950: level statistics, bitplane encoding with the
// per-plane error table and per-group lossless statistics, and the device-side
// hybrid selection of Alg. 2 (Sec. 4.2) with its Huffman codebook.
#include <climits>
#include <type_traits>

#include "device_bits.hpp"
#include "mdr_internal.hpp"

namespace mdr {
namespace {

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

__global__ void k_init_stats(LevelStats* st, int count)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    st[i].emax = INT_MIN;
    st[i].nonfinite = 0;
    st[i].minkey = ~0ull;
    st[i].maxkey = 0;
    st[i].maxabs_bits = 0;
    st[i].small_bits = 0;
}

// ------------------------------------------------------------------ level statistics
// One streaming pass: largest frexp exponent of the nonzero values (Alg. 1's
// alignment exponent), min / max / max|x|, and a non-finite flag.
template <bool F64>
__global__ __launch_bounds__(kThreads) void k_stats(const void* xv, uint64_t n, LevelStats* st)
{
    using U = std::conditional_t<F64, uint64_t, uint32_t>;
    const U* x = static_cast<const U*>(xv);
    int emax = INT_MIN;
    uint32_t bad = 0;
    uint64_t kmin = ~0ull, kmax = 0;
    U amax = 0;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        U b = x[i];
        U ab;
        int ex;
        uint64_t key;
        bool finite;
        if constexpr (F64) {
            ab = b & 0x7FFFFFFFFFFFFFFFull;
            finite = ab < 0x7FF0000000000000ull;
            ex = ab ? frexp_exp_f64(ab) : INT_MIN;
            key = order_key_f64(b);
        } else {
            ab = b & 0x7FFFFFFFu;
            finite = ab < 0x7F800000u;
            ex = ab ? frexp_exp_f32(ab) : INT_MIN;
            key = order_key_f32(b);
        }
        if (!finite) {
            bad = 1;
            continue;
        }
        emax = ex > emax ? ex : emax;
        kmin = key < kmin ? key : kmin;
        kmax = key > kmax ? key : kmax;
        amax = ab > amax ? ab : amax;
    }
    emax = wave_max(emax);
    kmin = wave_min(kmin);
    kmax = wave_max(kmax);
    amax = wave_max(amax);
    bad = __any(bad) ? 1u : 0u;
    if ((threadIdx.x & 63) == 0) {
        if (emax != INT_MIN) atomicMax(&st->emax, emax);
        if (bad) atomicOr(&st->nonfinite, 1u);
        atomicMin((unsigned long long*)&st->minkey, (unsigned long long)kmin);
        atomicMax((unsigned long long*)&st->maxkey, (unsigned long long)kmax);
        atomicMax((unsigned long long*)&st->maxabs_bits, (unsigned long long)amax);
    }
}

// ------------------------------------------------------------------ bitplane encoder
// One thread owns one block of 32 consecutive values (one u32 word of every
// plane); a workgroup covers a tile of 256 blocks and walks a contiguous range
// of tiles.  Per block:
//   y = |x| * 2^(B-e) (exact), mag = floor(y), sign bit;
//   error keys: for every k, fract(y * 2^(k-B)) = (|x| mod 2^(e-k)) / 2^(e-k),
//     a running maximum per k (values with mag = 0 lie below every cut: their
//     error is |x| for every k and is tracked separately as `small`);
//   32x32 in-register bit transpose (two of them for f64) -> plane words;
//   coalesced stores of each plane row, per-unit byte histograms (LDS), and
//   counts of W-bit word transitions for the run-length estimate.
template <bool F64, bool VEC>
__global__ __launch_bounds__(kThreads) void k_encode(EncodeJob job)
{
    using T = std::conditional_t<F64, double, float>;
    constexpr int G = F64 ? 2 : 1;  // u32 words per W-bit word
    constexpr int NK = F64 ? 65 : 33;
    extern __shared__ uint32_t s_hist[];  // [nunits][256]
    __shared__ uint32_t s_last[2][4][kMaxRows][G];
    __shared__ uint32_t s_trans[kMaxRows];
    __shared__ unsigned long long s_ek[4][F64 ? kMaxRows : 1];

    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t B = job.B, nbd = job.nbd, m = job.m;
    const uint64_t n = job.n;
    const int e = job.stats->emax == INT_MIN ? 0 : job.stats->emax;
    const T* x = static_cast<const T*>(job.x);

    for (uint32_t i = tid; i < job.nunits * 256; i += kThreads) s_hist[i] = 0;
    if (tid < kMaxRows) s_trans[tid] = 0;
    if constexpr (F64) {
        for (uint32_t i = tid; i < 4 * kMaxRows; i += kThreads) (&s_ek[0][0])[i] = 0;
    }
    __syncthreads();

    float kmax[F64 ? 1 : 33];
#pragma unroll
    for (int k = 0; k < (F64 ? 1 : 33); ++k) kmax[k] = 0.0f;
    T small = 0;

    const uint32_t t0 = blockIdx.x * job.tiles_per_wg;
    const uint32_t t1 = min(job.ntiles, t0 + job.tiles_per_wg);
    const uint32_t last_blk = min(nbd, t1 * kTileBlocks) - 1;

    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t blk = t * kTileBlocks + tid;
        const bool valid = blk < nbd;
        const uint64_t base = (uint64_t)blk * 32;

        // ---- load 32 consecutive values
        T v[32];
        if (VEC && valid && base + 32 <= n) {
            if constexpr (F64) {
                const double2* p = reinterpret_cast<const double2*>(x + base);
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    double2 q = p[j];
                    v[2 * j] = q.x;
                    v[2 * j + 1] = q.y;
                }
            } else {
                const float4* p = reinterpret_cast<const float4*>(x + base);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    float4 q = p[j];
                    v[4 * j] = q.x;
                    v[4 * j + 1] = q.y;
                    v[4 * j + 2] = q.z;
                    v[4 * j + 3] = q.w;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < 32; ++j) v[j] = (valid && base + j < n) ? x[base + j] : T(0);
        }

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
                double yh = __builtin_trunc(y * 0x1p-32);
                uint32_t h = (uint32_t)yh;
                uint32_t l = (uint32_t)(y - yh * 0x1p32);
                bool tiny = (h | l) == 0;
                small = (tiny && a > small) ? a : small;
                v[j] = tiny ? 0.0 : y;
                hi[j] = h;
                lo[j] = l;
            } else {
                uint32_t bits = __float_as_uint(v[j]);
                sgn |= (bits >> 31) << j;
                float a = __uint_as_float(bits & 0x7FFFFFFFu);
                float y = __builtin_amdgcn_ldexpf(a, (int)B - e);
                uint32_t mg = (uint32_t)y;
                bool tiny = mg == 0;
                small = (tiny && a > small) ? a : small;
                v[j] = tiny ? 0.0f : y;
                lo[j] = mg;
            }
        }

        // ---- exact error keys, k = 0..B
        if constexpr (F64) {
            for (int k = 0; k <= (int)B; ++k) {
                double km = 0.0;
#pragma unroll
                for (int j = 0; j < 32; ++j) {
                    double key = __builtin_amdgcn_fract(__builtin_amdgcn_ldexp(v[j], k - (int)B));
                    km = key > km ? key : km;
                }
                km = wave_max(km);
                if (lane == 0) {
                    unsigned long long kb = (unsigned long long)__double_as_longlong(km);
                    if (kb > s_ek[wave][k]) s_ek[wave][k] = kb;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < 33; ++k) {
                if (k <= (int)B) {
                    float km = kmax[k];
#pragma unroll
                    for (int j = 0; j < 32; j += 2) {
                        float k0 = __builtin_amdgcn_fractf(__builtin_amdgcn_ldexpf(v[j], k - (int)B));
                        float k1 = __builtin_amdgcn_fractf(__builtin_amdgcn_ldexpf(v[j + 1], k - (int)B));
                        km = fmaxf(km, fmaxf(k0, k1));
                    }
                    kmax[k] = km;
                }
            }
        }

        // ---- bit transpose: lo[c] (and hi[c]) become the plane words of bit c (32 + c)
        transpose32(lo);
        if constexpr (F64) transpose32(hi);

        // ---- store rows, histogram bytes, remember the last words of this wave
        // row 0 = sign; row r >= 1 = plane r-1 = bit B-r.
        const bool rec_last = valid && blk + G > last_blk;  // lanes holding the range's last word
        const bool rec_first = valid && t == t0 && wave == 0 && lane < G;
        auto emit = [&](uint32_t r, uint32_t w) {
            if (valid) {
                job.rows[(uint64_t)r * nbd + blk] = w;
                uint32_t u = r == 0 ? 0 : 1 + (r - 1) / m;
                uint32_t* h = s_hist + u * 256;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t byte = (w >> (8 * q)) & 0xFFu;
                    if (byte) atomicAdd(&h[byte], 1u);
                }
            }
            if (lane >= 64 - G) s_last[t & 1][wave][r][lane - (64 - G)] = w;
            uint32_t* rec = job.recs + ((uint64_t)blockIdx.x * kMaxRows + r) * 2 * G;
            if (rec_first) rec[lane] = w;
            if (rec_last) rec[G + (blk - (last_blk + 1 - G))] = w;
        };
        emit(0, sgn);
#pragma unroll
        for (int c = 31; c >= 0; --c)
            if (c < (int)B) emit(B - c, lo[c]);
        if constexpr (F64) {
#pragma unroll
            for (int c = 31; c >= 0; --c)
                if (32 + c < (int)B) emit(B - 32 - c, hi[c]);
        }
        __syncthreads();

        // ---- run-length statistics: transitions between consecutive W-bit words
        const bool have_prev = !(t == t0 && wave == 0);
        auto count = [&](uint32_t r, uint32_t w) {
            uint32_t prev = __shfl_up(w, G, 64);
            if (lane < G) {
                if (wave > 0)
                    prev = s_last[t & 1][wave - 1][r][lane];
                else if (have_prev)
                    prev = s_last[(t - 1) & 1][3][r][lane];
            }
            bool ne = w != prev;
            bool flag;
            if constexpr (G == 2) {
                bool ne1 = __shfl_down(ne ? 1 : 0, 1, 64) != 0;
                flag = ((lane & 1) == 0) && (ne || ne1);
            } else {
                flag = ne;
            }
            flag = flag && valid && (lane >= G || have_prev);
            unsigned long long bal = __ballot(flag);
            if (lane == 0 && bal) atomicAdd(&s_trans[r], (uint32_t)__popcll(bal));
        };
        count(0, sgn);
#pragma unroll
        for (int c = 31; c >= 0; --c)
            if (c < (int)B) count(B - c, lo[c]);
        if constexpr (F64) {
#pragma unroll
            for (int c = 31; c >= 0; --c)
                if (32 + c < (int)B) count(B - 32 - c, hi[c]);
        }
    }

    // ---- flush
    small = wave_max(small);
    if (lane == 0 && small > 0) {
        unsigned long long sb = F64 ? (unsigned long long)__double_as_longlong((double)small)
                                    : (unsigned long long)__float_as_uint((float)small);
        atomicMax((unsigned long long*)&job.stats->small_bits, sb);
    }
    if constexpr (F64) {
        __syncthreads();
        if (tid <= B) {
            unsigned long long mx = 0;
            for (int w = 0; w < 4; ++w) mx = s_ek[w][tid] > mx ? s_ek[w][tid] : mx;
            if (mx) atomicMax(&job.ekeys[tid], mx);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 33; ++k) {
            if (k <= (int)B) {
                float km = wave_max(kmax[k]);
                if (lane == 0 && km > 0.0f)
                    atomicMax(&job.ekeys[k], (unsigned long long)__float_as_uint(km));
            }
        }
        (void)NK;
    }
    __syncthreads();
    uint32_t* gh = job.hist + (uint64_t)blockIdx.x * job.nunits * 256;
    for (uint32_t i = tid; i < job.nunits * 256; i += kThreads) gh[i] = s_hist[i];
    if (tid <= B && s_trans[tid]) atomicAdd(&job.trans[tid], s_trans[tid]);
}

// ------------------------------------------------------------------ hybrid selection
// One workgroup per unit (Alg. 2): gather the byte histogram and the run count,
// build length-limited Huffman code lengths with the two-queue construction,
// canonical codes, both size estimates, and the method decision.
__global__ __launch_bounds__(kThreads) void k_select(SelectJob job)
{
    __shared__ unsigned long long s_f[256];     // working counts (halved when limiting)
    __shared__ unsigned long long s_f0[256];    // original counts
    __shared__ unsigned long long s_w[512];
    __shared__ int s_parent[512];
    __shared__ int s_sorted[256];
    __shared__ uint8_t s_len[256];
    __shared__ unsigned long long s_red[kThreads / 64];
    __shared__ int s_nl, s_maxlen;
    __shared__ uint32_t s_count[33], s_first[33];

    const uint32_t u = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t B = job.B, m = job.m, G = job.G, grid = job.grid;
    const uint32_t r0 = u == 0 ? 0 : 1 + (u - 1) * m;
    const uint32_t r1 = u == 0 ? 1 : min(B + 1, r0 + m);
    const uint64_t S = (uint64_t)(r1 - r0) * job.nbd * 4;

    auto block_sum = [&](unsigned long long v) -> unsigned long long {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) s_red[wave] = v;
        __syncthreads();
        unsigned long long t = s_red[0] + s_red[1] + s_red[2] + s_red[3];
        __syncthreads();
        return t;
    };

    // ---- byte histogram (zeros are implied: S minus the nonzero bytes)
    unsigned long long f = 0;
    for (uint32_t w = 0; w < grid; ++w) f += job.hist[((uint64_t)w * job.nunits + u) * 256 + tid];
    unsigned long long nz = block_sum(tid ? f : 0);
    if (tid == 0) f = S - nz;
    s_f[tid] = f;
    s_f0[tid] = f;

    // ---- runs of equal W-bit words: transitions inside workgroup ranges, at
    // range boundaries, and between consecutive planes of the group
    unsigned long long tr = 0;
    for (uint32_t r = r0 + tid; r < r1; r += kThreads) tr += job.trans[r];
    const uint32_t nrow = r1 - r0;
    for (uint32_t i = tid; i < (grid - 1) * nrow; i += kThreads) {
        uint32_t w = 1 + i / nrow, r = r0 + i % nrow;
        const uint32_t* cur = job.recs + ((uint64_t)w * kMaxRows + r) * 2 * G;
        const uint32_t* prv = job.recs + ((uint64_t)(w - 1) * kMaxRows + r) * 2 * G;
        bool ne = false;
        for (uint32_t g = 0; g < G; ++g) ne = ne || cur[g] != prv[G + g];
        tr += ne ? 1 : 0;
    }
    for (uint32_t r = r0 + 1 + tid; r < r1; r += kThreads) {
        const uint32_t* cur = job.recs + ((uint64_t)0 * kMaxRows + r) * 2 * G;
        const uint32_t* prv = job.recs + ((uint64_t)(grid - 1) * kMaxRows + (r - 1)) * 2 * G;
        bool ne = false;
        for (uint32_t g = 0; g < G; ++g) ne = ne || cur[g] != prv[G + g];
        tr += ne ? 1 : 0;
    }
    unsigned long long trans = block_sum(tr);
    const unsigned long long nruns = S ? 1 + trans : 0;
    __syncthreads();

    // ---- length-limited Huffman code lengths
    for (;;) {
        // rank of symbol tid among the nonzero counts, ordered by (count, symbol)
        unsigned long long ft = s_f[tid];
        int rank = 0;
        for (int s = 0; s < 256; ++s) {
            unsigned long long fs = s_f[s];
            rank += (fs && (fs < ft || (fs == ft && s < (int)tid))) ? 1 : 0;
        }
        if (tid == 0) s_nl = 0;
        __syncthreads();
        if (ft) {
            s_sorted[rank] = (int)tid;
            atomicAdd(&s_nl, 1);
        }
        s_len[tid] = 0;
        __syncthreads();
        const int nl = s_nl;
        if (tid == 0) {
            int maxlen = 0;
            if (nl == 1) {
                int s0 = s_sorted[0];
                s_len[s0] = 1;
                s_len[s0 == 0 ? 1 : 0] = 1;
                maxlen = 1;
            } else if (nl > 1) {
                for (int i = 0; i < nl; ++i) s_w[i] = s_f[s_sorted[i]];
                int q1 = 0, q2 = nl, next = nl;
                while ((nl - q1) + (next - q2) > 1) {
                    int pk[2];
                    for (int t = 0; t < 2; ++t) {
                        if (q1 < nl && (q2 == next || s_w[q1] <= s_w[q2]))
                            pk[t] = q1++;
                        else
                            pk[t] = q2++;
                    }
                    s_w[next] = s_w[pk[0]] + s_w[pk[1]];
                    s_parent[pk[0]] = next;
                    s_parent[pk[1]] = next;
                    ++next;
                }
                // depths, reusing s_w as storage (root has the largest index)
                int root = next - 1;
                s_w[root] = 0;
                for (int i = root - 1; i >= 0; --i) s_w[i] = s_w[s_parent[i]] + 1;
                for (int i = 0; i < nl; ++i) {
                    int d = (int)s_w[i];
                    s_len[s_sorted[i]] = (uint8_t)d;
                    maxlen = d > maxlen ? d : maxlen;
                }
            }
            s_maxlen = maxlen;
        }
        __syncthreads();
        if (s_maxlen <= (int)job.huf_lmax) break;
        unsigned long long h = s_f[tid];
        if (h) s_f[tid] = (h >> 1) ? (h >> 1) : 1;
        __syncthreads();
    }

    // ---- canonical codes: (length, symbol) order
    if (tid < 33) s_count[tid] = 0;
    __syncthreads();
    const uint32_t L = s_len[tid];
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
    uint32_t code = 0;
    if (L) {
        uint32_t before = 0;
        for (uint32_t s = 0; s < tid; ++s) before += s_len[s] == L ? 1u : 0u;
        code = s_first[L] + before;
    }
    job.lens[u * 256 + tid] = (uint8_t)L;
    job.codes[u * 256 + tid] = code;

    // ---- estimates and the decision
    unsigned long long bits = block_sum(s_f0[tid] * (unsigned long long)L);
    if (tid == 0) {
        const uint64_t nchunks = (S + job.huf_chunk - 1) / job.huf_chunk;
        const uint64_t est_huf = (bits + 7) / 8 + 8 + 256 + 4 * (nchunks + 1);
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
        job.units[u] = ui;
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

hipError_t launch_init_stats(LevelStats* st, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_stats, dim3((count + 63) / 64), dim3(64), 0, s, st, count);
    return hipGetLastError();
}

hipError_t launch_stats(const void* x, uint64_t n, bool f64, LevelStats* st, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    unsigned g = grid_for(n, kThreads * 16, 2048);
    if (f64)
        hipLaunchKernelGGL(k_stats<true>, dim3(g), dim3(kThreads), 0, s, x, n, st);
    else
        hipLaunchKernelGGL(k_stats<false>, dim3(g), dim3(kThreads), 0, s, x, n, st);
    return hipGetLastError();
}

hipError_t launch_encode(const EncodeJob& job, bool f64, hipStream_t s)
{
    if (job.nbd == 0) return hipSuccess;
    size_t shmem = (size_t)job.nunits * 256 * sizeof(uint32_t);
    bool vec = ((uintptr_t)job.x % 16) == 0;
    dim3 g(job.grid), b(kThreads);
    if (f64) {
        if (vec)
            hipLaunchKernelGGL((k_encode<true, true>), g, b, shmem, s, job);
        else
            hipLaunchKernelGGL((k_encode<true, false>), g, b, shmem, s, job);
    } else {
        if (vec)
            hipLaunchKernelGGL((k_encode<false, true>), g, b, shmem, s, job);
        else
            hipLaunchKernelGGL((k_encode<false, false>), g, b, shmem, s, job);
    }
    return hipGetLastError();
}

hipError_t launch_select(const SelectJob& job, hipStream_t s)
{
    hipLaunchKernelGGL(k_select, dim3(job.nunits), dim3(kThreads), 0, s, job);
    return hipGetLastError();
}

}  // namespace mdr
