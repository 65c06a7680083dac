// Lossless kernels for gfx950 (Sec. 4.1): device-wide exclusive scan, chunked
// canonical Huffman coding of byte symbols, and run-length coding of W-bit
// plane words.  Direct copy needs no kernel: its payload is the plane rows.
#include "device_bits.hpp"
#include "mdr_internal.hpp"

namespace mdr {
namespace {

constexpr int kScanItems = 4;                          // per thread
constexpr int kScanTile = kThreads * kScanItems;       // per workgroup

// Inclusive scan over the wavefront with data-parallel moves between lanes (no
// LDS traffic): within each row of 16 lanes by shifts of 1, 2, 4 and 8 (a lane
// whose source lies before its row adds 0), then row 0's last lane into row 1
// and row 2's into row 3, then lane 31 into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t lane)
{
    (void)lane;
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
    return (uint32_t)x;
}

// exclusive scan of one tile; returns the tile total
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_wave, uint32_t& excl)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t inc = wave_incl_scan(v, lane);
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t wbase = 0, total = 0;
    for (uint32_t w = 0; w < kThreads / 64; ++w) {
        wbase += w < wave ? s_wave[w] : 0;
        total += s_wave[w];
    }
    excl = wbase + inc - v;
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(kThreads) void k_scan_tiles(const uint32_t* in, uint32_t* out,
                                                         uint64_t n, uint32_t* sums)
{
    __shared__ uint32_t s_wave[kThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems], sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = base + j < n ? in[base + j] : 0;
        sum += v[j];
    }
    uint32_t excl;
    uint32_t total = block_excl_scan(sum, s_wave, excl);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) out[base + j] = excl;
        excl += v[j];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_add(uint32_t* out, uint64_t n,
                                                       const uint32_t* sums)
{
    const uint32_t add = sums[blockIdx.x];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < n) out[base + j] += add;
}

// ------------------------------------------------------------------ batch encode
// Huffman payload: u64 nsym | u8 len[256] | u32 off[nchunks+1] | u32 words[].
// Chunk c (huf_chunk symbols) starts at word off[c]; code bits are packed most
// significant first.  Run-length payload: u32 nruns | u32 wbytes |
// symbols[nruns] (W-bit) | u32 lengths[nruns].
//
// Every kernel below has a fixed grid and reads its amount of work from device
// memory (counts[]), so the whole stage runs without the host learning which
// units chose which method.
constexpr uint64_t kHufHeader = 8 + 256;

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v, uint32_t lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t o = __shfl_up(v, off, 64);
        if (lane >= (uint32_t)off) v += o;
    }
    return v;
}

// exclusive scan across a workgroup of NT threads (64-bit); returns the total
template <int NT>
__device__ uint64_t block_scan64(uint64_t v, uint64_t* s_wave, uint64_t& excl)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t inc = wave_incl_scan64(v, lane);
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint64_t wbase = 0, total = 0;
    for (uint32_t w = 0; w < NT / 64; ++w) {
        wbase += w < wave ? s_wave[w] : 0;
        total += s_wave[w];
    }
    excl = wbase + inc - v;
    __syncthreads();
    return total;
}

// largest u in [0, U) with base[u] <= c, for a non-decreasing base with base[0] = 0
__device__ __forceinline__ uint32_t find_unit(const uint32_t* base, uint32_t U, uint32_t c)
{
    uint32_t lo = 0, hi = U;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= c)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// first plane row of unit u (its rows are contiguous in the level's row array)
__device__ __forceinline__ const uint32_t* unit_rows(const LosslessArgs& A, uint32_t u)
{
    const uint32_t i = u % A.nunits;
    const EncodeJob& job = A.jobs[u / A.nunits];
    const uint32_t r0 = i == 0 ? 0 : 1 + (i - 1) * A.m;
    return job.rows + (uint64_t)r0 * job.nbd;
}

__global__ __launch_bounds__(1024) void k_unit_plan(const LosslessArgs* __restrict__ Ap)
{
    __shared__ uint64_t s_wave[16];
    const LosslessArgs& A = *Ap;
    uint64_t carry_c = 0, carry_t = 0;
    for (uint32_t b = 0; b < A.U; b += 1024) {
        const uint32_t u = b + threadIdx.x;
        uint64_t hc = 0, rt = 0;
        if (u < A.U) {
            const UnitInfo& ui = A.units[u];
            if (ui.method == 2) hc = ui.nchunks;
            if (ui.method == 1) rt = (ui.S / (4ull * A.G) + kRleTileWords - 1) / kRleTileWords;
        }
        uint64_t ec, et;
        const uint64_t tc = block_scan64<1024>(hc, s_wave, ec);
        const uint64_t tt = block_scan64<1024>(rt, s_wave, et);
        if (u < A.U) {
            A.chunk_base[u] = (uint32_t)(carry_c + ec);
            A.tile_base[u] = (uint32_t)(carry_t + et);
        }
        carry_c += tc;
        carry_t += tt;
    }
    if (threadIdx.x == 0) {
        A.chunk_base[A.U] = (uint32_t)carry_c;
        A.tile_base[A.U] = (uint32_t)carry_t;
        A.counts[0] = (uint32_t)carry_c;
        A.counts[1] = (uint32_t)carry_t;
        A.counts[2] = 0;
    }
}

// Huffman chunks are split among wavefronts in contiguous shares; a wavefront
// walks its share in batches of kHufLoads wave-wide loads of 256 words (lane l
// takes words 4l .. 4l+3 of each: sixteen consecutive symbols), never crossing
// a unit.  A chunk of huf_chunk symbols is huf_chunk / 4 words: 16, 32 or 64
// lanes of one load (chunks of 256, 512, 1024 symbols) or 2 or 4 whole loads
// (2048, 4096), so a batch holds 16 / (huf_chunk / 256) chunks.  Code lengths
// and codes of the current unit are cached in LDS.
constexpr uint32_t kHufLoads = 4;
static_assert(4096 / 256 <= 4 * kHufLoads, "a chunk of the largest size fits one batch");

// inclusive scan of v over segments of `seg` lanes (16, 32 or 64: a uniform
// value), by data-parallel moves: rows of 16 by shifts of 1, 2, 4, 8, then
// row 0's last lane into row 1 and row 2's into row 3, then lane 31 into rows
// 2 and 3
__device__ __forceinline__ uint32_t seg_incl_scan(uint32_t v, uint32_t seg)
{
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
    if (seg >= 32) x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    if (seg >= 64) x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return (uint32_t)x;
}

// a batch's words, lane l's four of each load (0 past the batch's chunks or
// the unit's end; `valid` counts the lane's words that are in)
struct HufBatch {
    uint32_t w[kHufLoads][4];
    uint32_t valid[kHufLoads];
};

__device__ __forceinline__ bool huf_load_batch(const uint32_t* g, uint64_t wb, uint32_t nwb, uint64_t nwu,
                                               uint32_t lane, HufBatch& hb)
{
    // a whole batch from a 16-byte boundary: one 16-byte load per lane and load
    if (nwb == 256 * kHufLoads && wb + 256 * kHufLoads <= nwu &&
        (reinterpret_cast<uintptr_t>(g + wb) & 15u) == 0) {
        const auto p = gmem(reinterpret_cast<const u32x4*>(g + wb));
#pragma unroll
        for (uint32_t r = 0; r < kHufLoads; ++r) {
            const u32x4 q = p[r * 64 + lane];
            hb.w[r][0] = q.x;
            hb.w[r][1] = q.y;
            hb.w[r][2] = q.z;
            hb.w[r][3] = q.w;
            hb.valid[r] = 4;
        }
        return true;
    }
    const auto gg = gmem(g);
#pragma unroll
    for (uint32_t r = 0; r < kHufLoads; ++r) {
        const uint32_t i0 = r * 256 + 4 * lane;
        uint32_t nv = 0;
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
            const bool ok = i0 + i < nwb && wb + i0 + i < nwu;
            hb.w[r][i] = ok ? gg[wb + i0 + i] : 0u;
            nv += ok ? 1u : 0u;
        }
        hb.valid[r] = nv;
    }
    return false;
}

__device__ __forceinline__ void wave_share(uint32_t total, uint32_t& c0, uint32_t& c1)
{
    const uint32_t nw = gridDim.x * (kThreads / 64), w = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const uint32_t per = (total + nw - 1) / nw;
    c0 = min(w * per, total);
    c1 = min(c0 + per, total);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// code bits of every Huffman chunk -> chunk_words[c] (words): per lane the
// code lengths of its sixteen symbols, summed over each chunk's lanes by a
// segmented scan (chunks over several loads carry their sum across them)
__device__ __forceinline__ void huf_count_body(const LosslessArgs& A)
{
    __shared__ uint32_t s_len[kThreads / 64][256];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t total = A.counts[0];
    if (blockIdx.x == 0 && tid == 0) A.chunk_words[total] = 0;
    uint32_t* L = s_len[wave];
    const uint32_t cw = A.huf_chunk / 4, wpl = A.huf_chunk / 256;  // words, 256-symbol groups per chunk
    const uint32_t cpb = 4 * kHufLoads / wpl;                       // chunks per batch
    const uint32_t seg = min(64u, 16 * wpl), lpc = wpl > 4 ? wpl / 4 : 1;  // lanes a chunk takes of a load; loads a chunk
    uint32_t c0, c1;
    wave_share(total, c0, c1);
    uint32_t u = 0, cb_lo = 1, cb_hi = 0;  // chunks [cb_lo, cb_hi) belong to unit u
    uint64_t nwu = 0;                      // words of unit u
    for (uint32_t c = c0; c < c1;) {
        if (c < cb_lo || c >= cb_hi) {
            u = find_unit(A.chunk_base, A.U, c);
            cb_lo = A.chunk_base[u];
            cb_hi = A.chunk_base[u + 1];
            nwu = A.units[u].S / 4;
            for (uint32_t k = lane; k < 256; k += 64) L[k] = A.lens[(uint64_t)u * 256 + k];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        const uint32_t nbt = min(cpb, min(c1, cb_hi) - c);  // chunks in this batch
        HufBatch hb;
        huf_load_batch(unit_rows(A, u), (uint64_t)(c - cb_lo) * cw, nbt * cw, nwu, lane, hb);
        uint32_t run = 0;  // bits of the chunk's earlier loads (chunks over several loads)
#pragma unroll
        for (uint32_t r = 0; r < kHufLoads; ++r) {
            uint32_t T = 0;
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) {
                const uint32_t w = hb.w[r][i];
                const uint32_t bits = L[w & 0xFF] + L[(w >> 8) & 0xFF] + L[(w >> 16) & 0xFF] + L[w >> 24];
                T += i < hb.valid[r] ? bits : 0u;
            }
            const uint32_t x = seg_incl_scan(T, seg);
            if (lpc == 1) {
                const uint32_t cj = (r * 256 + 4 * lane) / cw;
                if ((lane & (seg - 1)) == seg - 1 && cj < nbt) A.chunk_words[c + cj] = (x + 31) / 32;
            } else {
                if (r % lpc == 0) run = 0;
                run += (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
                const uint32_t cj = r / lpc;
                if (r % lpc == lpc - 1 && lane == 0 && cj < nbt) A.chunk_words[c + cj] = (run + 31) / 32;
            }
        }
        c += nbt;
    }
}

// runs starting inside each run-length tile -> tile_runs[t]; one workgroup per tile
__device__ __forceinline__ bool word_ne(const uint32_t* g, uint64_t i, uint64_t j, uint32_t G)
{
    bool ne = g[i * G] != g[j * G];
    if (G == 2) ne = ne || g[i * G + 1] != g[j * G + 1];
    return ne;
}

__device__ __forceinline__ void rle_count_body(const LosslessArgs& A)
{
    __shared__ uint32_t s_red[kThreads / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t total = A.counts[1];
    if (blockIdx.x == 0 && tid == 0) A.tile_runs[total] = 0;
    uint32_t u = 0, tb_lo = 1, tb_hi = 0;  // tiles [tb_lo, tb_hi) belong to unit u
    for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
        if (t < tb_lo || t >= tb_hi) {
            u = find_unit(A.tile_base, A.U, t);
            tb_lo = A.tile_base[u];
            tb_hi = A.tile_base[u + 1];
        }
        const uint32_t* g = unit_rows(A, u);
        const uint64_t nw = A.units[u].S / (4ull * A.G);
        const uint64_t i0 = (uint64_t)(t - tb_lo) * kRleTileWords;
        const uint64_t i1 = min(nw, i0 + kRleTileWords);
        uint32_t cnt = 0;
        for (uint64_t i = i0 + tid; i < i1; i += kThreads) cnt += (i == 0 || word_ne(g, i, i - 1, A.G)) ? 1u : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if (lane == 0) s_red[wave] = cnt;
        __syncthreads();
        if (tid == 0) {
            uint32_t sum = 0;
            for (int w = 0; w < kThreads / 64; ++w) sum += s_red[w];
            A.tile_runs[t] = sum;
        }
        __syncthreads();
    }
}

// Both statistics of the planned units in one launch: Huffman chunk sizes, then
// run counts per run-length tile.
__global__ __launch_bounds__(kThreads) void k_counts(const LosslessArgs* __restrict__ Ap)
{
    const LosslessArgs& A = *Ap;
    huf_count_body(A);
    rle_count_body(A);
}

// Exclusive scans, in place, of the first *count[a] + 1 entries of data[a] for
// both arrays at once, with a fixed grid: per-workgroup range sums, one scan of
// the sums, then each range rescanned from its base.
constexpr int kScanDevTile = kThreads * 4;

__device__ __forceinline__ void dev_range(uint32_t n, uint32_t& lo, uint32_t& hi)
{
    const uint32_t per = ((n + gridDim.x - 1) / gridDim.x + 3) & ~3u;
    lo = min(n, blockIdx.x * per);
    hi = min(n, lo + per);
}

struct ScanPair {
    uint32_t* data[2];
    const uint32_t* count[2];
    uint32_t* part[2];  // [gridDim.x] range sums, then their exclusive scan
};

__global__ __launch_bounds__(kThreads) void k_scan_dev_part(const ScanPair sp)
{
    __shared__ uint32_t s_red[2][kThreads / 64];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const uint32_t n = *sp.count[a] + 1;
        const uint32_t* data = sp.data[a];
        uint32_t lo, hi;
        dev_range(n, lo, hi);
        uint32_t sum = 0;
        for (uint32_t i = lo + threadIdx.x; i < hi; i += kThreads) sum += data[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if ((threadIdx.x & 63) == 0) s_red[a][threadIdx.x >> 6] = sum;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const uint32_t a = threadIdx.x;
        sp.part[a][blockIdx.x] = s_red[a][0] + s_red[a][1] + s_red[a][2] + s_red[a][3];
    }
}

__global__ __launch_bounds__(1024) void k_scan_dev_mid(const ScanPair sp, uint32_t np)
{
    __shared__ uint64_t s_wave[16];
    for (int a = 0; a < 2; ++a) {
        uint32_t* part = sp.part[a];
        uint64_t carry = 0;
        for (uint32_t b = 0; b < np; b += 1024) {
            const uint32_t i = b + threadIdx.x;
            const uint64_t v = i < np ? part[i] : 0;
            uint64_t ex;
            const uint64_t t = block_scan64<1024>(v, s_wave, ex);
            if (i < np) part[i] = (uint32_t)(carry + ex);
            carry += t;
        }
    }
}

// data[lo, hi) -> its exclusive scan plus carry, a tile of kScanDevTile at a time
__device__ __forceinline__ void scan_range(uint32_t* __restrict__ data, uint32_t lo, uint32_t hi,
                                           uint32_t carry, uint32_t* s_wave)
{
    for (uint32_t b = lo; b < hi; b += kScanDevTile) {
        const uint32_t i0 = b + threadIdx.x * 4;
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = i0 + j < hi ? data[i0 + j] : 0;
            sum += v[j];
        }
        uint32_t excl;
        const uint32_t total = block_excl_scan(sum, s_wave, excl);
        excl += carry;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i0 + j < hi) data[i0 + j] = excl;
            excl += v[j];
        }
        carry += total;
    }
}

__global__ __launch_bounds__(kThreads) void k_scan_dev_fin(const ScanPair sp)
{
    __shared__ uint32_t s_wave[kThreads / 64];
    for (int a = 0; a < 2; ++a) {
        uint32_t* __restrict__ data = sp.data[a];
        const uint32_t n = *sp.count[a] + 1;
        uint32_t lo, hi;
        dev_range(n, lo, hi);
        uint32_t carry = sp.part[a][blockIdx.x];
        scan_range(data, lo, hi, carry, s_wave);
    }
}

// stream bytes of every unit and its arena offset (exclusive scan of the
// 256-byte-aligned sizes); headers of empty streams
__global__ __launch_bounds__(1024) void k_unit_sizes(const LosslessArgs* __restrict__ Ap)
{
    __shared__ uint64_t s_wave[16];
    const LosslessArgs& A = *Ap;
    uint64_t carry = 0;
    for (uint32_t b = 0; b < A.U; b += 1024) {
        const uint32_t u = b + threadIdx.x;
        uint64_t bytes = 0, asz = 0;
        if (u < A.U) {
            const UnitInfo& ui = A.units[u];
            if (ui.method == 2) {
                const uint64_t words = A.chunk_words[A.chunk_base[u + 1]] - A.chunk_words[A.chunk_base[u]];
                bytes = kHufHeader + 4ull * (ui.nchunks + 1) + 4 * words;
            } else if (ui.method == 1) {
                bytes = 8 + ui.nruns * (4ull * A.G + 4);
            } else {
                bytes = ui.S;
            }
            asz = ui.method == 0 ? 0 : (bytes + 255) & ~255ull;
        }
        uint64_t ex;
        const uint64_t t = block_scan64<1024>(asz, s_wave, ex);
        if (u < A.U) {
            A.pay_off[u] = carry + ex;
            A.unit_bytes[u] = bytes;
        }
        carry += t;
    }
    __syncthreads();
    const bool over = carry > A.cap;
    if (threadIdx.x == 0) {
        A.counts[2] = over ? 1u : 0u;
        A.counts[4] = (uint32_t)carry;
        A.counts[5] = (uint32_t)(carry >> 32);
    }
    if (over) return;
    for (uint32_t u = threadIdx.x; u < A.U; u += 1024) {
        const UnitInfo& ui = A.units[u];
        if (ui.S != 0) continue;
        uint32_t* p = reinterpret_cast<uint32_t*>(A.arena + A.pay_off[u]);
        if (ui.method == 2) {  // nsym 0, no code lengths, off[0] = 0
            for (uint32_t k = 0; k < (kHufHeader + 4) / 4; ++k) p[k] = 0;
        } else if (ui.method == 1) {
            p[0] = 0;
            p[1] = 4 * A.G;
        }
    }
}

// Huffman payloads.  A batch's chunks go back to back into the wave's LDS
// buffer, each from a word boundary as in the stream: a lane's bits start at
// its chunk's word offset (the batch's earlier chunks, from their segment
// totals) plus the exclusive scan of its group plus the bits of the chunk's
// earlier loads.  A lane's sixteen codes go in as eight pairs (at most 24 bits,
// so one or two words each) with atomic ORs; the batch then leaves as one
// coalesced run of words, and each chunk's first lane writes its offset.  The
// first chunk's wavefront writes the header, the last one's the closing offset.
template <bool FULL>
__device__ __forceinline__ void huf_emit_load(const HufBatch& hb, uint32_t r, const uint32_t* LC, uint32_t* buf,
                                              uint32_t seg, uint32_t lpc, uint32_t nbt, uint32_t lane,
                                              uint32_t& boff, uint32_t& run, uint32_t* off, uint32_t gw)
{
    // the lane's eight code pairs (code, length), in stream order
    uint32_t cp[8], lp[8], T = 0;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
        const uint32_t w = hb.w[r][i];
        const bool in = FULL || i < hb.valid[r];
#pragma unroll
        for (uint32_t p = 0; p < 2; ++p) {
            const uint32_t a = LC[(w >> (16 * p)) & 0xFF], b = LC[(w >> (16 * p + 8)) & 0xFF];
            const uint32_t lb = b >> 16, L = (a >> 16) + lb;
            cp[2 * i + p] = in ? ((a & 0xFFFFu) << lb) | (b & 0xFFFFu) : 0u;
            lp[2 * i + p] = in ? L : 0u;
            T += in ? L : 0u;
        }
    }
    const uint32_t x = seg_incl_scan(T, seg);
    uint32_t pos;
    if (lpc == 1) {
        // chunks of this load: one per segment; the lane's chunk starts after
        // the earlier segments' words
        const uint32_t sg = lane / seg;
        uint32_t coff = boff, add = 0;
        for (uint32_t k = 0; k < 64 / seg; ++k) {
            const uint32_t wk = ((uint32_t)__builtin_amdgcn_readlane((int)x, (int)(k * seg + seg - 1)) + 31) / 32;
            coff += sg > k ? wk : 0u;
            add += wk;
        }
        const uint32_t cj = r * (64 / seg) + sg;
        if ((lane & (seg - 1)) == 0 && cj < nbt) *gmem(off + cj) = gw + coff;
        pos = 32 * coff + x - T;
        boff += add;
    } else {
        if (r % lpc == 0) {
            run = 0;
            if (lane == 0 && r / lpc < nbt) *gmem(off + r / lpc) = gw + boff;
        }
        pos = 32 * boff + run + x - T;
        run += (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
        if (r % lpc == lpc - 1) boff += (run + 31) / 32;
    }
    if (T != 0) {
        uint32_t P = pos;
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) {
            // bits [P, P + lp) of the stream, most significant first: in the
            // 64-bit window of words P / 32 and P / 32 + 1 the pair's last bit
            // sits 64 - lp - P % 32 bits up (an empty pair adds nothing)
            const uint64_t v = (uint64_t)cp[k] << ((64u - lp[k] - (P & 31u)) & 63u);
            uint32_t* q = buf + (P >> 5);
            atomicOr(q, (uint32_t)(v >> 32));
            atomicOr(q + 1, (uint32_t)v);
            P += lp[k];
        }
    }
}

// LDS words of one wave's batch buffer: cpb chunks of at most chunk * 12 bits,
// plus the word after the last (a pair's second OR may touch it), in 16-byte units
__host__ __device__ constexpr uint32_t huf_buf_words(uint32_t huf_chunk)
{
    return ((4 * kHufLoads / (huf_chunk / 256)) * ((huf_chunk * kLutBitsMax + 31) / 32) + 4 + 3) / 4 * 4;
}

__device__ __forceinline__ void huf_write_body(const LosslessArgs& A, uint32_t buf_words)
{
    extern __shared__ __align__(16) uint32_t s_buf[];  // [kThreads / 64][buf_words]
    __shared__ uint32_t s_lc[kThreads / 64][256];      // code | length << 16 of each symbol
    if (A.counts[2]) return;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t total = A.counts[0];
    uint32_t* LC = s_lc[wave];
    const uint32_t cw = A.huf_chunk / 4, wpl = A.huf_chunk / 256;
    const uint32_t cpb = 4 * kHufLoads / wpl;  // chunks per batch
    const uint32_t seg = min(64u, 16 * wpl), lpc = wpl > 4 ? wpl / 4 : 1;
    const uint32_t cmax = (A.huf_chunk * kLutBitsMax + 31) / 32;  // words of a chunk at most
    uint32_t* buf = s_buf + wave * buf_words;
    uint32_t c0, c1;
    wave_share(total, c0, c1);
    uint32_t u = 0, cb_lo = 1, cb_hi = 0, nch = 0, base = 0;
    uint64_t nwu = 0;
    uint8_t* pay = nullptr;
    auto sync_wave = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    for (uint32_t c = c0; c < c1;) {
        if (c < cb_lo || c >= cb_hi) {
            u = find_unit(A.chunk_base, A.U, c);
            cb_lo = A.chunk_base[u];
            cb_hi = A.chunk_base[u + 1];
            nwu = A.units[u].S / 4;
            nch = A.units[u].nchunks;
            base = A.chunk_words[cb_lo];
            pay = A.arena + A.pay_off[u];
            for (uint32_t k = lane; k < 256; k += 64)
                LC[k] = A.codes[(uint64_t)u * 256 + k] | ((uint32_t)A.lens[(uint64_t)u * 256 + k] << 16);
        }
        const uint32_t nbt = min(cpb, min(c1, cb_hi) - c);
        // zero the batch's words (and the one after them) for the ORs
        const uint32_t nclr = (nbt * cmax + 4) / 4;
        for (uint32_t i = lane; i < nclr; i += 64) reinterpret_cast<u32x4*>(buf)[i] = u32x4{0u, 0u, 0u, 0u};
        sync_wave();
        HufBatch hb;
        const bool full = huf_load_batch(unit_rows(A, u), (uint64_t)(c - cb_lo) * cw, nbt * cw, nwu, lane, hb);
        const uint32_t lc0 = c - cb_lo;               // the batch's first chunk in the unit
        const uint32_t gw = A.chunk_words[c] - base;  // and its first word in the stream
        uint32_t* const poff = reinterpret_cast<uint32_t*>(pay + kHufHeader);
        const auto off = gmem(poff);
        const auto words = off + nch + 1;
        uint32_t boff = 0, run = 0;  // words of the batch's finished chunks; bits of the chunk's earlier loads
        if (full) {
#pragma unroll
            for (uint32_t r = 0; r < kHufLoads; ++r)
                huf_emit_load<true>(hb, r, LC, buf, seg, lpc, nbt, lane, boff, run, poff + lc0, gw);
        } else {
#pragma unroll
            for (uint32_t r = 0; r < kHufLoads; ++r)
                huf_emit_load<false>(hb, r, LC, buf, seg, lpc, nbt, lane, boff, run, poff + lc0, gw);
        }
        sync_wave();
        for (uint32_t i = lane; i < boff; i += 64) words[gw + i] = buf[i];
        if (lane == 0 && lc0 + nbt == nch) off[nch] = gw + boff;
        if (lc0 == 0) {
            const UnitInfo& ui = A.units[u];
            if (lane == 0) *reinterpret_cast<uint64_t*>(pay) = ui.S;
            const uint32_t b4 = lane * 4;
            reinterpret_cast<uint32_t*>(pay + 8)[lane] = (LC[b4] >> 16) | ((LC[b4 + 1] >> 16) << 8) |
                                                         ((LC[b4 + 2] >> 16) << 16) | ((LC[b4 + 3] >> 16) << 24);
        }
        sync_wave();  // the buffer is cleared again by the next batch
        c += nbt;
    }
}

// run-length payloads.  Pass 1 (write): every run start stores its symbol and,
// in the lengths slot, its start position.  Pass 2 (len): every run's last
// word turns that slot into the length.  Run r of a unit = runs starting in
// its earlier tiles + starts before the word inside the tile.
constexpr int kRlePer = kRleTileWords / kThreads;  // consecutive words per thread

template <bool LEN>
__device__ __forceinline__ void rle_pass_body(const LosslessArgs& A)
{
    __shared__ uint32_t s_wave[kThreads / 64];
    if (A.counts[2]) return;
    const uint32_t tid = threadIdx.x;
    const uint32_t total = A.counts[1], G = A.G;
    uint32_t u = 0, tb_lo = 1, tb_hi = 0;  // tiles [tb_lo, tb_hi) belong to unit u
    for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
        if (t < tb_lo || t >= tb_hi) {
            u = find_unit(A.tile_base, A.U, t);
            tb_lo = A.tile_base[u];
            tb_hi = A.tile_base[u + 1];
        }
        const UnitInfo& ui = A.units[u];
        const uint32_t* g = unit_rows(A, u);
        const uint64_t nw = ui.S / (4ull * G), nruns = ui.nruns;
        uint8_t* pay = A.arena + A.pay_off[u];
        uint32_t* sym = reinterpret_cast<uint32_t*>(pay + 8);
        uint32_t* lslot = reinterpret_cast<uint32_t*>(pay + 8 + 4ull * G * nruns);
        const uint32_t lt = t - tb_lo;
        const uint64_t i0 = (uint64_t)lt * kRleTileWords + (uint64_t)tid * kRlePer;
        uint32_t flags = 0, cnt = 0;
        for (int k = 0; k < kRlePer; ++k) {
            const uint64_t i = i0 + k;
            const bool f = i < nw && (i == 0 || word_ne(g, i, i - 1, G));
            flags |= f ? (1u << k) : 0u;
            cnt += f ? 1u : 0u;
        }
        uint32_t excl;
        block_excl_scan(cnt, s_wave, excl);
        uint64_t r = (uint64_t)(A.tile_runs[t] - A.tile_runs[tb_lo]) + excl;
        if (!LEN && lt == 0 && tid == 0) {
            reinterpret_cast<uint32_t*>(pay)[0] = (uint32_t)nruns;
            reinterpret_cast<uint32_t*>(pay)[1] = 4 * G;
        }
        for (int k = 0; k < kRlePer; ++k) {
            const uint64_t i = i0 + k;
            if (i >= nw) break;
            const bool start = (flags >> k) & 1u;
            if (!LEN) {
                if (start && r < nruns) {
                    sym[r * G] = g[i * G];
                    if (G == 2) sym[r * G + 1] = g[i * G + 1];
                    lslot[r] = (uint32_t)i;
                }
                r += start ? 1 : 0;
            } else {
                r += start ? 1 : 0;  // now one past the run holding word i
                const bool end = i + 1 == nw || word_ne(g, i + 1, i, G);
                if (end && r - 1 < nruns) lslot[r - 1] = (uint32_t)(i + 1) - lslot[r - 1];
            }
        }
    }
}

// Payload writes: Huffman streams, then the first run-length pass (the two
// touch different units).
__global__ __launch_bounds__(kThreads) void k_write(const LosslessArgs* __restrict__ Ap, uint32_t buf_words)
{
    const LosslessArgs& A = *Ap;
    huf_write_body(A, buf_words);
    rle_pass_body<false>(A);
}

// the second run-length pass (lengths); it reads starts other workgroups wrote
__global__ __launch_bounds__(kThreads) void k_rle_len(const LosslessArgs* __restrict__ Ap)
{
    rle_pass_body<true>(*Ap);
}

// ------------------------------------------------------------------ Huffman decode
// The first-code table of a stream, built in LDS by a 256-thread workgroup
// from the 256 code lengths of its header: entry i of the 2^lmax-entry table
// holds (length << 8) | symbol of the code that the lmax-bit window i starts
// with (codes are prefix-free, so the bits after it do not matter).  A window
// that starts with no code (possible only for an incomplete code) consumes
// lmax bits as symbol 0.  Ends with a barrier.
__device__ void build_first_code_table(const uint8_t* __restrict__ payload, uint32_t lmax,
                                       uint16_t* s_one, uint32_t (*s_wcnt)[kLutBitsMax + 1],
                                       uint8_t* s_sym)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nent = 1u << lmax;
    // canonical code of symbol `tid`: the first code of its length plus the
    // smaller symbols of that length (wavefront ballots, then the counts of
    // the earlier wavefronts)
    const uint32_t L = payload[8 + tid];
    const bool has = L != 0 && L <= lmax;
    uint32_t before = 0;
    for (uint32_t l = 1; l <= lmax; ++l) {
        const unsigned long long bl = __ballot(has && L == l);
        if (lane == 0) s_wcnt[wave][l] = (uint32_t)__popcll(bl);
        if (has && L == l) before = (uint32_t)__popcll(bl & ((1ull << lane) - 1));
    }
    __syncthreads();
    // per length l (all in registers): lim[l] = end of the lmax-bit windows
    // whose first code has length <= l (non-decreasing in l); base[l] = index
    // of the first symbol of length l minus the first code of that length
    uint32_t lim[kLutBitsMax + 1], base[kLutBitsMax + 1], lim_all = 0;
    {
        uint32_t first = 0, idx = 0;
#pragma unroll
        for (int l = 1; l <= kLutBitsMax; ++l) {
            uint32_t cnt = 0;
            if (l <= (int)lmax)
                for (uint32_t w = 0; w < kThreads / 64; ++w) cnt += s_wcnt[w][l];
            if (has && (uint32_t)l == L) {
                for (uint32_t w = 0; w < wave; ++w) before += s_wcnt[w][l];
                s_sym[idx + before] = (uint8_t)tid;
            }
            base[l] = idx - first;
            lim[l] = l <= (int)lmax ? (first + cnt) << (lmax - l) : nent;
            if (l == (int)lmax) lim_all = lim[l];
            idx += cnt;
            first = (first + cnt) << 1;
        }
    }
    __syncthreads();
    // first code of every window (independent entries)
    for (uint32_t i = tid; i < nent; i += kThreads) {
        uint32_t Lx = 1, bx = base[1];
#pragma unroll
        for (int l = 1; l < kLutBitsMax; ++l) {
            const bool past = l < (int)lmax && lim[l] <= i;
            Lx += past ? 1u : 0u;
            bx = past ? base[l + 1] : bx;
        }
        const bool code = i < lim_all;  // then Lx is the leading code's length
        s_one[i] = code ? (uint16_t)((Lx << 8) | s_sym[bx + (i >> (lmax - Lx))]) : (uint16_t)(lmax << 8);
    }
    __syncthreads();
}

// The decode tables of a launch, one workgroup per stream, built once and
// stored to the job's table slot (the decoders' workgroups copy them to LDS
// instead of each building them).  MULTI: the multi-symbol table of the
// one-thread decoder, 2^lmax entries mapping the next lmax bits to up to
// three symbols (every code lying wholly inside the window is decoded by that
// one lookup): symbols | count << 24 | bits << 26.  Otherwise the first-code
// table (length << 8 | symbol) of the G-lane decoder.
template <bool MULTI>
__global__ __launch_bounds__(kThreads) void k_huf_tables(const DecodeJob* __restrict__ jobs)
{
    const DecodeJob& job = jobs[blockIdx.x];
    const uint32_t lmax = job.lmax, nent = 1u << lmax, mask = nent - 1, tid = threadIdx.x;
    __shared__ uint16_t s_one[1 << kLutBitsMax];
    __shared__ uint32_t s_wcnt[kThreads / 64][kLutBitsMax + 1];
    __shared__ uint8_t s_sym[256];
    build_first_code_table(job.payload, lmax, s_one, s_wcnt, s_sym);
    if (!MULTI) {
        const auto t = gmem(reinterpret_cast<uint32_t*>(job.table));
        for (uint32_t i = tid; i < nent / 2; i += kThreads)
            t[i] = reinterpret_cast<const uint32_t*>(s_one)[i];
        return;
    }
    // up to three whole codes per window: chains of first-code lookups, four
    // windows at a time so their LDS latencies overlap
    const auto t = gmem(reinterpret_cast<uint32_t*>(job.table));
    for (uint32_t i0 = tid; i0 < nent; i0 += 4 * kThreads) {
        uint32_t syms[4] = {0, 0, 0, 0}, k[4] = {0, 0, 0, 0}, used[4] = {0, 0, 0, 0};
        bool open[4] = {true, true, true, true};
#pragma unroll
        for (int step = 0; step < 3; ++step) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t i = i0 + q * kThreads;
                if (!open[q] || i >= nent) continue;
                const uint32_t e = s_one[(i << used[q]) & mask];
                const uint32_t l = e >> 8;
                if (used[q] + l > lmax) {
                    open[q] = false;  // the next code does not fit in the window
                    continue;
                }
                syms[q] |= (e & 0xFFu) << (8 * step);
                ++k[q];
                used[q] += l;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t i = i0 + q * kThreads;
            if (i < nent) t[i] = syms[q] | (k[q] << 24) | (used[q] << 26);
        }
    }
}

// copies a job's table of `words` 32-bit words to LDS with 16-byte loads
// (tables sit at 16 KiB strides, and 2^lmax / 2 words is a multiple of 4 for lmax >= 3)
__device__ __forceinline__ void load_table(const void* table, uint32_t words, uint32_t* lds)
{
    const auto src = gmem(reinterpret_cast<const u32x4*>(table));
    u32x4* dst = reinterpret_cast<u32x4*>(lds);
    for (uint32_t i = threadIdx.x; i < (words + 3) / 4; i += kThreads) dst[i] = src[i];
}

// One thread per chunk, kThreads chunks per workgroup (the launch for many
// chunks), through the multi-symbol table: skewed groups, whose frequent
// symbols have 1-3 bit codes, take a third of the dependent lookups of a
// one-symbol table; a 4-byte entry keeps the table at 16 KiB, so that eight
// workgroups fit a CU.  Compressed words arrive in 16-byte blocks one block
// ahead of their use, each iteration takes at most one word and makes two
// lookups, and decoded bytes leave in 64-byte pieces.
__global__ __launch_bounds__(kThreads) void k_huf_decode(const DecodeJob* __restrict__ jobs,
                                                         const uint32_t* __restrict__ wg_job)
{
    const DecodeJob& job = jobs[wg_job[blockIdx.x]];
    const uint8_t* payload = job.payload;
    const uint64_t S = job.S;
    const uint32_t chunk = job.chunk, lmax = job.lmax, nchunks = job.nchunks;
    __shared__ __align__(16) uint32_t s_multi[1 << kLutBitsMax];  // symbols | count << 24 | bits << 26
    const uint32_t tid = threadIdx.x;
    load_table(job.table, 1u << lmax, s_multi);
    __syncthreads();  // the only barrier

    const uint32_t c = (blockIdx.x - job.wg_base) * kThreads + tid;
    if (c >= nchunks) return;
    const auto off = gmem(reinterpret_cast<const uint32_t*>(payload + kHufHeader));
    const uint32_t wb = off[c], we = off[c + 1];
    // words past the chunk's end are never decoded: read the last one instead
    const uint32_t wl = we > wb ? we - 1 : wb;
    const uint64_t lo = (uint64_t)c * chunk;
    const uint32_t cnt = (uint32_t)((lo + chunk <= S) ? chunk : S - lo);  // a multiple of 4
    const auto dst4 = gmem(reinterpret_cast<u32x4*>(job.out + lo));
    // Compressed words arrive as aligned 16-byte blocks, two in flight: a
    // thread's stream is its own, and with one word per load every line came
    // from memory several times over before the thread had used it up.  Block
    // k holds words 4k - delta .. 4k - delta + 3 of the chunk data (delta puts
    // the data's start on its 16-byte grid); the first block may begin before
    // the chunk and the last may end past it (a stream's allocation is padded
    // to 256 bytes), but no block past the one holding word wl is read.
    const uintptr_t wbase = reinterpret_cast<uintptr_t>(payload + kHufHeader + 4ull * (nchunks + 1));
    const uint32_t delta = (uint32_t)((wbase & 15u) >> 2);
    const auto blk4 = gmem(reinterpret_cast<const u32x4*>(wbase & ~(uintptr_t)15));
    const uint32_t b0 = (wb + delta) >> 2, j0 = (wb + delta) & 3u, bl = (wl + delta) >> 2;
    u32x4 qa = blk4[b0], qb = blk4[min(b0 + 1, bl)];
    uint32_t bnext = b0 + 2, jq = j0;  // qa's next word (the first block may begin before the chunk)
    uint64_t buf = 0;
    int nb = 0;
    uint64_t pend = 0;  // decoded bytes not yet in a whole word (at most three between lookups)
    uint32_t npend = 0, done = 0, wo = 0, nob = 0, nsl = 0;
    // decoded words leave in whole 64-byte pieces: ob collects four words, the
    // slots s0..s2 the three vectors before it (a line written at once is
    // written once; 16-byte pieces of lines far apart were written back piecemeal)
    u32x4 ob = {0, 0, 0, 0}, s0 = {0, 0, 0, 0}, s1 = {0, 0, 0, 0}, s2 = {0, 0, 0, 0};
    // One lookup: up to three symbols into pend, and a whole word out of it
    // when there is one.  The window is whole: at least lmax bits are in the
    // buffer (or the chunk's data has ended; symbols from the bits past it lie
    // past its end, never complete a word, and are never stored).
    auto lookup = [&]() {
        const uint32_t e = s_multi[buf >> (64 - lmax)];
        const uint32_t k = (e >> 24) & 3u, used = e >> 26;
        pend |= (uint64_t)(e & 0xFFFFFFu) << (8 * npend);  // bytes past the k symbols are 0
        npend += k;
        done += k;
        buf <<= used;
        nb -= (int)used;
        if (npend >= 4) {
            ob = u32x4{ob.y, ob.z, ob.w, (uint32_t)pend};  // oldest word first once full
            pend >>= 32;
            npend -= 4;
            if (++nob == 4) {
                nob = 0;
                if (nsl == 3) {
                    dst4[wo] = s0;
                    dst4[wo + 1] = s1;
                    dst4[wo + 2] = s2;
                    dst4[wo + 3] = ob;
                    wo += 4;
                    nsl = 0;
                } else {
                    // the held vectors move down one slot: after three, s0..s2 hold them in order
                    s0 = s1;
                    s1 = s2;
                    s2 = ob;
                    ++nsl;
                }
            }
        }
    };
    // Every lane takes at most one word and makes two lookups per iteration
    // (a lookup uses at most lmax <= 12 bits, and after the refill at least 32
    // are held), so a wavefront iterates as often as its longest chunk needs
    // lookups, halved, instead of the sum over words of each word's slowest lane.
    while (done < cnt) {
        if (nb <= 32) {
            const uint32_t w = jq == 0 ? qa.x : jq == 1 ? qa.y : jq == 2 ? qa.z : qa.w;
            buf |= (uint64_t)w << (32 - nb);
            nb += 32;
            if (++jq == 4) {
                jq = 0;
                qa = qb;
                qb = blk4[min(bnext++, bl)];
            }
        }
        lookup();
        if (done < cnt) lookup();
    }
    // a chunk ends on a word: the whole vectors held in the slots, then up to
    // three words, the newest nob of ob (in order)
    if (nsl > 2) dst4[wo++] = s0;
    if (nsl > 1) dst4[wo++] = s1;
    if (nsl > 0) dst4[wo++] = s2;
    const auto dst = gmem(reinterpret_cast<uint32_t*>(job.out + lo)) + 4 * wo;
    if (nob == 3) {
        dst[0] = ob.y;
        dst[1] = ob.z;
        dst[2] = ob.w;
    } else if (nob == 2) {
        dst[0] = ob.z;
        dst[1] = ob.w;
    } else if (nob == 1) {
        dst[0] = ob.w;
    }
}

// ------------------------------------------------------------------ Huffman decode, G lanes a chunk
// For launches with too few chunks to fill the chip, where one thread per
// chunk leaves a 256-symbol chain of dependent lookups as the launch's
// latency.  A chunk's compressed bits are cut into G equal ranges and lane g
// of the chunk's G lanes decodes the codes that start in range g.  Only lane 0
// knows where its first code starts; lane g > 0 starts at its range's first
// bit, decodes to past its range's end, and the end it reaches becomes lane
// g+1's next start, until no start moves.  The chain of starts is then the
// one a serial decode passes through (lane 0's is right from the first round,
// and each round makes at least one more lane right, so G rounds always end
// it; a prefix code falls back into step with the true boundaries within a
// few codes, so two or three rounds are usual).  A prefix sum of the lanes'
// counts places their symbols, a last walk writes them to LDS, and the
// workgroup stores its chunks' bytes with 16-byte stores.
constexpr uint32_t kSplitOut = 16384;                            // decoded bytes a workgroup holds
constexpr uint32_t kSplitWords = kSplitOut * kLutBitsMax / 32;   // their compressed words, at most
constexpr uint32_t kSplitWordsPer = kSplitWords / kThreads;

// Walks the codes of a chunk (words W[qb..ql], bits MSB first) that start in
// [pos, hi); returns where the walk stops (the start of the first code at or
// past hi) and their count in n; kWrite: the first `room` symbols go to out.
template <bool kWrite>
__device__ __forceinline__ uint32_t huf_walk(const uint32_t* W, uint32_t qb, uint32_t ql,
                                             const uint16_t* tab, uint32_t lmax, uint32_t pos,
                                             uint32_t hi, uint32_t& n, uint8_t* out, uint32_t room)
{
    uint32_t q = qb + (pos >> 5);
    const uint32_t sh = pos & 31u;
    uint64_t buf = ((((uint64_t)W[min(q, ql)]) << 32) | W[min(q + 1, ql)]) << sh;
    uint32_t nb = 64 - sh;  // valid bits at the top of buf, never fewer than 32 at a lookup
    q += 2;
    uint32_t j = 0;
    while (pos < hi) {
        if (nb < 32) {
            buf |= (uint64_t)W[min(q, ql)] << (32 - nb);
            nb += 32;
            ++q;
        }
        const uint32_t e = tab[buf >> (64 - lmax)];
        const uint32_t L = e >> 8;
        if (kWrite && j < room) out[j] = (uint8_t)e;
        buf <<= L;
        nb -= L;
        pos += L;
        ++j;
    }
    n = j;
    return pos;
}

// Dynamic LDS of a launch whose largest chunk is cap_chunk symbols: the
// first-code table, then the compressed words and the decoded bytes of the
// workgroup's chunks.
__host__ __device__ constexpr uint32_t split_words_cap(uint32_t cpw, uint32_t cap_chunk)
{
    return cpw * cap_chunk * kLutBitsMax / 32;
}
__host__ __device__ constexpr uint32_t split_lds_bytes(uint32_t cpw, uint32_t cap_chunk)
{
    return (2u << kLutBitsMax) + 4 * split_words_cap(cpw, cap_chunk) + cpw * cap_chunk;
}

template <int G>
__global__ __launch_bounds__(kThreads) void k_huf_decode_split(const DecodeJob* __restrict__ jobs,
                                                               const uint32_t* __restrict__ wg_job,
                                                               uint32_t cap_chunk)
{
    static_assert(G >= 4 && G <= 64 && (G & (G - 1)) == 0, "G lanes a chunk: 4..64, a power of two");
    constexpr uint32_t kCpw = kThreads / G;  // chunks per workgroup
    const DecodeJob& job = jobs[wg_job[blockIdx.x]];
    const uint8_t* payload = job.payload;
    const uint64_t S = job.S;
    const uint32_t chunk = job.chunk, lmax = job.lmax, nchunks = job.nchunks;
    // the launcher sizes LDS for cap_chunk and raises G so that kCpw * cap_chunk <= kSplitOut
    if (chunk > cap_chunk || kCpw * cap_chunk > kSplitOut) return;
    extern __shared__ __align__(16) uint8_t s_dyn[];
    uint16_t* s_one = reinterpret_cast<uint16_t*>(s_dyn);
    const uint32_t wcap = split_words_cap(kCpw, cap_chunk);
    uint32_t* s_words = reinterpret_cast<uint32_t*>(s_dyn + (2u << kLutBitsMax));
    uint8_t* s_out = s_dyn + (2u << kLutBitsMax) + 4 * wcap;
    const uint32_t tid = threadIdx.x;
    const uint32_t c0 = (blockIdx.x - job.wg_base) * kCpw, c1 = min(c0 + kCpw, nchunks);
    const auto off = gmem(reinterpret_cast<const uint32_t*>(payload + kHufHeader));
    const auto wp = gmem(reinterpret_cast<const uint32_t*>(payload + kHufHeader + 4ull * (nchunks + 1)));
    // the workgroup's compressed words (its chunks are adjacent) and the
    // stream's table, both loads in flight at once
    const uint32_t w0 = off[c0], nw = min(off[c1] - w0, wcap);
    uint32_t held[kSplitWordsPer];
#pragma unroll
    for (uint32_t r = 0; r < kSplitWordsPer; ++r) {
        const uint32_t i = tid + r * kThreads;
        held[r] = i < nw ? wp[w0 + i] : 0u;
    }
    load_table(job.table, (1u << lmax) / 2, reinterpret_cast<uint32_t*>(s_one));
#pragma unroll
    for (uint32_t r = 0; r < kSplitWordsPer; ++r) {
        const uint32_t i = tid + r * kThreads;
        if (i < nw) s_words[i] = held[r];
    }
    __syncthreads();

    const uint32_t g = tid % G, cl = tid / G, c = c0 + cl;
    const bool live = c < c1;
    uint32_t qb = 0, ql = 0, nbits = 0, cnt = 0;
    if (live) {
        qb = min(off[c] - w0, wcap - 1);
        const uint32_t qe = min(off[c + 1] - w0, wcap);
        ql = qe > qb ? qe - 1 : qb;
        nbits = (qe > qb ? qe - qb : 0) * 32;
        const uint64_t lo = (uint64_t)c * chunk;
        cnt = (uint32_t)(lo + chunk <= S ? chunk : S - lo);
    }
    const uint32_t Lb = (nbits + G - 1) / G;
    const uint32_t lo_g = min(g * Lb, nbits), hi_g = min(lo_g + Lb, nbits);
    uint32_t start = lo_g, n = 0;
    for (int round = 0; round < G; ++round) {
        const uint32_t end = huf_walk<false>(s_words, qb, ql, s_one, lmax, start, hi_g, n, nullptr, 0);
        const uint32_t prev = __shfl_up(end, 1, G);
        // a lane whose range is empty (past the chunk's bits) decodes nothing
        // from any start: left out, it cannot hold the others up
        const bool moved = live && g != 0 && lo_g < hi_g && prev != start;
        if (__ballot(moved) == 0) break;  // every start is the end of the lane before
        if (moved) start = prev;
    }
    uint32_t incl = n;  // inclusive prefix sum of the counts over the chunk's lanes
#pragma unroll
    for (uint32_t d = 1; d < (uint32_t)G; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d, G);
        if (g >= d) incl += t;
    }
    const uint32_t o = incl - n;
    if (live && o < cnt)
        huf_walk<true>(s_words, qb, ql, s_one, lmax, start, hi_g, n, s_out + cl * chunk + o, cnt - o);
    __syncthreads();
    // the chunks' bytes are adjacent in the output too: a multiple of 4 bytes
    const uint64_t lo0 = (uint64_t)c0 * chunk;
    const uint32_t T = (uint32_t)(min((uint64_t)c1 * chunk, S) - lo0);
    const auto dst4 = gmem(reinterpret_cast<u32x4*>(job.out + lo0));
    const u32x4* src4 = reinterpret_cast<const u32x4*>(s_out);
    for (uint32_t i = tid; i < T / 16; i += kThreads) dst4[i] = src4[i];
    const uint32_t tw = (T & 15u) / 4;
    if (tid < tw) {
        const uint32_t i = (T & ~15u) / 4 + tid;
        gmem(reinterpret_cast<uint32_t*>(job.out + lo0))[i] = reinterpret_cast<const uint32_t*>(s_out)[i];
    }
}

// ------------------------------------------------------------------ RLE decode
// Every run-length group of a retrieval in one pass of three launches: the run
// lengths of all groups are gathered into one array, one exclusive scan turns
// them into run starts (a group's starts are its entries minus its first, so
// the scan's sums may wrap), and every W-bit word of every group finds its run
// by binary search over its group's starts.
__global__ __launch_bounds__(kThreads) void k_rle_gather(const RleJob* __restrict__ jobs,
                                                         const uint32_t* __restrict__ wg_job,
                                                         uint32_t* __restrict__ lens)
{
    const RleJob& job = jobs[wg_job[blockIdx.x]];
    const uint64_t r0 = (uint64_t)(blockIdx.x - job.wg_gather) * kRlePerWg;
    const uint64_t r1 = min(r0 + kRlePerWg, job.nruns);
    const auto src = gmem(reinterpret_cast<const uint32_t*>(job.payload + 8 + 4ull * job.G * job.nruns));
    for (uint64_t r = r0 + threadIdx.x; r < r1; r += kThreads) lens[job.run_base + r] = src[r];
}

__global__ __launch_bounds__(kThreads) void k_rle_expand(const RleJob* __restrict__ jobs,
                                                         const uint32_t* __restrict__ wg_job,
                                                         const uint32_t* __restrict__ starts)
{
    const RleJob& job = jobs[wg_job[blockIdx.x]];
    const uint32_t* st = starts + job.run_base;
    const uint32_t s0 = st[0];
    const auto sym = gmem(reinterpret_cast<const uint32_t*>(job.payload + 8));
    const auto g = gmem(reinterpret_cast<uint32_t*>(job.out));
    const uint32_t G = job.G;
    const uint64_t i0 = (uint64_t)(blockIdx.x - job.wg_expand) * kRlePerWg;
    const uint64_t i1 = min(i0 + kRlePerWg, job.nwords);
    for (uint64_t i = i0 + threadIdx.x; i < i1; i += kThreads) {
        // last run whose start is <= i (starts relative to the group's first)
        uint64_t lo = 0, hi = job.nruns;  // invariant: start[lo] <= i, answer in [lo, hi)
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) / 2;
            if ((uint64_t)(uint32_t)(st[mid] - s0) <= i)
                lo = mid;
            else
                hi = mid;
        }
        for (uint32_t q = 0; q < G; ++q) g[i * G + q] = sym[lo * G + q];
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers
static unsigned blocks_for(uint64_t items, uint64_t per, unsigned cap)
{
    uint64_t b = (items + per - 1) / per;
    if (b < 1) b = 1;
    return (unsigned)(b > cap ? cap : b);
}

uint64_t scan_temp_words(uint64_t n)
{
    uint64_t t = 0;
    while (n > 1) {
        n = (n + kScanTile - 1) / kScanTile;
        t += n + 64;
    }
    return t + 64;
}

hipError_t launch_scan_exclusive(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* temp,
                                 hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint64_t tiles = (n + kScanTile - 1) / kScanTile;
    uint32_t* sums = temp;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kThreads), 0, s, in, out, n, sums);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess || tiles == 1) return err;
    err = launch_scan_exclusive(sums, sums, tiles, temp + tiles + 64, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(kThreads), 0, s, out, n, sums);
    return hipGetLastError();
}

hipError_t launch_lossless_batch(const LosslessArgs& a, const LosslessArgs* a_dev, uint32_t* scan_part,
                                 hipStream_t s)
{
    if (a.U == 0) return hipSuccess;
    const dim3 P(kPersistWg), T(kThreads);
    hipLaunchKernelGGL(k_unit_plan, dim3(1), dim3(1024), 0, s, a_dev);
    hipLaunchKernelGGL(k_counts, P, T, 0, s, a_dev);
    ScanPair sp{};
    sp.data[0] = a.chunk_words;
    sp.count[0] = a.counts + 0;
    sp.part[0] = scan_part;
    sp.data[1] = a.tile_runs;
    sp.count[1] = a.counts + 1;
    sp.part[1] = scan_part + kPersistWg + 32;
    hipLaunchKernelGGL(k_scan_dev_part, P, T, 0, s, sp);
    hipLaunchKernelGGL(k_scan_dev_mid, dim3(1), dim3(1024), 0, s, sp, kPersistWg);
    hipLaunchKernelGGL(k_scan_dev_fin, P, T, 0, s, sp);
    hipLaunchKernelGGL(k_unit_sizes, dim3(1), dim3(1024), 0, s, a_dev);
    const uint32_t buf_words = huf_buf_words(a.huf_chunk);
    const size_t shmem = (size_t)(kThreads / 64) * buf_words * sizeof(uint32_t);
    hipLaunchKernelGGL(k_write, P, T, shmem, s, a_dev, buf_words);
    hipLaunchKernelGGL(k_rle_len, P, T, 0, s, a_dev);
    return hipGetLastError();
}

hipError_t launch_huf_decode_batch(const DecodeJob* jobs, uint32_t njobs, const uint32_t* wg_job,
                                   uint32_t grid, uint32_t lanes, uint32_t cap_chunk, hipStream_t s)
{
    if (grid == 0 || njobs == 0) return hipSuccess;
    const dim3 P(grid), T(kThreads);
    if (lanes == 1)
        hipLaunchKernelGGL(k_huf_tables<true>, dim3(njobs), T, 0, s, jobs);
    else
        hipLaunchKernelGGL(k_huf_tables<false>, dim3(njobs), T, 0, s, jobs);
    switch (lanes) {
    case 1: hipLaunchKernelGGL(k_huf_decode, P, T, 0, s, jobs, wg_job); break;
#define MDR_SPLIT(g)                                                                              \
    case g:                                                                                       \
        hipLaunchKernelGGL(k_huf_decode_split<g>, P, T, split_lds_bytes(kThreads / g, cap_chunk), s, jobs, \
                           wg_job, cap_chunk);                                                    \
        break;
    MDR_SPLIT(4)
    MDR_SPLIT(8)
    MDR_SPLIT(16)
    MDR_SPLIT(32)
    MDR_SPLIT(64)
#undef MDR_SPLIT
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

uint32_t huf_decode_lanes(uint32_t want, uint64_t total_chunks, uint32_t max_chunk)
{
    uint32_t g = want;
    if (g == 0) {
        // measured on 256-symbol chunks: 16 lanes (16 symbols a lane) were
        // fastest from 112 to 131040 chunks, 1.3-3.6x faster than one thread a
        // chunk; at 262080 chunks one thread a chunk was 4% ahead of 8 lanes
        if (total_chunks * max_chunk >= kHufOneLaneSymbols) return 1;
        g = min(64u, 16 * max(1u, max_chunk / 256));
    }
    if (g == 1) return 1;
    while (g < 64 && (uint64_t)g * kSplitOut < (uint64_t)kThreads * max_chunk) g <<= 1;  // staging fits
    return g;
}

hipError_t launch_rle_decode_batch(const RleJob* jobs, const uint32_t* wg_gather, uint32_t n_gather,
                                   const uint32_t* wg_expand, uint32_t n_expand, uint64_t total_runs,
                                   uint32_t* lens, uint32_t* starts, uint32_t* temp, hipStream_t s)
{
    if (n_gather == 0 || n_expand == 0 || total_runs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rle_gather, dim3(n_gather), dim3(kThreads), 0, s, jobs, wg_gather, lens);
    hipError_t err = launch_scan_exclusive(lens, starts, total_runs, temp, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_rle_expand, dim3(n_expand), dim3(kThreads), 0, s, jobs, wg_expand, starts);
    return hipGetLastError();
}

}  // namespace mdr
