// Lossless kernels for gfx950 (Sec. 4.1): device-wide exclusive scan, chunked
// canonical Huffman coding of byte symbols, and run-length coding of W-bit
// plane words.  Direct copy needs no kernel: its payload is the plane rows.
#include "mdr_internal.hpp"

namespace mdr {
namespace {

constexpr int kScanItems = 4;                          // per thread
constexpr int kScanTile = kThreads * kScanItems;       // per workgroup

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(v, off, 64);
        if (lane >= (uint32_t)off) v += o;
    }
    return v;
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

// ------------------------------------------------------------------ Huffman encode
// Payload: u64 nsym | u8 len[256] | u32 off[nchunks+1] | u32 words[].
// Chunk c (chunk symbols) starts at word off[c]; code bits are packed most
// significant first.  One wavefront per chunk; each lane owns chunk/64
// consecutive symbols (a multiple of 4 bytes).
constexpr uint64_t kHufHeader = 8 + 256;

__global__ __launch_bounds__(kThreads) void k_huf_count(const uint8_t* g, uint64_t S,
                                                        uint32_t chunk, const uint8_t* lens,
                                                        uint8_t* payload, uint32_t nchunks)
{
    __shared__ uint32_t s_len[256];
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    s_len[tid] = lens[tid];
    if (blockIdx.x == 0) {
        payload[8 + tid] = lens[tid];
        if (tid == 0) *reinterpret_cast<uint64_t*>(payload) = S;
    }
    __syncthreads();
    uint32_t* off = reinterpret_cast<uint32_t*>(payload + kHufHeader);
    const uint32_t c = blockIdx.x * (kThreads / 64) + (tid >> 6);
    if (c > nchunks) return;
    if (c == nchunks) {
        if (lane == 0) off[c] = 0;
        return;
    }
    const uint32_t per = chunk / 64;
    const uint64_t lo = (uint64_t)c * chunk + (uint64_t)lane * per;
    uint32_t bits = 0;
    for (uint32_t q = 0; q < per; q += 4) {
        if (lo + q >= S) break;
        uint32_t w = *reinterpret_cast<const uint32_t*>(g + lo + q);
        bits += s_len[w & 0xFF] + s_len[(w >> 8) & 0xFF] + s_len[(w >> 16) & 0xFF] + s_len[w >> 24];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bits += __shfl_xor(bits, o, 64);
    if (lane == 0) off[c] = (bits + 31) / 32;
}

__global__ __launch_bounds__(kThreads) void k_huf_write(const uint8_t* g, uint64_t S,
                                                        uint32_t chunk, const uint8_t* lens,
                                                        const uint32_t* codes, uint8_t* payload,
                                                        uint32_t nchunks, uint32_t buf_words)
{
    extern __shared__ uint32_t s_buf[];  // [4][buf_words]
    __shared__ uint32_t s_len[256], s_code[256];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    s_len[tid] = lens[tid];
    s_code[tid] = codes[tid];
    uint32_t* buf = s_buf + wave * buf_words;
    for (uint32_t i = lane; i < buf_words; i += 64) buf[i] = 0;
    __syncthreads();
    const uint32_t c = blockIdx.x * (kThreads / 64) + wave;
    if (c >= nchunks) return;
    const uint32_t* off = reinterpret_cast<const uint32_t*>(payload + kHufHeader);
    uint32_t* words = reinterpret_cast<uint32_t*>(payload + kHufHeader + 4ull * (nchunks + 1));
    const uint32_t per = chunk / 64;
    const uint64_t lo = (uint64_t)c * chunk + (uint64_t)lane * per;
    uint32_t bits = 0;
    for (uint32_t q = 0; q < per; q += 4) {
        if (lo + q >= S) break;
        uint32_t w = *reinterpret_cast<const uint32_t*>(g + lo + q);
        bits += s_len[w & 0xFF] + s_len[(w >> 8) & 0xFF] + s_len[(w >> 16) & 0xFF] + s_len[w >> 24];
    }
    uint32_t pos = wave_incl_scan(bits, lane) - bits;
    for (uint32_t q = 0; q < per; q += 4) {
        if (lo + q >= S) break;
        uint32_t w = *reinterpret_cast<const uint32_t*>(g + lo + q);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            uint32_t sym = (w >> (8 * b)) & 0xFF;
            uint32_t L = s_len[sym], cd = s_code[sym];
            uint32_t wi = pos >> 5, o = pos & 31;
            if (o + L <= 32) {
                atomicOr(&buf[wi], cd << (32 - o - L));
            } else {
                atomicOr(&buf[wi], cd >> (o + L - 32));
                atomicOr(&buf[wi + 1], cd << (64 - o - L));
            }
            pos += L;
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    const uint32_t w0 = off[c], nw = off[c + 1] - w0;
    for (uint32_t i = lane; i < nw; i += 64) words[w0 + i] = buf[i];
}

// ------------------------------------------------------------------ Huffman decode
// One thread per chunk; a 2^lmax-entry table in LDS maps the next lmax bits to
// (symbol, length).
__global__ __launch_bounds__(kThreads) void k_huf_decode(const uint8_t* payload, uint64_t S,
                                                         uint32_t chunk, uint32_t lmax,
                                                         uint8_t* g, uint32_t nchunks)
{
    __shared__ uint16_t s_lut[1 << kLutBitsMax];
    __shared__ uint8_t s_len[256];
    __shared__ uint32_t s_count[33], s_first[33], s_offset[33];
    __shared__ uint8_t s_sorted[256];
    const uint32_t tid = threadIdx.x;
    s_len[tid] = payload[8 + tid];
    if (tid < 33) s_count[tid] = 0;
    __syncthreads();
    const uint32_t L = s_len[tid];
    if (L && L <= lmax) atomicAdd(&s_count[L], 1u);
    __syncthreads();
    if (tid == 0) {
        uint32_t c = 0, o = 0;
        for (int l = 1; l <= 32; ++l) {
            s_first[l] = c;
            s_offset[l] = o;
            o += s_count[l];
            c = (c + s_count[l]) << 1;
        }
    }
    __syncthreads();
    if (L && L <= lmax) {
        uint32_t before = 0;
        for (uint32_t s = 0; s < tid; ++s) before += s_len[s] == L ? 1u : 0u;
        s_sorted[s_offset[L] + before] = (uint8_t)tid;
    }
    __syncthreads();
    for (uint32_t i = tid; i < (1u << lmax); i += kThreads) {
        uint16_t ent = (uint16_t)(lmax << 8);  // invalid prefix: consume lmax bits
        for (uint32_t l = 1; l <= lmax; ++l) {
            uint32_t p = i >> (lmax - l);
            if (s_count[l] && p >= s_first[l] && p - s_first[l] < s_count[l]) {
                ent = (uint16_t)((l << 8) | s_sorted[s_offset[l] + p - s_first[l]]);
                break;
            }
        }
        s_lut[i] = ent;
    }
    __syncthreads();
    const uint32_t c = blockIdx.x * kThreads + tid;
    if (c >= nchunks) return;
    const uint32_t* off = reinterpret_cast<const uint32_t*>(payload + kHufHeader);
    const uint32_t* words = reinterpret_cast<const uint32_t*>(payload + kHufHeader + 4ull * (nchunks + 1));
    uint32_t wp = off[c];
    const uint32_t wend = off[c + 1];
    uint64_t buf = 0;
    int nb = 0;
    const uint64_t lo = (uint64_t)c * chunk;
    const uint64_t cnt = (lo + chunk <= S) ? chunk : S - lo;
    uint32_t* dst = reinterpret_cast<uint32_t*>(g + lo);
    for (uint64_t i = 0; i < cnt; i += 4) {
        uint32_t out = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (nb <= 32) {
                uint32_t w = wp < wend ? words[wp] : 0u;
                ++wp;
                buf |= (uint64_t)w << (32 - nb);
                nb += 32;
            }
            uint32_t ent = s_lut[buf >> (64 - lmax)];
            uint32_t l = ent >> 8;
            out |= (ent & 0xFFu) << (8 * b);
            buf <<= l;
            nb -= (int)l;
        }
        dst[i / 4] = out;
    }
}

// ------------------------------------------------------------------ RLE
// Payload: u32 nruns | u32 wbytes | symbols[nruns] (W-bit) | u32 lengths[nruns].
__device__ __forceinline__ bool word_ne(const uint32_t* g, uint64_t i, uint64_t j, uint32_t G)
{
    bool ne = false;
    for (uint32_t q = 0; q < G; ++q) ne = ne || g[i * G + q] != g[j * G + q];
    return ne;
}

__global__ void k_rle_flags(const uint32_t* g, uint64_t nwords, uint32_t G, uint32_t* flags)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride)
        flags[i] = (i == 0 || word_ne(g, i, i - 1, G)) ? 1u : 0u;
}

__global__ void k_rle_scatter(const uint32_t* g, uint64_t nwords, uint32_t G, const uint32_t* idx,
                              uint8_t* payload, uint32_t* starts, uint64_t nruns)
{
    uint32_t* sym = reinterpret_cast<uint32_t*>(payload + 8);
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride) {
        if (i == 0 || word_ne(g, i, i - 1, G)) {
            uint64_t r = idx[i];
            if (r < nruns) {
                for (uint32_t q = 0; q < G; ++q) sym[r * G + q] = g[i * G + q];
                starts[r] = (uint32_t)i;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        reinterpret_cast<uint32_t*>(payload)[0] = (uint32_t)nruns;
        reinterpret_cast<uint32_t*>(payload)[1] = 4 * G;
    }
}

__global__ void k_rle_lengths(const uint32_t* starts, uint64_t nruns, uint64_t nwords, uint32_t G,
                              uint8_t* payload)
{
    uint32_t* lens = reinterpret_cast<uint32_t*>(payload + 8 + 4ull * G * nruns);
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nruns; r += stride) {
        uint64_t end = r + 1 < nruns ? starts[r + 1] : nwords;
        lens[r] = (uint32_t)(end - starts[r]);
    }
}

__global__ void k_rle_expand(const uint8_t* payload, uint64_t nwords, uint32_t G, uint64_t nruns,
                             const uint32_t* starts, uint32_t* g)
{
    const uint32_t* sym = reinterpret_cast<const uint32_t*>(payload + 8);
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride) {
        // last run whose start is <= i
        uint64_t lo = 0, hi = nruns;  // invariant: starts[lo] <= i, answer in [lo, hi)
        while (hi - lo > 1) {
            uint64_t mid = (lo + hi) / 2;
            if (starts[mid] <= i)
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

hipError_t launch_huf_encode(const uint8_t* g, uint64_t S, uint32_t chunk, const uint8_t* lens,
                             const uint32_t* codes, uint8_t* payload, uint32_t* temp,
                             hipStream_t s)
{
    const uint32_t nchunks = (uint32_t)((S + chunk - 1) / chunk);
    const unsigned wgs = blocks_for((uint64_t)nchunks + 1, kThreads / 64, 1u << 30);
    hipLaunchKernelGGL(k_huf_count, dim3(wgs), dim3(kThreads), 0, s, g, S, chunk, lens, payload,
                       nchunks);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    uint32_t* off = reinterpret_cast<uint32_t*>(payload + kHufHeader);
    err = launch_scan_exclusive(off, off, (uint64_t)nchunks + 1, temp, s);
    if (err != hipSuccess || nchunks == 0) return err;
    const uint32_t buf_words = (chunk * kLutBitsMax + 31) / 32 + 2;
    const size_t shmem = 4ull * buf_words * sizeof(uint32_t);
    hipLaunchKernelGGL(k_huf_write, dim3(blocks_for(nchunks, kThreads / 64, 1u << 30)),
                       dim3(kThreads), shmem, s, g, S, chunk, lens, codes, payload, nchunks,
                       buf_words);
    return hipGetLastError();
}

hipError_t launch_huf_decode(const uint8_t* payload, uint64_t S, uint32_t chunk, uint32_t lmax,
                             uint8_t* g, hipStream_t s)
{
    const uint32_t nchunks = (uint32_t)((S + chunk - 1) / chunk);
    if (nchunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_huf_decode, dim3(blocks_for(nchunks, kThreads, 1u << 30)), dim3(kThreads),
                       0, s, payload, S, chunk, lmax, g, nchunks);
    return hipGetLastError();
}

uint64_t rle_temp_words(uint64_t nwords)
{
    return 2 * nwords + scan_temp_words(nwords) + 64;
}

hipError_t launch_rle_encode(const uint8_t* g, uint64_t nwords, uint32_t G, uint64_t nruns,
                             uint8_t* payload, uint32_t* temp, hipStream_t s)
{
    const uint32_t* gw = reinterpret_cast<const uint32_t*>(g);
    uint32_t* flags = temp;
    uint32_t* starts = temp + nwords;
    uint32_t* scratch = temp + 2 * nwords + 64;
    unsigned b = blocks_for(nwords, kThreads, 8192);
    if (nwords) {
        hipLaunchKernelGGL(k_rle_flags, dim3(b), dim3(kThreads), 0, s, gw, nwords, G, flags);
        hipError_t err = launch_scan_exclusive(flags, flags, nwords, scratch, s);
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k_rle_scatter, dim3(b), dim3(kThreads), 0, s, gw, nwords, G, flags, payload,
                       starts, nruns);
    if (nruns)
        hipLaunchKernelGGL(k_rle_lengths, dim3(blocks_for(nruns, kThreads, 8192)), dim3(kThreads),
                           0, s, starts, nruns, nwords, G, payload);
    return hipGetLastError();
}

hipError_t launch_rle_decode(const uint8_t* payload, uint64_t nwords, uint32_t G, uint64_t nruns,
                             uint8_t* g, uint32_t* temp, hipStream_t s)
{
    if (nwords == 0 || nruns == 0) return hipSuccess;
    const uint32_t* lens = reinterpret_cast<const uint32_t*>(payload + 8 + 4ull * G * nruns);
    uint32_t* starts = temp;
    uint32_t* scratch = temp + nruns + 64;
    hipError_t err = launch_scan_exclusive(lens, starts, nruns, scratch, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_rle_expand, dim3(blocks_for(nwords, kThreads, 8192)), dim3(kThreads), 0,
                       s, payload, nwords, G, nruns, starts, reinterpret_cast<uint32_t*>(g));
    return hipGetLastError();
}

}  // namespace mdr
