// Internal declarations shared by the library's kernels (.hip) and its host
// orchestration (.cpp).  Not part of the C ABI (include/mdr.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mdr {

constexpr int kThreads = 256;     // threads per workgroup: 4 wavefronts of 64
constexpr int kTileBlocks = 256;  // 32-value blocks per tile: one per thread
constexpr int kMaxRows = 65;      // sign row + up to 64 magnitude planes
constexpr int kMaxWgEncode = 1024;
constexpr int kLutBitsMax = 12;   // Huffman decode table: 2^lmax entries

// Per-level statistics gathered on the device (zeroed by k_fill before use).
struct LevelStats {
    int32_t emax;          // largest frexp exponent over nonzero values (INT32_MIN: none)
    uint32_t nonfinite;    // nonzero if a NaN / Inf was seen
    uint64_t minkey;       // order-preserving integer key of the minimum
    uint64_t maxkey;       // order-preserving integer key of the maximum
    uint64_t maxabs_bits;  // bit pattern of max |x|
    uint64_t small_bits;   // bit pattern of max |x| over values below 2^(e-B)
    uint64_t pad[3];
};

// Selection result of one lossless unit (sign plane, or a group of m planes).
struct UnitInfo {
    uint64_t S;        // bytes of the unit's concatenated planes
    uint64_t est_huf;  // Huffman size estimate
    uint64_t est_rle;  // RLE size (exact)
    uint64_t nruns;    // runs of equal W-bit words
    uint32_t method;   // MDR_DC / MDR_RLE / MDR_HUF
    uint32_t nchunks;  // Huffman chunks
    uint32_t maxlen;   // longest Huffman code
    uint32_t pad;
};

struct EncodeJob {
    const void* x;          // level values (f32 or f64)
    uint64_t n;
    uint32_t nbd;           // 32-value blocks == u32 words per plane row
    uint32_t B;             // planes
    uint32_t m;             // planes per group
    uint32_t nunits;        // 1 + ceil(B / m)
    uint32_t ntiles;        // ceil(nbd / kTileBlocks)
    uint32_t tiles_per_wg;
    uint32_t grid;          // workgroups of the encode launch
    uint32_t pad;
    uint32_t* rows;         // [(B+1)][nbd]: row 0 sign, row 1+p plane p (bit B-1-p)
    LevelStats* stats;
    uint32_t* hist;         // [grid][nunits][256] nonzero-byte counts
    uint32_t* trans;        // [B+1] word transitions inside each workgroup's range
    uint32_t* recs;         // [grid][B+1][2G] first / last words of each workgroup's range
    unsigned long long* ekeys;  // [B+1] max error keys (float / double bit patterns)
};

struct SelectJob {
    uint64_t nbd;
    uint32_t B, m, nunits, grid, G;  // G: u32 words per W-bit word (1 f32, 2 f64)
    uint32_t t_cr_milli, huf_chunk, huf_lmax;
    int32_t force_method;
    uint64_t t_s;
    const uint32_t* hist;
    const uint32_t* trans;
    const uint32_t* recs;
    UnitInfo* units;        // [nunits]
    uint8_t* lens;          // [nunits][256]
    uint32_t* codes;        // [nunits][256]
};

// ---- launchers (k_refactor.hip) ----
hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s);
hipError_t launch_init_stats(LevelStats* st, int count, hipStream_t s);
hipError_t launch_stats(const void* x, uint64_t n, bool f64, LevelStats* st, hipStream_t s);
hipError_t launch_encode(const EncodeJob& job, bool f64, hipStream_t s);
hipError_t launch_select(const SelectJob& job, hipStream_t s);

// ---- launchers (k_lossless.hip) ----
// exclusive scan of n u32 values (out may alias in); temp: scan_temp_words(n) u32
uint64_t scan_temp_words(uint64_t n);
hipError_t launch_scan_exclusive(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* temp,
                                 hipStream_t s);
// Huffman: payload layout u64 nsym | u8 len[256] | u32 off[nchunks+1] | u32 words[]
hipError_t launch_huf_encode(const uint8_t* g, uint64_t S, uint32_t chunk, const uint8_t* lens,
                             const uint32_t* codes, uint8_t* payload, uint32_t* temp,
                             hipStream_t s);
hipError_t launch_huf_decode(const uint8_t* payload, uint64_t S, uint32_t chunk, uint32_t lmax,
                             uint8_t* g, hipStream_t s);
// RLE: payload u32 nruns | u32 wbytes | symbols[nruns] | u32 lengths[nruns]
hipError_t launch_rle_encode(const uint8_t* g, uint64_t nwords, uint32_t G, uint64_t nruns,
                             uint8_t* payload, uint32_t* temp, hipStream_t s);
hipError_t launch_rle_decode(const uint8_t* payload, uint64_t nwords, uint32_t G, uint64_t nruns,
                             uint8_t* g, uint32_t* temp, hipStream_t s);
uint64_t rle_temp_words(uint64_t nwords);

// ---- launchers (k_retrieve.hip) ----
struct ReconJob {
    const uint32_t* rows[kMaxRows];  // row pointers (row 0 = sign, 1+p = plane p), by value
    void* out;
    uint64_t n;
    uint32_t nbd, B, k;
    int32_t e;
};
hipError_t launch_reconstruct(const ReconJob& job, bool f64, hipStream_t s);

}  // namespace mdr
