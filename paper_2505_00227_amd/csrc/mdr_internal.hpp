// Internal declarations shared by the library's kernels (.hip) and its host
// orchestration (.cpp).  Not part of the C ABI (include/mdr.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mdr {

constexpr int kThreads = 256;     // threads per workgroup: 4 wavefronts of 64
constexpr int kTileBlocks = 256;  // 32-value blocks per tile: one per thread
constexpr int kMaxRows = 65;      // sign row + up to 64 magnitude planes
constexpr int kMaxWgEncode = 768;  // three encoder workgroups per CU run at once
constexpr int kLutBitsMax = 12;   // Huffman decode table: 2^lmax entries
constexpr int kKeyStride = 66;    // error keys k = 0..64, then [65] = max |x| below 2^(e-B)

// Per-level statistics gathered on the device (zeroed by k_fill before use).
// The bit pattern of max |x| also gives the alignment exponent (the largest
// frexp exponent over nonzero values is that of max |x|; 0 when all are zero)
// and reveals NaN / Inf, whose patterns are the largest.
struct LevelStats {
    uint64_t minkey;       // order-preserving integer key of the minimum
    uint64_t maxkey;       // order-preserving integer key of the maximum
    uint64_t maxabs_bits;  // bit pattern of max |x|
    uint64_t pad[5];
};

// statistics workgroups: threads, and at most this many per level (each
// publishes with three device atomics when it ends)
constexpr uint32_t kStatsThreads = 1024;
constexpr uint32_t kStatsMaxWg = 256;

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

// Work of one level in a flattened batch launch.  The tables below live in
// device memory; a workgroup finds its job through a per-launch map
// (workgroup -> job index) and its rank within the job as blockIdx - wg_base.
struct StatsJob {
    const void* x;
    uint64_t n;
    LevelStats* stats;
    uint32_t wg_base;       // first workgroup of this job in its launch
    uint32_t grid;          // workgroups of this job
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
    uint32_t grid;          // workgroups of this job
    uint32_t wg_base;       // first workgroup of this job in its launch
    uint32_t* rows;         // [(B+1)][nbd]: row 0 sign, row 1+p plane p (bit B-1-p)
    LevelStats* stats;
    // level totals, zeroed before the pass; workgroups add (max) theirs in
    uint32_t* hist;         // [nunits][256] nonzero-byte counts
    uint32_t* trans;        // [kMaxRows] word transitions inside workgroup ranges
    unsigned long long* keys;  // [kKeyStride] max error keys (float/double bits), small
    uint32_t* recs;         // [grid][kMaxRows][2G] first / last words of each workgroup's range
    uint16_t hist_off[kMaxRows];   // row r -> its unit's histogram offset (unit * 256)
};

// Per-level inputs / outputs of the selection kernel.
struct SelectLevel {
    uint64_t nbd;           // 0 for an empty level
    uint32_t grid;          // workgroups of that level's encode job
    uint32_t pad;
    const uint32_t* hist;   // [nunits][256] level totals from the encoder
    const uint32_t* trans;  // [kMaxRows] level totals from the encoder
    const uint32_t* recs;   // [grid][kMaxRows][2G]
    UnitInfo* units;        // [nunits]
    uint8_t* lens;          // [nunits][256]
    uint32_t* codes;        // [nunits][256]
};

struct SelectParams {
    uint32_t B, m, nunits, G;  // G: u32 words per W-bit word (1 f32, 2 f64)
    uint32_t t_cr_milli, huf_chunk, huf_lmax;
    int32_t force_method;
    uint32_t threads;  // workgroup size of the selection kernel: 256, 512 or 1024
    uint64_t t_s;
};

// Lossless stage of a batch.  Units are numbered level-major over the batch
// (unit u = job * nunits + i); unit i of a level holds rows [r0, r1) with
// r0 = i == 0 ? 0 : 1 + (i - 1) m.  Sizes are decided on the device, so the
// stage needs no host round trip; payloads go to one arena of capacity `cap`.
constexpr uint32_t kRleTileWords = 4096;  // W-bit words per run-length tile
constexpr uint32_t kPersistWg = 1024;     // workgroups of the persistent lossless kernels
constexpr uint32_t kSelectManyUnits = 1024;  // units of a pass from which the selection runs 256-thread workgroups

struct LosslessArgs {
    const EncodeJob* jobs;  // rows and nbd of each level
    const UnitInfo* units;  // [U] selection results
    const uint8_t* lens;    // [U][256]
    const uint32_t* codes;  // [U][256]
    uint32_t* chunk_base;   // [U+1] first Huffman chunk of each unit (0 if not HUF)
    uint32_t* tile_base;    // [U+1] first run-length tile of each unit
    uint32_t* chunk_words;  // [chunks+1] words per chunk, scanned in place to offsets
    uint32_t* tile_runs;    // [tiles+1] runs starting in each tile, scanned in place
    uint64_t* pay_off;      // [U] payload offset in the arena (DC: unused)
    uint64_t* unit_bytes;   // [U] stream bytes
    uint32_t* counts;       // [0] chunks, [1] tiles, [2] arena overflow, [3] pad, [4..5] arena bytes
    uint8_t* arena;
    uint64_t cap;
    uint32_t U, nunits, B, m, G, huf_chunk;
};

// ---- launchers (k_refactor.hip) ----
hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s);
// copy `bytes` (a multiple of 8) from pinned host memory (hipHostMalloc) to
// device memory with a kernel on `s`: no copy-engine transfer, so the kernels
// behind it start without waiting on another engine; under capture the kernel
// reads the host memory at every replay
hipError_t launch_copy_in(void* dst, const void* host, uint64_t bytes, hipStream_t s);
// level statistics [count] to their neutral values, z0[n0] and z1[n1] to zero
hipError_t launch_init_pass(LevelStats* st, uint32_t count, uint32_t* z0, uint64_t n0, uint32_t* z1,
                            uint64_t n1, hipStream_t s);
// statistics of every job; wg_job maps each of `grid` workgroups to its job
hipError_t launch_stats_batch(const StatsJob* jobs, const uint32_t* wg_job, uint32_t grid, bool f64,
                              bool vec, hipStream_t s);
size_t encode_lds_bytes(uint32_t nunits, uint32_t B, uint32_t m, bool f64);
// raise the encoder kernels' dynamic LDS limit (call outside graph capture)
hipError_t encode_set_lds(uint32_t nunits, uint32_t B, uint32_t m, bool f64);
hipError_t launch_encode_batch(const EncodeJob* jobs, const uint32_t* wg_job, uint32_t grid,
                               uint32_t nunits, uint32_t B, uint32_t m, bool f64, bool vec, hipStream_t s);
hipError_t launch_select_batch(const SelectParams& p, const SelectLevel* lv, uint32_t nlev,
                               hipStream_t s);

// ---- launchers (k_lossless.hip) ----
// exclusive scan of n u32 values (out may alias in); temp: scan_temp_words(n) u32
uint64_t scan_temp_words(uint64_t n);
hipError_t launch_scan_exclusive(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* temp,
                                 hipStream_t s);
// Huffman and run-length encoding of every unit the selection chose, sizes
// and arena offsets decided on the device (grid sizes fixed: graph-capturable).
// scan_part: 2 * kPersistWg + 64 u32 of scratch.
hipError_t launch_lossless_batch(const LosslessArgs& a, const LosslessArgs* a_dev, uint32_t* scan_part,
                                 hipStream_t s);
// Huffman decode of many streams in one launch (payload u64 nsym | u8 len[256] |
// u32 off[nchunks+1] | u32 words[]); kThreads chunks per workgroup
struct DecodeJob {
    const uint8_t* payload;
    uint8_t* out;           // S decoded bytes
    void* table;            // kHufTableBytes of device scratch, 16-byte aligned: the stream's decode table
    uint64_t S;
    uint32_t nchunks, chunk, lmax;
    uint32_t wg_base;       // first workgroup of this job in the launch
};
constexpr uint64_t kHufTableBytes = 4ull << kLutBitsMax;  // 2^lmax 32-bit entries at most
// lanes per chunk: 1 (kThreads chunks per workgroup) or 4..64 (kThreads / lanes
// chunks per workgroup); cap_chunk: the largest chunk of the jobs.  A first
// launch builds every job's decode table into its table slot, which the
// decoding workgroups copy
hipError_t launch_huf_decode_batch(const DecodeJob* jobs, uint32_t njobs, const uint32_t* wg_job,
                                   uint32_t grid, uint32_t lanes, uint32_t cap_chunk, hipStream_t s);
// lanes per chunk for a launch of total_chunks chunks, the largest chunk
// max_chunk symbols: want = 0 picks by the symbol count (16 symbols a lane
// below kHufOneLaneSymbols); 1 stays 1; 4..64 is raised where a workgroup's
// chunks would not fit its LDS staging
constexpr uint64_t kHufOneLaneSymbols = 196608ull * 256;  // one thread a chunk from this many symbols on
uint32_t huf_decode_lanes(uint32_t want, uint64_t total_chunks, uint32_t max_chunk);
// RLE decode of every run-length group of a retrieval: payload u32 nruns |
// u32 wbytes | symbols[nruns][G] | u32 lengths[nruns]
struct RleJob {
    const uint8_t* payload;
    uint8_t* out;        // nwords W-bit words (G 32-bit words each)
    uint64_t nwords, nruns;
    uint64_t run_base;   // first run of this group in the launch's run arrays
    uint32_t G;
    uint32_t wg_gather;  // first workgroup of this group in the gather launch
    uint32_t wg_expand;  // first workgroup of this group in the expand launch
};
constexpr uint32_t kRlePerWg = kThreads * 16;  // runs (gather) or words (expand) per workgroup
// lens, starts: total_runs u32 each; temp: scan_temp_words(total_runs) u32
hipError_t launch_rle_decode_batch(const RleJob* jobs, const uint32_t* wg_gather, uint32_t n_gather,
                                   const uint32_t* wg_expand, uint32_t n_expand, uint64_t total_runs,
                                   uint32_t* lens, uint32_t* starts, uint32_t* temp, hipStream_t s);

// ---- launchers (k_retrieve.hip) ----
struct ReconJob {
    const uint32_t* rows[kMaxRows];  // row pointers (row 0 = sign, 1+p = plane p)
    void* out;
    uint64_t n;
    uint32_t nbd, B, k;
    int32_t e;
    uint32_t wg_base;  // first workgroup of this job in the launch
    uint32_t vec;      // out is 16-byte aligned
};
// reconstruction of many levels (one dtype) in one launch; kThreads blocks per workgroup
// streaming: the launch reads most of its levels' planes (streaming loads and stores)
hipError_t launch_reconstruct_batch(const ReconJob* jobs, const uint32_t* wg_job, uint32_t grid,
                                   bool f64, bool streaming, hipStream_t s);
// V_total estimate of many (request, level) jobs of one dtype; acc must hold 0 first
// QoI families, as mdr_qoi_kind numbers them
constexpr uint32_t kQoiSumsq = 0, kQoiMagnitude = 1, kQoiProduct = 2;
struct QoiJob {
    const void* x;
    const void* y;
    const void* z;
    uint64_t n;
    double eps[3];
    unsigned long long* acc;  // max of the estimate's bit patterns (non-negative doubles)
    unsigned long long* arg;  // first point attaining it (argmax launch only)
    uint64_t base;            // index of the job's first point in its variable
    uint32_t kind, nvars;     // QoI family (kQoi*) and its variables (absent ones: zero bounds)
    uint32_t wg_base, grid;   // this job's workgroups in the launch
    uint32_t vec;             // x, y and z are 16-byte aligned (set by the launcher)
};
hipError_t launch_qoi_vtotal_batch(const QoiJob* jobs, const uint32_t* wg_job, uint32_t grid, bool f64,
                                   hipStream_t s);
// ---- device values to pinned host memory by a kernel (k_retrieve.hip): up to
// kCopySpans spans of 4-byte words, each from device memory to the device
// address of pinned host memory
constexpr int kCopySpans = 16;
struct CopySpans {
    const uint32_t* src[kCopySpans];
    uint32_t* dst[kCopySpans];
    uint64_t words[kCopySpans];
    uint32_t n;
};
hipError_t launch_copy_out(const CopySpans& sp, hipStream_t s);

// ---- squared-L2 per-plane table (k_l2.hip)
// fixed scratch of the allocation-free variant (mdr_l2_table_noalloc): at most
// kL2NoAllocLevels levels per call; its device address is resolved once per
// device (l2_scratch_init, with the device current or made current), after
// which l2_scratch hands out the partial-row and table areas
constexpr uint32_t kL2RowMax = 66;  // a level's L2 row: E2[0..B] and the largest |x|, B <= 64
constexpr uint32_t kL2NoAllocLevels = 64;
hipError_t l2_scratch_init(int device);
hipError_t l2_scratch(int device, double** part, double** out);
// part: l2_table_workgroups(n) * (B + 2) doubles; out: B + 2 doubles (the table, then the
// largest |x| read); B <= 32 for f32, <= 64 for f64
uint32_t l2_table_workgroups(uint64_t n);
hipError_t launch_l2_table(bool f64, const void* x, uint64_t n, int e, uint32_t B, double* part, double* out,
                           hipStream_t s);

// ---- multilevel decomposition (k_multilevel.hip): field <-> coefficient levels
constexpr uint32_t kMlMaxSteps = 30;
struct MlOffsets {
    uint64_t off[kMlMaxSteps + 1];  // first value of each level, coarsest first
};
// n0, n1 < 65536 (grid y/z); n2 < 2^31; `out` / `u` must not overlap the input
hipError_t launch_decompose(bool f64, const void* u, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t nsteps,
                            const MlOffsets& off, void* out, hipStream_t s);
hipError_t launch_recompose(bool f64, const void* c, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t nsteps,
                            const MlOffsets& off, void* u, hipStream_t s);

// ---- encoder-design ablation (k_ablation.hip): 32-bit words <-> 32 planes
constexpr int kAblLocality = 0, kAblBallot = 1, kAblShift = 2, kAblButterfly = 3, kAblRegBlock = 4;
uint64_t ablation_plane_words(int design, uint64_t n);
// encode: in[n] -> planes[32][words]; decode: planes -> out[n]
hipError_t launch_ablation(int design, bool encode, const uint32_t* in, uint64_t n, uint32_t* planes,
                           uint32_t* out, hipStream_t s);

// after launch_qoi_vtotal_batch on the same jobs: min over points whose estimate
// equals *acc of base + index, into *arg (which starts at ~0)
hipError_t launch_qoi_vtotal_argmax_batch(const QoiJob* jobs, const uint32_t* wg_job, uint32_t grid, bool f64,
                                          hipStream_t s);

}  // namespace mdr
