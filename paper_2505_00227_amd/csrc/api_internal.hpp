// Host-side objects behind the C ABI handles.
#pragma once

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "mdr.h"
#include "mdr_internal.hpp"

struct mdr_context;

namespace mdr {

// Owned device allocation (hipFree on destruction).
struct DevBuf {
    void* p = nullptr;
    uint64_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr, o.bytes = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept
    {
        reset();
        p = o.p, bytes = o.bytes;
        o.p = nullptr, o.bytes = 0;
        return *this;
    }
    ~DevBuf() { reset(); }
    void reset()
    {
        if (p) (void)hipFree(p);
        p = nullptr, bytes = 0;
    }
    hipError_t alloc(uint64_t n)
    {
        reset();
        if (n == 0) return hipSuccess;
        hipError_t e = hipMalloc(&p, n);
        if (e == hipSuccess) bytes = n;
        else p = nullptr;
        return e;
    }
};

// Freed device blocks a context keeps for reuse, at most.
constexpr uint64_t kPoolCacheBytes = 8ull << 30;

// Caching device allocator of one context.  Blocks come back to a size-sorted
// free list and are reused by later requests that fit them (within 2x); the
// list keeps at most `cap` bytes.  Callers return a block only after the work
// using it has completed (the handles' destroy calls synchronize the device).
class DevicePool {
public:
    explicit DevicePool(uint64_t cap) : cap_(cap) {}
    ~DevicePool();
    hipError_t alloc(uint64_t bytes, void** p, uint64_t* got);
    void release(void* p, uint64_t bytes);
    uint64_t cached() const { return cached_; }
private:
    std::mutex mu_;
    std::multimap<uint64_t, void*> free_;
    uint64_t cached_ = 0, cap_;
};

// A block from a DevicePool (returned to it on destruction).
struct PoolBuf {
    std::shared_ptr<DevicePool> pool;
    void* p = nullptr;
    uint64_t bytes = 0;
    PoolBuf() = default;
    PoolBuf(const PoolBuf&) = delete;
    PoolBuf& operator=(const PoolBuf&) = delete;
    PoolBuf(PoolBuf&& o) noexcept : pool(std::move(o.pool)), p(o.p), bytes(o.bytes) { o.p = nullptr, o.bytes = 0; }
    PoolBuf& operator=(PoolBuf&& o) noexcept
    {
        reset();
        pool = std::move(o.pool), p = o.p, bytes = o.bytes;
        o.p = nullptr, o.bytes = 0;
        return *this;
    }
    ~PoolBuf() { reset(); }
    void reset()
    {
        if (p && pool) pool->release(p, bytes);
        p = nullptr, bytes = 0;
    }
    hipError_t alloc(const std::shared_ptr<DevicePool>& pl, uint64_t n)
    {
        reset();
        pool = pl;
        if (n == 0) return hipSuccess;
        return pool->alloc(n, &p, &bytes);
    }
};

struct UnitRec {
    int32_t method = MDR_PLACEHOLDER;
    uint64_t bytes = 0;    // payload bytes (0 for placeholders)
    uint64_t S = 0;        // decoded bytes of the unit
    uint64_t nruns = 0;    // RLE runs
    uint64_t est_huf = 0, est_rle = 0;
    uint32_t nchunks = 0;  // Huffman chunks
    uint32_t maxlen = 0;   // longest Huffman code
    uint8_t* dev = nullptr;  // payload (DC: the plane rows themselves)
};

struct LevelRec {
    uint64_t n = 0;
    uint32_t nbd = 0;  // u32 words per plane row
    int32_t e = 0;
    double vmin = 0, vmax = 0, vmaxabs = 0;
    std::vector<double> E;      // B+1
    std::vector<double> E2;     // B+1 squared-L2 errors, once mdr_l2_table has run (else empty)
    uint32_t* rows = nullptr;   // [(B+1)][nbd]
    UnitRec units[kMaxRows];    // slot 0 = sign, 1+p = plane p
};

// first row / row count of the unit at table slot s
inline void slot_rows(uint32_t slot, uint32_t B, uint32_t m, uint32_t& r0, uint32_t& r1)
{
    if (slot == 0) {
        r0 = 0, r1 = 1;
    } else {
        r0 = slot;
        r1 = r0 + m < B + 1 ? r0 + m : B + 1;
    }
}

void set_error(const std::string& msg);

// Bracket one stage's launches with timing events when the context asks for it.
class StageTimer {
public:
    StageTimer(mdr_context* ctx, int stage, hipStream_t s);
    ~StageTimer();
private:
    mdr_context* ctx_;
    int stage_;
    hipStream_t s_;
    hipEvent_t start_ = nullptr;
};
mdr_status fail(mdr_status st, const std::string& msg);
mdr_status hip_fail(hipError_t e, const char* what);

#define MDR_HIP(expr)                                            \
    do {                                                         \
        hipError_t _e = (expr);                                  \
        if (_e != hipSuccess) return ::mdr::hip_fail(_e, #expr); \
    } while (0)

inline uint64_t align256(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

// grow-only buffers of a context (synchronize the device before a regrowth)
mdr_status ensure_dev(DevBuf& b, uint64_t need);
mdr_status ensure_stage(mdr_context* ctx, uint64_t need);
mdr_status check_params(const mdr_codec_params& p, uint32_t B);

// The levels of one variable of a batch.
struct VarLevels {
    const mdr_level_view* levels;
    uint32_t nlevels;
};

// Refactor every variable in one flattened pass: one launch per stage over all
// levels of all variables, sizes decided on the device, one host round trip at
// the end.  With `graph`, the pass is captured once per shape and replayed.
mdr_status refactor_batch(mdr_context* ctx, const VarLevels* vars, uint32_t nvars, mdr_dtype dtype,
                          uint32_t B, const mdr_codec_params& prm, hipStream_t s, bool graph,
                          mdr_refactored** outs);
void release_graphs(mdr_context* ctx);

// One retriever's share of a batched retrieval.
struct RetrieveTask {
    mdr_retriever* rt = nullptr;
    std::vector<uint32_t> knew;         // planes per level after the call
    void* const* out = nullptr;         // per-level outputs
    double tol_abs = 0.0;
    mdr_retrieve_info* info = nullptr;  // may be NULL
    bool all_levels = true;             // false: skip levels whose planes did not change
    bool reconstruct = true;            // false: decode only (a shared decode cache)
};
// A reconstruction from a retriever's decoded groups at k (each k_l no more
// than the planes it holds after the call's decodes), written to out.
struct ReconOnly {
    const mdr_retriever* rt = nullptr;
    std::vector<uint32_t> k;
    const std::vector<uint32_t>* kprev = nullptr;  // skip levels where k equals this (may be NULL)
    void* const* out = nullptr;
};
// Decode and reconstruct for every task at once (each retriever at most once),
// plus the extra reconstructions.
mdr_status retrieve_many(mdr_context* ctx, RetrieveTask* tasks, size_t ntasks, hipStream_t s,
                         const ReconOnly* extra = nullptr, size_t nextra = 0);
// V_total estimates: jobs (acc pointers included) in one launch per dtype,
// after clearing `nacc` accumulators at acc0.  argmax: also the first point
// attaining each maximum (jobs' arg pointers, nacc slots from acc0 + nacc).
mdr_status enqueue_qoi(mdr_context* ctx, const std::vector<QoiJob>& jobs, const std::vector<bool>& f64,
                       unsigned long long* acc0, uint32_t nacc, hipStream_t s, bool argmax = false);

// tolerance planner (greedy over levels, exact error tables)
// the greedy planner over an error table of each level: E (L-infinity, the
// default) or E2 (squared L2, with tol the squared tolerance)
using ErrTable = const std::vector<double> LevelRec::*;
double plan_bound(const mdr_refactored* r, const std::vector<uint32_t>& k, ErrTable tab = &LevelRec::E);
bool plan_step(const mdr_refactored* r, std::vector<uint32_t>& k, ErrTable tab = &LevelRec::E);
double plan_to(const mdr_refactored* r, double tol, std::vector<uint32_t>& k, ErrTable tab = &LevelRec::E);
double value_range(const mdr_refactored* r);

// Staging for the job tables of asynchronous launches: pinned host memory and
// its device copy, reused once the event recorded behind their readers fires.
constexpr int kDescSlots = 4;
struct DescSlot {
    DevBuf dev;
    void* host = nullptr;
    uint64_t bytes = 0;       // of host (the descriptor)
    uint64_t dev_bytes = 0;   // of dev (the descriptor and device-only scratch after it)
    hipEvent_t done = nullptr;
    bool pending = false;
    DescSlot() = default;
    DescSlot(const DescSlot&) = delete;
    DescSlot& operator=(const DescSlot&) = delete;
    ~DescSlot();
};

}  // namespace mdr

namespace mdr {
// A captured batch refactor: replayed whenever a batch of the same shape comes
// again.  Its kernels address `ws`; input and output pointers reach them
// through the descriptor the host rewrites in `stage` before each replay.
struct BatchGraph {
    std::string key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    PoolBuf ws;
    void* stage = nullptr;  // pinned: descriptor, then the metadata read back
    uint64_t stage_bytes = 0;
    uint64_t last_use = 0;
    ~BatchGraph();
};
}  // namespace mdr

namespace mdr {
// one tuning-table entry: key = (dtype, nplanes, group size, floor(log2(values
// in the pass)), floor(log2(levels in the pass))) and the launch shape to use
struct TuneEntry {
    uint32_t key[5];
    mdr_launch_shape shape;
    double ms;
};
void tune_key(mdr_dtype dtype, uint32_t B, uint32_t m, uint64_t values, uint64_t levels, uint32_t key[5]);
// the shape a pass with this key runs at: its table entry, else the context's default
mdr_launch_shape effective_shape(const mdr_context* ctx, const uint32_t key[5]);
// MDR_AUTOTUNE: tune the pass's key first when the table has no entry for it
mdr_status tune_on_first_use(mdr_context* ctx, const VarLevels* vars, uint32_t nvars, mdr_dtype dtype,
                             uint32_t B, const mdr_codec_params& prm, hipStream_t s);
// MDR_TUNE_CACHE / MDR_AUTOTUNE at context creation
void tune_from_env(mdr_context* ctx);
}  // namespace mdr

struct mdr_context {
    int device = 0;
    std::shared_ptr<mdr::DevicePool> pool;  // device memory of refactored data and retrievers
    // per-stage timing (mdr_context_set_timing)
    bool timing = false;
    struct Mark {
        int stage;
        hipEvent_t start, stop;
    };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> event_pool;
    double stage_ms[MDR_STAGE_COUNT] = {};
    uint64_t stage_launches[MDR_STAGE_COUNT] = {};
    mdr::DevBuf ws;    // refactor workspace (statistics, histograms, codebooks)
    mdr::DevBuf qacc;  // V_total estimate accumulator
    // batch refactor: launch shape and captured graphs
    uint32_t enc_target_wg = 2304;   // encoder workgroups a batch aims for
    uint32_t stats_wg_values = 65536;  // values per statistics workgroup (at most kStatsMaxWg per level)
    uint32_t select_threads = 0;       // selection workgroup size (0: by the pass's unit count)
    // launch-shape tuning table, its file, and tune-on-first-use
    std::vector<mdr::TuneEntry> tune;
    std::string tune_path;
    bool autotune = false;
    bool tuning = false;  // inside a sweep: passes use the candidate shape as the default
    bool graphs = true;
    hipStream_t capture_stream = nullptr;
    std::vector<std::unique_ptr<mdr::BatchGraph>> graph_cache;
    uint64_t graph_clock = 0;
    // Huffman decode: lanes per chunk (0 = chosen per launch by its chunk count)
    uint32_t decode_lanes = 0;
    // job tables of retrieval launches
    mdr::DescSlot ring[mdr::kDescSlots];
    uint32_t ring_next = 0;
    uint64_t ring_hw_host = 0, ring_hw_dev = 0;  // largest descriptor / device part requested
    void* stage = nullptr;  // pinned host staging
    uint64_t stage_bytes = 0;
};

struct mdr_refactored {
    mdr_context* ctx = nullptr;
    mdr_dtype dtype = MDR_F32;
    uint32_t B = 0, m = 0, G = 1;
    mdr_codec_params prm{};
    std::vector<mdr::LevelRec> levels;
    // plane rows and lossless payloads; shared by the variables of one batch
    std::shared_ptr<mdr::PoolBuf> rows_arena;
    std::shared_ptr<mdr::PoolBuf> payload_arena;
};

struct mdr_retriever {
    mdr_context* ctx = nullptr;
    const mdr_refactored* r = nullptr;
    std::vector<uint32_t> k;                      // planes held per level
    std::vector<std::vector<mdr::PoolBuf>> dec;   // [level][slot] decoded non-DC units
    uint64_t bytes_held = 0;
};
