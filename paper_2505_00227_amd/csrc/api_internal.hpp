// Host-side objects behind the C ABI handles.
#pragma once

#include <cstdint>
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

}  // namespace mdr

struct mdr_context {
    int device = 0;
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
    mdr::DevBuf tmp;   // refactor scratch for the lossless encoders
    void* stage = nullptr;  // pinned host staging
    uint64_t stage_bytes = 0;
};

struct mdr_refactored {
    mdr_context* ctx = nullptr;
    mdr_dtype dtype = MDR_F32;
    uint32_t B = 0, m = 0, G = 1;
    mdr_codec_params prm{};
    std::vector<mdr::LevelRec> levels;
    mdr::DevBuf rows_arena;
    mdr::DevBuf payload_arena;
};

struct mdr_retriever {
    mdr_context* ctx = nullptr;
    const mdr_refactored* r = nullptr;
    std::vector<uint32_t> k;                      // planes held per level
    std::vector<std::vector<mdr::DevBuf>> dec;    // [level][slot] decoded non-DC units
    mdr::DevBuf temp;                             // RLE decode scratch
    uint64_t bytes_held = 0;
};
