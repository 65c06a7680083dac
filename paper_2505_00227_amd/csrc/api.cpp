// C ABI: context, refactor orchestration, retriever and the tolerance planner.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>

#include "api_internal.hpp"

namespace mdr {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

mdr_status fail(mdr_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

mdr_status hip_fail(hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(e == hipErrorOutOfMemory ? MDR_ERR_OUT_OF_MEMORY : MDR_ERR_HIP, m);
}

#define MDR_HIP(expr)                                            \
    do {                                                         \
        hipError_t _e = (expr);                                  \
        if (_e != hipSuccess) return ::mdr::hip_fail(_e, #expr); \
    } while (0)

// ------------------------------------------------------------------ stage timing
static hipEvent_t take_event(mdr_context* ctx)
{
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

StageTimer::StageTimer(mdr_context* ctx, int stage, hipStream_t s) : ctx_(ctx), stage_(stage), s_(s)
{
    if (ctx_ && ctx_->timing) {
        start_ = take_event(ctx_);
        if (start_ && hipEventRecord(start_, s_) != hipSuccess) {
            ctx_->event_pool.push_back(start_);
            start_ = nullptr;
        }
    }
}

StageTimer::~StageTimer()
{
    if (!start_) return;
    hipEvent_t stop = take_event(ctx_);
    if (stop && hipEventRecord(stop, s_) == hipSuccess) {
        ctx_->marks.push_back({stage_, start_, stop});
    } else {
        ctx_->event_pool.push_back(start_);
        if (stop) ctx_->event_pool.push_back(stop);
    }
}

static uint64_t align256(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

static mdr_status ensure_dev(DevBuf& b, uint64_t need)
{
    if (b.bytes >= need) return MDR_OK;
    MDR_HIP(hipDeviceSynchronize());  // previous users of the buffer have finished
    hipError_t e = b.alloc(need + need / 4);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
    return MDR_OK;
}

static mdr_status ensure_stage(mdr_context* ctx, uint64_t need)
{
    if (ctx->stage_bytes >= need) return MDR_OK;
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    ctx->stage = nullptr;
    ctx->stage_bytes = 0;
    MDR_HIP(hipHostMalloc(&ctx->stage, need + need / 4, hipHostMallocDefault));
    ctx->stage_bytes = need + need / 4;
    return MDR_OK;
}

static mdr_status check_params(const mdr_codec_params& p, uint32_t B)
{
    if (p.group_planes < 1 || p.group_planes > B)
        return fail(MDR_ERR_INVALID_ARG, "group_planes must be in [1, nplanes]");
    if (p.huf_chunk < 256 || p.huf_chunk > 4096 || p.huf_chunk % 256)
        return fail(MDR_ERR_UNSUPPORTED, "huf_chunk must be a multiple of 256 in [256, 4096]");
    if (p.huf_lmax < 8 || p.huf_lmax > (uint32_t)kLutBitsMax)
        return fail(MDR_ERR_UNSUPPORTED, "huf_lmax must be in [8, 12]");
    if (p.force_method < -1 || p.force_method > MDR_HUF)
        return fail(MDR_ERR_INVALID_ARG, "force_method must be -1, MDR_DC, MDR_RLE or MDR_HUF");
    if (p.t_cr_milli == 0) return fail(MDR_ERR_INVALID_ARG, "t_cr_milli must be positive");
    return MDR_OK;
}

// value of an order-preserving key (see the statistics kernel)
static double key_value(uint64_t key, bool f64)
{
    double v;
    if (f64) {
        uint64_t bits = (key >> 63) ? (key ^ 0x8000000000000000ull) : ~key;
        std::memcpy(&v, &bits, 8);
    } else {
        uint32_t k32 = (uint32_t)key;
        uint32_t bits = (k32 >> 31) ? (k32 ^ 0x80000000u) : ~k32;
        float f;
        std::memcpy(&f, &bits, 4);
        v = f;
    }
    return v == 0.0 ? 0.0 : v;
}

static double bits_value(uint64_t bits, bool f64)
{
    if (f64) {
        double d;
        std::memcpy(&d, &bits, 8);
        return d;
    }
    uint32_t b = (uint32_t)bits;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

// Huffman payload of an empty unit (0 symbols, no chunks) and RLE of no runs
static std::vector<uint8_t> empty_payload(int method, uint32_t G)
{
    std::vector<uint8_t> p;
    if (method == MDR_HUF) {
        p.assign(8 + 256 + 4, 0);
    } else if (method == MDR_RLE) {
        p.assign(8, 0);
        uint32_t wb = 4 * G;
        std::memcpy(p.data() + 4, &wb, 4);
    }
    return p;
}

// ------------------------------------------------------------------ planner
// bound(k) = sum over levels of E_l[k_l], in level order.  Greedy: one more
// merged group in the level of largest (error drop) / (bytes to fetch),
// ties to the smallest level; when every drop is zero, the level whose
// current error is largest.
double plan_bound(const mdr_refactored* r, const std::vector<uint32_t>& k)
{
    double s = 0.0;
    for (size_t l = 0; l < r->levels.size(); ++l) s += r->levels[l].E[k[l]];
    return s;
}

static uint64_t group_cost(const mdr_refactored* r, size_t l, uint32_t kl)
{
    const LevelRec& L = r->levels[l];
    uint64_t c = L.units[1 + kl].bytes + (kl == 0 ? L.units[0].bytes : 0);
    return c ? c : 1;
}

bool plan_step(const mdr_refactored* r, std::vector<uint32_t>& k)
{
    const uint32_t B = r->B, m = r->m;
    int best = -1;
    double best_gain = 0.0;
    for (size_t l = 0; l < r->levels.size(); ++l) {
        if (k[l] >= B) continue;
        uint32_t nxt = std::min(B, k[l] + m);
        const std::vector<double>& E = r->levels[l].E;
        double gain = (E[k[l]] - E[nxt]) / (double)group_cost(r, l, k[l]);
        if (best < 0 || gain > best_gain) {
            best = (int)l;
            best_gain = gain;
        }
    }
    if (best < 0) return false;
    if (best_gain == 0.0) {
        best = -1;
        double worst = 0.0;
        for (size_t l = 0; l < r->levels.size(); ++l) {
            if (k[l] >= B) continue;
            double el = r->levels[l].E[k[l]];
            if (best < 0 || el > worst) {
                best = (int)l;
                worst = el;
            }
        }
    }
    k[best] = std::min(B, k[best] + m);
    return true;
}

double plan_to(const mdr_refactored* r, double tol, std::vector<uint32_t>& k)
{
    double b = plan_bound(r, k);
    while (b > tol) {
        if (!plan_step(r, k)) break;
        b = plan_bound(r, k);
    }
    return b;
}

double value_range(const mdr_refactored* r)
{
    double lo = 0.0, hi = 0.0;
    bool have = false;
    for (const LevelRec& L : r->levels) {
        if (L.n == 0) continue;
        if (!have || L.vmin < lo) lo = L.vmin;
        if (!have || L.vmax > hi) hi = L.vmax;
        have = true;
    }
    return hi - lo;
}

// ------------------------------------------------------------------ refactor
struct LevelPlan {
    uint64_t n;
    uint32_t nbd, ntiles, grid, tpw;
    uint64_t rows_off, recs_off, hist_off;
};

mdr_status refactor_impl(mdr_context* ctx, const mdr_level_view* levels, uint32_t nlevels,
                         mdr_dtype dtype, uint32_t B, const mdr_codec_params& prm, hipStream_t s,
                         mdr_refactored** out)
{
    const bool f64 = dtype == MDR_F64;
    const uint32_t G = f64 ? 2 : 1;
    const uint32_t m = prm.group_planes;
    const uint32_t nunits = 1 + (B + m - 1) / m;
    MDR_HIP(hipSetDevice(ctx->device));

    auto R = std::make_unique<mdr_refactored>();
    R->ctx = ctx;
    R->dtype = dtype;
    R->B = B;
    R->m = m;
    R->G = G;
    R->prm = prm;
    R->levels.resize(nlevels);

    // ---- sizes
    std::vector<LevelPlan> lp(nlevels);
    uint64_t rows_bytes = 0, recs_bytes = 0, hist_bytes = 0;
    for (uint32_t l = 0; l < nlevels; ++l) {
        LevelPlan& p = lp[l];
        p.n = levels[l].n;
        if (p.n > 0xFFFFFFFFull) return fail(MDR_ERR_UNSUPPORTED, "a level may hold at most 2^32-1 values");
        if (p.n && !levels[l].data) return fail(MDR_ERR_INVALID_ARG, "level data is NULL");
        p.nbd = f64 ? (uint32_t)(2 * ((p.n + 63) / 64)) : (uint32_t)((p.n + 31) / 32);
        p.ntiles = (p.nbd + kTileBlocks - 1) / kTileBlocks;
        p.grid = std::min<uint32_t>(std::max<uint32_t>(p.ntiles, 1), kMaxWgEncode);
        p.tpw = std::max<uint32_t>(1, (p.ntiles + p.grid - 1) / p.grid);
        p.grid = std::max<uint32_t>(1, (p.ntiles + p.tpw - 1) / p.tpw);
        p.rows_off = rows_bytes;
        rows_bytes += align256(4ull * (B + 1) * p.nbd);
        p.recs_off = recs_bytes;
        recs_bytes += align256(4ull * p.grid * kMaxRows * 2 * G);
        p.hist_off = hist_bytes;
        hist_bytes += align256(4ull * p.grid * nunits * 256);
    }
    {
        hipError_t e = R->rows_arena.alloc(rows_bytes);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(planes)");
    }
    const uint64_t L = nlevels;
    const uint64_t off_stats = 0;
    const uint64_t off_ekeys = off_stats + align256(sizeof(LevelStats) * L);
    const uint64_t off_trans = off_ekeys + align256(8ull * kMaxRows * L);
    const uint64_t off_units = off_trans + align256(4ull * kMaxRows * L);
    const uint64_t off_lens = off_units + align256(sizeof(UnitInfo) * kMaxRows * L);
    const uint64_t off_codes = off_lens + align256(256ull * kMaxRows * L);
    const uint64_t off_recs = off_codes + align256(1024ull * kMaxRows * L);
    const uint64_t off_hist = off_recs + recs_bytes;
    const uint64_t ws_total = off_hist + hist_bytes;
    mdr_status st = ensure_dev(ctx->ws, ws_total);
    if (st) return st;
    uint8_t* ws = static_cast<uint8_t*>(ctx->ws.p);
    LevelStats* d_stats = reinterpret_cast<LevelStats*>(ws + off_stats);
    unsigned long long* d_ekeys = reinterpret_cast<unsigned long long*>(ws + off_ekeys);
    uint32_t* d_trans = reinterpret_cast<uint32_t*>(ws + off_trans);
    UnitInfo* d_units = reinterpret_cast<UnitInfo*>(ws + off_units);
    uint8_t* d_lens = ws + off_lens;
    uint32_t* d_codes = reinterpret_cast<uint32_t*>(ws + off_codes);

    // ---- statistics, encoding, selection
    MDR_HIP(launch_init_stats(d_stats, (int)L, s));
    MDR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(d_ekeys), 2ull * kMaxRows * L, 0u, s));
    MDR_HIP(launch_fill_u32(d_trans, (uint64_t)kMaxRows * L, 0u, s));
    uint8_t* rows_base = static_cast<uint8_t*>(R->rows_arena.p);
    for (uint32_t l = 0; l < nlevels; ++l) {
        LevelRec& LR = R->levels[l];
        LR.n = lp[l].n;
        LR.nbd = lp[l].nbd;
        LR.rows = reinterpret_cast<uint32_t*>(rows_base + lp[l].rows_off);
        if (LR.n == 0) continue;
        {
            StageTimer tm(ctx, MDR_STAGE_STATS, s);
            MDR_HIP(launch_stats(levels[l].data, LR.n, f64, d_stats + l, s));
        }
        EncodeJob job{};
        job.x = levels[l].data;
        job.n = LR.n;
        job.nbd = LR.nbd;
        job.B = B;
        job.m = m;
        job.nunits = nunits;
        job.ntiles = lp[l].ntiles;
        job.tiles_per_wg = lp[l].tpw;
        job.grid = lp[l].grid;
        job.rows = LR.rows;
        job.stats = d_stats + l;
        job.hist = reinterpret_cast<uint32_t*>(ws + off_hist + lp[l].hist_off);
        job.trans = d_trans + (uint64_t)l * kMaxRows;
        job.recs = reinterpret_cast<uint32_t*>(ws + off_recs + lp[l].recs_off);
        job.ekeys = d_ekeys + (uint64_t)l * kMaxRows;
        {
            StageTimer tm(ctx, MDR_STAGE_ENCODE, s);
            MDR_HIP(launch_encode(job, f64, s));
        }
        SelectJob sj{};
        sj.nbd = LR.nbd;
        sj.B = B;
        sj.m = m;
        sj.nunits = nunits;
        sj.grid = lp[l].grid;
        sj.G = G;
        sj.t_cr_milli = prm.t_cr_milli;
        sj.huf_chunk = prm.huf_chunk;
        sj.huf_lmax = prm.huf_lmax;
        sj.force_method = prm.force_method;
        sj.t_s = prm.t_s_bytes;
        sj.hist = job.hist;
        sj.trans = job.trans;
        sj.recs = job.recs;
        sj.units = d_units + (uint64_t)l * kMaxRows;
        sj.lens = d_lens + (uint64_t)l * kMaxRows * 256;
        sj.codes = d_codes + (uint64_t)l * kMaxRows * 256;
        {
            StageTimer tm(ctx, MDR_STAGE_SELECT, s);
            MDR_HIP(launch_select(sj, s));
        }
    }

    // ---- small metadata to the host
    const uint64_t h_stats = 0, h_ekeys = align256(sizeof(LevelStats) * L);
    const uint64_t h_units = h_ekeys + align256(8ull * kMaxRows * L);
    const uint64_t h_total = h_units + align256(sizeof(UnitInfo) * kMaxRows * L);
    st = ensure_stage(ctx, h_total + 8ull * kMaxRows * L);
    if (st) return st;
    uint8_t* hs = static_cast<uint8_t*>(ctx->stage);
    MDR_HIP(hipMemcpyAsync(hs + h_stats, d_stats, sizeof(LevelStats) * L, hipMemcpyDeviceToHost, s));
    MDR_HIP(hipMemcpyAsync(hs + h_ekeys, d_ekeys, 8ull * kMaxRows * L, hipMemcpyDeviceToHost, s));
    MDR_HIP(hipMemcpyAsync(hs + h_units, d_units, sizeof(UnitInfo) * kMaxRows * L,
                           hipMemcpyDeviceToHost, s));
    MDR_HIP(hipStreamSynchronize(s));
    const LevelStats* hst = reinterpret_cast<const LevelStats*>(hs + h_stats);
    const unsigned long long* hek = reinterpret_cast<const unsigned long long*>(hs + h_ekeys);
    const UnitInfo* hun = reinterpret_cast<const UnitInfo*>(hs + h_units);

    uint64_t payload_bytes = 0, temp_words = 0;
    std::vector<uint64_t> payload_off(L * kMaxRows, 0);
    for (uint32_t l = 0; l < nlevels; ++l) {
        LevelRec& LR = R->levels[l];
        LR.E.assign(B + 1, 0.0);
        if (LR.n == 0) {
            for (uint32_t slot = 0; slot <= B; slot = slot == 0 ? 1 : slot + m) {
                UnitRec& u = LR.units[slot];
                u.method = prm.force_method >= 0 ? prm.force_method : MDR_DC;
                u.S = 0;
                u.bytes = empty_payload(u.method, G).size();
                u.est_huf = 8 + 256 + 4;
                u.est_rle = 8;
                payload_off[l * kMaxRows + slot] = payload_bytes;
                payload_bytes += align256(u.bytes);
            }
            continue;
        }
        const LevelStats& ls = hst[l];
        if (ls.nonfinite)
            return fail(MDR_ERR_INVALID_ARG, "level " + std::to_string(l) + " holds NaN or Inf");
        LR.e = ls.emax == INT_MIN ? 0 : ls.emax;
        LR.vmin = key_value(ls.minkey, f64);
        LR.vmax = key_value(ls.maxkey, f64);
        LR.vmaxabs = bits_value(ls.maxabs_bits, f64);
        const double small = bits_value(ls.small_bits, f64);
        for (uint32_t k = 0; k <= B; ++k) {
            double key = bits_value(hek[(uint64_t)l * kMaxRows + k], f64);
            double ek = std::ldexp(key, LR.e - (int)k);
            LR.E[k] = ek > small ? ek : small;
        }
        for (uint32_t u = 0; u < nunits; ++u) {
            const UnitInfo& ui = hun[(uint64_t)l * kMaxRows + u];
            uint32_t slot = u == 0 ? 0 : 1 + (u - 1) * m;
            UnitRec& ur = LR.units[slot];
            ur.method = (int32_t)ui.method;
            ur.S = ui.S;
            ur.nruns = ui.nruns;
            ur.est_huf = ui.est_huf;
            ur.est_rle = ui.est_rle;
            ur.nchunks = ui.nchunks;
            ur.maxlen = ui.maxlen;
            if (ur.method == MDR_HUF) {
                uint64_t words = ui.nchunks + (ui.S * (uint64_t)std::max<uint32_t>(ui.maxlen, 1) + 31) / 32;
                uint64_t cap = 8 + 256 + 4ull * (ui.nchunks + 1) + 4 * words;
                payload_off[l * kMaxRows + slot] = payload_bytes;
                payload_bytes += align256(cap);
                temp_words = std::max(temp_words, scan_temp_words((uint64_t)ui.nchunks + 1));
            } else if (ur.method == MDR_RLE) {
                ur.bytes = 8 + ui.nruns * (4ull * G + 4);
                payload_off[l * kMaxRows + slot] = payload_bytes;
                payload_bytes += align256(ur.bytes);
                temp_words = std::max(temp_words, rle_temp_words(ui.S / 4 / G));
            } else {
                ur.bytes = ui.S;
            }
        }
    }
    {
        hipError_t e = R->payload_arena.alloc(payload_bytes);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(payloads)");
    }
    if (temp_words) {
        st = ensure_dev(ctx->tmp, 4 * temp_words);
        if (st) return st;
    }
    uint8_t* pay = static_cast<uint8_t*>(R->payload_arena.p);
    uint32_t* tmp = static_cast<uint32_t*>(ctx->tmp.p);
    std::vector<std::pair<uint32_t, uint32_t>> huf_units;  // (level, slot)
    for (uint32_t l = 0; l < nlevels; ++l) {
        LevelRec& LR = R->levels[l];
        for (uint32_t slot = 0; slot <= B; slot = slot == 0 ? 1 : slot + m) {
            UnitRec& ur = LR.units[slot];
            uint32_t r0, r1;
            slot_rows(slot, B, m, r0, r1);
            if (LR.n == 0) {
                ur.dev = pay + payload_off[l * kMaxRows + slot];
                std::vector<uint8_t> ep = empty_payload(ur.method, G);
                if (!ep.empty())
                    MDR_HIP(hipMemcpy(ur.dev, ep.data(), ep.size(), hipMemcpyHostToDevice));
                continue;
            }
            const uint8_t* g = reinterpret_cast<const uint8_t*>(LR.rows + (uint64_t)r0 * LR.nbd);
            uint32_t u = slot == 0 ? 0 : 1 + (slot - 1) / m;
            if (ur.method == MDR_DC) {
                ur.dev = const_cast<uint8_t*>(g);
            } else if (ur.method == MDR_HUF) {
                ur.dev = pay + payload_off[l * kMaxRows + slot];
                StageTimer tm(ctx, MDR_STAGE_HUF_ENCODE, s);
                MDR_HIP(launch_huf_encode(g, ur.S, prm.huf_chunk,
                                          d_lens + ((uint64_t)l * kMaxRows + u) * 256,
                                          d_codes + ((uint64_t)l * kMaxRows + u) * 256, ur.dev, tmp,
                                          s));
                huf_units.push_back({l, slot});
            } else {
                ur.dev = pay + payload_off[l * kMaxRows + slot];
                StageTimer tm(ctx, MDR_STAGE_RLE_ENCODE, s);
                MDR_HIP(launch_rle_encode(g, ur.S / 4 / G, G, ur.nruns, ur.dev, tmp, s));
            }
        }
    }
    if (!huf_units.empty()) {
        uint32_t* hw = reinterpret_cast<uint32_t*>(hs);
        for (size_t i = 0; i < huf_units.size(); ++i) {
            const UnitRec& ur = R->levels[huf_units[i].first].units[huf_units[i].second];
            MDR_HIP(hipMemcpyAsync(hw + i, ur.dev + 8 + 256 + 4ull * ur.nchunks, 4,
                                   hipMemcpyDeviceToHost, s));
        }
        MDR_HIP(hipStreamSynchronize(s));
        for (size_t i = 0; i < huf_units.size(); ++i) {
            UnitRec& ur = R->levels[huf_units[i].first].units[huf_units[i].second];
            ur.bytes = 8 + 256 + 4ull * (ur.nchunks + 1) + 4ull * hw[i];
        }
    } else {
        MDR_HIP(hipStreamSynchronize(s));
    }
    *out = R.release();
    return MDR_OK;
}

// ------------------------------------------------------------------ retrieve
mdr_status retrieve_impl(mdr_retriever* rt, const std::vector<uint32_t>& knew,
                         void* const* level_out, hipStream_t s, double tol_abs,
                         mdr_retrieve_info* info)
{
    const mdr_refactored* r = rt->r;
    const bool f64 = r->dtype == MDR_F64;
    const uint32_t B = r->B, m = r->m, G = r->G;
    MDR_HIP(hipSetDevice(rt->ctx->device));
    for (size_t l = 0; l < r->levels.size(); ++l)
        if (r->levels[l].n && !level_out[l])
            return fail(MDR_ERR_INVALID_ARG, "level_out[" + std::to_string(l) + "] is NULL");

    // decode the units entering [k_old, k_new); state is committed at the end
    std::vector<std::pair<size_t, uint32_t>> fresh;
    std::vector<DevBuf> fresh_bufs;
    uint64_t fetched = 0;
    uint32_t groups = 0;
    for (size_t l = 0; l < r->levels.size(); ++l) {
        const LevelRec& LR = r->levels[l];
        const uint32_t k0 = rt->k[l], k1 = knew[l];
        for (uint32_t slot = 0; slot <= B; slot = slot == 0 ? 1 : slot + m) {
            bool needed_before = slot == 0 ? k0 > 0 : (slot - 1) < k0;
            bool needed_now = slot == 0 ? k1 > 0 : (slot - 1) < k1;
            if (!needed_now || needed_before) continue;
            const UnitRec& ur = LR.units[slot];
            fetched += ur.bytes;
            ++groups;
            if (ur.method == MDR_DC || LR.n == 0) continue;
            DevBuf buf;
            hipError_t e = buf.alloc(std::max<uint64_t>(ur.S, 4));
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(decoded group)");
            if (ur.method == MDR_HUF) {
                StageTimer tm(rt->ctx, MDR_STAGE_HUF_DECODE, s);
                MDR_HIP(launch_huf_decode(ur.dev, ur.S, r->prm.huf_chunk, r->prm.huf_lmax,
                                          static_cast<uint8_t*>(buf.p), s));
            } else if (ur.method == MDR_RLE) {
                uint64_t need = 4 * (ur.nruns + 64 + scan_temp_words(ur.nruns));
                if (rt->temp.bytes < need) {
                    MDR_HIP(hipStreamSynchronize(s));
                    hipError_t e2 = rt->temp.alloc(need);
                    if (e2 != hipSuccess) return hip_fail(e2, "hipMalloc(decode scratch)");
                }
                StageTimer tm(rt->ctx, MDR_STAGE_RLE_DECODE, s);
                MDR_HIP(launch_rle_decode(ur.dev, ur.S / 4 / G, G, ur.nruns,
                                          static_cast<uint8_t*>(buf.p),
                                          static_cast<uint32_t*>(rt->temp.p), s));
            } else {
                return fail(MDR_ERR_CORRUPT_STREAM, "unknown lossless method");
            }
            fresh.push_back({l, slot});
            fresh_bufs.push_back(std::move(buf));
        }
    }
    auto source = [&](size_t l, uint32_t slot) -> const uint8_t* {
        for (size_t i = 0; i < fresh.size(); ++i)
            if (fresh[i].first == l && fresh[i].second == slot)
                return static_cast<const uint8_t*>(fresh_bufs[i].p);
        const DevBuf& d = rt->dec[l][slot];
        if (d.p) return static_cast<const uint8_t*>(d.p);
        return r->levels[l].units[slot].dev;  // direct copy: the payload is the plane rows
    };
    for (size_t l = 0; l < r->levels.size(); ++l) {
        const LevelRec& LR = r->levels[l];
        if (LR.n == 0) continue;
        ReconJob job{};
        job.out = level_out[l];
        job.n = LR.n;
        job.nbd = LR.nbd;
        job.B = B;
        job.k = knew[l];
        job.e = LR.e;
        if (knew[l] > 0) {
            for (uint32_t row = 0; row <= B; ++row) {
                uint32_t slot = row == 0 ? 0 : 1 + ((row - 1) / m) * m;
                if (row > 0 && row - 1 >= knew[l]) break;
                uint32_t r0, r1;
                slot_rows(slot, B, m, r0, r1);
                job.rows[row] = reinterpret_cast<const uint32_t*>(source(l, slot)) +
                                (uint64_t)(row - r0) * LR.nbd;
            }
        }
        StageTimer tm(rt->ctx, MDR_STAGE_RECONSTRUCT, s);
        MDR_HIP(launch_reconstruct(job, f64, s));
    }
    // commit
    for (size_t i = 0; i < fresh.size(); ++i)
        rt->dec[fresh[i].first][fresh[i].second] = std::move(fresh_bufs[i]);
    rt->k = knew;
    rt->bytes_held += fetched;
    if (info) {
        info->tol_abs = tol_abs;
        info->bound = plan_bound(r, knew);
        info->bytes_fetched = fetched;
        info->bytes_held = rt->bytes_held;
        info->groups_fetched = groups;
        info->met = info->bound <= tol_abs ? 1 : 0;
    }
    return MDR_OK;
}

}  // namespace mdr

using namespace mdr;

// ================================================================== C ABI
extern "C" {

const char* mdr_version(void) { return "mdr-mi355x 0.1 (gfx950)"; }

const char* mdr_last_error(void) { return g_err.c_str(); }

mdr_status mdr_codec_params_default(mdr_codec_params* out)
{
    if (!out) return fail(MDR_ERR_INVALID_ARG, "out is NULL");
    out->group_planes = 4;
    out->t_cr_milli = 2000;
    out->t_s_bytes = 4096;
    out->huf_chunk = 1024;
    out->huf_lmax = 12;
    out->force_method = -1;
    return MDR_OK;
}

mdr_status mdr_context_create(int hip_device, mdr_context** out)
{
    g_err.clear();
    if (!out) return fail(MDR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    MDR_HIP(hipGetDeviceCount(&count));
    if (hip_device < 0 || hip_device >= count)
        return fail(MDR_ERR_INVALID_ARG, "no such HIP device");
    MDR_HIP(hipSetDevice(hip_device));
    auto* c = new mdr_context();
    c->device = hip_device;
    *out = c;
    return MDR_OK;
}

void mdr_context_destroy(mdr_context* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    for (auto& mk : ctx->marks) {
        (void)hipEventDestroy(mk.start);
        (void)hipEventDestroy(mk.stop);
    }
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    delete ctx;
}

mdr_status mdr_context_set_timing(mdr_context* ctx, int enable)
{
    if (!ctx) return fail(MDR_ERR_INVALID_ARG, "ctx is NULL");
    ctx->timing = enable != 0;
    return MDR_OK;
}

mdr_status mdr_context_timing(mdr_context* ctx, double* ms, uint64_t* launches, int reset)
{
    if (!ctx) return fail(MDR_ERR_INVALID_ARG, "ctx is NULL");
    MDR_HIP(hipSetDevice(ctx->device));
    for (auto& mk : ctx->marks) {
        MDR_HIP(hipEventSynchronize(mk.stop));
        float t = 0.0f;
        MDR_HIP(hipEventElapsedTime(&t, mk.start, mk.stop));
        ctx->stage_ms[mk.stage] += t;
        ctx->stage_launches[mk.stage] += 1;
        ctx->event_pool.push_back(mk.start);
        ctx->event_pool.push_back(mk.stop);
    }
    ctx->marks.clear();
    for (int i = 0; i < MDR_STAGE_COUNT; ++i) {
        if (ms) ms[i] = ctx->stage_ms[i];
        if (launches) launches[i] = ctx->stage_launches[i];
        if (reset) {
            ctx->stage_ms[i] = 0.0;
            ctx->stage_launches[i] = 0;
        }
    }
    return MDR_OK;
}

mdr_status mdr_refactor(mdr_context* ctx, const mdr_level_view* levels, uint32_t nlevels,
                        mdr_dtype dtype, uint32_t nplanes, const mdr_codec_params* params,
                        void* stream, mdr_refactored** out)
{
    g_err.clear();
    if (!out) return fail(MDR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(MDR_ERR_INVALID_ARG, "ctx is NULL");
    if (nlevels == 0 || !levels) return fail(MDR_ERR_INVALID_ARG, "no levels");
    if (dtype != MDR_F32 && dtype != MDR_F64) return fail(MDR_ERR_INVALID_ARG, "bad dtype");
    const uint32_t W = dtype == MDR_F32 ? 32 : 64;
    if (nplanes < 1 || nplanes > W)
        return fail(MDR_ERR_UNSUPPORTED, "nplanes must be in [1, 32] for f32 and [1, 64] for f64");
    mdr_codec_params prm;
    mdr_codec_params_default(&prm);
    if (params) prm = *params;
    // a group never spans more than every plane (m larger than nplanes means one group)
    if (prm.group_planes > nplanes) prm.group_planes = nplanes;
    mdr_status st = check_params(prm, nplanes);
    if (st) return st;
    return refactor_impl(ctx, levels, nlevels, dtype, nplanes, prm,
                         static_cast<hipStream_t>(stream), out);
}

void mdr_refactored_destroy(mdr_refactored* r)
{
    if (!r) return;
    (void)hipSetDevice(r->ctx->device);
    (void)hipDeviceSynchronize();
    delete r;
}

mdr_status mdr_refactored_shape(const mdr_refactored* r, uint32_t* nlevels, mdr_dtype* dtype,
                                uint32_t* nplanes, mdr_codec_params* params)
{
    if (!r) return fail(MDR_ERR_INVALID_ARG, "r is NULL");
    if (nlevels) *nlevels = (uint32_t)r->levels.size();
    if (dtype) *dtype = r->dtype;
    if (nplanes) *nplanes = r->B;
    if (params) *params = r->prm;
    return MDR_OK;
}

mdr_status mdr_refactored_info(const mdr_refactored* r, uint32_t level, int32_t* e, uint64_t* n,
                               double* vmin, double* vmax, double* error_table)
{
    if (!r) return fail(MDR_ERR_INVALID_ARG, "r is NULL");
    if (level >= r->levels.size()) return fail(MDR_ERR_INVALID_ARG, "level out of range");
    const LevelRec& L = r->levels[level];
    if (e) *e = L.e;
    if (n) *n = L.n;
    if (vmin) *vmin = L.vmin;
    if (vmax) *vmax = L.vmax;
    if (error_table)
        for (uint32_t k = 0; k <= r->B; ++k) error_table[k] = L.E[k];
    return MDR_OK;
}

mdr_status mdr_refactored_stream(const mdr_refactored* r, uint32_t level, int32_t stream,
                                 const void** dev_ptr, uint64_t* bytes, mdr_method* method)
{
    if (!r) return fail(MDR_ERR_INVALID_ARG, "r is NULL");
    if (level >= r->levels.size()) return fail(MDR_ERR_INVALID_ARG, "level out of range");
    if (stream < -1 || stream >= (int32_t)r->B) return fail(MDR_ERR_INVALID_ARG, "stream out of range");
    const UnitRec& u = r->levels[level].units[stream + 1];
    if (dev_ptr) *dev_ptr = u.method == MDR_PLACEHOLDER ? nullptr : u.dev;
    if (bytes) *bytes = u.method == MDR_PLACEHOLDER ? 0 : u.bytes;
    if (method) *method = (mdr_method)u.method;
    return MDR_OK;
}

mdr_status mdr_retriever_create(mdr_context* ctx, const mdr_refactored* r, mdr_retriever** out)
{
    g_err.clear();
    if (!out) return fail(MDR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx || !r) return fail(MDR_ERR_INVALID_ARG, "ctx or r is NULL");
    if (ctx->device != r->ctx->device)
        return fail(MDR_ERR_INVALID_ARG, "context and refactored data live on different devices");
    auto* rt = new mdr_retriever();
    rt->ctx = ctx;
    rt->r = r;
    rt->k.assign(r->levels.size(), 0);
    rt->dec.resize(r->levels.size());
    for (auto& v : rt->dec) v.resize(kMaxRows);
    *out = rt;
    return MDR_OK;
}

void mdr_retriever_destroy(mdr_retriever* rt)
{
    if (!rt) return;
    (void)hipSetDevice(rt->ctx->device);
    (void)hipDeviceSynchronize();
    delete rt;
}

mdr_status mdr_retriever_planes(const mdr_retriever* rt, uint32_t* k)
{
    if (!rt || !k) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    for (size_t l = 0; l < rt->k.size(); ++l) k[l] = rt->k[l];
    return MDR_OK;
}

mdr_status mdr_retrieve(mdr_retriever* rt, mdr_bound kind, double tol, void* const* level_out,
                        void* stream, mdr_retrieve_info* info)
{
    g_err.clear();
    if (!rt || !level_out) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    if (!(tol >= 0.0) || std::isinf(tol)) return fail(MDR_ERR_INVALID_ARG, "tolerance must be finite and >= 0");
    if (kind != MDR_ABS && kind != MDR_REL) return fail(MDR_ERR_INVALID_ARG, "bad bound kind");
    double tol_abs = kind == MDR_REL ? tol * value_range(rt->r) : tol;
    std::vector<uint32_t> k = rt->k;
    plan_to(rt->r, tol_abs, k);
    return retrieve_impl(rt, k, level_out, static_cast<hipStream_t>(stream), tol_abs, info);
}

mdr_status mdr_retrieve_planes(mdr_retriever* rt, const uint32_t* kreq, void* const* level_out,
                               void* stream, mdr_retrieve_info* info)
{
    g_err.clear();
    if (!rt || !kreq || !level_out) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    const uint32_t B = rt->r->B, m = rt->r->m;
    std::vector<uint32_t> k = rt->k;
    for (size_t l = 0; l < k.size(); ++l) {
        if (kreq[l] > B) return fail(MDR_ERR_INVALID_ARG, "planes beyond nplanes");
        uint32_t want = std::min(B, (kreq[l] + m - 1) / m * m);
        k[l] = std::max(k[l], want);
    }
    return retrieve_impl(rt, k, level_out, static_cast<hipStream_t>(stream), 0.0, info);
}

}  // extern "C"
