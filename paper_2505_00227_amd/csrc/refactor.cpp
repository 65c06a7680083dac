// Batch refactor orchestration: Alg. 1 (bitplane encoding with the exact
// per-plane error table) and Alg. 2 (hybrid lossless selection and encoding)
// over every level of every variable of a batch, as one flattened pass.
//
// The host only lays out the work: per-level jobs, workgroup maps, arena
// offsets and capacities.  Everything that depends on the data (exponents,
// error tables, methods, stream sizes, payload offsets) is decided on the
// device, and the metadata comes back in one copy at the end.  Because no
// launch shape depends on the data, the pass can be captured into a HIP graph
// once per batch shape and replayed; inputs and outputs reach the kernels
// through a descriptor the host rewrites before each replay.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>

#include "api_internal.hpp"

namespace mdr {

BatchGraph::~BatchGraph()
{
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (stage) (void)hipHostFree(stage);
}

void release_graphs(mdr_context* ctx)
{
    ctx->graph_cache.clear();
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    ctx->capture_stream = nullptr;
}

namespace {

constexpr size_t kGraphCacheMax = 8;

// value of an order-preserving key (see the statistics kernel)
double key_value(uint64_t key, bool f64)
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

double bits_value(uint64_t bits, bool f64)
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

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Largest stream the encoders can produce for a unit of S bytes: the arena is
// sized from these before launch, so that no size has to come back first.
// Under Alg. 2 a Huffman stream is chosen only when T_cr * est_H < S, and the
// written stream exceeds est_H by at most 4 bytes per chunk (word-aligned
// chunks); a run-length stream is chosen only when T_cr * est_R < S and is
// exactly est_R.  Forced methods take the largest size the format allows.
uint64_t unit_cap(uint64_t S, const mdr_codec_params& prm, uint32_t G)
{
    if (S == 0) return 512;  // empty Huffman / run-length header
    const uint64_t nch = ceil_div(S, prm.huf_chunk);
    const uint64_t huf = 8 + 256 + 4 * (nch + 1) + 4 * (ceil_div(S * prm.huf_lmax, 32) + nch);
    const uint64_t rle = 8 + (S / (4ull * G)) * (4ull * G + 4);
    uint64_t cap;
    if (prm.force_method == MDR_HUF)
        cap = huf;
    else if (prm.force_method == MDR_RLE)
        cap = rle;
    else if (prm.force_method == MDR_DC)
        cap = 0;
    else if (S <= prm.t_s_bytes)
        cap = 0;
    else
        cap = std::min(std::max(huf, rle), 1000 * S / prm.t_cr_milli + 4 * nch + 16);
    return align256(cap);
}

struct JobPlan {
    uint32_t var = 0, level = 0;
    const void* x = nullptr;
    uint64_t n = 0;
    uint32_t nbd = 0, ntiles = 0, tpw = 0, grid_e = 0, grid_s = 0;
    uint32_t wg_base_s = 0, wg_base_e = 0;
    bool vec = false;
    uint64_t rows_off = 0, hist_off = 0, recs_off = 0, trans_off = 0;
};

struct Layout {
    bool f64 = false;
    uint32_t G = 1, B = 0, m = 0, nunits = 0, J = 0, U = 0;
    std::vector<JobPlan> jobs;
    std::vector<uint32_t> var_first;  // first job of each variable, plus J
    uint64_t rows_bytes = 0, pay_cap = 0, max_chunks = 0, max_tiles = 0;
    // workspace: metadata block (read back in one copy), then scratch
    uint64_t o_stats = 0, o_keys = 0, o_units = 0, o_payoff = 0, o_ubytes = 0, o_counts = 0,
             meta_bytes = 0;
    uint64_t o_lens = 0, o_codes = 0, o_hist = 0, o_recs = 0, o_trans = 0, o_tot_end = 0, o_cbase = 0,
             o_tbase = 0, o_cwords = 0, o_truns = 0, o_scan = 0, o_desc = 0, ws_bytes = 0;
    // descriptor (uploaded before every pass)
    uint64_t d_sjobs = 0, d_ejobs = 0, d_slev = 0, d_largs = 0, d_map[4] = {}, desc_bytes = 0;
    std::vector<uint32_t> map[4];  // workgroup -> job: stats (unaligned, aligned), encode (same)
    std::string key;               // launch shape, for the graph cache
    mdr_launch_shape shape{};      // the knobs this pass runs with
};

mdr_status make_layout(const mdr_context* ctx, const VarLevels* vars, uint32_t nvars, mdr_dtype dtype,
                       uint32_t B, const mdr_codec_params& prm, Layout& L)
{
    L.f64 = dtype == MDR_F64;
    L.G = L.f64 ? 2 : 1;
    L.B = B;
    L.m = prm.group_planes;
    L.nunits = 1 + (B + L.m - 1) / L.m;
    uint64_t total_tiles = 0, total_values = 0;
    for (uint32_t v = 0; v < nvars; ++v) {
        L.var_first.push_back((uint32_t)L.jobs.size());
        for (uint32_t l = 0; l < vars[v].nlevels; ++l) {
            const mdr_level_view& lv = vars[v].levels[l];
            if (lv.n > 0xFFFFFFFFull)
                return fail(MDR_ERR_UNSUPPORTED, "a level may hold at most 2^32-1 values");
            if (lv.n && !lv.data)
                return fail(MDR_ERR_INVALID_ARG, "variable " + std::to_string(v) + " level " +
                                                     std::to_string(l) + ": data is NULL");
            JobPlan jp;
            jp.var = v;
            jp.level = l;
            jp.x = lv.data;
            jp.n = lv.n;
            jp.nbd = L.f64 ? (uint32_t)(2 * ceil_div(lv.n, 64)) : (uint32_t)ceil_div(lv.n, 32);
            jp.ntiles = (uint32_t)ceil_div(jp.nbd, kTileBlocks);
            jp.vec = ((uintptr_t)lv.data % 16) == 0;
            total_tiles += jp.ntiles;
            total_values += lv.n;
            L.jobs.push_back(jp);
        }
    }
    L.var_first.push_back((uint32_t)L.jobs.size());
    L.J = (uint32_t)L.jobs.size();
    L.U = L.J * L.nunits;
    if (L.J == 0) return MDR_OK;
    {
        uint32_t tk[5];
        tune_key(dtype, B, L.m, total_values, L.J, tk);
        L.shape = effective_shape(ctx, tk);
        // the selection builds each unit's code on one lane: with many units,
        // smaller workgroups let more of them build at once (the 4896 units
        // of 32 slabs of the 1024^3 field: 0.19 ms at 256 threads, 0.25 at
        // 512), with few the larger ones' faster histogram and rank steps win
        if (L.shape.select_threads == 0) L.shape.select_threads = L.U >= kSelectManyUnits ? 256u : 512u;
    }

    // every encoder workgroup walks about the same number of tiles, so that a
    // batch of mixed level sizes finishes together
    const uint64_t tpw_all = std::max<uint64_t>(1, ceil_div(total_tiles, std::max<uint32_t>(1, L.shape.enc_target_wg)));
    uint64_t hist = 0, recs = 0, trans = 0;
    for (JobPlan& jp : L.jobs) {
        if (jp.ntiles) {
            jp.tpw = (uint32_t)std::min<uint64_t>(jp.ntiles, tpw_all);
            jp.grid_e = (uint32_t)ceil_div(jp.ntiles, jp.tpw);
            jp.grid_s = (uint32_t)std::min<uint64_t>(kStatsMaxWg, ceil_div(jp.n, std::max<uint32_t>(1024, L.shape.stats_wg_values)));
        }
        jp.rows_off = L.rows_bytes;
        L.rows_bytes += align256(4ull * (B + 1) * jp.nbd);
        jp.hist_off = hist;
        hist += 4ull * L.nunits * 256;
        jp.recs_off = recs;
        recs += align256(4ull * jp.grid_e * kMaxRows * 2 * L.G);
        jp.trans_off = trans;
        trans += 4ull * kMaxRows;
        for (uint32_t i = 0; i < L.nunits; ++i) {
            const uint32_t r0 = i == 0 ? 0 : 1 + (i - 1) * L.m;
            const uint32_t r1 = i == 0 ? 1 : std::min(B + 1, r0 + L.m);
            const uint64_t S = 4ull * (r1 - r0) * jp.nbd;
            L.pay_cap += unit_cap(S, prm, L.G);
            L.max_chunks += ceil_div(S, prm.huf_chunk);
            L.max_tiles += ceil_div(S / (4ull * L.G), kRleTileWords);
        }
    }

    // workgroup maps; the encoder's longest workgroups are dispatched first
    for (uint32_t j = 0; j < L.J; ++j) {
        JobPlan& jp = L.jobs[j];
        std::vector<uint32_t>& ms = L.map[jp.vec ? 1 : 0];
        jp.wg_base_s = (uint32_t)ms.size();
        ms.insert(ms.end(), jp.grid_s, j);
    }
    std::vector<uint32_t> order(L.J);
    for (uint32_t j = 0; j < L.J; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return L.jobs[a].tpw > L.jobs[b].tpw; });
    for (uint32_t j : order) {
        JobPlan& jp = L.jobs[j];
        std::vector<uint32_t>& me = L.map[jp.vec ? 3 : 2];
        jp.wg_base_e = (uint32_t)me.size();
        me.insert(me.end(), jp.grid_e, j);
    }

    // workspace
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o += align256(bytes);
        return at;
    };
    L.o_stats = take(sizeof(LevelStats) * L.J);
    L.o_keys = take(8ull * kKeyStride * L.J);
    L.o_units = take(sizeof(UnitInfo) * L.U);
    L.o_payoff = take(8ull * L.U);
    L.o_ubytes = take(8ull * L.U);
    L.o_counts = take(4 * 8);
    L.meta_bytes = o;
    L.o_lens = take(256ull * L.U);
    L.o_codes = take(1024ull * L.U);
    L.o_recs = take(recs);
    L.o_hist = take(hist);  // level totals: histograms, then transitions, zeroed per pass
    L.o_trans = take(trans);
    L.o_tot_end = o;
    L.o_cbase = take(4ull * (L.U + 1));
    L.o_tbase = take(4ull * (L.U + 1));
    L.o_cwords = take(4ull * (L.max_chunks + 1));
    L.o_truns = take(4ull * (L.max_tiles + 1));
    L.o_scan = take(4ull * (2 * kPersistWg + 64));
    // descriptor
    uint64_t d = 0;
    auto dtake = [&](uint64_t bytes) {
        uint64_t at = d;
        d += align256(bytes);
        return at;
    };
    L.d_sjobs = dtake(sizeof(StatsJob) * L.J);
    L.d_ejobs = dtake(sizeof(EncodeJob) * L.J);
    L.d_slev = dtake(sizeof(SelectLevel) * L.J);
    L.d_largs = dtake(sizeof(LosslessArgs));
    for (int k = 0; k < 4; ++k) L.d_map[k] = dtake(4ull * L.map[k].size());
    L.desc_bytes = d;
    L.o_desc = take(L.desc_bytes);
    L.ws_bytes = o;

    // shape key: everything the captured launches depend on
    std::string& key = L.key;
    auto put = [&](uint64_t v) { key.append(reinterpret_cast<const char*>(&v), 8); };
    put((uint64_t)dtype);
    put(B);
    put(L.m);
    put(prm.t_cr_milli);
    put(prm.t_s_bytes);
    put(prm.huf_chunk);
    put(prm.huf_lmax);
    put((uint64_t)(int64_t)prm.force_method);
    put(L.shape.enc_target_wg);
    put(L.shape.stats_wg_values);
    put(L.shape.select_threads);
    put(nvars);
    for (const JobPlan& jp : L.jobs) {
        put(jp.n);
        put(((uint64_t)jp.var << 1) | (jp.vec ? 1u : 0u));
    }
    return MDR_OK;
}

// descriptor with the pointers of this pass
void fill_descriptor(const Layout& L, const mdr_codec_params& prm, uint8_t* ws, uint8_t* rows_base,
                     uint8_t* pay_base, uint8_t* desc)
{
    std::memset(desc, 0, L.desc_bytes);
    StatsJob* sj = reinterpret_cast<StatsJob*>(desc + L.d_sjobs);
    EncodeJob* ej = reinterpret_cast<EncodeJob*>(desc + L.d_ejobs);
    SelectLevel* sl = reinterpret_cast<SelectLevel*>(desc + L.d_slev);
    LevelStats* stats = reinterpret_cast<LevelStats*>(ws + L.o_stats);
    for (uint32_t j = 0; j < L.J; ++j) {
        const JobPlan& jp = L.jobs[j];
        sj[j].x = jp.x;
        sj[j].n = jp.n;
        sj[j].stats = stats + j;
        sj[j].wg_base = jp.wg_base_s;
        sj[j].grid = jp.grid_s;

        EncodeJob& e = ej[j];
        e.x = jp.x;
        e.n = jp.n;
        e.nbd = jp.nbd;
        e.B = L.B;
        e.m = L.m;
        e.nunits = L.nunits;
        e.ntiles = jp.ntiles;
        e.tiles_per_wg = jp.tpw;
        e.grid = jp.grid_e;
        e.wg_base = jp.wg_base_e;
        e.rows = reinterpret_cast<uint32_t*>(rows_base + jp.rows_off);
        e.stats = stats + j;
        e.hist = reinterpret_cast<uint32_t*>(ws + L.o_hist + jp.hist_off);
        e.trans = reinterpret_cast<uint32_t*>(ws + L.o_trans + jp.trans_off);
        e.recs = reinterpret_cast<uint32_t*>(ws + L.o_recs + jp.recs_off);
        e.keys = reinterpret_cast<unsigned long long*>(ws + L.o_keys) + (uint64_t)j * kKeyStride;
        for (uint32_t r = 0; r <= L.B; ++r)
            e.hist_off[r] = (uint16_t)((r == 0 ? 0 : 1 + (r - 1) / L.m) * 256);

        SelectLevel& s = sl[j];
        s.nbd = jp.nbd;
        s.grid = jp.grid_e;
        s.hist = e.hist;
        s.trans = e.trans;
        s.recs = e.recs;
        s.units = reinterpret_cast<UnitInfo*>(ws + L.o_units) + (uint64_t)j * L.nunits;
        s.lens = ws + L.o_lens + (uint64_t)j * L.nunits * 256;
        s.codes = reinterpret_cast<uint32_t*>(ws + L.o_codes) + (uint64_t)j * L.nunits * 256;
    }
    LosslessArgs* la = reinterpret_cast<LosslessArgs*>(desc + L.d_largs);
    la->jobs = reinterpret_cast<const EncodeJob*>(ws + L.o_desc + L.d_ejobs);
    la->units = reinterpret_cast<const UnitInfo*>(ws + L.o_units);
    la->lens = ws + L.o_lens;
    la->codes = reinterpret_cast<const uint32_t*>(ws + L.o_codes);
    la->chunk_base = reinterpret_cast<uint32_t*>(ws + L.o_cbase);
    la->tile_base = reinterpret_cast<uint32_t*>(ws + L.o_tbase);
    la->chunk_words = reinterpret_cast<uint32_t*>(ws + L.o_cwords);
    la->tile_runs = reinterpret_cast<uint32_t*>(ws + L.o_truns);
    la->pay_off = reinterpret_cast<uint64_t*>(ws + L.o_payoff);
    la->unit_bytes = reinterpret_cast<uint64_t*>(ws + L.o_ubytes);
    la->counts = reinterpret_cast<uint32_t*>(ws + L.o_counts);
    la->arena = pay_base;
    la->cap = L.pay_cap;
    la->U = L.U;
    la->nunits = L.nunits;
    la->B = L.B;
    la->m = L.m;
    la->G = L.G;
    la->huf_chunk = prm.huf_chunk;
    for (int k = 0; k < 4; ++k)
        if (!L.map[k].empty())
            std::memcpy(desc + L.d_map[k], L.map[k].data(), 4 * L.map[k].size());
}

// the pass itself: descriptor upload, every stage, metadata read-back
mdr_status enqueue_pass(mdr_context* ctx, const Layout& L, const mdr_codec_params& prm, uint8_t* ws,
                        uint8_t* stage, hipStream_t s, bool timed)
{
    // the launch checks read the thread's last HIP error: drop one left by a
    // call outside this library (another runtime client on the thread)
    (void)hipGetLastError();
    mdr_context* tctx = timed ? ctx : nullptr;
    uint8_t* desc = ws + L.o_desc;
    MDR_HIP(launch_copy_in(desc, stage, L.desc_bytes, s));
    const StatsJob* sj = reinterpret_cast<const StatsJob*>(desc + L.d_sjobs);
    const EncodeJob* ej = reinterpret_cast<const EncodeJob*>(desc + L.d_ejobs);
    const SelectLevel* sl = reinterpret_cast<const SelectLevel*>(desc + L.d_slev);
    const uint32_t* map[4];
    for (int k = 0; k < 4; ++k) map[k] = reinterpret_cast<const uint32_t*>(desc + L.d_map[k]);
    {
        StageTimer tm(tctx, MDR_STAGE_STATS, s);
        // the encoder adds its workgroups' histograms, transitions and key
        // maxima into zeroed level totals (a kernel: safe under capture)
        MDR_HIP(launch_init_pass(reinterpret_cast<LevelStats*>(ws + L.o_stats), L.J,
                                 reinterpret_cast<uint32_t*>(ws + L.o_keys), 2ull * kKeyStride * L.J,
                                 reinterpret_cast<uint32_t*>(ws + L.o_hist), (L.o_tot_end - L.o_hist) / 4, s));
        MDR_HIP(launch_stats_batch(sj, map[0], (uint32_t)L.map[0].size(), L.f64, false, s));
        MDR_HIP(launch_stats_batch(sj, map[1], (uint32_t)L.map[1].size(), L.f64, true, s));
    }
    {
        StageTimer tm(tctx, MDR_STAGE_ENCODE, s);
        MDR_HIP(launch_encode_batch(ej, map[2], (uint32_t)L.map[2].size(), L.nunits, L.B, L.m, L.f64, false, s));
        MDR_HIP(launch_encode_batch(ej, map[3], (uint32_t)L.map[3].size(), L.nunits, L.B, L.m, L.f64, true, s));
    }
    {
        StageTimer tm(tctx, MDR_STAGE_SELECT, s);
        SelectParams sp{};
        sp.B = L.B;
        sp.m = L.m;
        sp.nunits = L.nunits;
        sp.G = L.G;
        sp.t_cr_milli = prm.t_cr_milli;
        sp.huf_chunk = prm.huf_chunk;
        sp.huf_lmax = prm.huf_lmax;
        sp.force_method = prm.force_method;
        sp.threads = L.shape.select_threads;
        sp.t_s = prm.t_s_bytes;
        for (uint32_t j0 = 0; j0 < L.J; j0 += 65535)
            MDR_HIP(launch_select_batch(sp, sl + j0, std::min<uint32_t>(65535, L.J - j0), s));
    }
    {
        StageTimer tm(tctx, MDR_STAGE_LOSSLESS, s);
        LosslessArgs a{};
        a.chunk_words = reinterpret_cast<uint32_t*>(ws + L.o_cwords);
        a.tile_runs = reinterpret_cast<uint32_t*>(ws + L.o_truns);
        a.counts = reinterpret_cast<uint32_t*>(ws + L.o_counts);
        a.U = L.U;
        a.huf_chunk = prm.huf_chunk;
        MDR_HIP(launch_lossless_batch(a, reinterpret_cast<const LosslessArgs*>(desc + L.d_largs),
                                      reinterpret_cast<uint32_t*>(ws + L.o_scan), s));
    }
    {
        StageTimer tm(tctx, MDR_STAGE_ASSEMBLE, s);
        MDR_HIP(hipMemcpyAsync(stage + L.desc_bytes, ws + L.o_stats, L.meta_bytes, hipMemcpyDeviceToHost, s));
    }
    return MDR_OK;
}

// handles from the metadata read back after the pass
// x * 2^n rounded once, as std::ldexp: a product with the power of two when
// that power is a double (-1074 <= n <= 1023; the product of x and an exact
// power of two is the exact value rounded), ldexp otherwise.  A level's error
// table takes B of these per pass, and ldexp's library call cost about 6 ns
// each: 0.1 ms of host time for the 288 levels of 32 slabs.
static inline double scale2(double x, int n)
{
    if (n < -1074 || n > 1023) return std::ldexp(x, n);
    const uint64_t bits = n >= -1022 ? (uint64_t)(n + 1023) << 52 : 1ull << (n + 1074);
    double p;
    std::memcpy(&p, &bits, sizeof p);
    return x * p;
}

mdr_status assemble(mdr_context* ctx, const Layout& L, mdr_dtype dtype, const mdr_codec_params& prm,
                    const uint8_t* meta, const std::shared_ptr<PoolBuf>& rows,
                    const std::shared_ptr<PoolBuf>& pay, uint32_t nvars, mdr_refactored** outs)
{
    const LevelStats* hst = reinterpret_cast<const LevelStats*>(meta + L.o_stats);
    const unsigned long long* hek = reinterpret_cast<const unsigned long long*>(meta + L.o_keys);
    const UnitInfo* hun = reinterpret_cast<const UnitInfo*>(meta + L.o_units);
    const uint64_t* hoff = reinterpret_cast<const uint64_t*>(meta + L.o_payoff);
    const uint64_t* hbytes = reinterpret_cast<const uint64_t*>(meta + L.o_ubytes);
    const uint32_t* hcnt = reinterpret_cast<const uint32_t*>(meta + L.o_counts);
    const uint64_t inf_bits = L.f64 ? 0x7FF0000000000000ull : 0x7F800000ull;
    for (uint32_t j = 0; j < L.J; ++j)
        if (L.jobs[j].n && hst[j].maxabs_bits >= inf_bits)
            return fail(MDR_ERR_INVALID_ARG, "variable " + std::to_string(L.jobs[j].var) + " level " +
                                                 std::to_string(L.jobs[j].level) + " holds NaN or Inf");
    if (hcnt[2]) return fail(MDR_ERR_HIP, "internal: lossless streams exceed their arena");

    std::vector<std::unique_ptr<mdr_refactored>> made(nvars);
    uint8_t* rows_base = static_cast<uint8_t*>(rows->p);
    uint8_t* pay_base = static_cast<uint8_t*>(pay->p);
    for (uint32_t v = 0; v < nvars; ++v) {
        auto R = std::make_unique<mdr_refactored>();
        R->ctx = ctx;
        R->dtype = dtype;
        R->B = L.B;
        R->m = L.m;
        R->G = L.G;
        R->prm = prm;
        R->rows_arena = rows;
        R->payload_arena = pay;
        const uint32_t j0 = L.var_first[v], j1 = L.var_first[v + 1];
        R->levels.resize(j1 - j0);
        for (uint32_t j = j0; j < j1; ++j) {
            const JobPlan& jp = L.jobs[j];
            LevelRec& LR = R->levels[j - j0];
            LR.n = jp.n;
            LR.nbd = jp.nbd;
            LR.rows = reinterpret_cast<uint32_t*>(rows_base + jp.rows_off);
            LR.E.assign(L.B + 1, 0.0);
            if (jp.n) {
                const LevelStats& ls = hst[j];
                LR.vmin = key_value(ls.minkey, L.f64);
                LR.vmax = key_value(ls.maxkey, L.f64);
                LR.vmaxabs = bits_value(ls.maxabs_bits, L.f64);
                // alignment exponent: frexp's of max |x| (exact in double), 0 if all zero
                LR.e = 0;
                if (LR.vmaxabs != 0.0) (void)std::frexp(LR.vmaxabs, &LR.e);
                const unsigned long long* keys = hek + (uint64_t)j * kKeyStride;
                const double small = bits_value(keys[kKeyStride - 1], L.f64);
                LR.E[0] = LR.vmaxabs;  // nothing fetched: the error is max |x|
                for (uint32_t k = 1; k <= L.B; ++k) {
                    const double ek = scale2(bits_value(keys[k], L.f64), LR.e - (int)k);
                    LR.E[k] = ek > small ? ek : small;
                }
            }
            for (uint32_t i = 0; i < L.nunits; ++i) {
                const uint64_t u = (uint64_t)j * L.nunits + i;
                const UnitInfo& ui = hun[u];
                const uint32_t slot = i == 0 ? 0 : 1 + (i - 1) * L.m;
                UnitRec& ur = LR.units[slot];
                ur.method = (int32_t)ui.method;
                ur.S = ui.S;
                ur.nruns = ui.nruns;
                ur.est_huf = ui.est_huf;
                ur.est_rle = ui.est_rle;
                ur.nchunks = ui.nchunks;
                ur.maxlen = ui.maxlen;
                ur.bytes = hbytes[u];
                ur.dev = ur.method == MDR_DC ? reinterpret_cast<uint8_t*>(LR.rows + (uint64_t)slot * jp.nbd)
                                             : pay_base + hoff[u];
            }
        }
        made[v] = std::move(R);
    }
    for (uint32_t v = 0; v < nvars; ++v) outs[v] = made[v].release();
    return MDR_OK;
}

}  // namespace

mdr_status refactor_batch(mdr_context* ctx, const VarLevels* vars, uint32_t nvars, mdr_dtype dtype,
                          uint32_t B, const mdr_codec_params& prm, hipStream_t s, bool graph,
                          mdr_refactored** outs)
{
    MDR_HIP(hipSetDevice(ctx->device));
    if (ctx->autotune && !ctx->tuning) {
        mdr_status ts = tune_on_first_use(ctx, vars, nvars, dtype, B, prm, s);
        if (ts) return ts;
    }
    Layout L;
    mdr_status st = make_layout(ctx, vars, nvars, dtype, B, prm, L);
    if (st) return st;

    auto rows = std::make_shared<PoolBuf>();
    auto pay = std::make_shared<PoolBuf>();
    {
        hipError_t e = rows->alloc(ctx->pool, L.rows_bytes);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(planes)");
        e = pay->alloc(ctx->pool, L.pay_cap + 256);  // padded for the Huffman decoder's block reads
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(payloads)");
    }
    if (L.J == 0) return assemble(ctx, L, dtype, prm, nullptr, rows, pay, nvars, outs);
    MDR_HIP(encode_set_lds(L.nunits, L.B, L.m, L.f64));

    // on failure after the first launch, let queued work end before the pool reuses the memory
    struct SyncOnFail {
        hipStream_t s;
        bool armed = true;
        ~SyncOnFail()
        {
            if (armed) (void)hipStreamSynchronize(s);
        }
    } sync_on_fail{s};

    const uint8_t* meta = nullptr;
    if (!graph) {
        st = ensure_dev(ctx->ws, L.ws_bytes);
        if (st) return st;
        st = ensure_stage(ctx, L.desc_bytes + L.meta_bytes);
        if (st) return st;
        uint8_t* ws = static_cast<uint8_t*>(ctx->ws.p);
        uint8_t* stage = static_cast<uint8_t*>(ctx->stage);
        fill_descriptor(L, prm, ws, static_cast<uint8_t*>(rows->p), static_cast<uint8_t*>(pay->p), stage);
        st = enqueue_pass(ctx, L, prm, ws, stage, s, true);
        if (st) return st;
        MDR_HIP(hipStreamSynchronize(s));
        meta = stage + L.desc_bytes;
    } else {
        BatchGraph* g = nullptr;
        for (auto& e : ctx->graph_cache)
            if (e->key == L.key) g = e.get();
        if (!g) {
            auto ng = std::make_unique<BatchGraph>();
            ng->key = L.key;
            hipError_t e = ng->ws.alloc(ctx->pool, L.ws_bytes);
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(batch workspace)");
            MDR_HIP(hipHostMalloc(&ng->stage, L.desc_bytes + L.meta_bytes, hipHostMallocDefault));
            std::memset(ng->stage, 0, L.desc_bytes + L.meta_bytes);  // fault the pages in before capture
            ng->stage_bytes = L.desc_bytes + L.meta_bytes;
            if (!ctx->capture_stream)
                MDR_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
            hipStream_t cs = ctx->capture_stream;
            MDR_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
            st = enqueue_pass(ctx, L, prm, static_cast<uint8_t*>(ng->ws.p), static_cast<uint8_t*>(ng->stage),
                              cs, false);
            hipGraph_t gr = nullptr;
            hipError_t ee = hipStreamEndCapture(cs, &gr);
            if (st) {
                if (gr) (void)hipGraphDestroy(gr);
                return st;
            }
            if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
            ng->graph = gr;
            MDR_HIP(hipGraphInstantiate(&ng->exec, gr, nullptr, nullptr, 0));
            if (ctx->graph_cache.size() >= kGraphCacheMax) {
                auto lru = std::min_element(ctx->graph_cache.begin(), ctx->graph_cache.end(),
                                            [](const std::unique_ptr<BatchGraph>& a,
                                               const std::unique_ptr<BatchGraph>& b) {
                                                return a->last_use < b->last_use;
                                            });
                ctx->graph_cache.erase(lru);
            }
            g = ng.get();
            ctx->graph_cache.push_back(std::move(ng));
        }
        g->last_use = ++ctx->graph_clock;
        uint8_t* stage = static_cast<uint8_t*>(g->stage);
        fill_descriptor(L, prm, static_cast<uint8_t*>(g->ws.p), static_cast<uint8_t*>(rows->p),
                        static_cast<uint8_t*>(pay->p), stage);
        MDR_HIP(hipGraphLaunch(g->exec, s));
        MDR_HIP(hipStreamSynchronize(s));
        meta = stage + L.desc_bytes;
    }
    sync_on_fail.armed = false;
    return assemble(ctx, L, dtype, prm, meta, rows, pay, nvars, outs);
}

}  // namespace mdr
