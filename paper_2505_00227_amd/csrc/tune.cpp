// Launch-shape autotuner of the refactor pass: the pass's block and tile
// shapes (encoder workgroups, statistics workgroup values, selection
// workgroup size) are picked per pass shape by timing candidate shapes on the
// caller's own data, and kept in a per-context table that persists as JSON.
// No knob changes a result; the table only decides which shape a pass runs at.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>

#include "api_internal.hpp"

namespace mdr {

namespace {

uint32_t floor_log2(uint64_t v)
{
    uint32_t r = 0;
    while (v > 1) {
        v >>= 1;
        ++r;
    }
    return r;
}

const TuneEntry* find_entry(const mdr_context* ctx, const uint32_t key[5])
{
    for (const TuneEntry& e : ctx->tune)
        if (std::equal(e.key, e.key + 5, key)) return &e;
    return nullptr;
}

mdr_launch_shape default_shape(const mdr_context* ctx)
{
    return mdr_launch_shape{ctx->enc_target_wg, ctx->stats_wg_values, ctx->select_threads};
}

void record(mdr_context* ctx, const uint32_t key[5], const mdr_launch_shape& sh, double ms)
{
    for (TuneEntry& e : ctx->tune)
        if (std::equal(e.key, e.key + 5, key)) {
            e.shape = sh;
            e.ms = ms;
            return;
        }
    TuneEntry e;
    std::copy(key, key + 5, e.key);
    e.shape = sh;
    e.ms = ms;
    ctx->tune.push_back(e);
}

// values and levels of a pass (for its key)
void pass_size(const VarLevels* vars, uint32_t nvars, uint64_t& values, uint64_t& levels)
{
    values = levels = 0;
    for (uint32_t v = 0; v < nvars; ++v) {
        levels += vars[v].nlevels;
        for (uint32_t l = 0; l < vars[v].nlevels; ++l) values += vars[v].levels[l].n;
    }
}

// One timed pass at `sh` (wall clock of the whole call: launches, the pass, the
// metadata read-back and the handles), fastest of `reps`.
mdr_status time_shape(mdr_context* ctx, const VarLevels* vars, uint32_t nvars, mdr_dtype dtype, uint32_t B,
                      const mdr_codec_params& prm, hipStream_t s, uint32_t reps, const mdr_launch_shape& sh,
                      double& best_ms)
{
    const mdr_launch_shape keep = default_shape(ctx);
    ctx->enc_target_wg = sh.enc_target_wg;
    ctx->stats_wg_values = sh.stats_wg_values;
    ctx->select_threads = sh.select_threads;
    std::vector<mdr_refactored*> outs(nvars, nullptr);
    mdr_status st = MDR_OK;
    best_ms = 0.0;
    for (uint32_t r = 0; r < reps && st == MDR_OK; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        st = refactor_batch(ctx, vars, nvars, dtype, B, prm, s, false, outs.data());
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (mdr_refactored*& o : outs) {
            delete o;
            o = nullptr;
        }
        if (st == MDR_OK && (r == 0 || ms < best_ms)) best_ms = ms;
    }
    ctx->enc_target_wg = keep.enc_target_wg;
    ctx->stats_wg_values = keep.stats_wg_values;
    ctx->select_threads = keep.select_threads;
    return st;
}

// coordinate descent over the three knobs from the default shape
mdr_status sweep(mdr_context* ctx, const VarLevels* vars, uint32_t nvars, mdr_dtype dtype, uint32_t B,
                 const mdr_codec_params& prm, hipStream_t s, uint32_t reps, mdr_tune_result& res)
{
    static const uint32_t kEnc[] = {768, 1152, 2304, 4608, 9216};
    static const uint32_t kStats[] = {16384, 65536, 262144};
    static const uint32_t kSel[] = {256, 512, 1024};
    res.dflt = default_shape(ctx);
    ctx->tuning = true;
    struct Unset {
        mdr_context* c;
        ~Unset() { c->tuning = false; }
    } unset{ctx};
    double ms = 0.0;
    mdr_status st = time_shape(ctx, vars, nvars, dtype, B, prm, s, reps, res.dflt, ms);
    if (st) return st;
    res.default_ms = ms;
    mdr_launch_shape best = res.dflt;
    double best_ms = ms;
    uint32_t timed = 1;
    auto try_shape = [&](const mdr_launch_shape& c) -> mdr_status {
        if (c.enc_target_wg == best.enc_target_wg && c.stats_wg_values == best.stats_wg_values &&
            c.select_threads == best.select_threads)
            return MDR_OK;
        double t = 0.0;
        mdr_status e = time_shape(ctx, vars, nvars, dtype, B, prm, s, reps, c, t);
        if (e) return e;
        ++timed;
        if (t < best_ms) {
            best_ms = t;
            best = c;
        }
        return MDR_OK;
    };
    for (uint32_t v : kEnc) {
        mdr_launch_shape c = best;
        c.enc_target_wg = v;
        if ((st = try_shape(c))) return st;
    }
    for (uint32_t v : kStats) {
        mdr_launch_shape c = best;
        c.stats_wg_values = v;
        if ((st = try_shape(c))) return st;
    }
    for (uint32_t v : kSel) {
        mdr_launch_shape c = best;
        c.select_threads = v;
        if ((st = try_shape(c))) return st;
    }
    res.best = best;
    res.best_ms = best_ms;
    res.candidates = timed;
    return MDR_OK;
}

bool json_uint(const std::string& line, const char* name, uint64_t& v)
{
    const std::string k = std::string("\"") + name + "\":";
    const size_t at = line.find(k);
    if (at == std::string::npos) return false;
    const char* p = line.c_str() + at + k.size();
    char* end = nullptr;
    const unsigned long long x = std::strtoull(p, &end, 10);
    if (end == p) return false;
    v = x;
    return true;
}

mdr_status load_file(mdr_context* ctx, const std::string& path)
{
    std::ifstream f(path);
    if (!f) return fail(MDR_ERR_INVALID_ARG, "cannot open tuning file " + path);
    std::string line;
    bool header = false;
    std::vector<TuneEntry> got;
    while (std::getline(f, line)) {
        if (line.find("\"mdr_tune\":1") != std::string::npos) {
            header = true;
            continue;
        }
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        uint64_t d, B, m, vb, lb, enc, sv, sel;
        if (!json_uint(line, "dtype", d) || !json_uint(line, "nplanes", B) || !json_uint(line, "group_planes", m) ||
            !json_uint(line, "value_bucket", vb) || !json_uint(line, "level_bucket", lb) ||
            !json_uint(line, "enc_target_wg", enc) || !json_uint(line, "stats_wg_values", sv) ||
            !json_uint(line, "select_threads", sel))
            return fail(MDR_ERR_CORRUPT_STREAM, "malformed tuning entry in " + path + ": " + line);
        if (d > 1 || B < 1 || B > 64 || m < 1 || enc < 64 || enc > 65536 || sv < 1024 || sv > (1u << 24) ||
            (sel != 0 && sel != 256 && sel != 512 && sel != 1024))
            return fail(MDR_ERR_CORRUPT_STREAM, "tuning entry out of range in " + path + ": " + line);
        TuneEntry e;
        e.key[0] = (uint32_t)d, e.key[1] = (uint32_t)B, e.key[2] = (uint32_t)m, e.key[3] = (uint32_t)vb,
        e.key[4] = (uint32_t)lb;
        e.shape = mdr_launch_shape{(uint32_t)enc, (uint32_t)sv, (uint32_t)sel};
        e.ms = 0.0;
        got.push_back(e);
    }
    if (!header) return fail(MDR_ERR_CORRUPT_STREAM, "not a tuning file (no header line): " + path);
    for (const TuneEntry& e : got) record(ctx, e.key, e.shape, e.ms);
    return MDR_OK;
}

mdr_status save_file(const mdr_context* ctx, const std::string& path)
{
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return fail(MDR_ERR_INVALID_ARG, "cannot write tuning file " + path);
        f << "{\"mdr_tune\":1}\n";
        for (const TuneEntry& e : ctx->tune) {
            f << "{\"dtype\":" << e.key[0] << ",\"nplanes\":" << e.key[1] << ",\"group_planes\":" << e.key[2]
              << ",\"value_bucket\":" << e.key[3] << ",\"level_bucket\":" << e.key[4]
              << ",\"enc_target_wg\":" << e.shape.enc_target_wg << ",\"stats_wg_values\":" << e.shape.stats_wg_values
              << ",\"select_threads\":" << e.shape.select_threads << ",\"ms\":" << e.ms << "}\n";
        }
        if (!f) return fail(MDR_ERR_INVALID_ARG, "cannot write tuning file " + path);
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) return fail(MDR_ERR_INVALID_ARG, "cannot replace " + path);
    return MDR_OK;
}

mdr_status tune(mdr_context* ctx, const VarLevels* vars, uint32_t nvars, mdr_dtype dtype, uint32_t B,
                const mdr_codec_params& prm, hipStream_t s, uint32_t reps, bool force, mdr_tune_result& res)
{
    std::memset(&res, 0, sizeof(res));
    uint64_t values = 0, levels = 0;
    pass_size(vars, nvars, values, levels);
    uint32_t key[5];
    tune_key(dtype, B, prm.group_planes, values, levels, key);
    res.value_bucket = key[3];
    res.level_bucket = key[4];
    res.dflt = default_shape(ctx);
    if (!force)
        if (const TuneEntry* e = find_entry(ctx, key)) {
            res.best = e->shape;
            return MDR_OK;
        }
    mdr_status st = sweep(ctx, vars, nvars, dtype, B, prm, s, std::max<uint32_t>(1, reps), res);
    if (st) return st;
    record(ctx, key, res.best, res.best_ms);
    return MDR_OK;
}

}  // namespace

void tune_key(mdr_dtype dtype, uint32_t B, uint32_t m, uint64_t values, uint64_t levels, uint32_t key[5])
{
    key[0] = (uint32_t)dtype;
    key[1] = B;
    key[2] = m;
    key[3] = floor_log2(std::max<uint64_t>(1, values));
    key[4] = floor_log2(std::max<uint64_t>(1, levels));
}

mdr_launch_shape effective_shape(const mdr_context* ctx, const uint32_t key[5])
{
    if (!ctx->tuning)
        if (const TuneEntry* e = find_entry(ctx, key)) return e->shape;
    return default_shape(ctx);
}

mdr_status tune_on_first_use(mdr_context* ctx, const VarLevels* vars, uint32_t nvars, mdr_dtype dtype, uint32_t B,
                             const mdr_codec_params& prm, hipStream_t s)
{
    uint64_t values = 0, levels = 0;
    pass_size(vars, nvars, values, levels);
    uint32_t key[5];
    tune_key(dtype, B, prm.group_planes, values, levels, key);
    if (find_entry(ctx, key) || values == 0) return MDR_OK;
    mdr_tune_result res;
    mdr_status st = tune(ctx, vars, nvars, dtype, B, prm, s, 2, true, res);
    if (st) return st;
    return ctx->tune_path.empty() ? MDR_OK : save_file(ctx, ctx->tune_path);
}

// the environment's tuning file and tune-on-first-use switch (context creation)
void tune_from_env(mdr_context* ctx)
{
    if (const char* p = std::getenv("MDR_TUNE_CACHE")) {
        ctx->tune_path = p;
        std::ifstream probe(ctx->tune_path);
        if (probe.good()) {
            probe.close();
            if (load_file(ctx, ctx->tune_path) != MDR_OK) ctx->tune.clear();  // a bad file is ignored
        }
    }
    if (const char* a = std::getenv("MDR_AUTOTUNE")) ctx->autotune = std::strcmp(a, "1") == 0;
}

}  // namespace mdr

using namespace mdr;

extern "C" {

mdr_status mdr_context_set_select_threads(mdr_context* ctx, uint32_t threads)
{
    if (!ctx) return fail(MDR_ERR_INVALID_ARG, "ctx is NULL");
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return fail(MDR_ERR_INVALID_ARG, "select_threads must be 0 (by the pass), 256, 512 or 1024");
    ctx->select_threads = threads;
    return MDR_OK;
}

mdr_status mdr_autotune_refactor(mdr_context* ctx, const mdr_level_view* const* vars, const uint32_t* nlevels,
                                 uint32_t nvars, mdr_dtype dtype, uint32_t nplanes, const mdr_codec_params* params,
                                 void* stream, uint32_t reps, int force, mdr_tune_result* out)
{
    if (!ctx || !out) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    if (nvars == 0 || !vars || !nlevels) return fail(MDR_ERR_INVALID_ARG, "no variables");
    std::vector<VarLevels> vl(nvars);
    for (uint32_t v = 0; v < nvars; ++v) {
        if (nlevels[v] == 0 || !vars[v]) return fail(MDR_ERR_INVALID_ARG, "variable " + std::to_string(v) + " has no levels");
        vl[v] = {vars[v], nlevels[v]};
    }
    if (dtype != MDR_F32 && dtype != MDR_F64) return fail(MDR_ERR_INVALID_ARG, "bad dtype");
    const uint32_t W = dtype == MDR_F32 ? 32 : 64;
    if (nplanes < 1 || nplanes > W)
        return fail(MDR_ERR_UNSUPPORTED, "nplanes must be in [1, 32] for f32 and [1, 64] for f64");
    mdr_codec_params prm;
    mdr_codec_params_default(&prm);
    if (params) prm = *params;
    if (prm.group_planes > nplanes) prm.group_planes = nplanes;
    mdr_status st = check_params(prm, nplanes);
    if (st) return st;
    MDR_HIP(hipSetDevice(ctx->device));
    return tune(ctx, vl.data(), nvars, dtype, nplanes, prm, static_cast<hipStream_t>(stream), reps, force != 0, *out);
}

mdr_status mdr_tune_save(const mdr_context* ctx, const char* path)
{
    if (!ctx || !path) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    return save_file(ctx, path);
}

mdr_status mdr_tune_load(mdr_context* ctx, const char* path)
{
    if (!ctx || !path) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    return load_file(ctx, path);
}

mdr_status mdr_tune_entries(const mdr_context* ctx, uint32_t* count)
{
    if (!ctx || !count) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    *count = (uint32_t)ctx->tune.size();
    return MDR_OK;
}

mdr_status mdr_tune_entry(const mdr_context* ctx, uint32_t i, uint32_t key[5], mdr_launch_shape* shape)
{
    if (!ctx || !key || !shape) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    if (i >= ctx->tune.size()) return fail(MDR_ERR_INVALID_ARG, "no such tuning entry");
    std::copy(ctx->tune[i].key, ctx->tune[i].key + 5, key);
    *shape = ctx->tune[i].shape;
    return MDR_OK;
}

}  // extern "C"
