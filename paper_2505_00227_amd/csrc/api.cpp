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


// ------------------------------------------------------------------ device pool
DevicePool::~DevicePool()
{
    for (auto& kv : free_) (void)hipFree(kv.second);
}

hipError_t DevicePool::alloc(uint64_t bytes, void** p, uint64_t* got)
{
    bytes = align256(bytes);
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = free_.lower_bound(bytes);
        if (it != free_.end() && it->first <= 2 * bytes) {
            *p = it->second;
            *got = it->first;
            cached_ -= it->first;
            free_.erase(it);
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipErrorOutOfMemory) {
        // give the cached blocks back to the device and try once more
        (void)hipGetLastError();
        std::multimap<uint64_t, void*> drop;
        {
            std::lock_guard<std::mutex> lk(mu_);
            drop.swap(free_);
            cached_ = 0;
        }
        for (auto& kv : drop) (void)hipFree(kv.second);
        e = hipMalloc(p, bytes);
    }
    if (e != hipSuccess) {
        *p = nullptr;
        *got = 0;
        return e;
    }
    *got = bytes;
    return hipSuccess;
}

void DevicePool::release(void* p, uint64_t bytes)
{
    std::unique_lock<std::mutex> lk(mu_);
    if (cached_ + bytes > cap_) {
        lk.unlock();
        (void)hipFree(p);
        return;
    }
    free_.emplace(bytes, p);
    cached_ += bytes;
}

mdr_status ensure_dev(DevBuf& b, uint64_t need)
{
    if (b.bytes >= need) return MDR_OK;
    MDR_HIP(hipDeviceSynchronize());  // previous users of the buffer have finished
    hipError_t e = b.alloc(need + need / 4);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
    return MDR_OK;
}

mdr_status ensure_stage(mdr_context* ctx, uint64_t need)
{
    if (ctx->stage_bytes >= need) return MDR_OK;
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    ctx->stage = nullptr;
    ctx->stage_bytes = 0;
    MDR_HIP(hipHostMalloc(&ctx->stage, need + need / 4, hipHostMallocDefault));
    std::memset(ctx->stage, 0, need + need / 4);  // fault the pages in now, not in the calls that write them
    ctx->stage_bytes = need + need / 4;
    return MDR_OK;
}

mdr_status check_params(const mdr_codec_params& p, uint32_t B)
{
    if (p.group_planes < 1 || p.group_planes > B)
        return fail(MDR_ERR_INVALID_ARG, "group_planes must be in [1, nplanes]");
    if (p.huf_chunk < 256 || p.huf_chunk > 4096 || (p.huf_chunk & (p.huf_chunk - 1)))
        return fail(MDR_ERR_UNSUPPORTED, "huf_chunk must be 256, 512, 1024, 2048 or 4096");
    if (p.huf_lmax < 8 || p.huf_lmax > (uint32_t)kLutBitsMax)
        return fail(MDR_ERR_UNSUPPORTED, "huf_lmax must be in [8, 12]");
    if (p.force_method < -1 || p.force_method > MDR_HUF)
        return fail(MDR_ERR_INVALID_ARG, "force_method must be -1, MDR_DC, MDR_RLE or MDR_HUF");
    if (p.t_cr_milli == 0) return fail(MDR_ERR_INVALID_ARG, "t_cr_milli must be positive");
    return MDR_OK;
}

// ------------------------------------------------------------------ planner
// bound(k) = sum over levels of E_l[k_l], in level order.  Greedy: one more
// merged group in the level of largest (error drop) / (bytes to fetch),
// ties to the smallest level; when every drop is zero, the level whose
// current error is largest.
double plan_bound(const mdr_refactored* r, const std::vector<uint32_t>& k, ErrTable tab)
{
    double s = 0.0;
    for (size_t l = 0; l < r->levels.size(); ++l) s += (r->levels[l].*tab)[k[l]];
    return s;
}

static uint64_t group_cost(const mdr_refactored* r, size_t l, uint32_t kl)
{
    const LevelRec& L = r->levels[l];
    uint64_t c = L.units[1 + kl].bytes + (kl == 0 ? L.units[0].bytes : 0);
    return c ? c : 1;
}

bool plan_step(const mdr_refactored* r, std::vector<uint32_t>& k, ErrTable tab)
{
    const uint32_t B = r->B, m = r->m;
    int best = -1;
    double best_gain = 0.0;
    for (size_t l = 0; l < r->levels.size(); ++l) {
        if (k[l] >= B) continue;
        uint32_t nxt = std::min(B, k[l] + m);
        const std::vector<double>& E = r->levels[l].*tab;
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
            double el = (r->levels[l].*tab)[k[l]];
            if (best < 0 || el > worst) {
                best = (int)l;
                worst = el;
            }
        }
    }
    k[best] = std::min(B, k[best] + m);
    return true;
}

double plan_to(const mdr_refactored* r, double tol, std::vector<uint32_t>& k, ErrTable tab)
{
    double b = plan_bound(r, k, tab);
    if (b <= tol) return b;
    // When every table is non-increasing along the steps the greedy can take,
    // so is the bound (a sum in fixed order of non-increasing terms), and if
    // even every plane of every level leaves it above tol the greedy can only
    // end with all of them: take that plan at once (a retrieval of everything
    // would otherwise walk one group at a time through every level).
    {
        const uint32_t B = r->B, m = r->m;
        bool monotone = true;
        for (size_t l = 0; l < r->levels.size() && monotone; ++l) {
            const std::vector<double>& E = r->levels[l].*tab;
            for (uint32_t kl = k[l]; kl < B && monotone; kl = std::min(B, kl + m))
                monotone = E[std::min(B, kl + m)] <= E[kl];
        }
        if (monotone) {
            std::vector<uint32_t> all(k.size(), B);
            const double ball = plan_bound(r, all, tab);
            if (ball > tol) {
                k = all;
                return ball;
            }
        }
    }
    while (b > tol) {
        if (!plan_step(r, k, tab)) break;
        b = plan_bound(r, k, tab);
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

// ------------------------------------------------------------------ retrieve
static mdr_status retrieve_one(mdr_retriever* rt, const std::vector<uint32_t>& knew,
                               void* const* level_out, hipStream_t s, double tol_abs,
                               mdr_retrieve_info* info)
{
    RetrieveTask t;
    t.rt = rt;
    t.knew = knew;
    t.out = level_out;
    t.tol_abs = tol_abs;
    t.info = info;
    return retrieve_many(rt->ctx, &t, 1, s);
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
    out->huf_chunk = 256;
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
    MDR_HIP(l2_scratch_init(hip_device));  // the fixed scratch of mdr_l2_table_noalloc, on this device
    auto* c = new mdr_context();
    c->device = hip_device;
    // freed device blocks are kept for reuse up to an eighth of the device's
    // memory (at least kPoolCacheBytes): a resident working set of passes
    // (plane rows, payload arenas, decoded groups) then cycles through the
    // cache instead of through hipFree / hipMalloc, which synchronise
    size_t mem_free = 0, mem_total = 0;
    MDR_HIP(hipMemGetInfo(&mem_free, &mem_total));
    c->pool = std::make_shared<DevicePool>(std::max<uint64_t>(kPoolCacheBytes, mem_total / 8));
    tune_from_env(c);
    *out = c;
    return MDR_OK;
}

void mdr_context_destroy(mdr_context* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    release_graphs(ctx);
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
    VarLevels v{levels, nlevels};
    return refactor_batch(ctx, &v, 1, dtype, nplanes, prm, static_cast<hipStream_t>(stream), false, out);
}

mdr_status mdr_refactor_batch(mdr_context* ctx, const mdr_level_view* const* vars,
                              const uint32_t* nlevels, uint32_t nvars, mdr_dtype dtype,
                              uint32_t nplanes, const mdr_codec_params* params, void* stream,
                              mdr_refactored** outs)
{
    g_err.clear();
    if (!outs) return fail(MDR_ERR_INVALID_ARG, "outs is NULL");
    for (uint32_t v = 0; v < nvars; ++v) outs[v] = nullptr;
    if (!ctx) return fail(MDR_ERR_INVALID_ARG, "ctx is NULL");
    if (nvars == 0 || !vars || !nlevels) return fail(MDR_ERR_INVALID_ARG, "no variables");
    std::vector<VarLevels> vl(nvars);
    for (uint32_t v = 0; v < nvars; ++v) {
        if (nlevels[v] == 0 || !vars[v])
            return fail(MDR_ERR_INVALID_ARG, "variable " + std::to_string(v) + " has no levels");
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
    return refactor_batch(ctx, vl.data(), nvars, dtype, nplanes, prm, static_cast<hipStream_t>(stream),
                          ctx->graphs, outs);
}

mdr_status mdr_context_set_launch(mdr_context* ctx, uint32_t enc_target_wg, uint32_t stats_wg_values,
                                  int graphs)
{
    g_err.clear();
    if (!ctx) return fail(MDR_ERR_INVALID_ARG, "ctx is NULL");
    if (enc_target_wg && (enc_target_wg < 64 || enc_target_wg > 65536))
        return fail(MDR_ERR_INVALID_ARG, "enc_target_wg must be in [64, 65536]");
    if (stats_wg_values && (stats_wg_values < 1024 || stats_wg_values > (1u << 24)))
        return fail(MDR_ERR_INVALID_ARG, "stats_wg_values must be in [1024, 2^24]");
    if (graphs < -1 || graphs > 1) return fail(MDR_ERR_INVALID_ARG, "graphs must be -1, 0 or 1");
    if (enc_target_wg) ctx->enc_target_wg = enc_target_wg;
    if (stats_wg_values) ctx->stats_wg_values = stats_wg_values;
    if (graphs >= 0) ctx->graphs = graphs != 0;
    return MDR_OK;
}

mdr_status mdr_context_set_decode_lanes(mdr_context* ctx, uint32_t lanes)
{
    g_err.clear();
    if (!ctx) return fail(MDR_ERR_INVALID_ARG, "ctx is NULL");
    if (lanes != 0 && lanes != 1 && lanes != 4 && lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64)
        return fail(MDR_ERR_INVALID_ARG, "decode lanes must be 0, 1, 4, 8, 16, 32 or 64");
    ctx->decode_lanes = lanes;
    return MDR_OK;
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
    if (kind != MDR_ABS && kind != MDR_REL && kind != MDR_L2) return fail(MDR_ERR_INVALID_ARG, "bad bound kind");
    std::vector<uint32_t> k = rt->k;
    if (kind == MDR_L2) {
        for (const LevelRec& L : rt->r->levels)
            if (L.E2.size() != rt->r->B + 1) return fail(MDR_ERR_INVALID_ARG, "no L2 table: call mdr_l2_table first");
        plan_to(rt->r, tol * tol, k, &LevelRec::E2);
        mdr_status st = retrieve_one(rt, k, level_out, static_cast<hipStream_t>(stream), tol, info);
        if (!st && info) {  // report the L2 bound, not the squared one
            info->bound = std::sqrt(plan_bound(rt->r, k, &LevelRec::E2));
            info->met = info->bound <= tol;
        }
        return st;
    }
    double tol_abs = kind == MDR_REL ? tol * value_range(rt->r) : tol;
    plan_to(rt->r, tol_abs, k);
    return retrieve_one(rt, k, level_out, static_cast<hipStream_t>(stream), tol_abs, info);
}

mdr_status mdr_retrieve_qoi_vtotal(mdr_retriever* vx, mdr_retriever* vy, mdr_retriever* vz,
                                   mdr_bound kind, double tau, double mape_c,
                                   void* const* out_x, void* const* out_y, void* const* out_z,
                                   void* stream, mdr_qoi_info* info)
{
    mdr_qoi_params prm{};
    prm.estimator = MDR_QOI_MAPE;
    prm.mape_c = mape_c;
    return mdr_retrieve_qoi_vtotal_with(vx, vy, vz, kind, tau, &prm, out_x, out_y, out_z, stream, info);
}

mdr_status mdr_retrieve_qoi_vtotal_with(mdr_retriever* vx, mdr_retriever* vy, mdr_retriever* vz,
                                        mdr_bound kind, double tau, const mdr_qoi_params* params,
                                        void* const* out_x, void* const* out_y, void* const* out_z,
                                        void* stream, mdr_qoi_info* info)
{
    mdr_retriever* const rts[3] = {vx, vy, vz};
    void* const* const outs[3] = {out_x, out_y, out_z};
    return mdr_retrieve_qoi(MDR_QOI_SUMSQ, rts, 3, kind, tau, params, outs, stream, info);
}

}  // extern "C"

namespace {

static_assert(MDR_QOI_SUMSQ == kQoiSumsq && MDR_QOI_MAGNITUDE == kQoiMagnitude && MDR_QOI_PRODUCT == kQoiProduct,
              "QoI family numbers");

// A family's score at one point from the absolute values a[c] and bounds e[c],
// in the kernel's order of operations (see k_qoi_batch)
double qoi_score_at(int kind, uint32_t nv, const double* a, const double* e)
{
    if (kind == MDR_QOI_PRODUCT) return ((a[0] * e[1]) + (a[1] * e[0])) + (e[0] * e[1]);
    double d = 0.0;
    for (uint32_t c = 0; c < nv; ++c) d = d + e[c] * ((2.0 * a[c]) + e[c]);
    if (kind == MDR_QOI_SUMSQ) return d;
    double sh = 0.0;
    for (uint32_t c = 0; c < nv; ++c) sh = sh + (a[c] * a[c]);
    return sh == 0.0 ? INFINITY : (d * d) / sh;
}

// tau' from the largest score: the score itself, or for the magnitude the root
// of its minimum with sum eps^2; inflated by (1 + 2^-40) for rounding
double qoi_estimate_of(int kind, uint32_t nv, double score, const double* e)
{
    double t = score;
    if (kind == MDR_QOI_MAGNITUDE) {
        double s2 = 0.0;
        for (uint32_t c = 0; c < nv; ++c) s2 = s2 + (e[c] * e[c]);
        t = std::sqrt(score < s2 ? score : s2);
    }
    return t * (1.0 + std::ldexp(1.0, -40));
}

}  // namespace

extern "C" {

mdr_status mdr_retrieve_qoi(mdr_qoi_kind qkind, mdr_retriever* const* rts, uint32_t nv, mdr_bound kind, double tau,
                            const mdr_qoi_params* params, void* const* const* outs, void* stream,
                            mdr_qoi_info* info)
{
    g_err.clear();
    mdr_qoi_params prm{};
    prm.estimator = MDR_QOI_MAPE;
    if (params) prm = *params;
    if (qkind != MDR_QOI_SUMSQ && qkind != MDR_QOI_MAGNITUDE && qkind != MDR_QOI_PRODUCT)
        return fail(MDR_ERR_INVALID_ARG, "unknown QoI family");
    if (!rts || !outs) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    if (qkind == MDR_QOI_PRODUCT ? nv != 2 : (nv < 1 || nv > 3))
        return fail(MDR_ERR_INVALID_ARG, "a product takes 2 variables, a sum of squares or magnitude 1 to 3");
    if (prm.estimator != MDR_QOI_MAPE && prm.estimator != MDR_QOI_MA && prm.estimator != MDR_QOI_CP)
        return fail(MDR_ERR_INVALID_ARG, "unknown QoI estimator");
    if (!(prm.cp_decay < 1.0)) return fail(MDR_ERR_INVALID_ARG, "cp_decay must be below 1");
    const double mape_c = prm.mape_c;
    const double decay = prm.cp_decay > 0.0 ? prm.cp_decay : 0.5;
    const bool cp = prm.estimator == MDR_QOI_CP;
    for (uint32_t c = 0; c < nv; ++c)
        if (!rts[c] || !outs[c]) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    if (!(tau >= 0.0) || std::isinf(tau)) return fail(MDR_ERR_INVALID_ARG, "tolerance must be finite and >= 0");
    if (kind != MDR_ABS && kind != MDR_REL) return fail(MDR_ERR_INVALID_ARG, "bad bound kind");
    const mdr_refactored* r0 = rts[0]->r;
    for (uint32_t c = 1; c < nv; ++c) {
        const mdr_refactored* rc = rts[c]->r;
        if (rc->dtype != r0->dtype || rc->levels.size() != r0->levels.size())
            return fail(MDR_ERR_INVALID_ARG, "the variables must share dtype and level structure");
        for (size_t l = 0; l < r0->levels.size(); ++l)
            if (rc->levels[l].n != r0->levels[l].n)
                return fail(MDR_ERR_INVALID_ARG, "the variables must hold the same points per level");
        if (rts[c]->ctx->device != rts[0]->ctx->device) return fail(MDR_ERR_INVALID_ARG, "retrievers on different devices");
        for (uint32_t d = 0; d < c; ++d)
            if (rts[d] == rts[c]) return fail(MDR_ERR_INVALID_ARG, "a retriever appears twice");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    mdr_context* ctx = rts[0]->ctx;
    MDR_HIP(hipSetDevice(ctx->device));
    mdr_status st = ensure_dev(ctx->qacc, 256);
    if (st) return st;
    st = ensure_stage(ctx, 64);
    if (st) return st;
    unsigned long long* acc = static_cast<unsigned long long*>(ctx->qacc.p);

    // the family's scale (relative tolerances) and Alg. 3's initial bounds
    double amax[3] = {0, 0, 0}, range[3] = {0, 0, 0};
    for (uint32_t c = 0; c < nv; ++c) {
        double lo = 0.0, hi = 0.0;
        bool have = false;
        for (const LevelRec& L : rts[c]->r->levels) {
            if (L.n == 0) continue;
            if (!have || L.vmin < lo) lo = L.vmin;
            if (!have || L.vmax > hi) hi = L.vmax;
            have = true;
        }
        amax[c] = std::max(std::fabs(lo), std::fabs(hi));
        range[c] = value_range(rts[c]->r);
    }
    double qmax = 0.0;
    for (uint32_t c = 0; c < nv; ++c) qmax = qmax + amax[c] * amax[c];
    double scale = qmax;
    if (qkind == MDR_QOI_MAGNITUDE) scale = std::sqrt(qmax);
    if (qkind == MDR_QOI_PRODUCT) scale = amax[0] * amax[1];
    const double tau_abs = kind == MDR_REL ? tau * scale : tau;
    double e0[3] = {0, 0, 0};
    for (uint32_t c = 0; c < nv; ++c) {
        if (qkind == MDR_QOI_SUMSQ)
            e0[c] = qmax == 0.0 ? 0.0 : (tau_abs / qmax) * range[c];
        else if (qkind == MDR_QOI_MAGNITUDE)
            e0[c] = tau_abs / std::sqrt((double)nv);
        else
            e0[c] = amax[1 - c] > 0.0 ? tau_abs / (2.0 * amax[1 - c]) : INFINITY;
    }
    const double cmape = mape_c > 0.0 ? mape_c : 10.0;
    std::vector<uint32_t> ks[3];
    for (uint32_t c = 0; c < nv; ++c) {
        ks[c] = rts[c]->k;
        plan_to(rts[c]->r, e0[c], ks[c]);
    }
    const bool f64 = r0->dtype == MDR_F64;
    uint64_t fetched = 0;
    uint32_t it = 0;
    double tprime = 0.0, eps[3] = {0, 0, 0};
    for (;;) {
        ++it;
        {
            RetrieveTask tk[3];
            mdr_retrieve_info ri[3];
            for (uint32_t c = 0; c < nv; ++c) {
                tk[c].rt = rts[c];
                tk[c].knew = ks[c];
                tk[c].out = outs[c];
                tk[c].info = &ri[c];
                tk[c].all_levels = it == 1;
            }
            st = retrieve_many(ctx, tk, nv, s);
            if (st) return st;
            for (uint32_t c = 0; c < nv; ++c) {
                fetched += ri[c].bytes_fetched;
                eps[c] = plan_bound(rts[c]->r, ks[c]);
            }
        }
        {
            // absent components read the first variable with a zero bound (their
            // terms add exact zeros)
            std::vector<QoiJob> jobs;
            uint64_t base = 0;
            for (size_t l = 0; l < r0->levels.size(); ++l) {
                QoiJob j{};
                j.x = outs[0][l];
                j.y = nv > 1 ? outs[1][l] : outs[0][l];
                j.z = nv > 2 ? outs[2][l] : outs[0][l];
                j.n = r0->levels[l].n;
                for (uint32_t c = 0; c < nv; ++c) j.eps[c] = eps[c];
                j.kind = (uint32_t)qkind;
                j.nvars = nv;
                j.acc = acc;
                j.arg = acc + 1;
                j.base = base;
                base += j.n;
                jobs.push_back(j);
            }
            st = enqueue_qoi(ctx, jobs, std::vector<bool>(jobs.size(), f64), acc, 1, s, cp);
            if (st) return st;
        }
        unsigned long long* hb = static_cast<unsigned long long*>(ctx->stage);
        MDR_HIP(hipMemcpyAsync(hb, acc, cp ? 16 : 8, hipMemcpyDeviceToHost, s));
        MDR_HIP(hipStreamSynchronize(s));
        double worst;
        std::memcpy(&worst, hb, 8);
        tprime = qoi_estimate_of(qkind, nv, worst, eps);
        bool full = true;
        for (uint32_t c = 0; c < nv; ++c)
            for (uint32_t kl : ks[c]) full = full && kl == rts[c]->r->B;
        if (tprime <= tau_abs || full) break;
        // next bounds from the estimator; none: minimal augmentation only
        bool have_target = false;
        double target[3] = {0, 0, 0};
        if (prm.estimator == MDR_QOI_MAPE) {
            const double p = tau_abs > 0.0 ? tprime / tau_abs : INFINITY;
            if (p > cmape) {
                for (uint32_t c = 0; c < nv; ++c) target[c] = eps[c] / p;
                have_target = true;
            }
        } else if (cp) {
            // the worst point's current values, then its bounds decayed until
            // its own estimate (as tau' is evaluated) is within tau
            uint64_t at = hb[1];
            size_t l = 0;
            while (l < r0->levels.size() && at >= r0->levels[l].n) at -= r0->levels[l++].n;
            if (l == r0->levels.size()) return fail(MDR_ERR_HIP, "internal: no point attains the estimate");
            const size_t es = f64 ? 8 : 4;
            uint8_t* hv = reinterpret_cast<uint8_t*>(hb + 2);
            for (uint32_t c = 0; c < nv; ++c)
                MDR_HIP(hipMemcpyAsync(hv + 8 * c, static_cast<const uint8_t*>(outs[c][l]) + at * es, es,
                                       hipMemcpyDeviceToHost, s));
            MDR_HIP(hipStreamSynchronize(s));
            double a[3] = {0, 0, 0};
            for (uint32_t c = 0; c < nv; ++c) {
                if (f64) {
                    std::memcpy(&a[c], hv + 8 * c, 8);
                } else {
                    float fv;
                    std::memcpy(&fv, hv + 8 * c, 4);
                    a[c] = fv;
                }
                a[c] = std::fabs(a[c]);
                target[c] = eps[c];
            }
            auto at_point = [&](const double* e) {
                return qoi_estimate_of(qkind, nv, qoi_score_at(qkind, nv, a, e), e);
            };
            for (int step = 0; step < 2200 && at_point(target) > tau_abs; ++step)
                for (uint32_t c = 0; c < nv; ++c) target[c] = target[c] * decay;
            have_target = true;
        }
        bool moved = false;
        if (have_target) {
            for (uint32_t c = 0; c < nv; ++c) {
                std::vector<uint32_t> knew = ks[c];
                plan_to(rts[c]->r, target[c], knew);
                moved = moved || knew != ks[c];
                ks[c] = knew;
            }
        }
        if (!moved)
            for (uint32_t c = 0; c < nv; ++c) plan_step(rts[c]->r, ks[c]);
    }
    if (info) {
        info->tau_abs = tau_abs;
        info->tau_est = tprime;
        for (int c = 0; c < 3; ++c) info->eps[c] = c < (int)nv ? eps[c] : 0.0;
        info->bytes_fetched = fetched;
        info->iterations = it;
        info->met = tprime <= tau_abs ? 1 : 0;
    }
    return MDR_OK;
}

mdr_status mdr_retrieve_batch(mdr_retriever* const* rts, uint32_t n, mdr_bound kind,
                              const double* tols, void* const* const* level_out, void* stream,
                              mdr_retrieve_info* infos)
{
    g_err.clear();
    if (n == 0) return MDR_OK;
    if (!rts || !tols || !level_out) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    if (kind != MDR_ABS && kind != MDR_REL) return fail(MDR_ERR_INVALID_ARG, "bad bound kind");
    std::vector<RetrieveTask> tk(n);
    for (uint32_t i = 0; i < n; ++i) {
        if (!rts[i] || !level_out[i]) return fail(MDR_ERR_INVALID_ARG, "NULL retriever or outputs");
        if (!(tols[i] >= 0.0) || std::isinf(tols[i]))
            return fail(MDR_ERR_INVALID_ARG, "tolerance must be finite and >= 0");
        tk[i].rt = rts[i];
        tk[i].tol_abs = kind == MDR_REL ? tols[i] * value_range(rts[i]->r) : tols[i];
        tk[i].knew = rts[i]->k;
        plan_to(rts[i]->r, tk[i].tol_abs, tk[i].knew);
        tk[i].out = level_out[i];
        tk[i].info = infos ? infos + i : nullptr;
    }
    return retrieve_many(rts[0]->ctx, tk.data(), n, static_cast<hipStream_t>(stream));
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
    return retrieve_one(rt, k, level_out, static_cast<hipStream_t>(stream), 0.0, info);
}

uint64_t mdr_ablation_plane_words(int32_t design, uint64_t n)
{
    if (design < MDR_ABL_LOCALITY || design > MDR_ABL_REGBLOCK) return 0;
    return ablation_plane_words(design, n);
}

static mdr_status ablation_run(int32_t design, bool encode, const uint32_t* in, uint32_t* planes, uint32_t* out,
                               uint64_t n, void* stream)
{
    g_err.clear();
    if (design < MDR_ABL_LOCALITY || design > MDR_ABL_REGBLOCK) return fail(MDR_ERR_INVALID_ARG, "unknown design");
    if (n == 0) return MDR_OK;
    const void* ptrs[2] = {encode ? static_cast<const void*>(in) : static_cast<const void*>(planes),
                           encode ? static_cast<const void*>(planes) : static_cast<const void*>(out)};
    for (const void* p : ptrs) {
        if (!p) return fail(MDR_ERR_INVALID_ARG, "NULL buffer");
        if (reinterpret_cast<uintptr_t>(p) % 16) return fail(MDR_ERR_INVALID_ARG, "buffers must be 16-byte aligned");
    }
    (void)hipGetLastError();
    MDR_HIP(launch_ablation(design, encode, in, n, planes, out, static_cast<hipStream_t>(stream)));
    return MDR_OK;
}

mdr_status mdr_ablation_encode(int32_t design, const uint32_t* in, uint64_t n, uint32_t* planes, void* stream)
{
    return ablation_run(design, true, in, planes, nullptr, n, stream);
}

mdr_status mdr_ablation_decode(int32_t design, const uint32_t* planes, uint64_t n, uint32_t* out, void* stream)
{
    return ablation_run(design, false, nullptr, const_cast<uint32_t*>(planes), out, n, stream);
}

}  // extern "C"

// ---- multilevel decomposition ----------------------------------------------

static mdr_status ml_check(uint64_t n0, uint64_t n1, uint64_t n2, uint32_t nsteps, mdr::MlOffsets* off,
                           uint64_t* total)
{
    if (nsteps > mdr::kMlMaxSteps) return fail(MDR_ERR_INVALID_ARG, "nsteps must be at most 30");
    if (n0 > 65535 || n1 > 65535 || n2 > 0x7fffffffull)
        return fail(MDR_ERR_UNSUPPORTED, "grid too large: n0 and n1 must be below 65536, n2 below 2^31");
    uint64_t sizes[mdr::kMlMaxSteps + 1];
    mdr_level_sizes(n0, n1, n2, nsteps, sizes);
    uint64_t acc = 0;
    for (uint32_t l = 0; l <= nsteps; ++l) {
        if (off) off->off[l] = acc;
        acc += sizes[l];
    }
    *total = acc;
    return MDR_OK;
}

static bool ranges_overlap(const void* a, const void* b, uint64_t bytes)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bytes && y < x + bytes;
}

// [p, p + bytes) inside one device allocation (a host pointer, or a buffer too
// small for the grid, would fault in the kernels)
static bool device_range(const void* p, uint64_t bytes)
{
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const uintptr_t b = reinterpret_cast<uintptr_t>(base), x = reinterpret_cast<uintptr_t>(p);
    return x >= b && x - b + bytes <= size;
}

static mdr_status ml_run(bool decompose, mdr_dtype dtype, const void* in, uint64_t n0, uint64_t n1, uint64_t n2,
                         uint32_t nsteps, void* out, void* stream)
{
    g_err.clear();
    if (dtype != MDR_F32 && dtype != MDR_F64) return fail(MDR_ERR_INVALID_ARG, "dtype must be MDR_F32 or MDR_F64");
    mdr::MlOffsets off{};
    uint64_t total = 0;
    if (mdr_status st = ml_check(n0, n1, n2, nsteps, &off, &total)) return st;
    if (total == 0) return MDR_OK;
    const uint64_t w = dtype == MDR_F64 ? 8 : 4;
    if (!in || !out) return fail(MDR_ERR_INVALID_ARG, "NULL buffer");
    if (reinterpret_cast<uintptr_t>(in) % w || reinterpret_cast<uintptr_t>(out) % w)
        return fail(MDR_ERR_INVALID_ARG, "buffers must be aligned to the value size");
    if (ranges_overlap(in, out, total * w)) return fail(MDR_ERR_INVALID_ARG, "input and output overlap");
    (void)hipGetLastError();
    if (!device_range(in, total * w) || !device_range(out, total * w))
        return fail(MDR_ERR_INVALID_ARG, "buffers must be device memory holding n0*n1*n2 values");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (decompose)
        MDR_HIP(mdr::launch_decompose(dtype == MDR_F64, in, (uint32_t)n0, (uint32_t)n1, (uint32_t)n2, nsteps, off, out, s));
    else
        MDR_HIP(mdr::launch_recompose(dtype == MDR_F64, in, (uint32_t)n0, (uint32_t)n1, (uint32_t)n2, nsteps, off, out, s));
    return MDR_OK;
}

extern "C" {

mdr_status mdr_level_sizes(uint64_t n0, uint64_t n1, uint64_t n2, uint32_t nsteps, uint64_t* sizes)
{
    if (!sizes) return fail(MDR_ERR_INVALID_ARG, "sizes is NULL");
    if (nsteps > mdr::kMlMaxSteps) return fail(MDR_ERR_INVALID_ARG, "nsteps must be at most 30");
    auto count = [&](uint32_t j) -> uint64_t {
        auto m = [&](uint64_t n) { return n == 0 ? 0 : ((n - 1) >> j) + 1; };
        return m(n0) * m(n1) * m(n2);
    };
    sizes[0] = count(nsteps);
    for (uint32_t l = 1; l <= nsteps; ++l) sizes[l] = count(nsteps - l) - count(nsteps - l + 1);
    return MDR_OK;
}

mdr_status mdr_decompose(mdr_dtype dtype, const void* field, uint64_t n0, uint64_t n1, uint64_t n2, uint32_t nsteps,
                         void* coeffs, void* stream)
{
    return ml_run(true, dtype, field, n0, n1, n2, nsteps, coeffs, stream);
}

mdr_status mdr_recompose(mdr_dtype dtype, const void* coeffs, uint64_t n0, uint64_t n1, uint64_t n2, uint32_t nsteps,
                         void* field, void* stream)
{
    return ml_run(false, dtype, coeffs, n0, n1, n2, nsteps, field, stream);
}

}  // extern "C"

// ---- squared-L2 per-plane table ---------------------------------------------

namespace {

// argument checks shared by both table entry points; nmax = the largest level
mdr_status l2_check(const mdr_refactored* r, const mdr_level_view* levels, uint32_t nlevels, uint64_t& nmax)
{
    if (!r || (nlevels && !levels)) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    if (nlevels != r->levels.size()) return fail(MDR_ERR_INVALID_ARG, "level count differs from the refactored one");
    const uint64_t w = r->dtype == MDR_F64 ? 8 : 4;
    nmax = 0;
    for (uint32_t l = 0; l < nlevels; ++l) {
        if (levels[l].n != r->levels[l].n) return fail(MDR_ERR_INVALID_ARG, "level sizes differ from the refactored ones");
        if (levels[l].n == 0) continue;
        if (!levels[l].data || reinterpret_cast<uintptr_t>(levels[l].data) % w)
            return fail(MDR_ERR_INVALID_ARG, "level data must be non-NULL and aligned to the value size");
        (void)hipGetLastError();
        if (!device_range(levels[l].data, levels[l].n * w))
            return fail(MDR_ERR_INVALID_ARG, "level data must be device memory holding n values");
        nmax = std::max(nmax, levels[l].n);
    }
    return MDR_OK;
}

// every level's table into `out` (nlevels * (B + 1) doubles, device) through
// `part` (partial rows, device), then one copy to `host`; waits for the stream,
// also when a launch fails, so that no queued kernel outlives the buffers
mdr_status l2_run(mdr_refactored* r, const mdr_level_view* levels, uint32_t nlevels, uint64_t nmax, double* part,
                  double* out, double* host, hipStream_t s)
{
    const uint32_t B = r->B;
    hipError_t err = hipSuccess;
    const char* what = nullptr;
    const size_t W = (size_t)B + 2;  // a level's row: the table, then the largest |x| read
    for (uint32_t l = 0; l < nlevels && err == hipSuccess; ++l) {
        if (levels[l].n == 0) continue;
        // the next level reuses the partial sums: the launches stay in stream order
        err = launch_l2_table(r->dtype == MDR_F64, levels[l].data, levels[l].n, r->levels[l].e, B, part,
                              out + (size_t)l * W, s);
        what = "launch_l2_table";
    }
    // one copy of every level's row (a copy to pageable memory costs a staging round trip each)
    if (err == hipSuccess && nmax) {
        err = hipMemcpyAsync(host, out, (size_t)nlevels * W * 8, hipMemcpyDeviceToHost, s);
        what = "hipMemcpyAsync(tables)";
    }
    const hipError_t es = hipStreamSynchronize(s);
    if (err != hipSuccess) return hip_fail(err, what);
    if (es != hipSuccess) return hip_fail(es, "hipStreamSynchronize");
    // the values must be the refactored ones: the largest |x| the tables read
    // equals the level's from the refactor, else no table is installed (a
    // table of other data would make an L2 bound a false guarantee)
    for (uint32_t l = 0; l < nlevels; ++l) {
        const LevelRec& L = r->levels[l];
        if (levels[l].n == 0) continue;
        const double amax = std::max(std::fabs(L.vmin), std::fabs(L.vmax));
        if (host[(size_t)l * W + B + 1] != amax)
            return fail(MDR_ERR_INVALID_ARG, "level " + std::to_string(l) +
                                                 ": the values differ from the refactored ones (largest |x|)");
    }
    for (uint32_t l = 0; l < nlevels; ++l) {
        double* t = host + (size_t)l * W;
        if (levels[l].n == 0) std::fill(t, t + B + 1, 0.0);
        r->levels[l].E2.assign(t, t + B + 1);
    }
    return MDR_OK;
}

}  // namespace

extern "C" {

mdr_status mdr_l2_table(mdr_refactored* r, const mdr_level_view* levels, uint32_t nlevels, void* stream)
{
    g_err.clear();
    uint64_t nmax = 0;
    mdr_status st = l2_check(r, levels, nlevels, nmax);
    if (st) return st;
    const uint32_t B = r->B;
    MDR_HIP(hipSetDevice(r->ctx->device));
    PoolBuf part, out;
    MDR_HIP(part.alloc(r->ctx->pool, (uint64_t)l2_table_workgroups(nmax) * (B + 2) * 8));
    MDR_HIP(out.alloc(r->ctx->pool, (uint64_t)nlevels * (B + 2) * 8));
    std::vector<double> host((size_t)nlevels * (B + 2), 0.0);
    return l2_run(r, levels, nlevels, nmax, static_cast<double*>(part.p), static_cast<double*>(out.p), host.data(),
                  static_cast<hipStream_t>(stream));
}

mdr_status mdr_l2_table_noalloc(mdr_refactored* r, const mdr_level_view* levels, uint32_t nlevels, void* stream)
{
    g_err.clear();
    uint64_t nmax = 0;
    mdr_status st = l2_check(r, levels, nlevels, nmax);
    if (st) return st;
    if (nlevels > kL2NoAllocLevels)
        return fail(MDR_ERR_UNSUPPORTED, "mdr_l2_table_noalloc takes at most " + std::to_string(kL2NoAllocLevels) +
                                             " levels (its fixed scratch); use mdr_l2_table");
    MDR_HIP(hipSetDevice(r->ctx->device));
    double *part = nullptr, *out = nullptr;
    MDR_HIP(l2_scratch(r->ctx->device, &part, &out));
    double host[kL2NoAllocLevels * kL2RowMax];  // nlevels * (B + 2) <= 64 * 66
    return l2_run(r, levels, nlevels, nmax, part, out, host, static_cast<hipStream_t>(stream));
}

mdr_status mdr_refactored_l2(const mdr_refactored* r, uint32_t level, double* E2)
{
    if (!r || !E2) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    if (level >= r->levels.size()) return fail(MDR_ERR_INVALID_ARG, "no such level");
    const std::vector<double>& t = r->levels[level].E2;
    if (t.size() != r->B + 1) return fail(MDR_ERR_INVALID_ARG, "no L2 table: call mdr_l2_table first");
    std::copy(t.begin(), t.end(), E2);
    return MDR_OK;
}

}  // extern "C"
