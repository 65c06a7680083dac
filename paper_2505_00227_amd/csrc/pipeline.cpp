// Chunked pipeline for fields larger than one pass should hold (the paper's
// sub-domain pipeline, Sec. 5.1 and 6.2): chunk c of a host field is an
// independent sub-domain with its own levels.  Refactor: the H2D copy of chunk
// c+1, the refactor of chunk c and the D2H copy of chunk c-1's streams run at
// the same time on three streams.  Retrieve: the H2D copy of chunk c+1's
// streams, the decode / reconstruction of chunk c and the D2H copy of chunk
// c-1's values likewise.  Refactored streams stay in pinned host memory between
// the two, laid out exactly as on the device (plane rows, then payloads), so a
// chunk comes back with two copies.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <string>
#include <utility>

#include "api_internal.hpp"

using namespace mdr;

namespace {

struct HostChunk {
    std::vector<LevelRec> levels;  // metadata; unit `dev` fields hold offsets (see below)
    std::vector<uint64_t> unit_off;  // [level * kMaxRows + slot]: offset in rows (DC) or payload blob
    void* rows = nullptr;            // pinned: plane rows as laid out on the device
    uint64_t rows_bytes = 0;
    // byte spans of `rows` that direct-copy units occupy, ascending and merged; only these
    // cross PCIe, since the rows of coded groups are never read once their payloads exist
    std::vector<std::pair<uint64_t, uint64_t>> dc;
    void* pay = nullptr;             // pinned: compressed payloads
    uint64_t pay_bytes = 0, pay_cap = 0;
    ~HostChunk()
    {
        if (rows) (void)hipHostFree(rows);
        if (pay) (void)hipHostFree(pay);
    }
};

}  // namespace

struct mdr_pipeline {
    mdr_context* ctx = nullptr;
    uint32_t nchunks = 0, nlevels = 0, B = 0;
    mdr_dtype dtype = MDR_F32;
    mdr_codec_params prm{};
    std::vector<uint64_t> sizes;  // values per level of one chunk
    uint64_t chunk_values = 0, chunk_bytes = 0;
    std::vector<std::unique_ptr<HostChunk>> chunks;
    bool have = false;  // refactored data present
    hipStream_t st[3] = {nullptr, nullptr, nullptr};  // H2D, compute, D2H
    PoolBuf dev_in[2], dev_rows[2], dev_pay[2], dev_out[2];
    std::vector<hipEvent_t> events;
    double value_lo = 0.0, value_hi = 0.0;
};

namespace {

hipEvent_t make_event(mdr_pipeline* p, bool timing)
{
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, timing ? hipEventDefault : hipEventDisableTiming) != hipSuccess)
        return nullptr;
    p->events.push_back(e);
    return e;
}

uint64_t elem(const mdr_pipeline* p) { return p->dtype == MDR_F64 ? 8 : 4; }

// device-resident view of a host chunk whose rows / payload blobs were copied to rows / pay
std::unique_ptr<mdr_refactored> device_view(const mdr_pipeline* p, const HostChunk& hc, uint8_t* rows,
                                            uint8_t* pay)
{
    auto R = std::make_unique<mdr_refactored>();
    R->ctx = p->ctx;
    R->dtype = p->dtype;
    R->B = p->B;
    R->m = p->prm.group_planes;
    R->G = p->dtype == MDR_F64 ? 2 : 1;
    R->prm = p->prm;
    R->levels = hc.levels;
    uint64_t roff = 0;
    for (uint32_t l = 0; l < p->nlevels; ++l) {
        LevelRec& L = R->levels[l];
        L.rows = reinterpret_cast<uint32_t*>(rows + roff);
        roff += align256(4ull * (p->B + 1) * L.nbd);
        for (uint32_t s = 0; s <= p->B; ++s) {
            UnitRec& u = L.units[s];
            if (u.method == MDR_PLACEHOLDER) continue;
            const uint64_t o = hc.unit_off[(uint64_t)l * kMaxRows + s];
            u.dev = (u.method == MDR_DC ? rows : pay) + o;
        }
    }
    return R;
}

// keep a refactored chunk's metadata, with unit offsets instead of pointers
void keep_meta(const mdr_refactored* R, HostChunk& hc, uint64_t& pay_used)
{
    hc.levels = R->levels;
    hc.unit_off.assign(R->levels.size() * kMaxRows, 0);
    const uint8_t* rows0 = reinterpret_cast<const uint8_t*>(R->levels.empty() ? nullptr : R->levels[0].rows);
    const uint8_t* pay0 = static_cast<const uint8_t*>(R->payload_arena->p);
    pay_used = 0;
    hc.dc.clear();
    for (size_t l = 0; l < R->levels.size(); ++l)
        for (uint32_t s = 0; s <= R->B; ++s) {
            const UnitRec& u = R->levels[l].units[s];
            if (u.method == MDR_PLACEHOLDER) continue;
            uint64_t o;
            if (u.method == MDR_DC) {
                o = (uint64_t)(u.dev - rows0);
                if (u.bytes) hc.dc.emplace_back(o, u.bytes);
            } else {
                o = (uint64_t)(u.dev - pay0);
                pay_used = std::max(pay_used, o + u.bytes);
            }
            hc.unit_off[l * kMaxRows + s] = o;
            hc.levels[l].units[s].dev = nullptr;
        }
    for (LevelRec& L : hc.levels) L.rows = nullptr;
    std::sort(hc.dc.begin(), hc.dc.end());
    size_t k = 0;
    for (size_t i = 0; i < hc.dc.size(); ++i) {
        if (k && hc.dc[k - 1].first + hc.dc[k - 1].second == hc.dc[i].first)
            hc.dc[k - 1].second += hc.dc[i].second;
        else
            hc.dc[k++] = hc.dc[i];
    }
    hc.dc.resize(k);
}

// bytes of a chunk's rows that cross PCIe
uint64_t dc_bytes(const HostChunk& hc)
{
    uint64_t b = 0;
    for (const auto& d : hc.dc) b += d.second;
    return b;
}

// Byte spans of the units that planes k (per level) need, in the rows region
// (direct-copy units) and the payload blob (coded units), each list ascending
// and merged: the retrieval uploads only these (Sec. 5.1's retrieval moves just
// the precision segments the bound needs).
void fetch_spans(const mdr_pipeline* p, const HostChunk& hc, const std::vector<uint32_t>& k,
                 std::vector<std::pair<uint64_t, uint64_t>>& rows, std::vector<std::pair<uint64_t, uint64_t>>& pay)
{
    rows.clear();
    pay.clear();
    for (uint32_t l = 0; l < p->nlevels; ++l) {
        if (k[l] == 0) continue;
        for (uint32_t s = 0; s <= p->B; ++s) {
            const UnitRec& u = hc.levels[l].units[s];
            if (u.method == MDR_PLACEHOLDER || u.bytes == 0) continue;
            if (s > 0 && s - 1 >= k[l]) break;  // the group's first plane is past k: so are the rest
            auto& v = u.method == MDR_DC ? rows : pay;
            v.emplace_back(hc.unit_off[(uint64_t)l * kMaxRows + s], u.bytes);
        }
    }
    for (auto* v : {&rows, &pay}) {
        std::sort(v->begin(), v->end());
        size_t n = 0;
        for (size_t i = 0; i < v->size(); ++i) {
            if (n && (*v)[n - 1].first + (*v)[n - 1].second == (*v)[i].first)
                (*v)[n - 1].second += (*v)[i].second;
            else
                (*v)[n++] = (*v)[i];
        }
        v->resize(n);
    }
}

double elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return ms;
}

}  // namespace

extern "C" {

mdr_status mdr_pipeline_create(mdr_context* ctx, uint32_t nchunks, const uint64_t* level_sizes, uint32_t nlevels,
                               mdr_dtype dtype, uint32_t nplanes, const mdr_codec_params* params,
                               mdr_pipeline** out)
{
    if (!out) return fail(MDR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx || !level_sizes || nlevels == 0 || nchunks == 0) return fail(MDR_ERR_INVALID_ARG, "bad argument");
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
    auto p = std::make_unique<mdr_pipeline>();
    p->ctx = ctx;
    p->nchunks = nchunks;
    p->nlevels = nlevels;
    p->B = nplanes;
    p->dtype = dtype;
    p->prm = prm;
    p->sizes.assign(level_sizes, level_sizes + nlevels);
    for (uint64_t n : p->sizes) p->chunk_values += n;
    p->chunk_bytes = p->chunk_values * elem(p.get());
    MDR_HIP(hipSetDevice(ctx->device));
    for (int i = 0; i < 3; ++i) MDR_HIP(hipStreamCreateWithFlags(&p->st[i], hipStreamNonBlocking));
    p->chunks.resize(nchunks);
    *out = p.release();
    return MDR_OK;
}

void mdr_pipeline_destroy(mdr_pipeline* p)
{
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    for (int i = 0; i < 3; ++i)
        if (p->st[i]) (void)hipStreamSynchronize(p->st[i]);
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    for (int i = 0; i < 3; ++i)
        if (p->st[i]) (void)hipStreamDestroy(p->st[i]);
    delete p;
}

mdr_status mdr_pipeline_refactor(mdr_pipeline* p, const void* host_values, int overlap, mdr_pipeline_info* info)
{
    if (!p || !host_values) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    MDR_HIP(hipSetDevice(p->ctx->device));
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t A = p->st[0], Bs = p->st[1], C = p->st[2];
    for (int s = 0; s < 2; ++s)
        if (!p->dev_in[s].p) {
            hipError_t e = p->dev_in[s].alloc(p->ctx->pool, p->chunk_bytes);
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(pipeline input)");
        }
    const uint8_t* host = static_cast<const uint8_t*>(host_values);
    std::vector<hipEvent_t> h2d_a(p->nchunks), h2d_b(p->nchunks), cmp_a(p->nchunks), cmp_b(p->nchunks),
        d2h_a(p->nchunks), d2h_b(p->nchunks);
    for (uint32_t c = 0; c < p->nchunks; ++c) {
        h2d_a[c] = make_event(p, true), h2d_b[c] = make_event(p, true);
        cmp_a[c] = make_event(p, true), cmp_b[c] = make_event(p, true);
        d2h_a[c] = make_event(p, true), d2h_b[c] = make_event(p, true);
        if (!h2d_a[c] || !h2d_b[c] || !cmp_a[c] || !cmp_b[c] || !d2h_a[c] || !d2h_b[c])
            return fail(MDR_ERR_HIP, "hipEventCreate");
    }
    auto h2d = [&](uint32_t c) -> mdr_status {
        MDR_HIP(hipEventRecord(h2d_a[c], A));
        MDR_HIP(hipMemcpyAsync(p->dev_in[c & 1].p, host + (uint64_t)c * p->chunk_bytes, p->chunk_bytes,
                               hipMemcpyHostToDevice, A));
        MDR_HIP(hipEventRecord(h2d_b[c], A));
        return MDR_OK;
    };
    std::vector<std::unique_ptr<mdr_refactored>> live(p->nchunks);
    uint64_t h2d_bytes = 0, d2h_bytes = 0, stream_bytes = 0;
    mdr_status st = h2d(0);
    if (st) return st;
    h2d_bytes += p->chunk_bytes;
    double lo = 0.0, hi = 0.0;
    bool have_range = false;
    for (uint32_t c = 0; c < p->nchunks; ++c) {
        if (overlap && c + 1 < p->nchunks) {  // next input while this chunk is refactored
            st = h2d(c + 1);
            if (st) return st;
            h2d_bytes += p->chunk_bytes;
        }
        MDR_HIP(hipStreamWaitEvent(Bs, h2d_b[c], 0));
        std::vector<mdr_level_view> views(p->nlevels);
        uint64_t o = 0;
        for (uint32_t l = 0; l < p->nlevels; ++l) {
            views[l].data = static_cast<uint8_t*>(p->dev_in[c & 1].p) + o * elem(p);
            views[l].n = p->sizes[l];
            o += p->sizes[l];
        }
        VarLevels v{views.data(), p->nlevels};
        mdr_refactored* R = nullptr;
        MDR_HIP(hipEventRecord(cmp_a[c], Bs));
        st = refactor_batch(p->ctx, &v, 1, p->dtype, p->B, p->prm, Bs, p->ctx->graphs, &R);
        if (st) return st;
        MDR_HIP(hipEventRecord(cmp_b[c], Bs));
        live[c].reset(R);
        for (const LevelRec& L : R->levels) {
            if (L.n == 0) continue;
            if (!have_range || L.vmin < lo) lo = L.vmin;
            if (!have_range || L.vmax > hi) hi = L.vmax;
            have_range = true;
        }
        // streams of this chunk to pinned host memory
        if (!p->chunks[c]) p->chunks[c] = std::make_unique<HostChunk>();
        HostChunk& hc = *p->chunks[c];
        uint64_t pay_used = 0;
        keep_meta(R, hc, pay_used);
        const uint64_t rows_bytes = R->rows_arena->bytes;
        if (hc.rows_bytes < rows_bytes) {
            if (hc.rows) (void)hipHostFree(hc.rows);
            hc.rows = nullptr;
            MDR_HIP(hipHostMalloc(&hc.rows, rows_bytes, hipHostMallocDefault));
            hc.rows_bytes = rows_bytes;
        }
        if (hc.pay_cap < pay_used) {
            if (hc.pay) (void)hipHostFree(hc.pay);
            hc.pay = nullptr;
            MDR_HIP(hipHostMalloc(&hc.pay, pay_used, hipHostMallocDefault));
            hc.pay_cap = pay_used;
        }
        hc.pay_bytes = pay_used;
        MDR_HIP(hipStreamWaitEvent(C, cmp_b[c], 0));
        MDR_HIP(hipEventRecord(d2h_a[c], C));
        for (const auto& d : hc.dc)
            MDR_HIP(hipMemcpyAsync(static_cast<uint8_t*>(hc.rows) + d.first,
                                   static_cast<const uint8_t*>(R->rows_arena->p) + d.first, d.second,
                                   hipMemcpyDeviceToHost, C));
        if (pay_used) MDR_HIP(hipMemcpyAsync(hc.pay, R->payload_arena->p, pay_used, hipMemcpyDeviceToHost, C));
        MDR_HIP(hipEventRecord(d2h_b[c], C));
        d2h_bytes += dc_bytes(hc) + pay_used;
        for (const LevelRec& L : R->levels)
            for (uint32_t s = 0; s <= p->B; ++s)
                if (L.units[s].method != MDR_PLACEHOLDER) stream_bytes += L.units[s].bytes;
        if (!overlap) {  // one stage at a time
            MDR_HIP(hipEventSynchronize(d2h_b[c]));
            if (c + 1 < p->nchunks) {
                st = h2d(c + 1);
                if (st) return st;
                h2d_bytes += p->chunk_bytes;
            }
        }
        // the previous chunk's device arenas go back once its copies are done
        if (c >= 1 && live[c - 1]) {
            MDR_HIP(hipEventSynchronize(d2h_b[c - 1]));
            live[c - 1].reset();
        }
    }
    MDR_HIP(hipStreamSynchronize(C));
    live.clear();
    p->have = true;
    p->value_lo = lo;
    p->value_hi = hi;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (uint32_t c = 0; c < p->nchunks; ++c) {
            info->h2d_ms += elapsed(h2d_a[c], h2d_b[c]);
            info->compute_ms += elapsed(cmp_a[c], cmp_b[c]);
            info->d2h_ms += elapsed(d2h_a[c], d2h_b[c]);
        }
        info->h2d_bytes = h2d_bytes;
        info->d2h_bytes = d2h_bytes;
        info->stream_bytes = stream_bytes;
    }
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    p->events.clear();
    return MDR_OK;
}

mdr_status mdr_pipeline_retrieve(mdr_pipeline* p, mdr_bound kind, double tol, void* host_out, int overlap,
                                 mdr_pipeline_info* info)
{
    if (!p || !host_out) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    if (!p->have) return fail(MDR_ERR_INVALID_ARG, "nothing refactored yet");
    if (kind != MDR_ABS && kind != MDR_REL) return fail(MDR_ERR_INVALID_ARG, "bad bound kind");
    if (!(tol >= 0.0) || std::isinf(tol)) return fail(MDR_ERR_INVALID_ARG, "tolerance must be finite and >= 0");
    MDR_HIP(hipSetDevice(p->ctx->device));
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t A = p->st[0], Bs = p->st[1], C = p->st[2];
    uint64_t rows_max = 0, pay_max = 0;
    for (auto& hc : p->chunks) {
        rows_max = std::max(rows_max, hc->rows_bytes);
        pay_max = std::max(pay_max, hc->pay_bytes);
    }
    for (int s = 0; s < 2; ++s) {
        if (p->dev_rows[s].bytes < rows_max) {
            hipError_t e = p->dev_rows[s].alloc(p->ctx->pool, rows_max);
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(pipeline rows)");
        }
        // 256 bytes past the last payload: the Huffman decoder reads whole aligned
        // 16-byte blocks, the last of which may end past its stream
        if (p->dev_pay[s].bytes < pay_max + 256) {
            hipError_t e = p->dev_pay[s].alloc(p->ctx->pool, pay_max + 256);
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(pipeline payloads)");
        }
        if (!p->dev_out[s].p) {
            hipError_t e = p->dev_out[s].alloc(p->ctx->pool, p->chunk_bytes + 256ull * p->nlevels);
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(pipeline output)");
        }
    }
    // one absolute tolerance for every chunk: relative to the whole field's range
    const double tol_abs = kind == MDR_REL ? tol * (p->value_hi - p->value_lo) : tol;
    uint8_t* out = static_cast<uint8_t*>(host_out);
    // pinned output: the values leave through a kernel writing the host memory's
    // device address (the copy engine's downloads slowed to half speed while
    // the next chunk's streams were uploading); pageable output: copies
    uint8_t* out_dev = nullptr;
    {
        void* dp = nullptr;
        if (hipHostGetDevicePointer(&dp, host_out, 0) == hipSuccess)
            out_dev = static_cast<uint8_t*>(dp);
        else
            (void)hipGetLastError();
    }
    const uint32_t N = p->nchunks;
    std::vector<hipEvent_t> h2d_a(N), h2d_b(N), cmp_a(N), cmp_b(N), d2h_a(N), d2h_b(N);
    for (uint32_t c = 0; c < N; ++c) {
        h2d_a[c] = make_event(p, true), h2d_b[c] = make_event(p, true);
        cmp_a[c] = make_event(p, true), cmp_b[c] = make_event(p, true);
        d2h_a[c] = make_event(p, true), d2h_b[c] = make_event(p, true);
        if (!h2d_a[c] || !h2d_b[c] || !cmp_a[c] || !cmp_b[c] || !d2h_a[c] || !d2h_b[c])
            return fail(MDR_ERR_HIP, "hipEventCreate");
    }
    std::vector<std::unique_ptr<mdr_refactored>> views(N);
    std::vector<mdr_retriever*> rts(N, nullptr);
    struct Cleanup {
        std::vector<mdr_retriever*>& r;
        ~Cleanup()
        {
            for (mdr_retriever* x : r)
                if (x) delete x;
        }
    } cleanup{rts};
    uint64_t h2d_bytes = 0, d2h_bytes = 0, fetched = 0;
    // every chunk's plan first, on the host from its error tables: the uploads
    // carry only the units the plan reads
    std::vector<std::vector<uint32_t>> plans(N);
    for (uint32_t c = 0; c < N; ++c) {
        const int s = c & 1;
        views[c] = device_view(p, *p->chunks[c], static_cast<uint8_t*>(p->dev_rows[s].p),
                               static_cast<uint8_t*>(p->dev_pay[s].p));
        plans[c].assign(p->nlevels, 0);
        plan_to(views[c].get(), tol_abs, plans[c]);
    }
    std::vector<std::pair<uint64_t, uint64_t>> span_rows, span_pay;
    auto h2d = [&](uint32_t c) -> mdr_status {
        const HostChunk& hc = *p->chunks[c];
        const int s = c & 1;
        if (c >= 2) MDR_HIP(hipStreamWaitEvent(A, cmp_b[c - 2], 0));  // slot free once chunk c-2 is rebuilt
        MDR_HIP(hipEventRecord(h2d_a[c], A));
        fetch_spans(p, hc, plans[c], span_rows, span_pay);
        for (const auto& d : span_rows) {
            MDR_HIP(hipMemcpyAsync(static_cast<uint8_t*>(p->dev_rows[s].p) + d.first,
                                   static_cast<const uint8_t*>(hc.rows) + d.first, d.second,
                                   hipMemcpyHostToDevice, A));
            h2d_bytes += d.second;
        }
        for (const auto& d : span_pay) {
            MDR_HIP(hipMemcpyAsync(static_cast<uint8_t*>(p->dev_pay[s].p) + d.first,
                                   static_cast<const uint8_t*>(hc.pay) + d.first, d.second,
                                   hipMemcpyHostToDevice, A));
            h2d_bytes += d.second;
        }
        MDR_HIP(hipEventRecord(h2d_b[c], A));
        return MDR_OK;
    };
    mdr_status st = h2d(0);
    if (st) return st;
    for (uint32_t c = 0; c < N; ++c) {
        if (overlap && c + 1 < N) {
            st = h2d(c + 1);
            if (st) return st;
        }
        const int s = c & 1;
        rts[c] = new mdr_retriever();
        rts[c]->ctx = p->ctx;
        rts[c]->r = views[c].get();
        rts[c]->k.assign(p->nlevels, 0);
        rts[c]->dec.resize(p->nlevels);
        for (auto& d : rts[c]->dec) d.resize(kMaxRows);
        RetrieveTask t;
        t.rt = rts[c];
        t.knew = plans[c];
        t.tol_abs = tol_abs;
        std::vector<void*> lo(p->nlevels);
        uint64_t o = 0;
        for (uint32_t l = 0; l < p->nlevels; ++l) {
            lo[l] = static_cast<uint8_t*>(p->dev_out[s].p) + o;
            o += align256(p->sizes[l] * elem(p));
        }
        t.out = lo.data();
        mdr_retrieve_info ri{};
        t.info = &ri;
        MDR_HIP(hipStreamWaitEvent(Bs, h2d_b[c], 0));
        if (c >= 2) MDR_HIP(hipStreamWaitEvent(Bs, d2h_b[c - 2], 0));  // output slot free
        MDR_HIP(hipEventRecord(cmp_a[c], Bs));
        st = retrieve_many(p->ctx, &t, 1, Bs);
        if (st) return st;
        MDR_HIP(hipEventRecord(cmp_b[c], Bs));
        fetched += ri.bytes_fetched;
        // values of this chunk back to the host, levels concatenated
        MDR_HIP(hipStreamWaitEvent(C, cmp_b[c], 0));
        MDR_HIP(hipEventRecord(d2h_a[c], C));
        o = 0;
        uint64_t ho = (uint64_t)c * p->chunk_bytes;
        CopySpans sp{};
        for (uint32_t l = 0; l < p->nlevels; ++l) {
            const uint64_t nb = p->sizes[l] * elem(p);
            const uint8_t* src = static_cast<uint8_t*>(p->dev_out[s].p) + o;
            if (nb && out_dev && sp.n < (uint32_t)kCopySpans) {
                sp.src[sp.n] = reinterpret_cast<const uint32_t*>(src);
                sp.dst[sp.n] = reinterpret_cast<uint32_t*>(out_dev + ho);
                sp.words[sp.n] = nb / 4;
                ++sp.n;
            } else if (nb) {
                MDR_HIP(hipMemcpyAsync(out + ho, src, nb, hipMemcpyDeviceToHost, C));
            }
            ho += nb;
            o += align256(nb);
        }
        MDR_HIP(launch_copy_out(sp, C));
        MDR_HIP(hipEventRecord(d2h_b[c], C));
        d2h_bytes += p->chunk_bytes;
        if (!overlap) {
            MDR_HIP(hipEventSynchronize(d2h_b[c]));
            if (c + 1 < N) {
                st = h2d(c + 1);
                if (st) return st;
            }
        }
        // chunk c-1's decoded groups go back once it is rebuilt
        if (c >= 1 && rts[c - 1]) {
            MDR_HIP(hipEventSynchronize(cmp_b[c - 1]));
            delete rts[c - 1];
            rts[c - 1] = nullptr;
        }
    }
    MDR_HIP(hipStreamSynchronize(C));
    MDR_HIP(hipStreamSynchronize(Bs));
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (uint32_t c = 0; c < N; ++c) {
            info->h2d_ms += elapsed(h2d_a[c], h2d_b[c]);
            info->compute_ms += elapsed(cmp_a[c], cmp_b[c]);
            info->d2h_ms += elapsed(d2h_a[c], d2h_b[c]);
        }
        info->h2d_bytes = h2d_bytes;
        info->d2h_bytes = d2h_bytes;
        info->stream_bytes = fetched;
    }
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    p->events.clear();
    return MDR_OK;
}

mdr_status mdr_pipeline_chunk(const mdr_pipeline* p, uint32_t chunk, mdr_context* ctx, mdr_refactored** out)
{
    if (!out) return fail(MDR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!p || !ctx) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    if (!p->have || chunk >= p->nchunks) return fail(MDR_ERR_INVALID_ARG, "no such refactored chunk");
    const HostChunk& hc = *p->chunks[chunk];
    MDR_HIP(hipSetDevice(ctx->device));
    auto rows = std::make_shared<PoolBuf>();
    auto pay = std::make_shared<PoolBuf>();
    hipError_t e = rows->alloc(ctx->pool, hc.rows_bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(chunk rows)");
    e = pay->alloc(ctx->pool, hc.pay_bytes + 256);  // padded for the decoder's block reads
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(chunk payloads)");
    for (const auto& d : hc.dc)
        MDR_HIP(hipMemcpy(static_cast<uint8_t*>(rows->p) + d.first, static_cast<const uint8_t*>(hc.rows) + d.first,
                          d.second, hipMemcpyHostToDevice));
    if (hc.pay_bytes) MDR_HIP(hipMemcpy(pay->p, hc.pay, hc.pay_bytes, hipMemcpyHostToDevice));
    auto R = device_view(p, hc, static_cast<uint8_t*>(rows->p), static_cast<uint8_t*>(pay->p));
    R->ctx = ctx;
    R->rows_arena = rows;
    R->payload_arena = pay;
    *out = R.release();
    return MDR_OK;
}

}  // extern "C"
