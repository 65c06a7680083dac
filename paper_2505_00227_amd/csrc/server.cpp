// Retrieval server: refactored fields stay resident in HBM and an engine
// thread serves retrieval requests with continuous batching.  Every engine
// step advances every admitted request by one round of its retrieval (a raw
// request finishes in one round; a V_total request takes the rounds of Alg. 3
// with MAPE, Sec. 5.2) with one batched decode, one batched reconstruction and
// one batched estimate for all of them.  Requests are admitted whenever a slot
// and enough of the HBM budget for their outputs are free, also while others
// are in flight.  Decoded groups are cached per field and shared by every
// request on it; a request's result depends only on its own planes, so it is
// the same alone and in any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>

#include "api_internal.hpp"

using namespace mdr;

namespace {

struct Field {
    const mdr_refactored* r = nullptr;
    mdr_retriever* cache = nullptr;  // decoded groups shared by every request on the field
    uint64_t out_bytes = 0;          // one reconstruction (all levels, 256-byte aligned)
    double range = 0.0;              // max - min over the field's values
    double absmax = 0.0;             // max(|min|, |max|)
};

struct Req {
    uint64_t ticket = 0;
    mdr_request q{};
    int ncomp = 1;
    uint32_t field[3] = {0, 0, 0};
    std::vector<uint32_t> k[3];      // planes per level (current plan)
    std::vector<uint32_t> kdone[3];  // planes already in the output
    std::vector<uint32_t> kstart[3]; // planes held by the parent session at the start
    void* out[3] = {nullptr, nullptr, nullptr};  // one device block per component
    uint64_t need = 0;               // budget charged for the outputs (all blocks)
    std::vector<void*> outp[3];
    double tol_abs = 0.0, eps[3] = {0, 0, 0}, est = 0.0;
    uint32_t it = 0;
    bool first = true;
    mdr_completion c{};
};

double now_ms(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct mdr_server {
    mdr_context* ctx = nullptr;  // the server's own context (pool, staging), same device
    hipStream_t stream = nullptr;
    uint64_t budget = 0, in_use = 0;
    uint32_t max_slots = 0;
    std::vector<Field> fields;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::thread engine;
    uint64_t next_ticket = 1;
    std::deque<Req*> pending;
    std::vector<Req*> active;                    // owned by the engine thread
    std::unordered_map<uint64_t, Req*> done;     // completed, outputs held until released
    std::deque<mdr_completion> completions;      // not yet polled
    std::unordered_map<uint64_t, int> state;     // ticket -> 0 pending, 1 active, 2 done/released
    std::unordered_map<uint64_t, std::vector<uint32_t>> final_k;  // ticket -> planes at completion (3 x nlevels)
    // Output blocks (one component's reconstruction each) of released
    // requests, kept by size for the next block of that size: serving then
    // allocates and frees no device memory in steady state (a free would also
    // wait for the whole device).  `held` counts every output block, in use or
    // kept; it never exceeds the budget.
    std::multimap<uint64_t, void*> spare;
    uint64_t held = 0;
    uint64_t steps = 0, step_requests = 0;
    DevBuf acc;                                  // V_total accumulators, one per active request
    void* acc_host = nullptr;
};

namespace {

// bytes of one component's output block (all levels, each 256-byte aligned)
uint64_t block_bytes(const mdr_server* S, uint32_t field) { return S->fields[field].out_bytes; }

void keep_blocks(mdr_server* S, Req* q);

void complete(mdr_server* S, Req* q, mdr_status st)
{
    q->c.ticket = q->ticket;
    q->c.tag = q->q.tag;
    q->c.status = st;
    q->c.t_done_ms = now_ms(S->t0);
    q->c.iterations = q->it;
    std::vector<uint32_t> fk;
    for (int c = 0; c < q->ncomp; ++c) fk.insert(fk.end(), q->k[c].begin(), q->k[c].end());
    std::lock_guard<std::mutex> lk(S->mu);
    if (st == MDR_OK) S->final_k[q->ticket] = std::move(fk);  // a session later requests may refine
    S->state[q->ticket] = 2;
    S->completions.push_back(q->c);
    if (st != MDR_OK) {
        S->in_use -= q->need;
        keep_blocks(S, q);
        delete q;
    } else {
        S->done[q->ticket] = q;
    }
    S->cv.notify_all();
}

// a request's blocks back to the kept ones (caller holds the mutex)
void keep_blocks(mdr_server* S, Req* q)
{
    for (int c = 0; c < 3; ++c)
        if (q->out[c]) {
            S->spare.emplace(block_bytes(S, q->field[c]), q->out[c]);
            q->out[c] = nullptr;
        }
}

// an output block of `need` bytes: a kept one of that size, else a new one
// after giving back kept blocks (largest first) until it fits the budget
mdr_status take_block(mdr_server* S, uint64_t need, void** p)
{
    *p = nullptr;
    std::vector<void*> drop;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->spare.find(need);
        if (it != S->spare.end()) {
            *p = it->second;
            S->spare.erase(it);
            return MDR_OK;
        }
        while (S->held + need > S->budget && !S->spare.empty()) {
            auto last = std::prev(S->spare.end());
            S->held -= last->first;
            drop.push_back(last->second);
            S->spare.erase(last);
        }
        S->held += need;  // the blocks in use are the admitted outputs: within the budget
    }
    for (void* d : drop) (void)hipFree(d);
    hipError_t e = hipMalloc(p, need);
    if (e != hipSuccess) {
        *p = nullptr;
        std::lock_guard<std::mutex> lk(S->mu);
        S->held -= need;
        return hip_fail(e, "hipMalloc(request outputs)");
    }
    return MDR_OK;
}

// set up a request at admission: outputs, starting planes, first plan
mdr_status start(mdr_server* S, Req* q)
{
    const Field& f0 = S->fields[q->field[0]];
    const size_t nl = f0.r->levels.size();
    for (int c = 0; c < q->ncomp; ++c) {
        mdr_status bst = take_block(S, block_bytes(S, q->field[c]), &q->out[c]);
        if (bst) return bst;
    }
    for (int c = 0; c < q->ncomp; ++c) {
        const mdr_refactored* r = S->fields[q->field[c]].r;
        uint8_t* base = static_cast<uint8_t*>(q->out[c]);
        q->outp[c].resize(nl);
        uint64_t o = 0;
        for (size_t l = 0; l < nl; ++l) {
            q->outp[c][l] = base + o;
            o += align256(r->levels[l].n * (r->dtype == MDR_F64 ? 8 : 4));
        }
        q->kdone[c].assign(nl, 0);
    }
    // starting planes: the parent's final planes, or none
    for (int c = 0; c < q->ncomp; ++c) q->k[c].assign(nl, 0);
    if (q->q.parent) {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->final_k.find(q->q.parent);
        if (it == S->final_k.end()) return fail(MDR_ERR_INVALID_ARG, "parent request is unknown or failed");
        if (it->second.size() != nl * q->ncomp)
            return fail(MDR_ERR_INVALID_ARG, "parent request has another kind or shape");
        for (int c = 0; c < q->ncomp; ++c)
            q->k[c].assign(it->second.begin() + c * nl, it->second.begin() + (c + 1) * nl);
    }
    for (int c = 0; c < q->ncomp; ++c) q->kstart[c] = q->k[c];
    if (q->ncomp == 1) {
        const Field& f = S->fields[q->field[0]];
        q->tol_abs = q->q.bound == MDR_REL ? q->q.tol * f.range : q->q.tol;
        plan_to(f.r, q->tol_abs, q->k[0]);
    } else {
        double qmax = 0.0;
        for (int c = 0; c < 3; ++c) qmax = qmax + S->fields[q->field[c]].absmax * S->fields[q->field[c]].absmax;
        q->tol_abs = q->q.bound == MDR_REL ? q->q.tol * qmax : q->q.tol;
        for (int c = 0; c < 3; ++c) {
            const double e0 = qmax == 0.0 ? 0.0 : (q->tol_abs / qmax) * S->fields[q->field[c]].range;
            plan_to(S->fields[q->field[c]].r, e0, q->k[c]);
        }
    }
    q->c.t_start_ms = now_ms(S->t0);
    return MDR_OK;
}

// bytes of the groups in k that the starting planes did not hold
uint64_t new_bytes(const mdr_refactored* r, const std::vector<uint32_t>& k0, const std::vector<uint32_t>& k1)
{
    uint64_t b = 0;
    for (size_t l = 0; l < r->levels.size(); ++l) {
        const LevelRec& L = r->levels[l];
        for (uint32_t slot = 0; slot <= r->B; slot = slot == 0 ? 1 : slot + r->m) {
            const bool before = slot == 0 ? k0[l] > 0 : (slot - 1) < k0[l];
            const bool now = slot == 0 ? k1[l] > 0 : (slot - 1) < k1[l];
            if (now && !before) b += L.units[slot].bytes;
        }
    }
    return b;
}

// one engine step over every active request
mdr_status step(mdr_server* S)
{
    std::vector<Req*>& act = S->active;
    hipStream_t s = S->stream;
    // decode targets: per field, the most planes any active request needs
    std::map<uint32_t, std::vector<uint32_t>> target;
    for (Req* q : act)
        for (int c = 0; c < q->ncomp; ++c) {
            const uint32_t fi = q->field[c];
            auto it = target.find(fi);
            if (it == target.end()) it = target.emplace(fi, S->fields[fi].cache->k).first;
            for (size_t l = 0; l < q->k[c].size(); ++l) it->second[l] = std::max(it->second[l], q->k[c][l]);
        }
    std::vector<RetrieveTask> tasks;
    for (auto& kv : target) {
        mdr_retriever* cache = S->fields[kv.first].cache;
        if (kv.second == cache->k) continue;
        RetrieveTask t;
        t.rt = cache;
        t.knew = kv.second;
        t.reconstruct = false;
        tasks.push_back(std::move(t));
    }
    std::vector<ReconOnly> rec;
    for (Req* q : act)
        for (int c = 0; c < q->ncomp; ++c) {
            ReconOnly ro;
            ro.rt = S->fields[q->field[c]].cache;
            ro.k = q->k[c];
            ro.kprev = q->first ? nullptr : &q->kdone[c];
            ro.out = q->outp[c].data();
            rec.push_back(std::move(ro));
        }
    mdr_status st = retrieve_many(S->ctx, tasks.data(), tasks.size(), s, rec.data(), rec.size());
    if (st) return st;
    // V_total estimates of the QoI requests
    std::vector<QoiJob> jobs;
    std::vector<bool> f64;
    uint32_t nq = 0;
    std::vector<int> slot_of(act.size(), -1);
    for (size_t i = 0; i < act.size(); ++i) {
        Req* q = act[i];
        if (q->ncomp != 3) continue;
        slot_of[i] = (int)nq++;
        for (int c = 0; c < 3; ++c) q->eps[c] = plan_bound(S->fields[q->field[c]].r, q->k[c]);
    }
    if (nq) {
        if (S->acc.bytes < 8ull * nq) {
            MDR_HIP(hipStreamSynchronize(s));
            hipError_t e = S->acc.alloc(8ull * nq + 4096);
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(accumulators)");
            if (S->acc_host) (void)hipHostFree(S->acc_host);
            S->acc_host = nullptr;
            MDR_HIP(hipHostMalloc(&S->acc_host, S->acc.bytes, hipHostMallocDefault));
        }
        unsigned long long* acc = static_cast<unsigned long long*>(S->acc.p);
        for (size_t i = 0; i < act.size(); ++i) {
            if (slot_of[i] < 0) continue;
            Req* q = act[i];
            const mdr_refactored* r0 = S->fields[q->field[0]].r;
            for (size_t l = 0; l < r0->levels.size(); ++l) {
                QoiJob j{};
                j.x = q->outp[0][l];
                j.y = q->outp[1][l];
                j.z = q->outp[2][l];
                j.n = r0->levels[l].n;
                for (int c = 0; c < 3; ++c) j.eps[c] = q->eps[c];
                j.kind = kQoiSumsq;  // V_total: the sum of squares of three variables
                j.nvars = 3;
                j.acc = acc + slot_of[i];
                jobs.push_back(j);
                f64.push_back(r0->dtype == MDR_F64);
            }
        }
        st = enqueue_qoi(S->ctx, jobs, f64, acc, nq, s);
        if (st) return st;
        MDR_HIP(hipMemcpyAsync(S->acc_host, acc, 8ull * nq, hipMemcpyDeviceToHost, s));
    }
    MDR_HIP(hipStreamSynchronize(s));
    ++S->steps;
    S->step_requests += act.size();

    // advance each request
    std::vector<Req*> keep;
    for (size_t i = 0; i < act.size(); ++i) {
        Req* q = act[i];
        ++q->it;
        for (int c = 0; c < q->ncomp; ++c) q->kdone[c] = q->k[c];
        q->first = false;
        if (q->ncomp == 1) {
            const mdr_refactored* r = S->fields[q->field[0]].r;
            q->c.bound = plan_bound(r, q->k[0]);
            q->c.met = q->c.bound <= q->tol_abs ? 1 : 0;
            q->c.bytes_fetched = new_bytes(r, q->kstart[0], q->k[0]);
            q->c.tol_abs = q->tol_abs;
            complete(S, q, MDR_OK);
            continue;
        }
        double worst;
        std::memcpy(&worst, static_cast<unsigned long long*>(S->acc_host) + slot_of[i], 8);
        const double tprime = worst * (1.0 + std::ldexp(1.0, -40));
        bool full = true;
        for (int c = 0; c < 3; ++c)
            for (uint32_t kl : q->k[c]) full = full && kl == S->fields[q->field[c]].r->B;
        if (tprime <= q->tol_abs || full) {
            q->c.bound = tprime;
            q->c.met = tprime <= q->tol_abs ? 1 : 0;
            q->c.tol_abs = q->tol_abs;
            q->c.bytes_fetched = 0;
            for (int c = 0; c < 3; ++c)
                q->c.bytes_fetched += new_bytes(S->fields[q->field[c]].r, q->kstart[c], q->k[c]);
            complete(S, q, MDR_OK);
            continue;
        }
        const double mape = q->q.mape_c > 0.0 ? q->q.mape_c : 10.0;
        const double p = q->tol_abs > 0.0 ? tprime / q->tol_abs : INFINITY;
        bool moved = false;
        if (p > mape) {
            for (int c = 0; c < 3; ++c) {
                std::vector<uint32_t> knew = q->k[c];
                plan_to(S->fields[q->field[c]].r, q->eps[c] / p, knew);
                moved = moved || knew != q->k[c];
                q->k[c] = knew;
            }
        }
        if (!moved)
            for (int c = 0; c < 3; ++c) plan_step(S->fields[q->field[c]].r, q->k[c]);
        keep.push_back(q);
    }
    act.swap(keep);
    return MDR_OK;
}

void engine_main(mdr_server* S)
{
    (void)hipSetDevice(S->ctx->device);
    for (;;) {
        std::vector<Req*> admit;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || !S->pending.empty() || !S->active.empty(); });
            if (S->stop) break;
            // admission: FIFO while a slot and the outputs' memory are free; a
            // request whose parent is still running waits without blocking others
            for (auto it = S->pending.begin(); it != S->pending.end();) {
                Req* q = *it;
                if (S->active.size() + admit.size() >= S->max_slots) break;
                if (q->q.parent && S->state.count(q->q.parent) && S->state[q->q.parent] != 2) {
                    ++it;
                    continue;
                }
                uint64_t need = 0;
                for (int c = 0; c < q->ncomp; ++c) need += block_bytes(S, q->field[c]);
                if (S->in_use + need > S->budget) break;
                S->in_use += need;
                q->need = need;
                S->state[q->ticket] = 1;
                admit.push_back(q);
                it = S->pending.erase(it);
            }
            if (admit.empty() && S->active.empty()) {
                // nothing runnable: wait for a release or a completion
                S->cv.wait_for(lk, std::chrono::milliseconds(1));
                continue;
            }
        }
        for (Req* q : admit) {
            mdr_status st = start(S, q);
            if (st) {
                q->c.status = st;
                complete(S, q, st);
            } else {
                S->active.push_back(q);
            }
        }
        if (S->active.empty()) continue;
        mdr_status st = step(S);
        if (st) {
            std::vector<Req*> act;
            act.swap(S->active);
            for (Req* q : act) complete(S, q, st);
        }
    }
}

}  // namespace

extern "C" {

mdr_status mdr_server_create(mdr_context* ctx, uint64_t hbm_budget, uint32_t max_slots, mdr_server** out)
{
    if (!out) return fail(MDR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(MDR_ERR_INVALID_ARG, "ctx is NULL");
    if (hbm_budget == 0 || max_slots == 0) return fail(MDR_ERR_INVALID_ARG, "budget and slots must be positive");
    auto* S = new mdr_server();
    mdr_status st = mdr_context_create(ctx->device, &S->ctx);
    if (st) {
        delete S;
        return st;
    }
    hipError_t e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        mdr_context_destroy(S->ctx);
        delete S;
        return hip_fail(e, "hipStreamCreate");
    }
    S->budget = hbm_budget;
    S->max_slots = max_slots;
    S->t0 = std::chrono::steady_clock::now();
    S->engine = std::thread(engine_main, S);
    *out = S;
    return MDR_OK;
}

mdr_status mdr_server_add_field(mdr_server* S, const mdr_refactored* r, uint32_t* field_id)
{
    if (!S || !r || !field_id) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    if (r->ctx->device != S->ctx->device) return fail(MDR_ERR_INVALID_ARG, "field lives on another device");
    mdr_retriever* cache = nullptr;
    mdr_status st = mdr_retriever_create(S->ctx, r, &cache);
    if (st) return st;
    Field f;
    f.r = r;
    f.cache = cache;
    for (const LevelRec& L : r->levels) f.out_bytes += align256(L.n * (r->dtype == MDR_F64 ? 8 : 4));
    f.range = value_range(r);
    double lo = 0.0, hi = 0.0;
    bool have = false;
    for (const LevelRec& L : r->levels) {
        if (L.n == 0) continue;
        if (!have || L.vmin < lo) lo = L.vmin;
        if (!have || L.vmax > hi) hi = L.vmax;
        have = true;
    }
    f.absmax = std::max(std::fabs(lo), std::fabs(hi));
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->active.empty() || !S->pending.empty())
        return fail(MDR_ERR_BUSY, "fields are added while the server is idle");
    *field_id = (uint32_t)S->fields.size();
    S->fields.push_back(f);
    return MDR_OK;
}

mdr_status mdr_server_submit(mdr_server* S, const mdr_request* rq, uint64_t* ticket)
{
    if (!S || !rq || !ticket) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    *ticket = 0;
    const int ncomp = rq->kind == MDR_REQ_QOI_VTOTAL ? 3 : 1;
    if (rq->kind != MDR_REQ_FIELD && rq->kind != MDR_REQ_QOI_VTOTAL) return fail(MDR_ERR_INVALID_ARG, "bad request kind");
    if (rq->bound != MDR_ABS && rq->bound != MDR_REL) return fail(MDR_ERR_INVALID_ARG, "bad bound kind");
    if (!(rq->tol >= 0.0) || std::isinf(rq->tol)) return fail(MDR_ERR_INVALID_ARG, "tolerance must be finite and >= 0");
    std::lock_guard<std::mutex> lk(S->mu);
    for (int c = 0; c < ncomp; ++c)
        if (rq->field[c] >= S->fields.size()) return fail(MDR_ERR_INVALID_ARG, "no such field");
    if (ncomp == 3) {
        const mdr_refactored* a = S->fields[rq->field[0]].r;
        for (int c = 1; c < 3; ++c) {
            const mdr_refactored* b = S->fields[rq->field[c]].r;
            if (b->dtype != a->dtype || b->levels.size() != a->levels.size())
                return fail(MDR_ERR_INVALID_ARG, "QoI fields must share dtype and levels");
            for (size_t l = 0; l < a->levels.size(); ++l)
                if (a->levels[l].n != b->levels[l].n)
                    return fail(MDR_ERR_INVALID_ARG, "QoI fields must hold the same points per level");
        }
    }
    uint64_t need = 0;
    for (int c = 0; c < ncomp; ++c) need += block_bytes(S, rq->field[c]);
    if (need > S->budget) return fail(MDR_ERR_INVALID_ARG, "the request's outputs exceed the HBM budget");
    if (rq->parent && !S->state.count(rq->parent)) return fail(MDR_ERR_INVALID_ARG, "unknown parent ticket");
    auto* q = new Req();
    q->ticket = S->next_ticket++;
    q->q = *rq;
    q->ncomp = ncomp;
    for (int c = 0; c < ncomp; ++c) q->field[c] = rq->field[c];
    q->c.t_submit_ms = now_ms(S->t0);
    S->state[q->ticket] = 0;
    S->pending.push_back(q);
    *ticket = q->ticket;
    S->cv.notify_all();
    return MDR_OK;
}

mdr_status mdr_server_poll(mdr_server* S, mdr_completion* out, uint32_t cap, uint32_t* n)
{
    if (!S || !n || (cap && !out)) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    uint32_t k = 0;
    while (k < cap && !S->completions.empty()) {
        out[k++] = S->completions.front();
        S->completions.pop_front();
    }
    *n = k;
    return MDR_OK;
}

mdr_status mdr_server_output(mdr_server* S, uint64_t ticket, uint32_t comp, uint32_t level, void** dev_ptr,
                             uint64_t* n)
{
    if (!S || !dev_ptr) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->done.find(ticket);
    if (it == S->done.end()) return fail(MDR_ERR_INVALID_ARG, "no completed, unreleased request with this ticket");
    Req* q = it->second;
    if ((int)comp >= q->ncomp || level >= q->outp[comp].size()) return fail(MDR_ERR_INVALID_ARG, "no such output");
    *dev_ptr = q->outp[comp][level];
    if (n) *n = S->fields[q->field[comp]].r->levels[level].n;
    return MDR_OK;
}

mdr_status mdr_server_release(mdr_server* S, uint64_t ticket)
{
    if (!S) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->done.find(ticket);
    if (it == S->done.end()) return fail(MDR_ERR_INVALID_ARG, "no completed, unreleased request with this ticket");
    Req* q = it->second;
    S->in_use -= q->need;
    keep_blocks(S, q);
    delete q;
    S->done.erase(it);
    S->cv.notify_all();
    return MDR_OK;
}

mdr_status mdr_server_stats(mdr_server* S, mdr_server_info* info)
{
    if (!S || !info) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    info->pending = (uint32_t)S->pending.size();
    info->active = (uint32_t)S->active.size();
    info->completed_unreleased = (uint32_t)S->done.size();
    info->steps = S->steps;
    info->step_requests = S->step_requests;
    info->hbm_in_use = S->in_use;
    info->hbm_budget = S->budget;
    info->hbm_held = S->held;
    return MDR_OK;
}

void mdr_server_destroy(mdr_server* S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->engine.joinable()) S->engine.join();
    (void)hipSetDevice(S->ctx->device);
    (void)hipStreamSynchronize(S->stream);
    for (Req* q : S->pending) delete q;
    for (Req* q : S->active) {
        keep_blocks(S, q);
        delete q;
    }
    for (auto& kv : S->done) {
        keep_blocks(S, kv.second);
        delete kv.second;
    }
    for (auto& kv : S->spare) (void)hipFree(kv.second);
    for (Field& f : S->fields) mdr_retriever_destroy(f.cache);
    if (S->acc_host) (void)hipHostFree(S->acc_host);
    S->acc.reset();
    (void)hipStreamDestroy(S->stream);
    mdr_context_destroy(S->ctx);
    delete S;
}

}  // extern "C"
