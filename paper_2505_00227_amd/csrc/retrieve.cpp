// Batched progressive retrieval (the inverse of Alg. 1 and Alg. 2): for any
// number of retrievers at once, decode the lossless groups that enter each
// one's plan (one Huffman launch for all of them), then rebuild every level of
// every variable from its sign plane and first k magnitude planes (one launch
// per dtype).  Plans are made on the host from the exact error tables.
#include <algorithm>
#include <cstring>
#include <string>

#include "api_internal.hpp"

namespace mdr {

namespace {

// A descriptor slot: pinned host staging plus its device copy, whose host
// buffer holds `bytes` and whose device buffer holds `dev_bytes` (>= bytes:
// device-only scratch follows the descriptor).  A slot is reused only after
// the event recorded behind the kernels that read it.
// Grow a slot that no launch still reads to the ring's high-water sizes.
static mdr_status grow_slot(mdr_context* ctx, DescSlot& d)
{
    if (d.bytes < ctx->ring_hw_host) {
        const uint64_t want = std::max<uint64_t>(ctx->ring_hw_host + ctx->ring_hw_host / 2, 64 << 10);
        if (d.host) (void)hipHostFree(d.host);
        d.host = nullptr;
        d.bytes = 0;
        hipError_t e = hipHostMalloc(&d.host, want, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "hipHostMalloc(descriptor)");
        // touch every page now: the first writes to fresh pinned pages fault
        // one page at a time (about 0.3 ms for a retrieval's tables)
        std::memset(d.host, 0, want);
        d.bytes = want;
    }
    if (d.dev_bytes < ctx->ring_hw_dev) {
        const uint64_t want = std::max<uint64_t>(ctx->ring_hw_dev + ctx->ring_hw_dev / 2, 64 << 10);
        d.dev_bytes = 0;
        hipError_t e = d.dev.alloc(want);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(descriptor)");
        d.dev_bytes = want;
    }
    return MDR_OK;
}

DescSlot* acquire_slot(mdr_context* ctx, uint64_t bytes, uint64_t dev_bytes, mdr_status& st)
{
    dev_bytes = std::max(dev_bytes, bytes);
    // Calls of different kinds (a refactor's tables, a retrieval's with its
    // decode-table scratch) take turns on the ring, so a slot sized for one
    // kind meets the other a few calls later.  Every slot is therefore sized
    // to the largest request seen so far, and a new largest one grows the idle
    // slots too, at once: otherwise the calls after the first would each pay a
    // pinned and a device reallocation.
    const bool larger = bytes > ctx->ring_hw_host || dev_bytes > ctx->ring_hw_dev;
    ctx->ring_hw_host = std::max(ctx->ring_hw_host, bytes);
    ctx->ring_hw_dev = std::max(ctx->ring_hw_dev, dev_bytes);
    DescSlot& d = ctx->ring[ctx->ring_next++ % kDescSlots];
    st = MDR_OK;
    if (d.pending) {
        hipError_t e = hipEventSynchronize(d.done);
        if (e != hipSuccess) {
            st = hip_fail(e, "hipEventSynchronize(descriptor slot)");
            return nullptr;
        }
        d.pending = false;
    }
    if (!d.done) {
        hipError_t e = hipEventCreateWithFlags(&d.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            st = hip_fail(e, "hipEventCreate");
            return nullptr;
        }
    }
    if ((st = grow_slot(ctx, d)) != MDR_OK) return nullptr;
    if (larger)
        for (DescSlot& o : ctx->ring) {
            if (&o == &d) continue;
            if (o.pending) {
                const hipError_t q = hipEventQuery(o.done);
                (void)hipGetLastError();  // a not-ready answer must not reach the launch checks
                if (q != hipSuccess) continue;  // still read: grown on its next turn
                o.pending = false;
            }
            if ((st = grow_slot(ctx, o)) != MDR_OK) return nullptr;
        }
    return &d;
}

struct Fresh {
    size_t task;
    uint32_t level, slot;
    PoolBuf buf;
};

}  // namespace

DescSlot::~DescSlot()
{
    if (done) (void)hipEventDestroy(done);
    if (host) (void)hipHostFree(host);
}

mdr_status retrieve_many(mdr_context* ctx, RetrieveTask* tasks, size_t ntasks, hipStream_t s,
                         const ReconOnly* extra, size_t nextra)
{
    (void)hipGetLastError();  // as in enqueue_pass: only this call's launches are checked
    MDR_HIP(hipSetDevice(ctx->device));
    for (size_t t = 0; t < ntasks; ++t) {
        const mdr_refactored* r = tasks[t].rt->r;
        for (size_t u = 0; u < t; ++u)
            if (tasks[u].rt == tasks[t].rt) return fail(MDR_ERR_INVALID_ARG, "a retriever appears twice in one batch");
        if (tasks[t].rt->ctx->device != ctx->device)
            return fail(MDR_ERR_INVALID_ARG, "retrievers on different devices");
        if (tasks[t].reconstruct) {  // decode-only tasks have no outputs
            if (!tasks[t].out) return fail(MDR_ERR_INVALID_ARG, "level_out is NULL");
            for (size_t l = 0; l < r->levels.size(); ++l)
                if (r->levels[l].n && !tasks[t].out[l])
                    return fail(MDR_ERR_INVALID_ARG, "level_out[" + std::to_string(l) + "] is NULL");
        }
    }
    for (size_t i = 0; i < nextra; ++i) {
        if (!extra[i].rt || !extra[i].out || extra[i].k.size() != extra[i].rt->r->levels.size())
            return fail(MDR_ERR_INVALID_ARG, "bad reconstruction request");
        for (size_t l = 0; l < extra[i].k.size(); ++l)
            if (extra[i].rt->r->levels[l].n && !extra[i].out[l])
                return fail(MDR_ERR_INVALID_ARG, "level_out[" + std::to_string(l) + "] is NULL");
    }

    // groups entering each plan; state is committed only at the end
    std::vector<Fresh> fresh;
    std::vector<DecodeJob> dec;
    std::vector<RleJob> rle;
    uint64_t rle_runs = 0;
    std::vector<uint64_t> fetched(ntasks, 0);
    std::vector<uint32_t> groups(ntasks, 0);
    struct SyncOnFail {
        hipStream_t s;
        bool armed = true;
        ~SyncOnFail()
        {
            if (armed) (void)hipStreamSynchronize(s);
        }
    } sync_on_fail{s};
    for (size_t t = 0; t < ntasks; ++t) {
        mdr_retriever* rt = tasks[t].rt;
        const mdr_refactored* r = rt->r;
        const uint32_t B = r->B, m = r->m, G = r->G;
        for (uint32_t l = 0; l < r->levels.size(); ++l) {
            const LevelRec& LR = r->levels[l];
            const uint32_t k0 = rt->k[l], k1 = tasks[t].knew[l];
            for (uint32_t slot = 0; slot <= B; slot = slot == 0 ? 1 : slot + m) {
                const bool before = slot == 0 ? k0 > 0 : (slot - 1) < k0;
                const bool now = slot == 0 ? k1 > 0 : (slot - 1) < k1;
                if (!now || before) continue;
                const UnitRec& ur = LR.units[slot];
                fetched[t] += ur.bytes;
                ++groups[t];
                if (ur.method == MDR_DC || LR.n == 0) continue;
                Fresh f{t, l, slot, PoolBuf()};
                hipError_t e = f.buf.alloc(rt->ctx->pool, std::max<uint64_t>(ur.S, 4));
                if (e != hipSuccess) return hip_fail(e, "hipMalloc(decoded group)");
                if (ur.method == MDR_HUF) {
                    DecodeJob dj{};
                    dj.payload = ur.dev;
                    dj.out = static_cast<uint8_t*>(f.buf.p);
                    dj.S = ur.S;
                    dj.nchunks = ur.nchunks;
                    dj.chunk = r->prm.huf_chunk;
                    dj.lmax = r->prm.huf_lmax;
                    dec.push_back(dj);
                } else if (ur.method == MDR_RLE) {
                    RleJob rj{};
                    rj.payload = ur.dev;
                    rj.out = static_cast<uint8_t*>(f.buf.p);
                    rj.nwords = ur.S / 4 / G;
                    rj.nruns = ur.nruns;
                    rj.G = G;
                    if (rj.nwords >= (1ull << 32)) return fail(MDR_ERR_UNSUPPORTED, "run-length group of 2^32 words");
                    if (rj.nwords && rj.nruns) {
                        rj.run_base = rle_runs;
                        rle_runs += rj.nruns;
                        rle.push_back(rj);
                    }
                } else {
                    return fail(MDR_ERR_CORRUPT_STREAM, "unknown lossless method");
                }
                fresh.push_back(std::move(f));
            }
        }
    }

    // reconstruction jobs, one list per dtype
    std::vector<std::vector<const uint8_t*>> fsrc(ntasks);
    for (size_t t = 0; t < ntasks; ++t) fsrc[t].assign(tasks[t].rt->r->levels.size() * kMaxRows, nullptr);
    for (const Fresh& f : fresh) fsrc[f.task][(size_t)f.level * kMaxRows + f.slot] = static_cast<const uint8_t*>(f.buf.p);
    std::vector<ReconJob> rj[2];
    // t: the task whose fresh groups apply (ntasks: none)
    auto add_jobs = [&](size_t t, const mdr_retriever* rt, const std::vector<uint32_t>& k,
                        const std::vector<uint32_t>* kprev, void* const* out) {
        const mdr_refactored* r = rt->r;
        const uint32_t B = r->B, m = r->m;
        for (uint32_t l = 0; l < r->levels.size(); ++l) {
            const LevelRec& LR = r->levels[l];
            if (LR.n == 0) continue;
            if (kprev && k[l] == (*kprev)[l]) continue;  // output already holds these planes
            ReconJob job{};
            job.out = out[l];
            job.n = LR.n;
            job.nbd = LR.nbd;
            job.B = B;
            job.k = k[l];
            job.e = LR.e;
            job.vec = ((uintptr_t)job.out % 16) == 0 ? 1u : 0u;
            if (job.k > 0) {
                for (uint32_t row = 0; row <= B; ++row) {
                    if (row > 0 && row - 1 >= job.k) break;
                    const uint32_t slot = row == 0 ? 0 : 1 + ((row - 1) / m) * m;
                    uint32_t r0, r1;
                    slot_rows(slot, B, m, r0, r1);
                    const uint8_t* src = nullptr;
                    if (t < ntasks) src = fsrc[t][(size_t)l * kMaxRows + slot];
                    if (!src) src = static_cast<const uint8_t*>(rt->dec[l][slot].p);
                    if (!src) src = r->levels[l].units[slot].dev;  // direct copy: the payload is the plane rows
                    job.rows[row] = reinterpret_cast<const uint32_t*>(src) + (uint64_t)(row - r0) * LR.nbd;
                }
            }
            rj[r->dtype == MDR_F64 ? 1 : 0].push_back(job);
        }
    };
    for (size_t t = 0; t < ntasks; ++t)
        if (tasks[t].reconstruct)
            add_jobs(t, tasks[t].rt, tasks[t].knew, tasks[t].all_levels ? nullptr : &tasks[t].rt->k, tasks[t].out);
    for (size_t i = 0; i < nextra; ++i) {
        size_t t = ntasks;
        for (size_t u = 0; u < ntasks; ++u)
            if (tasks[u].rt == extra[i].rt) t = u;
        const std::vector<uint32_t>& held = t < ntasks ? tasks[t].knew : extra[i].rt->k;
        for (size_t l = 0; l < held.size(); ++l)
            if (extra[i].k[l] > held[l]) return fail(MDR_ERR_INVALID_ARG, "reconstruction beyond the planes held");
        add_jobs(t, extra[i].rt, extra[i].k, extra[i].kprev, extra[i].out);
    }

    // descriptor: decode jobs, reconstruction jobs, workgroup maps
    std::vector<uint32_t> map_dec, map_r[2];
    uint64_t dec_chunks = 0;
    uint32_t dec_chunk_max = 0;
    for (const DecodeJob& d : dec) {
        dec_chunks += d.nchunks;
        dec_chunk_max = std::max(dec_chunk_max, d.chunk);
    }
    std::vector<uint32_t> map_rg, map_re;
    for (uint32_t i = 0; i < rle.size(); ++i) {
        rle[i].wg_gather = (uint32_t)map_rg.size();
        map_rg.insert(map_rg.end(), (rle[i].nruns + kRlePerWg - 1) / kRlePerWg, i);
        rle[i].wg_expand = (uint32_t)map_re.size();
        map_re.insert(map_re.end(), (rle[i].nwords + kRlePerWg - 1) / kRlePerWg, i);
    }
    const uint32_t lanes = huf_decode_lanes(ctx->decode_lanes, dec_chunks, dec_chunk_max);
    const uint32_t cpw = kThreads / lanes;
    for (uint32_t i = 0; i < dec.size(); ++i) {
        dec[i].wg_base = (uint32_t)map_dec.size();
        map_dec.insert(map_dec.end(), (dec[i].nchunks + cpw - 1) / cpw, i);
    }
    for (int d = 0; d < 2; ++d)
        for (uint32_t i = 0; i < rj[d].size(); ++i) {
            rj[d][i].wg_base = (uint32_t)map_r[d].size();
            map_r[d].insert(map_r[d].end(), (rj[d][i].nbd + kThreads - 1) / kThreads, i);
        }
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o += align256(bytes);
        return at;
    };
    const uint64_t o_dec = take(sizeof(DecodeJob) * dec.size());
    const uint64_t o_r0 = take(sizeof(ReconJob) * rj[0].size());
    const uint64_t o_r1 = take(sizeof(ReconJob) * rj[1].size());
    const uint64_t o_md = take(4 * map_dec.size());
    const uint64_t o_m0 = take(4 * map_r[0].size());
    const uint64_t o_m1 = take(4 * map_r[1].size());
    const uint64_t o_rle = take(sizeof(RleJob) * rle.size());
    const uint64_t o_mrg = take(4 * map_rg.size());
    const uint64_t o_mre = take(4 * map_re.size());
    if (o) {
        // after the descriptor, on the device only (never copied): the decode
        // tables, then the run lengths, run starts and scan scratch
        const uint64_t o_tab = o, tab_bytes = kHufTableBytes * dec.size();
        const uint64_t o_lens = o_tab + tab_bytes, o_starts = o_lens + align256(4 * rle_runs);
        const uint64_t o_stemp = o_starts + align256(4 * rle_runs);
        const uint64_t dev_bytes = rle_runs ? o_stemp + 4 * scan_temp_words(rle_runs) : o_lens;
        mdr_status st;
        DescSlot* slot = acquire_slot(ctx, o, dev_bytes, st);
        if (!slot) return st;
        uint8_t* h = static_cast<uint8_t*>(slot->host);
        uint8_t* dv = static_cast<uint8_t*>(slot->dev.p);
        for (size_t i = 0; i < dec.size(); ++i) dec[i].table = dv + o_tab + kHufTableBytes * i;
        auto put = [&](uint64_t at, const void* src, uint64_t bytes) {
            if (bytes) std::memcpy(h + at, src, bytes);
        };
        put(o_dec, dec.data(), sizeof(DecodeJob) * dec.size());
        put(o_r0, rj[0].data(), sizeof(ReconJob) * rj[0].size());
        put(o_r1, rj[1].data(), sizeof(ReconJob) * rj[1].size());
        put(o_md, map_dec.data(), 4 * map_dec.size());
        put(o_m0, map_r[0].data(), 4 * map_r[0].size());
        put(o_m1, map_r[1].data(), 4 * map_r[1].size());
        put(o_rle, rle.data(), sizeof(RleJob) * rle.size());
        put(o_mrg, map_rg.data(), 4 * map_rg.size());
        put(o_mre, map_re.data(), 4 * map_re.size());
        MDR_HIP(launch_copy_in(dv, h, o, s));
        if (!rle.empty()) {
            StageTimer tm(ctx, MDR_STAGE_RLE_DECODE, s);
            MDR_HIP(launch_rle_decode_batch(reinterpret_cast<const RleJob*>(dv + o_rle),
                                            reinterpret_cast<const uint32_t*>(dv + o_mrg), (uint32_t)map_rg.size(),
                                            reinterpret_cast<const uint32_t*>(dv + o_mre), (uint32_t)map_re.size(),
                                            rle_runs, reinterpret_cast<uint32_t*>(dv + o_lens),
                                            reinterpret_cast<uint32_t*>(dv + o_starts),
                                            reinterpret_cast<uint32_t*>(dv + o_stemp), s));
        }
        if (!map_dec.empty()) {
            StageTimer tm(ctx, MDR_STAGE_HUF_DECODE, s);
            MDR_HIP(launch_huf_decode_batch(reinterpret_cast<const DecodeJob*>(dv + o_dec), (uint32_t)dec.size(),
                                            reinterpret_cast<const uint32_t*>(dv + o_md),
                                            (uint32_t)map_dec.size(), lanes, dec_chunk_max, s));
        }
        for (int d = 0; d < 2; ++d) {
            if (map_r[d].empty()) continue;
            // streaming loads and stores when the launch reads at least half of its planes
            uint64_t held = 0, all = 0;
            for (const ReconJob& j : rj[d]) {
                held += (uint64_t)j.k * j.nbd;
                all += (uint64_t)j.B * j.nbd;
            }
            StageTimer tm(ctx, MDR_STAGE_RECONSTRUCT, s);
            MDR_HIP(launch_reconstruct_batch(reinterpret_cast<const ReconJob*>(dv + (d ? o_r1 : o_r0)),
                                             reinterpret_cast<const uint32_t*>(dv + (d ? o_m1 : o_m0)),
                                             (uint32_t)map_r[d].size(), d == 1, 2 * held >= all, s));
        }
        MDR_HIP(hipEventRecord(slot->done, s));
        slot->pending = true;
    }

    // commit
    sync_on_fail.armed = false;
    for (Fresh& f : fresh) tasks[f.task].rt->dec[f.level][f.slot] = std::move(f.buf);
    for (size_t t = 0; t < ntasks; ++t) {
        mdr_retriever* rt = tasks[t].rt;
        rt->k = tasks[t].knew;
        rt->bytes_held += fetched[t];
        if (mdr_retrieve_info* info = tasks[t].info) {
            info->tol_abs = tasks[t].tol_abs;
            info->bound = plan_bound(rt->r, rt->k);
            info->bytes_fetched = fetched[t];
            info->bytes_held = rt->bytes_held;
            info->groups_fetched = groups[t];
            info->met = info->bound <= tasks[t].tol_abs ? 1 : 0;
        }
    }
    return MDR_OK;
}

mdr_status enqueue_qoi(mdr_context* ctx, const std::vector<QoiJob>& jobs, const std::vector<bool>& f64,
                       unsigned long long* acc0, uint32_t nacc, hipStream_t s, bool argmax)
{
    (void)hipGetLastError();
    MDR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(acc0), 2ull * nacc, 0u, s));
    if (argmax) MDR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(acc0 + nacc), 2ull * nacc, ~0u, s));
    std::vector<QoiJob> js[2];
    std::vector<uint32_t> maps[2];
    for (size_t i = 0; i < jobs.size(); ++i) {
        if (jobs[i].n == 0) continue;
        const int d = f64[i] ? 1 : 0;
        QoiJob j = jobs[i];
        const auto a16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
        j.vec = a16(j.x) && a16(j.y) && a16(j.z) ? 1u : 0u;
        j.grid = (uint32_t)std::min<uint64_t>(1024, (j.n + kThreads * 8 - 1) / (kThreads * 8));
        j.wg_base = (uint32_t)maps[d].size();
        maps[d].insert(maps[d].end(), j.grid, (uint32_t)js[d].size());
        js[d].push_back(j);
    }
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o += align256(bytes);
        return at;
    };
    const uint64_t oj[2] = {take(sizeof(QoiJob) * js[0].size()), take(sizeof(QoiJob) * js[1].size())};
    const uint64_t om[2] = {take(4 * maps[0].size()), take(4 * maps[1].size())};
    if (!o) return MDR_OK;
    mdr_status st;
    DescSlot* slot = acquire_slot(ctx, o, o, st);
    if (!slot) return st;
    uint8_t* h = static_cast<uint8_t*>(slot->host);
    uint8_t* dv = static_cast<uint8_t*>(slot->dev.p);
    for (int d = 0; d < 2; ++d) {
        if (!js[d].empty()) std::memcpy(h + oj[d], js[d].data(), sizeof(QoiJob) * js[d].size());
        if (!maps[d].empty()) std::memcpy(h + om[d], maps[d].data(), 4 * maps[d].size());
    }
    MDR_HIP(launch_copy_in(dv, h, o, s));
    for (int d = 0; d < 2; ++d)
        MDR_HIP(launch_qoi_vtotal_batch(reinterpret_cast<const QoiJob*>(dv + oj[d]),
                                        reinterpret_cast<const uint32_t*>(dv + om[d]), (uint32_t)maps[d].size(),
                                        d == 1, s));
    if (argmax)
        for (int d = 0; d < 2; ++d)
            MDR_HIP(launch_qoi_vtotal_argmax_batch(reinterpret_cast<const QoiJob*>(dv + oj[d]),
                                                   reinterpret_cast<const uint32_t*>(dv + om[d]),
                                                   (uint32_t)maps[d].size(), d == 1, s));
    MDR_HIP(hipEventRecord(slot->done, s));
    slot->pending = true;
    return MDR_OK;
}

}  // namespace mdr
