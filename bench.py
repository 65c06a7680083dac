"""Benchmark of the refactor / progressive-retrieve hot path on one MI355X.

Default workload: the 1024^3 float64 field (8 GiB) as 32 slabs of
32x1024x1024 values, each its own 9-level sub-domain, 64 planes, groups of 4
planes, resident in HBM before the timed region.  One step = one batched
refactor pass over the 32 slabs + one batched retrieval of every plane of the
32 slabs, each writing the full reconstruction.  Prints one JSON line; the
host-to-host chunked pipeline, per-slab retrieval latencies (cold), and short
runs of the 512^3 float32 field, the 256-variable batch and the serving loop
ride along as extra keys.

value = original bytes moved through the path per second: the field once for
refactor plus once for the retrieval (the paper's GB/s-of-original-data
convention).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2505_00227_amd", "csrc")
# kernel -> the source file it is built from (a traffic figure is valid only
# for the source it was measured on)
KERNEL_SRC = {"k_encode": "k_refactor.hip", "k_stats": "k_refactor.hip", "k_select": "k_refactor.hip",
              "k_reconstruct": "k_retrieve.hip", "k_huf_decode": "k_lossless.hip",
              "lossless": "k_lossless.hip"}
# stage timed by the library -> kernel it launches
STAGE_KERNEL = {"encode": "k_encode", "stats": "k_stats", "select": "k_select",
                "reconstruct": "k_reconstruct", "huf_decode": "k_huf_decode", "lossless": "lossless"}


def source_hash(kernel: str) -> str:
    import hashlib
    return hashlib.sha256(open(os.path.join(CSRC, KERNEL_SRC[kernel]), "rb").read()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter runs (profiles/<kernel>_<workload>_traffic.md: FETCH_SIZE
    and WRITE_SIZE, each scaled by the same counter on a plain copy of known
    size), or None when the kernel's source changed since they were taken."""
    note = os.path.join(ROOT, "profiles", "%s_%s_traffic.md" % (kernel, workload))
    try:
        vals = {}
        for line in open(note):
            if line.startswith("machine: "):
                for kv in line[len("machine: "):].split():
                    k, v = kv.split("=")
                    vals[k] = v
        if vals.get("source_sha") != source_hash(kernel):
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 4, 5],
                    help="3 (default): the 1024^3 float64 field resident in HBM; --pipeline: host to host")
    ap.add_argument("--pipeline", action="store_true",
                    help="the 1024^3 float64 field through the chunked host-to-host pipeline only")
    ap.add_argument("--chunks", type=int, default=32, help="chunked workload: 32x1024x1024 f64 slabs")
    ap.add_argument("--serve-requests", type=int, default=10000, help="serving workload: requests per load")
    ap.add_argument("--serve-edge", type=int, default=512, help="serving workload: field edge")
    ap.add_argument("--serve-loads", type=str, default="0.5,0.9,2.0",
                    help="serving workload: offered loads (x measured sequential capacity)")
    ap.add_argument("--batch-vars", type=int, default=256, help="variables of the batched workload")
    ap.add_argument("--no-tune", action="store_true", help="batched workload: skip the launch-shape sweep")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--multilevel", action="store_true",
                    help="multilevel decomposition of the 512^3 field, and the field through the whole path")
    ap.add_argument("--ablation", action="store_true",
                    help="encoder-design ablation: 32-bit words <-> 32 planes by each design, 2^20..2^28 words")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: leave out the short runs of the other workloads")
    ap.add_argument("--no-qoi-estimators", dest="qoi_estimators", action="store_false",
                    help="serving workload: skip the estimator comparison")
    ap.add_argument("--cpu-sample", type=int, default=1 << 25,
                    help="values of the finest level the oracle baseline refactors")
    return ap.parse_args()


def workload(cfg: int):
    import numpy as np
    import workloads
    if cfg == 1:
        levels = [workloads.plain_level(seed=1, n=1 << 20)]
        return {"name": "plain-2^20-f32-laplace", "levels": levels, "B": 32, "m": 1,
                "tols": [1e-1, 1e-3, 1e-6]}
    levels = workloads.field_levels(seed=2, edge=512, nlevels=9, dtype=np.float32)
    return {"name": "field-512^3-f32-9-levels", "levels": levels, "B": 32, "m": 4,
            "tols": [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6]}


def cpu_baseline(w, sample: int):
    """The oracle as it stands, on the host cores, over a bounded sample: the
    finest level truncated to `sample` values, refactored then retrieved to each
    bound.  Returns GB/s of original data on the same convention as `value`."""
    import oracle
    x = w["levels"][-1][:sample]
    p = oracle.Params(group_planes=w["m"])
    t0 = time.perf_counter()
    lv = oracle.refactor([x], w["B"], p)
    k = None
    for tol in w["tols"]:
        vals, k, bound, met = oracle.retrieve_to(lv, tol, k_in=k)
    t = time.perf_counter() - t0
    nbytes = x.nbytes * (1 + len(w["tols"]))
    cores = oracle.get_threads()
    # the same work on one thread, over a quarter of the sample
    x1 = x[: max(1, x.size // 4)]
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        lv = oracle.refactor([x1], w["B"], p)
        k = None
        for tol in w["tols"]:
            vals, k, bound, met = oracle.retrieve_to(lv, tol, k_in=k)
        t1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(cores)
    return {"value": nbytes / t / 1e9, "unit": "GB/s", "cores": cores,
            "kind": "oracle", "seconds": t,
            "single_thread_value": x1.nbytes * (1 + len(w["tols"])) / t1 / 1e9,
            "sample": "first %d values of the finest level (%.1f MiB): refactor + %d "
                      "incremental retrievals (single thread: first %d values)"
                      % (x.size, x.nbytes / 2 ** 20, len(w["tols"]), x1.size)}


def progress(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def bench_batched(args):
    """256 variables of uneven size (cube edge ~ U{16..256}, 5 Laplace levels,
    f32): refactor every variable in one batched pass (a replayed HIP graph) and
    retrieve all of them (every plane, then relative 1e-3) in one batched call,
    against the same work done one variable at a time (mdr_refactor /
    mdr_retrieve per variable) at identical bounds."""
    import numpy as np
    import torch

    import paper_2505_00227_amd as mdr
    import workloads

    B = 32
    edges, vs = workloads.batch_variables(seed=4, nvars=args.batch_vars, nlevels=5, lo=16, hi=256,
                                          dtype=np.float32)
    progress("generated", len(vs), "variables")
    nvals = sum(a.size for v in vs for a in v)
    nbytes = 4 * nvals
    dev = [[torch.from_numpy(a).cuda() for a in v] for v in vs]
    outs = [[torch.empty_like(t) for t in v] for v in dev]
    del vs
    ctx = mdr.Context(0)
    params = mdr.default_params(group_planes=4)
    tols = [0.0, 1e-3]  # 0 = every plane (relative bound 0 is met only by all planes)
    dev_views, out_ptrs = mdr.BatchViews(dev), mdr.BatchOutputs(outs)  # marshalled once
    torch.cuda.synchronize()

    def batched_step(times):
        t0 = time.perf_counter()
        rs = mdr.refactor_batch(ctx, dev_views, B, params)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tr = []
        for tol in tols:  # each bound from a fresh retriever
            rts = [mdr.Retriever(ctx, r) for r in rs]
            ta = time.perf_counter()
            mdr.retrieve_batch(rts, [tol] * len(rts), out_ptrs)
            torch.cuda.synchronize()
            tr.append(time.perf_counter() - ta)
            for rt in rts:
                rt.close()
        times.append((t1 - t0, tr))
        for r in rs:
            r.close()

    def single_step(times):
        t0 = time.perf_counter()
        rs = [mdr.refactor(ctx, v, B, params) for v in dev]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tr = []
        for tol in tols:
            rts = [mdr.Retriever(ctx, r) for r in rs]
            ta = time.perf_counter()
            for rt, o in zip(rts, outs):
                rt.retrieve(tol, o)
            torch.cuda.synchronize()
            tr.append(time.perf_counter() - ta)
            for rt in rts:
                rt.close()
        times.append((t1 - t0, tr))
        for r in rs:
            r.close()

    tune = None
    if not args.no_tune:
        # the library's autotuner times candidate launch shapes of this batch's
        # pass and records the fastest for its key; later passes of the same
        # shape run at it (results are identical for every shape)
        tune = ctx.autotune(dev, B, params, reps=2, force=True)
        tune["table"] = ctx.tune_table()
        progress("tune", tune)
    for _ in range(args.warmup):
        batched_step([])
        single_step([])
    bt, st = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batched_step(bt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for _ in range(args.steps):
        single_step(st)

    def summary(times):
        ref = statistics.median(x[0] for x in times)
        ret = [statistics.median(x[1][i] for x in times) for i in range(len(tols))]
        return {"refactor_ms": ref * 1e3, "refactor_gbps": nbytes / ref / 1e9,
                "retrieve_ms": {("all" if t == 0 else "%.0e" % t): r * 1e3 for t, r in zip(tols, ret)},
                "retrieve_gbps": {("all" if t == 0 else "%.0e" % t): nbytes / r / 1e9 for t, r in zip(tols, ret)},
                "step_ms": (ref + sum(ret)) * 1e3}
    sb, ss = summary(bt), summary(st)
    moved = nbytes * (1 + len(tols))
    res = {
        "metric": "refactor & retrieve GB/s (frac of HBM peak); p50/p99 retrieval latency",
        "value": moved / (elapsed / args.steps) / 1e9,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch-%d-vars-edge16..256-f32-5-levels" % len(dev), "values": nvals,
                   "nplanes": B, "group_planes": 4, "bounds_rel": ["all planes", 1e-3],
                   "parallelism": "single-gpu"},
        "batched": sb,
        "per_variable": ss,
        "speedup_batched_vs_per_variable": ss["step_ms"] / sb["step_ms"],
        "tune": tune,
        "tuned_gain_vs_default": (tune["default_ms"] / tune["best_ms"]) if tune else None,
    }
    return res


def bench_chunked(args):
    """1024^3 float64 field (8 GiB) in pinned host memory as 32 slabs of
    32x1024x1024 values, each its own 9-level sub-domain, 64 planes: end-to-end
    refactor (H2D / refactor / D2H overlapped on three streams) and
    full-precision retrieval back to host memory, against the same work one
    stage at a time."""
    import numpy as np
    import torch

    import paper_2505_00227_amd as mdr
    import workloads

    sizes = workloads.chunk_level_sizes()
    per = sum(sizes)
    n = args.chunks
    host = torch.empty(per * n, dtype=torch.float64).pin_memory()
    hv = host.numpy()
    for c in range(n):
        hv[c * per:(c + 1) * per] = np.concatenate(workloads.chunk_levels(seed=3, chunk=c))
    progress("generated", n, "chunks")
    out = torch.empty_like(host).pin_memory()
    ctx = mdr.Context(0)
    pipe = mdr.Pipeline(ctx, n, sizes, torch.float64, 64, mdr.default_params(group_planes=4))
    nbytes = host.numel() * 8
    runs = {}
    for name, fn in (("refactor", lambda ov: pipe.refactor(host, overlap=ov)),
                     ("retrieve_all", lambda ov: pipe.retrieve(0.0, out, overlap=ov))):
        for ov in (True, False):
            fn(ov)  # warm: graphs, pinned staging, pools
            best = None
            for _ in range(max(1, args.steps)):
                info = fn(ov)
                if best is None or info["wall_ms"] < best["wall_ms"]:
                    best = info
            best["gbps"] = nbytes / (best["wall_ms"] / 1e3) / 1e9
            best["kernel_gbps"] = nbytes / (best["compute_ms"] / 1e3) / 1e9 if best["compute_ms"] else None
            runs["%s_%s" % (name, "pipelined" if ov else "serial")] = best
            progress(name, "overlap" if ov else "serial", best)
    e2e = (runs["refactor_pipelined"]["wall_ms"] + runs["retrieve_all_pipelined"]["wall_ms"]) / 1e3
    res = {
        "metric": "refactor & retrieve GB/s (frac of HBM peak); p50/p99 retrieval latency",
        "value": 2 * nbytes / e2e / 1e9,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": e2e * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "chunked-1024^3-f64-%d-slabs-9-levels" % n, "values": host.numel(),
                   "nplanes": 64, "group_planes": 4, "parallelism": "single-gpu"},
        "runs": runs,
        "pipelining_speedup": {
            "refactor": runs["refactor_serial"]["wall_ms"] / runs["refactor_pipelined"]["wall_ms"],
            "retrieve": runs["retrieve_all_serial"]["wall_ms"] / runs["retrieve_all_pipelined"]["wall_ms"]},
    }
    print(json.dumps(res))


def bench_serving(args):
    """8 resident fields (edge^3 f32, 9 levels; fields 0..2 = vx, vy, vz), a
    Poisson stream of retrieval requests (tolerance log-uniform in 1e-7..1e-1,
    half raw fields, half V_total, 30% refining an earlier request), served with
    continuous batching under a 16 GiB output budget at several offered loads,
    against the same stream served one request at a time (one slot)."""
    import numpy as np
    import torch

    import paper_2505_00227_amd as mdr
    import workloads

    ctx = mdr.Context(0)
    params = mdr.default_params(group_planes=4)
    fields = []
    nbytes_field = 0
    level_sizes = []
    for f in range(8):
        levels = workloads.field_levels(seed=50 + f, edge=args.serve_edge, nlevels=9, dtype=np.float32)
        dev = [torch.from_numpy(a).cuda() for a in levels]
        nbytes_field = sum(a.nbytes for a in levels)
        level_sizes = [a.size for a in levels]
        fields.append(mdr.refactor(ctx, dev, 32, params))
        torch.cuda.synchronize()
        del dev, levels
        progress("field", f, "refactored")

    # The next-bound estimators of Sec. 5.2 on the velocity fields 0..2: bits per
    # value fetched, rounds and time per V_total tolerance (relative to the
    # largest V_total the ranges allow), each from fresh retrievers
    qoi_estimators = {}
    outs3 = [] if not args.qoi_estimators else [[torch.empty(n, dtype=torch.float32, device="cuda") for n in level_sizes] for _ in range(3)]
    nvals_field = sum(level_sizes)
    estimators = (("CP", "cp", 10.0), ("MA", "ma", 10.0), ("MAPE(c=2)", "mape", 2.0),
                  ("MAPE(c=10)", "mape", 10.0)) if args.qoi_estimators else ()
    for name, est, c in estimators:
        rows = {}
        for tol in (1e-1, 5e-1, 1e-2, 5e-2, 1e-3, 5e-3, 1e-4, 5e-4, 1e-5, 5e-5):
            rts = [mdr.Retriever(ctx, fields[i]) for i in range(3)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = mdr.retrieve_qoi_vtotal(*rts, tol, outs3, relative=True, mape_c=c, estimator=est)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rows["%.0e" % tol] = {"bitrate": info["bytes_fetched"] * 8.0 / (3 * nvals_field),
                                  "iterations": info["iterations"], "ms": dt * 1e3,
                                  "gbps": 3 * nbytes_field / dt / 1e9, "met": info["met"]}
            for rt in rts:
                rt.close()
        qoi_estimators[name] = rows
        progress("qoi estimator", name, rows)
    del outs3

    def make_requests(rate, n):
        reqs = workloads.serving_requests(seed=58, n=n, nfields=8, rate=rate)
        for q in reqs:  # a refinement continues its parent's kind and field
            if q["parent"] is not None:
                p = reqs[q["parent"]]
                q["kind"], q["field"] = p["kind"], p["field"]
        return reqs

    def run(reqs, slots):
        srv = mdr.Server(ctx, hbm_budget=16 << 30, max_slots=slots)
        for r in fields:
            srv.add_field(r)
        tickets = [0] * len(reqs)
        by_ticket = {}
        lat, served = [], 0
        t0 = time.perf_counter()
        i = 0
        while len(lat) < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i]["t"] <= now:
                q = reqs[i]
                parent = tickets[q["parent"]] if q["parent"] is not None else 0
                if q["kind"] == "raw":
                    t = srv.submit(mdr.MDR_REQ_FIELD, [q["field"]], q["tol"], parent=parent)
                else:
                    t = srv.submit(mdr.MDR_REQ_QOI_VTOTAL, [0, 1, 2], q["tol"], parent=parent)
                tickets[i] = t
                by_ticket[t] = q
                i += 1
            for c in srv.poll(1024):
                if c["status"] != 0:
                    raise RuntimeError("request failed: %r" % (c,))
                lat.append(c["t_done_ms"] - c["t_submit_ms"])
                served += nbytes_field * (1 if by_ticket[c["ticket"]]["kind"] == "raw" else 3)
                srv.release(c["ticket"])
            if i < len(reqs):
                time.sleep(max(0.0, min(0.0005, reqs[i]["t"] - (time.perf_counter() - t0))))
            else:
                time.sleep(0.0002)
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        lat.sort()
        pct = lambda p: lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))]
        return {"requests": len(reqs), "wall_s": wall, "gbps": served / wall / 1e9,
                "p50_ms": pct(50), "p99_ms": pct(99), "mean_ms": sum(lat) / len(lat),
                "batch_depth": st["step_requests"] / max(1, st["steps"])}

    # capacity: the request mix served back to back, one at a time
    n = args.serve_requests
    cap_reqs = make_requests(1e9, min(n, 300))
    cap = run(cap_reqs, 1)
    capacity = cap["requests"] / cap["wall_s"]
    progress("capacity %.1f req/s" % capacity)
    loads = {}
    for rho in [float(x) for x in args.serve_loads.split(",")]:
        reqs = make_requests(rho * capacity, n)
        b = run(reqs, 64)
        progress("load", rho, "batched", b)
        q = run(reqs, 1)
        progress("load", rho, "sequential", q)
        loads["%.1f" % rho] = {"batched": b, "sequential": q}
    main_load = loads.get("0.9") or next(iter(loads.values()))
    res = {
        "metric": "refactor & retrieve GB/s (frac of HBM peak); p50/p99 retrieval latency",
        "value": main_load["batched"]["gbps"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": n,
        "warmup": 0,
        "ms_per_step": main_load["batched"]["mean_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving-8-fields-%d^3-f32-9-levels" % args.serve_edge,
                   "requests": n, "budget_gib": 16, "slots": 64, "parallelism": "single-gpu"},
        "capacity_req_per_s": capacity,
        "qoi_estimators": qoi_estimators,
        "latency_ms": {"p50": main_load["batched"]["p50_ms"], "p99": main_load["batched"]["p99_ms"]},
        "loads": loads,
    }
    return res


def bench_ablation(args):
    """Sec. 3's encoding experiment on gfx950: n 32-bit words into 32 bitplanes
    and back by each parallelisation; GB/s of input words, HIP events on the
    stream the launches use (median of 10 after 2 warm-ups); every size is
    checked to round-trip."""
    import torch

    import paper_2505_00227_amd as mdr

    designs = list(mdr.ABLATION_DESIGNS)
    table = {}
    for lg in (20, 22, 24, 26, 28):
        n = 1 << lg
        x = torch.randint(-2 ** 31, 2 ** 31 - 1, (n,), dtype=torch.int32, device="cuda")
        out = torch.empty_like(x)
        for d in designs:
            planes = torch.empty(32 * mdr.ablation_plane_words(d, n), dtype=torch.int32, device="cuda")
            row = {}
            for kind, fn in (("encode", lambda: mdr.ablation_encode(d, x, planes)),
                             ("decode", lambda: mdr.ablation_decode(d, planes, out))):
                for _ in range(2):
                    fn()
                ts = []
                for _ in range(10):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    fn()
                    e1.record()
                    e1.synchronize()
                    ts.append(e0.elapsed_time(e1) / 1e3)
                t = statistics.median(ts)
                row[kind + "_gbps"] = 4 * n / t / 1e9
                row[kind + "_us"] = t * 1e6
            if not torch.equal(out, x):
                raise RuntimeError("ablation design %s does not round-trip at n=2^%d" % (d, lg))
            table.setdefault(d, {})["2^%d" % lg] = row
            del planes
            progress("ablation", d, "2^%d" % lg, row)
        del x, out
    res = {"metric": "bitplane encode / decode GB/s of 32-bit words by design (32 planes)",
           "unit": "GB/s", "n_gpus": 1, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "ablation-u32-32-planes", "sizes": ["2^%d" % k for k in (20, 22, 24, 26, 28)],
                      "designs": designs, "parallelism": "single-gpu"},
           "ablation": table}
    print(json.dumps(res))


def bench_multilevel(args):
    """Multilevel decomposition of the smooth 512^3 field (8 steps, 9 levels) in
    float32 and float64: decompose and recompose times (median of 10 after 2
    warm-ups, HIP events on the stream the launches use), GB/s of field data,
    and the fraction of HBM peak for 2 * n * s algorithmic bytes per pass (read
    the field and write the levels, or the reverse); then the field through the
    whole path: decompose, refactor, and six incremental retrievals from 1e-1
    to 1e-6 of the field's range, each recomposed."""
    import torch

    import paper_2505_00227_amd as mdr
    import workloads

    shape, nsteps = (512, 512, 512), 8
    n = shape[0] * shape[1] * shape[2]
    sizes = mdr.level_sizes(shape, nsteps)
    table = {}

    def timed(fn):
        for _ in range(2):
            fn()
        ts = []
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        return statistics.median(ts)

    u64 = workloads.smooth_field_tensor(2, shape, "cuda")
    for name, dt, B in (("f32", torch.float32, 32), ("f64", torch.float64, 64)):
        u = u64.to(dt)
        s = u.element_size()
        c = torch.empty(n, dtype=dt, device="cuda")
        v = torch.empty_like(u)
        td = timed(lambda: mdr.decompose(u, nsteps, c))
        tr = timed(lambda: mdr.recompose(c, nsteps, v))
        err = float((v.double() - u.double()).abs().max())
        if err > 4 * nsteps * torch.finfo(dt).eps * float(u.abs().max()):
            raise RuntimeError("recompose(decompose(u)) is off by %g" % err)
        row = {"decompose_ms": td * 1e3, "recompose_ms": tr * 1e3,
               "decompose_gbps": n * s / td / 1e9, "recompose_gbps": n * s / tr / 1e9,
               "decompose_hbm_frac": 2 * n * s / td / 8e12, "recompose_hbm_frac": 2 * n * s / tr / 8e12,
               "round_trip_max_err": err}
        # the field through the whole path
        ctx = mdr.Context(0)
        levels = list(torch.split(c, sizes))
        cat = torch.empty(n, dtype=dt, device="cuda")
        outs = list(torch.split(cat, sizes))  # retrieved levels land in one buffer
        rng_u = float(u.max() - u.min())
        bounds = [10.0 ** -k for k in range(1, 7)]

        def step():
            mdr.decompose(u, nsteps, c)
            r = mdr.refactor(ctx, levels, B)
            rt = mdr.Retriever(ctx, r)
            worst = 0.0
            for b in bounds:
                rt.retrieve(b * rng_u, outs, relative=False)
                mdr.recompose(cat, nsteps, v)
            torch.cuda.synchronize()
            worst = float((v.double() - u.double()).abs().max())
            rt.close()
            r.close()
            return worst

        step()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            worst = step()
            ts.append(time.perf_counter() - t0)
        if worst > 1e-6 * rng_u * (1 + 1e-6) + 4 * nsteps * torch.finfo(dt).eps * float(u.abs().max()):
            raise RuntimeError("field error %g above the 1e-6 bound" % worst)
        row["path_step_ms"] = statistics.median(ts) * 1e3
        row["path_gbps"] = n * s / statistics.median(ts) / 1e9
        row["path_final_max_err_rel"] = worst / rng_u
        # squared-L2 tables of the 9 levels (the MDR L2 option) and one L2 retrieval
        r = mdr.refactor(ctx, levels, B)
        tl = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r.l2_table(levels)          # waits for its stream
            tl.append(time.perf_counter() - t0)
        row["l2_table_ms"] = statistics.median(tl) * 1e3
        row["l2_table_gbps"] = n * s / statistics.median(tl) / 1e9
        norm = math.sqrt(sum(r.l2(l)[0] for l in range(len(sizes))))
        rt = mdr.Retriever(ctx, r)
        info = rt.retrieve_l2(1e-4 * norm, outs)
        torch.cuda.synchronize()
        row["l2_retrieve_1e-4_planes"] = rt.planes()
        row["l2_retrieve_1e-4_bound_rel"] = info["bound"] / norm
        rt.close()
        r.close()
        ctx.close()
        table[name] = row
        progress("multilevel", name, row)
        del u, c, v, levels, outs, cat
    res = {"metric": "multilevel decompose / recompose GB/s of field data (frac of HBM peak)",
           "unit": "GB/s", "n_gpus": 1, "dtype": "f32,f64", "data": "synthetic",
           "config": {"workload": "field-512^3-8-steps-9-levels", "level_sizes": sizes,
                      "parallelism": "single-gpu"},
           "multilevel": table}
    print(json.dumps(res))


def unit_table(r, B, m):
    """Per level of a refactored variable: (n, words per plane row, [(method,
    payload bytes, plane rows)] per unit in stream order, sign unit first)."""
    out = []
    for l in range(r.nlevels):
        n = r.info(l)["n"]
        nbd = -(-n // 32) if r.dtype == 0 else 2 * -(-n // 64)
        units = []
        for s in [-1] + list(range(0, B, m)):
            _, nb, meth = r.stream(l, s)
            rows = 1 if s < 0 else min(m, B - s)
            units.append((meth, nb, rows))
        out.append((n, nbd, units))
    return out


def kernel_bytes(tables, s, B, m, k_retrieved):
    """Algorithmic bytes per pass of each kernel: what its job must move.

    k_encode: the refactor's bytes of the method (read every value, write
    every final stream and the B+1 error bounds; the rows of Huffman- or
    run-length-coded groups, which the encoder also writes, are intermediate
    and not counted);
    k_stats: read every value; lossless: read the rows of each coded unit,
    write its payload; k_huf_decode: read the Huffman payloads of the fetched
    units, write their rows; k_reconstruct: read the sign row and the k plane
    rows of each level, write every value."""
    enc = stats = lossless = huf = rec = 0
    for t, k in zip(tables, k_retrieved):
        for (n, nbd, units), kl in zip(t, k):
            enc += n * s + sum(nb for _, nb, _ in units) + (B + 1) * s
            stats += n * s
            fetched = 1 + -(-kl // m) if kl else 0
            for i, (meth, nb, rows) in enumerate(units):
                if meth in (1, 2):
                    lossless += 4 * rows * nbd + nb
                if meth == 2 and i < fetched:
                    huf += nb + 4 * rows * nbd
            if kl:
                rec += 4 * (1 + kl) * nbd + n * s
    return {"k_encode": enc, "k_stats": stats, "lossless": lossless, "k_huf_decode": huf,
            "k_reconstruct": rec}


def path_bytes(tables, s, B, m, k_retrieved):
    """Algorithmic bytes of the whole path (refactor: values in, every stream
    out, the error tables; retrieval: the fetched streams in, every value out)."""
    ref = ret = 0
    for t, k in zip(tables, k_retrieved):
        for (n, nbd, units), kl in zip(t, k):
            coded = sum(nb for _, nb, _ in units)
            ref += n * s + coded + (B + 1) * s
            fetched = 1 + -(-kl // m) if kl else 0
            ret += sum(nb for _, nb, _ in units[:fetched]) + n * s
    return ref, ret


def roofline_from(stages, steps, kbytes, workload):
    """The step's dominant kernel (most time in the timed region, from HIP
    events on the library's stream) against the HBM peak."""
    times = {STAGE_KERNEL[st]: v[0] for st, v in stages.items() if st in STAGE_KERNEL and v[1]}
    kern = max((k for k in times if k in kbytes), key=times.get)
    launches = {STAGE_KERNEL[st]: v[1] for st, v in stages.items() if st in STAGE_KERNEL}
    ms_per_launch = times[kern] / max(1, launches[kern])
    bytes_per_launch = kbytes[kern] * steps / max(1, launches[kern])
    achieved = bytes_per_launch / (ms_per_launch / 1e3) / 1e9
    traffic = measured_traffic(kern, workload)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "kernel": kern, "source_sha": source_hash(kern), "launches_per_step": launches[kern] / steps,
            "ms_per_launch": ms_per_launch, "algorithmic_bytes_per_launch": bytes_per_launch,
            "kernel_ms_per_step": {k: v / steps for k, v in times.items()},
            "kernel_frac": {k: (kbytes[k] * steps / (v / 1e3) / 1e9 / HBM_PEAK_GBS if v else None)
                            for k, v in times.items() if k in kbytes}}


def copy_rate():
    """Measured device-to-device copy bandwidth (read + write) of 256 MiB: the
    practical ceiling.  The copy is a plain elementwise kernel (a negation of
    2^26 float32 values: 256 MiB read, 256 MiB written), so that it appears in
    a rocprofv3 counter run as a kernel of known traffic that scales the
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    ref = torch.zeros(1 << 26, dtype=torch.float32, device="cuda")
    ref_copy = torch.empty_like(ref)
    torch.neg(ref, out=ref_copy)  # warm (the first launch loads the kernel)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        torch.neg(ref, out=ref_copy)
    ev1.record()
    torch.cuda.synchronize()
    return 2 * ref.numel() * 4 * 10 / (ev0.elapsed_time(ev1) / 1e3) / 1e9


def cpu_baseline_slab(levels, B, m):
    """The oracle as it stands, on the host cores, over one 32x1024x1024 slab of
    the workload (2^25 float64 values, 9 levels): refactor + retrieval of every
    plane.  GB/s of original data on the same convention as `value`."""
    import oracle
    p = oracle.Params(group_planes=m)
    t0 = time.perf_counter()
    lv = oracle.refactor(levels, B, p)
    vals, k, bound, met = oracle.retrieve_to(lv, 0.0)
    t = time.perf_counter() - t0
    nbytes = sum(a.nbytes for a in levels)
    return {"value": 2 * nbytes / t / 1e9, "unit": "GB/s", "cores": oracle.get_threads(),
            "kind": "oracle", "seconds": t,
            "sample": "one 32x1024x1024 slab (2^25 float64 values, 9 levels, 256 MiB): "
                      "refactor + retrieval of every plane"}


def bench_field1024(args):
    """The 1024^3 float64 field (8 GiB) as 32 slabs of 32x1024x1024, each its
    own 9-level sub-domain (B = 64, m = 4), resident in HBM: one step = batched
    refactor of the slabs + batched retrieval of every plane."""
    import numpy as np
    import torch

    import paper_2505_00227_amd as mdr
    import workloads

    B, m, s = 64, 4, 8
    nch = args.chunks
    sizes = workloads.chunk_level_sizes()
    per = sum(sizes)
    host = torch.empty(per * nch, dtype=torch.float64).pin_memory()
    hv = host.numpy()
    for c in range(nch):
        hv[c * per:(c + 1) * per] = np.concatenate(workloads.chunk_levels(seed=3, chunk=c))
    progress("generated", nch, "slabs")
    dev_all = host.cuda()
    out_all = torch.empty_like(dev_all)
    dev = [list(torch.split(dev_all[c * per:(c + 1) * per], sizes)) for c in range(nch)]
    outs = [list(torch.split(out_all[c * per:(c + 1) * per], sizes)) for c in range(nch)]
    nbytes = dev_all.numel() * s
    ctx = mdr.Context(0)
    ctx.set_launch(graphs=0)
    params = mdr.default_params(group_planes=m)
    # the tensors' views and output pointers are marshalled once (resident inputs)
    dev_views, out_ptrs = mdr.BatchViews(dev), mdr.BatchOutputs(outs)
    torch.cuda.synchronize()

    state = {}

    def step(tr):
        t0 = time.perf_counter()
        rs = mdr.refactor_batch(ctx, dev_views, B, params)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rts = [mdr.Retriever(ctx, r) for r in rs]
        infos = mdr.retrieve_batch(rts, [0.0] * nch, out_ptrs)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tr.append((t1 - t0, t2 - t1))
        state["k"] = [rt.planes() for rt in rts]
        state["bounds"] = [i["bound"] for i in infos]
        for rt in rts:
            rt.close()
        if "tables" not in state:
            state["tables"] = [unit_table(r, B, m) for r in rs]
        for r in rs:
            r.close()

    for _ in range(args.warmup):
        step([])
    ctx.set_timing(True)
    ctx.timing(reset=True)
    tr = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(tr)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = ctx.timing(reset=True)
    ctx.set_timing(False)
    progress("timed", args.steps, "steps: %.1f ms/step" % (elapsed / args.steps * 1e3))
    # every plane held: each slab's error is within its table bound (the tails
    # below plane 64 of values far under the level maximum are all that is lost)
    for c in range(nch):
        err = float((out_all[c * per:(c + 1) * per] - dev_all[c * per:(c + 1) * per]).abs().max())
        if not err <= state["bounds"][c]:
            raise RuntimeError("slab %d: error %g above its bound %g" % (c, err, state["bounds"][c]))

    tables, k = state["tables"], state["k"]
    kb = kernel_bytes(tables, s, B, m, k)
    ref_b, ret_b = path_bytes(tables, s, B, m, k)
    t_ref = statistics.median(x[0] for x in tr)
    t_ret = statistics.median(x[1] for x in tr)
    stream_bytes = sum(nb for t in tables for (_, _, units) in t for _, nb, _ in units)

    # per-slab retrieval latency, cold: a fresh retriever per (slab, bound), with
    # 1 GiB of unrelated writes before each so that no stream is still in cache
    rs = mdr.refactor_batch(ctx, dev, B, params)
    flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    lat = {}
    bounds = [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 0.0]
    for c in range(nch):
        for tol in bounds:
            rt = mdr.Retriever(ctx, rs[c])
            flush.fill_(c & 0xFF)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            rt.retrieve(tol, outs[c])
            torch.cuda.synchronize()
            lat.setdefault(tol, []).append((time.perf_counter() - ta) * 1e3)
            rt.close()
    del flush
    for r in rs:
        r.close()
    all_lat = sorted(x for v in lat.values() for x in v)

    def pct(v, p):
        v = sorted(v)
        return v[min(len(v) - 1, int(round(p / 100.0 * (len(v) - 1))))]

    latency = {"p50": pct(all_lat, 50), "p99": pct(all_lat, 99), "count": len(all_lat),
               "per_bound": {("all" if t == 0 else "%.0e" % t): {"p50": pct(v, 50), "p99": pct(v, 99)}
                             for t, v in lat.items()},
               "note": "one 256 MiB slab per retrieval, fresh retriever, after 1 GiB of other writes"}
    progress("latency", latency)
    copy_gbps = copy_rate()
    out_keep = out_all[:per * 2].cpu()  # the first two slabs, all planes (the resident path's result)
    del dev, outs, dev_all, out_all

    # host to host through the chunked pipeline (pinned H2D / refactor / D2H on
    # three streams): PCIe-bound, reported beside the resident figures
    pipe = mdr.Pipeline(ctx, nch, sizes, torch.float64, B, params)
    hout = torch.empty_like(host).pin_memory()
    runs = {}
    for name, fn in (("refactor", lambda: pipe.refactor(host)), ("retrieve_all", lambda: pipe.retrieve(0.0, hout))):
        fn()
        best = min((fn() for _ in range(2)), key=lambda i: i["wall_ms"])
        best["gbps"] = nbytes / (best["wall_ms"] / 1e3) / 1e9
        runs[name] = best
    if not torch.equal(hout[:per * 2], out_keep):
        raise RuntimeError("pipelined retrieval differs from the resident one")
    pipe.close()
    del hout
    progress("pipeline", runs)

    res = {
        "metric": "refactor & retrieve GB/s (frac of HBM peak); p50/p99 retrieval latency",
        "value": 2 * nbytes / (elapsed / args.steps) / 1e9,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "chunked-1024^3-f64-%d-slabs-9-levels-resident" % nch, "values": nbytes // s,
                   "nplanes": B, "group_planes": m, "bounds_rel": ["all planes"],
                   "parallelism": "single-gpu"},
        "refactor_ms": t_ref * 1e3,
        "refactor_gbps": nbytes / t_ref / 1e9,
        "refactor_hbm_frac": ref_b / t_ref / 1e9 / HBM_PEAK_GBS,
        "retrieve_ms": t_ret * 1e3,
        "retrieve_gbps": nbytes / t_ret / 1e9,
        "retrieve_hbm_frac": ret_b / t_ret / 1e9 / HBM_PEAK_GBS,
        "algorithmic_bytes": {"refactor": ref_b, "retrieve": ret_b, "streams": stream_bytes},
        "latency_ms": latency,
        "roofline": roofline_from(stages, args.steps, kb, "field1024_f64"),
        "copy_gbps": copy_gbps,
        "host_to_host": {"gbps": 2 * nbytes / ((runs["refactor"]["wall_ms"] + runs["retrieve_all"]["wall_ms"]) / 1e3) / 1e9,
                         "runs": runs,
                         "note": "pinned host memory in and out, PCIe included (not `value`)"},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_slab(workloads.chunk_levels(seed=3, chunk=0), B, m)
    return res


def extras(args):
    """Short runs of the other workloads, as extra keys of the default line."""
    import argparse as _ap
    out = {}
    progress("extra: 512^3 float32 field")
    out["field512_f32"] = bench_field512(args, 2, 3, 1, cpu=False)
    progress("extra: 256-variable batch")
    a4 = _ap.Namespace(**vars(args))
    a4.no_tune, a4.steps, a4.warmup = False, 2, 1
    out["batched_256_vars"] = bench_batched(a4)
    progress("extra: serving")
    a5 = _ap.Namespace(**vars(args))
    a5.serve_requests, a5.serve_loads, a5.qoi_estimators = 1000, "0.9", False
    out["serving"] = bench_serving(a5)
    for v in out.values():
        for key in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
            v.pop(key, None)
    return out


def bench_field512(args, cfg, steps, warmup, cpu=True):
    """The 512^3 float32 field (9 levels; `cfg` 1: the plain 2^20 level): one
    step = refactor + incremental retrievals to relative bounds 1e-1 .. 1e-6."""
    import numpy as np
    import torch

    import paper_2505_00227_amd as mdr

    w = workload(cfg)
    levels = w["levels"]
    B, m = w["B"], w["m"]
    nvals = sum(a.size for a in levels)
    nbytes = sum(a.nbytes for a in levels)
    ctx = mdr.Context(0)
    dev = [torch.from_numpy(a).cuda() for a in levels]
    outs = [torch.empty_like(t) for t in dev]
    params = mdr.default_params(group_planes=m)
    torch.cuda.synchronize()

    def step(lat, tref):
        t0 = time.perf_counter()
        r = mdr.refactor(ctx, dev, B, params)
        torch.cuda.synchronize()
        tref.append(time.perf_counter() - t0)
        rt = mdr.Retriever(ctx, r)
        for tol in w["tols"]:
            t1 = time.perf_counter()
            info = rt.retrieve(tol, outs)
            torch.cuda.synchronize()
            lat.append((tol, time.perf_counter() - t1, info))
        rt.close()
        r.close()

    for _ in range(warmup):
        step([], [])
    ctx.set_timing(True)
    ctx.timing(reset=True)
    lat, tref = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(lat, tref)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = ctx.timing(reset=True)
    ctx.set_timing(False)
    copy_gbps = copy_rate()

    ms_step = elapsed / steps * 1e3
    moved = nbytes * (1 + len(w["tols"]))
    value = moved / (elapsed / steps) / 1e9
    lat_ms = sorted(t * 1e3 for _, t, _ in lat)

    def pct(p):
        return lat_ms[min(len(lat_ms) - 1, int(round(p / 100.0 * (len(lat_ms) - 1))))]

    per_tol = {}
    for tol, t, info in lat:
        per_tol.setdefault(tol, []).append((t, info))
    retrieve = {("%.0e" % tol): {"ms": statistics.median(x[0] for x in v) * 1e3,
                                 "gbps": nbytes / statistics.median(x[0] for x in v) / 1e9,
                                 "bound": v[0][1]["bound"], "met": v[0][1]["met"],
                                 "bytes_fetched": v[0][1]["bytes_fetched"]}
                for tol, v in per_tol.items()}

    # roofline of the dominant kernel (the bitplane encoder): the refactor's
    # bytes of the method (values in, final streams and error bounds out), per
    # launch; time from HIP events on its stream
    enc_ms, enc_n = stages["encode"]
    r = mdr.refactor(ctx, dev, B, params)
    s_bytes = levels[0].itemsize
    enc_bytes_per_step = sum(n * s_bytes + sum(nb for _, nb, _ in units) + (B + 1) * s_bytes
                             for n, _, units in unit_table(r, B, m))
    r.close()
    enc_launches_per_step = enc_n / steps
    achieved = (enc_bytes_per_step * steps) / (enc_ms / 1e3) / 1e9 if enc_ms else 0.0
    rec_ms, rec_n = stages["reconstruct"]
    res = {
        "metric": "refactor & retrieve GB/s (frac of HBM peak); p50/p99 retrieval latency",
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "values": nvals, "levels": len(levels), "nplanes": B,
                   "group_planes": m, "bounds_rel": w["tols"], "parallelism": "single-gpu"},
        "refactor_gbps": nbytes / statistics.median(tref) / 1e9,
        "refactor_ms": statistics.median(tref) * 1e3,
        "retrieve": retrieve,
        "latency_ms": {"p50": pct(50), "p99": pct(99), "count": len(lat_ms)},
        "stage_ms_per_step": {k: v[0] / steps for k, v in stages.items()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (measured_traffic("k_encode", "field512_f32") if cfg == 2 else None),
                     "traffic_unit": "HBM bytes per step (all encoder launches)",
                     "source_sha": source_hash("k_encode"),
                     "kernel": "k_encode", "launches_per_step": enc_launches_per_step,
                     "algorithmic_bytes_per_step": enc_bytes_per_step},
        "copy_gbps": copy_gbps,
        "reconstruct_kernel_gbps": ((nbytes * len(w["tols"]) * steps) / (rec_ms / 1e3) / 1e9
                                    if rec_ms else None),
    }
    if cpu:
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path has no multi-GPU component "
              "(variables and chunks shard independently); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.ablation:
        bench_ablation(args)
        return
    if args.multilevel:
        bench_multilevel(args)
        return
    if args.config == 4:
        print(json.dumps(bench_batched(args)))
        return
    if args.config == 5:
        print(json.dumps(bench_serving(args)))
        return
    if args.pipeline:
        bench_chunked(args)
        return
    if args.config in (1, 2):
        print(json.dumps(bench_field512(args, args.config, args.steps, args.warmup,
                                        cpu=not args.no_cpu_baseline)))
        return
    res = bench_field1024(args)
    if not args.no_extras:
        res["extras"] = extras(args)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
