"""Benchmark of the refactor / progressive-retrieve hot path on one MI355X.

Default workload: a 512^3 float32 field as 9 coefficient levels (2^27 values,
512 MiB), 32 planes, groups of 4 planes.  One step = refactor of every level +
progressive (incremental) retrieval to relative L-inf bounds 1e-1 ... 1e-6,
each writing the full reconstruction.  Inputs are resident in HBM before the
timed region.  Prints one JSON line.

value = original bytes moved through the path per second: the field once for
refactor plus once per retrieval (the paper's GB/s-of-original-data convention).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ENCODER_SRC = os.path.join(ROOT, "paper_2505_00227_amd", "csrc", "k_refactor.hip")
TRAFFIC_NOTE = os.path.join(ROOT, "profiles", "k_encode_field512_traffic.md")


def encoder_hash() -> str:
    import hashlib
    return hashlib.sha256(open(ENCODER_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per step of the encoder from the committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a plain copy of
    known size), or None when the encoder source changed since they were taken."""
    try:
        vals = {}
        for line in open(TRAFFIC_NOTE):
            if line.startswith("machine: "):
                for kv in line[len("machine: "):].split():
                    k, v = kv.split("=")
                    vals[k] = v
        if vals.get("source_sha") != encoder_hash():
            return None
        return float(vals["traffic_bytes_per_step"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 22,
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
    return {"value": nbytes / t / 1e9, "unit": "GB/s", "cores": oracle.get_threads(),
            "kind": "oracle", "seconds": t,
            "sample": "first %d values of the finest level (%.1f MiB): refactor + %d "
                      "incremental retrievals" % (x.size, x.nbytes / 2 ** 20, len(w["tols"]))}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path has no multi-GPU component "
              "(variables and chunks shard independently); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2505_00227_amd as mdr

    w = workload(args.config)
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

    for _ in range(args.warmup):
        step([], [])
    ctx.set_timing(True)
    ctx.timing(reset=True)
    lat, tref = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(lat, tref)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = ctx.timing(reset=True)
    ctx.set_timing(False)
    # a plain device copy of known size (256 MiB): the reference that scales the
    # FETCH_SIZE / WRITE_SIZE counters when this run is profiled
    ref = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    ref_copy = ref.clone()
    torch.cuda.synchronize()
    del ref, ref_copy

    ms_step = elapsed / args.steps * 1e3
    moved = nbytes * (1 + len(w["tols"]))
    value = moved / (elapsed / args.steps) / 1e9
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

    # roofline of the dominant kernel (the bitplane encoder): algorithmic bytes =
    # input values + all B+1 plane rows, per launch; time from HIP events on its stream
    enc_ms, enc_n = stages["encode"]
    plane_bytes = 0
    for a in levels:
        nbd = (a.size + 31) // 32
        plane_bytes += 4 * (B + 1) * nbd
    enc_bytes_per_step = nbytes + plane_bytes
    enc_launches_per_step = enc_n / args.steps
    achieved = (enc_bytes_per_step * args.steps) / (enc_ms / 1e3) / 1e9 if enc_ms else 0.0
    rec_ms, rec_n = stages["reconstruct"]
    res = {
        "metric": "refactor & retrieve GB/s (frac of HBM peak); p50/p99 retrieval latency",
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
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
        "stage_ms_per_step": {k: v[0] / args.steps for k, v in stages.items()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (measured_traffic() if args.config == 2 else None),
                     "traffic_unit": "HBM bytes per step (all encoder launches)",
                     "encoder_sha": encoder_hash(),
                     "kernel": "k_encode", "launches_per_step": enc_launches_per_step,
                     "algorithmic_bytes_per_step": enc_bytes_per_step},
        "reconstruct_kernel_gbps": ((nbytes * len(w["tols"]) * args.steps) / (rec_ms / 1e3) / 1e9
                                    if rec_ms else None),
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
