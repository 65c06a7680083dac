"""Serving (continuous batching over resident fields): every request's result is
the same, bit for bit, whether it runs alone or in a mix with others, equals the
oracle's retrieval from the same starting planes, and admission keeps the
outputs within the HBM budget."""
import time

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import say, to_oracle_params, upload

pytestmark = pytest.mark.gpu

SIZES = [8, 56, 448, 3584, 28672]


@pytest.fixture(scope="module")
def mdr():
    import paper_2505_00227_amd as m
    return m


@pytest.fixture(scope="module")
def setup(mdr):
    ctx = mdr.Context(0)
    rng = np.random.default_rng(70)
    raw = [workloads.laplace_levels(SIZES, 1.0 + f, rng, np.float32) for f in range(4)]
    p = mdr.default_params()
    rs = [mdr.refactor(ctx, upload(levels), 32, p) for levels in raw]
    orc = [oracle.refactor(levels, 32, to_oracle_params(p)) for levels in raw]
    yield ctx, raw, rs, orc
    ctx.close()


def _requests(seed, n, orc):
    """Mixed requests: raw fields (relative L-inf) and V_total on fields 0..2
    (absolute tolerance), some refining an earlier request of the same kind."""
    rng = np.random.default_rng(seed)
    vt = sum(np.concatenate([lv.reconstruct(32).astype(np.float64) for lv in orc[c]]) ** 2 for c in range(3))
    qrange = float(vt.max() - vt.min())
    reqs = []
    for i in range(n):
        kind = "qoi" if rng.random() < 0.4 else "raw"
        rel = float(np.exp(rng.uniform(np.log(1e-6), np.log(1e-1))))
        parent = None
        cands = [j for j in range(i) if reqs[j]["kind"] == kind]
        if cands and rng.random() < 0.3:
            parent = int(rng.choice(cands))
        field = int(rng.integers(0, 4)) if kind == "raw" else 0
        if parent is not None:
            field = reqs[parent]["field"]
        tol = rel if kind == "raw" else rel * qrange
        reqs.append({"kind": kind, "field": field, "tol": tol, "parent": parent})
    return reqs


def _submit(mdr, srv, q, tickets):
    parent = tickets[q["parent"]] if q["parent"] is not None else 0
    if q["kind"] == "raw":
        return srv.submit(mdr.MDR_REQ_FIELD, [q["field"]], q["tol"], relative=True, parent=parent)
    return srv.submit(mdr.MDR_REQ_QOI_VTOTAL, [0, 1, 2], q["tol"], relative=False, parent=parent)


def _collect(mdr, srv, q, c):
    ncomp = 1 if q["kind"] == "raw" else 3
    out = []
    for comp in range(ncomp):
        for l in range(len(SIZES)):
            ptr, n = srv.output(c["ticket"], comp, l)
            out.append(mdr.device_bytes(ptr, 4 * n))
    return out


def _wait(mdr, srv, reqs_by_ticket, want, timeout=60.0):
    """Collect completions; each one's outputs are copied out and released at
    once, as a client would, so the budget frees up for waiting requests."""
    got = {}
    t0 = time.time()
    while len(got) < want:
        for c in srv.poll():
            q = reqs_by_ticket[c["ticket"]]
            outs = _collect(mdr, srv, q, c) if c["status"] == 0 else None
            if c["status"] == 0:
                srv.release(c["ticket"])
            got[c["ticket"]] = (c, outs)
        st = srv.stats()
        assert st["hbm_in_use"] <= st["hbm_budget"] and st["hbm_held"] <= st["hbm_budget"]
        assert time.time() - t0 < timeout, ("server did not finish", len(got), want, st)
        time.sleep(0.001)
    return got


def test_alone_equals_mix_equals_oracle(mdr, setup):
    ctx, raw, rs, orc = setup
    reqs = _requests(71, 40, orc)
    out_bytes = sum(4 * n for n in SIZES) + 256 * len(SIZES)

    # mix: everything submitted at once; a budget of ~6 QoI requests' outputs
    srv = mdr.Server(ctx, hbm_budget=6 * 3 * out_bytes, max_slots=16)
    for r in rs:
        srv.add_field(r)
    tickets = []
    for q in reqs:
        tickets.append(_submit(mdr, srv, q, tickets))
    got = _wait(mdr, srv, dict(zip(tickets, reqs)), len(reqs))
    mix = []
    for q, t in zip(reqs, tickets):
        c, outs = got[t]
        assert c["status"] == 0, (q, c)
        mix.append((c, outs))
    st = srv.stats()
    say("mix stats", st)
    assert st["step_requests"] > st["steps"], "requests were never batched together"
    srv.close()

    # alone: one request at a time on a fresh server
    srv = mdr.Server(ctx, hbm_budget=6 * 3 * out_bytes, max_slots=16)
    for r in rs:
        srv.add_field(r)
    tickets = []
    for i, q in enumerate(reqs):
        t = _submit(mdr, srv, q, tickets)
        tickets.append(t)
        c, alone = _wait(mdr, srv, {t: q}, 1)[t]
        assert c["status"] == 0, (q, c)
        assert alone == mix[i][1], ("alone vs mix", i, q)
        for key in ("bound", "met", "iterations", "bytes_fetched"):
            assert c[key] == mix[i][0][key], ("alone vs mix", i, key, c[key], mix[i][0][key])
    srv.close()

    # oracle, from the same starting planes
    final_k = []
    for i, q in enumerate(reqs):
        say("oracle check", i, q)
        c, outs = mix[i]
        k_in = final_k[q["parent"]] if q["parent"] is not None else None
        if q["kind"] == "raw":
            vals, k, bound, met = oracle.retrieve_to(orc[q["field"]], q["tol"], k_in=k_in)
            assert c["bound"] == bound and c["met"] == int(met)
            ref = [np.asarray(v, np.float32).tobytes() for v in vals]
            final_k.append(k)
        else:
            vals, ks, tprime, met, it = oracle.retrieve_qoi_vtotal(orc[:3], q["tol"], k_in=k_in)
            assert c["bound"] == tprime and c["met"] == int(met) and c["iterations"] == it
            ref = []
            for comp in range(3):
                o = 0
                for n in SIZES:
                    ref.append(np.asarray(vals[comp][o:o + n], np.float32).tobytes())
                    o += n
            final_k.append(ks)
        assert outs == ref, ("oracle", i, q)


def test_rejects_requests_beyond_budget(mdr, setup):
    ctx, raw, rs, orc = setup
    srv = mdr.Server(ctx, hbm_budget=1 << 16, max_slots=4)
    srv.add_field(rs[0])
    with pytest.raises(mdr.MdrError) as ei:
        srv.submit(mdr.MDR_REQ_FIELD, [0], 1e-3)
    assert ei.value.status == mdr.MDR_ERR_INVALID_ARG
    srv.close()


def test_output_blocks_are_reused(mdr, setup):
    """Released outputs are kept and reused: serving one request at a time holds
    one block per component of the largest request so far, and never more than
    the budget."""
    ctx, raw, rs, orc = setup
    block = sum((4 * n + 255) // 256 * 256 for n in SIZES)
    srv = mdr.Server(ctx, hbm_budget=4 * block, max_slots=4)
    for r in rs:
        srv.add_field(r)
    held = []
    for i, kind in enumerate(["raw", "raw", "qoi", "raw", "qoi", "raw"]):
        q = {"kind": kind, "field": i % 4, "tol": 1e-3 if kind == "raw" else 1e-2, "parent": None}
        t = _submit(mdr, srv, q, [])
        c, _ = _wait(mdr, srv, {t: q}, 1)[t]
        assert c["status"] == 0, (q, c)
        held.append(srv.stats()["hbm_held"])
    assert held == [block, block, 3 * block, 3 * block, 3 * block, 3 * block], held
    srv.close()
