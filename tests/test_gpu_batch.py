"""GPU parity of the batched refactor: one flattened pass over every level of
every variable (optionally captured once as a HIP graph and replayed) must give,
per variable, exactly the oracle's streams, tables and reconstructions, and the
same bytes as a separate per-variable refactor."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import (assert_same_bits, compare_refactor, gpu_outputs, host, say,
                      to_oracle_params, upload)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdr():
    import paper_2505_00227_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mdr):
    c = mdr.Context(0)
    yield c
    c.close()


def _mixed_vars(seed, dtype, nvars=7):
    """Uneven variables: cube edges 3..40, 4 levels, plus one with an empty level."""
    edges, vs = workloads.batch_variables(seed=seed, nvars=nvars, nlevels=4, lo=3, hi=40, dtype=dtype)
    rng = np.random.default_rng(seed + 1)
    vs.append([rng.laplace(0, 1, 37).astype(dtype), np.zeros(0, dtype), rng.laplace(0, 0.5, 300).astype(dtype)])
    return vs


def _check_batch(mdr, ctx, vs, B, params, graphs):
    ctx.set_launch(graphs=1 if graphs else 0)
    dev = [upload(v) for v in vs]
    rs = mdr.refactor_batch(ctx, dev, B, params)
    assert len(rs) == len(vs)
    op = to_oracle_params(params)
    for i, (r, v) in enumerate(zip(rs, vs)):
        say("batch variable", i, "sizes", [a.size for a in v], "graphs", graphs)
        orc = oracle.refactor(v, B, op)
        compare_refactor(r, orc)
        single = mdr.refactor(ctx, dev[i], B, params)
        assert single.serialize() == r.serialize(), ("batch vs single", i)
        rt = mdr.Retriever(ctx, r)
        outs = gpu_outputs(v)
        m = min(params.group_planes, B)
        for k in sorted({m, B}):
            rt.retrieve_planes([k] * len(v), outs)
            for l, ol in enumerate(orc):
                assert_same_bits(host(outs[l]), ol.reconstruct(min(B, k)), ("var", i, "level", l, "k", k))
    return rs


@pytest.mark.parametrize("graphs", [False, True])
def test_batch_f32_matches_oracle_and_single(mdr, ctx, graphs):
    vs = _mixed_vars(41, np.float32)
    _check_batch(mdr, ctx, vs, 32, mdr.default_params(), graphs)


def test_batch_f64_forced_methods(mdr, ctx):
    vs = _mixed_vars(43, np.float64, nvars=4)
    for fm in (-1, 1, 2):
        say("f64 batch force", fm)
        _check_batch(mdr, ctx, vs, 52, mdr.default_params(force_method=fm), True)


def test_batch_graph_replay_new_data(mdr, ctx):
    """Same shape twice: the second call replays the captured graph with new
    inputs and new output arenas; both must match the oracle."""
    shape_a = _mixed_vars(45, np.float32, nvars=5)
    rng = np.random.default_rng(46)
    shape_b = [[rng.laplace(0, 3, a.size).astype(np.float32) for a in v] for v in shape_a]
    p = mdr.default_params(force_method=2, huf_chunk=512)
    first = _check_batch(mdr, ctx, shape_a, 32, p, True)
    second = _check_batch(mdr, ctx, shape_b, 32, p, True)
    # the first call's results are untouched by the replay
    op = to_oracle_params(p)
    for r, v in zip(first, shape_a):
        compare_refactor(r, oracle.refactor(v, 32, op))
    del second


def test_batch_launch_shapes_do_not_change_results(mdr, ctx):
    vs = _mixed_vars(47, np.float32, nvars=3)
    dev = [upload(v) for v in vs]
    p = mdr.default_params()
    ref = None
    for tgt, sv in ((64, 1024), (512, 4096), (8192, 1 << 20), (2304, 16384)):
        ctx.set_launch(enc_target_wg=tgt, stats_wg_values=sv, graphs=0)
        blobs = [r.serialize() for r in mdr.refactor_batch(ctx, dev, 32, p)]
        if ref is None:
            ref = blobs
        assert blobs == ref, ("launch shape", tgt, sv)
    ctx.set_launch(enc_target_wg=2304, stats_wg_values=65536, graphs=1)


def test_batch_rejects_nonfinite(mdr, ctx):
    good = [np.ones(100, np.float32)]
    bad = [np.array([1.0, np.inf, 2.0], np.float32)]
    with pytest.raises(mdr.MdrError) as ei:
        mdr.refactor_batch(ctx, [upload(good), upload(bad)], 32)
    assert ei.value.status == mdr.MDR_ERR_INVALID_ARG
    assert "variable 1" in str(ei.value)


def test_retrieve_batch_matches_oracle(mdr, ctx):
    """Batched retrieval (each variable its own tolerance, two rounds to check
    incremental state) equals the oracle's retrieval of each variable."""
    vs = _mixed_vars(49, np.float32, nvars=5)
    vs.append([a.astype(np.float64) for a in _mixed_vars(50, np.float32, nvars=1)[0]])  # one f64 variable
    p = mdr.default_params()
    op = to_oracle_params(p)
    rs = [mdr.refactor(ctx, upload(v), 32 if v[0].dtype == np.float32 else 52, p) for v in vs]
    orc = [oracle.refactor(v, 32 if v[0].dtype == np.float32 else 52, op) for v in vs]
    rts = [mdr.Retriever(ctx, r) for r in rs]
    outs = [gpu_outputs(v) for v in vs]
    k_prev = [None] * len(vs)
    rounds = [[10 ** -(1 + i) for i in range(len(vs))], [10 ** -(4 + i % 3) for i in range(len(vs))]]
    for rnd, tols in enumerate(rounds):
        say("retrieve batch round", rnd, "tols", tols)
        infos = mdr.retrieve_batch(rts, tols, outs)
        for i, v in enumerate(vs):
            vals, k, bound, met = oracle.retrieve_to(orc[i], tols[i], k_in=k_prev[i])
            assert rts[i].planes() == list(k), (i, rts[i].planes(), k)
            assert infos[i]["bound"] == bound and infos[i]["met"] == int(met)
            got = np.concatenate([host(o).astype(np.float64) for o in outs[i]])
            ref = np.concatenate([np.asarray(a, np.float64) for a in vals])
            assert_same_bits(got, ref, ("var", i, "round", rnd))
            k_prev[i] = k


def test_prepared_views_repeat_passes(mdr, ctx):
    """BatchViews / BatchOutputs marshal a batch once: passes repeated through
    them equal passes marshalled per call, for new data in the same tensors too,
    and the prepared objects keep their tensors alive."""
    import gc
    vs = _mixed_vars(53, np.float32, nvars=4)
    p = mdr.default_params()
    dev = [upload(v) for v in vs]
    bv = mdr.BatchViews(dev)
    outs = [gpu_outputs(v) for v in vs]
    bo = mdr.BatchOutputs(outs)
    del outs
    gc.collect()
    for rnd in range(2):
        if rnd:  # new values in the same device tensors
            rng = np.random.default_rng(54)
            vs = [[rng.laplace(0, 1, a.size).astype(np.float32) for a in v] for v in vs]
            for d, v in zip(dev, vs):
                for t, a in zip(d, v):
                    t.copy_(torch_from(a))
        say("prepared views round", rnd)
        a = [r.serialize() for r in mdr.refactor_batch(ctx, bv, 32, p)]
        rs = mdr.refactor_batch(ctx, dev, 32, p)
        assert [r.serialize() for r in rs] == a
        rts = [mdr.Retriever(ctx, r) for r in rs]
        infos = mdr.retrieve_batch(rts, [1e-3] * len(rts), bo)
        orc = [oracle.refactor(v, 32, to_oracle_params(p)) for v in vs]
        for i, v in enumerate(vs):
            vals, k, bound, met = oracle.retrieve_to(orc[i], 1e-3)
            assert rts[i].planes() == list(k) and infos[i]["bound"] == bound
            got = np.concatenate([host(o).astype(np.float64) for o in bo.outs[i]])
            assert_same_bits(got, np.concatenate([np.asarray(x, np.float64) for x in vals]), ("var", i))
    with pytest.raises(ValueError):
        mdr.retrieve_batch(rts[:2], [1e-3] * 2, bo)


def torch_from(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("dtype,B", [(np.float32, 32), (np.float64, 64)])
@pytest.mark.parametrize("graphs", [False, True])
def test_large_batch_matches_single_and_oracle(mdr, ctx, dtype, B, graphs):
    """A pass of more than 2^24 values over several variables (many tiles per
    encoder workgroup, a replayed graph): every variable equals its own
    single-variable refactor and the oracle."""
    ctx.set_launch(graphs=1 if graphs else 0)
    rng = np.random.default_rng(71)
    sizes = [workloads.level_sizes((e, e, e), 4) for e in (180, 200, 160)]
    vs = [workloads.laplace_levels(sz, 1.0 + i, rng, dtype) for i, sz in enumerate(sizes)]
    assert sum(a.size for v in vs for a in v) >= 1 << 24
    dev = [upload(v) for v in vs]
    p = mdr.default_params()
    say("large batch", np.dtype(dtype).name, "graphs", graphs, [sum(a.size for a in v) for v in vs])
    for rep in range(2):  # a replay of the captured pass too
        rs = mdr.refactor_batch(ctx, dev, B, p)
        for i, (r, v) in enumerate(zip(rs, vs)):
            single = mdr.refactor(ctx, dev[i], B, p)
            assert single.serialize() == r.serialize(), ("batch vs single", i, rep)
    compare_refactor(rs[1], oracle.refactor(vs[1], B, to_oracle_params(p)))
    ctx.set_launch(graphs=1)
