"""The launch-shape autotuner: it times candidate shapes of the refactor pass,
records the fastest per pass key, persists the table as JSON, and the shape it
picks changes no result (every stream equal to the default shape's and to the
oracle's, bit for bit)."""
import os

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import compare_refactor, say, to_oracle_params, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdr():
    import paper_2505_00227_amd as m
    return m


def _vars(seed, nvars=6):
    edges, vs = workloads.batch_variables(seed=seed, nvars=nvars, nlevels=4, lo=20, hi=90)
    return vs


def test_tuner_records_a_shape_that_changes_nothing(mdr, tmp_path):
    ctx = mdr.Context(0)
    ctx.set_launch(graphs=0)
    vs = _vars(61)
    dev = [upload(v) for v in vs]
    p = mdr.default_params()
    ref = [r.serialize() for r in mdr.refactor_batch(ctx, dev, 32, p)]
    res = ctx.autotune(dev, 32, p, reps=1)
    say("tune result", res)
    assert res["candidates"] >= 8 and res["best_ms"] > 0 and res["default_ms"] > 0
    assert res["best_ms"] <= res["default_ms"]
    assert res["best"]["select_threads"] in (0, 256, 512, 1024)  # 0: chosen by the pass's unit count
    table = ctx.tune_table()
    assert len(table) == 1 and table[0]["shape"] == res["best"]
    nvals = sum(a.size for v in vs for a in v)
    assert table[0]["key"] == [0, 32, 4, int(np.floor(np.log2(nvals))), int(np.floor(np.log2(4 * len(vs))))]
    # the tuned shape is used by the next pass of that key, and changes nothing
    got = [r.serialize() for r in mdr.refactor_batch(ctx, dev, 32, p)]
    assert got == ref
    op = to_oracle_params(p)
    r0 = mdr.refactor_batch(ctx, dev, 32, p)[0]
    compare_refactor(r0, oracle.refactor(vs[0], 32, op))
    # known key, no force: nothing timed
    again = ctx.autotune(dev, 32, p)
    assert again["candidates"] == 0 and again["best"] == res["best"]
    # the table persists and a new context reads it back
    path = str(tmp_path / "tune.json")
    ctx.tune_save(path)
    ctx2 = mdr.Context(0)
    ctx2.tune_load(path)
    assert ctx2.tune_table() == table
    with open(path, "a") as f:
        f.write('{"dtype":0,"nplanes":32}\n')
    with pytest.raises(mdr.MdrError) as ei:
        ctx2.tune_load(path)
    assert ei.value.status == mdr.MDR_ERR_CORRUPT_STREAM
    with pytest.raises(mdr.MdrError):
        ctx2.tune_load(str(tmp_path / "missing.json"))
    ctx2.close()
    ctx.close()


@pytest.mark.parametrize("threads", [0, 256, 512, 1024])
def test_selection_workgroup_sizes_agree(mdr, threads):
    """Every selection workgroup size gives the oracle's methods and streams,
    for a single field and for a batch, under Alg. 2 and forced Huffman."""
    ctx = mdr.Context(0)
    ctx.set_select_threads(threads)
    x = workloads.plain_level(seed=70, n=300_000)
    for force in (-1, 2):
        p = mdr.default_params(group_planes=4, force_method=force)
        r = mdr.refactor(ctx, upload([x]), 32, p)
        compare_refactor(r, oracle.refactor([x], 32, to_oracle_params(p)))
    vs = _vars(62, nvars=3)
    p = mdr.default_params()
    for r, v in zip(mdr.refactor_batch(ctx, [upload(v) for v in vs], 32, p), vs):
        compare_refactor(r, oracle.refactor(v, 32, to_oracle_params(p)))
    ctx.close()


def test_tune_on_first_use_from_the_environment(mdr, tmp_path, monkeypatch):
    path = str(tmp_path / "auto.json")
    monkeypatch.setenv("MDR_TUNE_CACHE", path)
    monkeypatch.setenv("MDR_AUTOTUNE", "1")
    ctx = mdr.Context(0)
    vs = _vars(63, nvars=4)
    dev = [upload(v) for v in vs]
    p = mdr.default_params()
    rs = mdr.refactor_batch(ctx, dev, 32, p)
    assert len(ctx.tune_table()) == 1 and os.path.exists(path)
    op = to_oracle_params(p)
    for r, v in zip(rs, vs):
        compare_refactor(r, oracle.refactor(v, 32, op))
    ctx.close()
    monkeypatch.delenv("MDR_AUTOTUNE")
    ctx2 = mdr.Context(0)  # reads the file the first context wrote
    assert len(ctx2.tune_table()) == 1
    ctx2.close()
