"""GPU parity of the QoI families beyond V_total (Sec. 5.2's error control for
derived quantities; mdr_retrieve_qoi): sum of squares of one or two
variables, the magnitude sqrt(sum of squares) of one to three, and the product
of two, each with the MAPE, MA and CP estimators, against the oracle's loop:
same planes per variable, the same estimate bit for bit, the same number of
rounds, the same reconstructions, and real error <= estimate <= tolerance."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_same_bits, gpu_outputs, host, say, upload

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


def _qoi(kind, v):
    if kind == "product":
        return v[0] * v[1]
    s = sum(x * x for x in v)
    return np.sqrt(s) if kind == "magnitude" else s


def _run(mdr, ctx, kind, nv, dtype, B, seed, rels, estimator, c=2.0, incremental=False):
    sizes = [8, 56, 448, 3584, 28672]
    rng = np.random.default_rng(seed)
    raw = [workloads.laplace_levels(sizes, 1.0 + 0.5 * i, rng, dtype) for i in range(nv)]
    op = oracle.Params(group_planes=4)
    orc = [oracle.refactor(levels, B, op) for levels in raw]
    gpu = [mdr.refactor(ctx, upload(levels), B, mdr.default_params(group_planes=4)) for levels in raw]
    q = _qoi(kind, [np.concatenate([a.astype(np.float64) for a in levels]) for levels in raw])
    scale = oracle.qoi_scale(kind, orc)
    rts = [mdr.Retriever(ctx, r) for r in gpu]
    k_prev = None
    for rel in rels:
        say("qoi family", kind, nv, np.dtype(dtype).name, estimator, "rel", rel, "incremental", incremental)
        if not incremental:
            rts = [mdr.Retriever(ctx, r) for r in gpu]
            k_prev = None
        outs = [gpu_outputs(levels) for levels in raw]
        info = mdr.retrieve_qoi(kind, rts, rel, outs, relative=True, mape_c=c, estimator=estimator)
        vals, ks, tp, met, it = oracle.retrieve_qoi(kind, orc, rel * scale, c=c, k_in=k_prev,
                                                    estimator=estimator)
        assert [rt.planes() for rt in rts] == ks, ([rt.planes() for rt in rts], ks)
        assert info["tau_abs"] == rel * scale
        assert info["tau_est"] == tp and info["iterations"] == it and info["met"] == int(met)
        got = []
        for i in range(nv):
            g = np.concatenate([host(o).astype(np.float64) for o in outs[i]])
            assert_same_bits(g, vals[i], ("variable", i))
            got.append(g)
        real = float(np.abs(_qoi(kind, got) - q).max())
        assert real <= info["tau_est"]
        if met:
            assert info["tau_est"] <= rel * scale
        k_prev = ks


@pytest.mark.parametrize("kind,nv", [("sumsq", 1), ("sumsq", 2), ("magnitude", 1), ("magnitude", 2),
                                     ("magnitude", 3), ("product", 2)])
@pytest.mark.parametrize("estimator", ["mape", "ma", "cp"])
def test_family_matches_oracle_f32(mdr, ctx, kind, nv, estimator):
    _run(mdr, ctx, kind, nv, np.float32, 32, 40 + nv, (1e-1, 1e-3, 1e-5), estimator)


@pytest.mark.parametrize("kind,nv", [("magnitude", 3), ("product", 2)])
def test_family_matches_oracle_f64_incremental(mdr, ctx, kind, nv):
    _run(mdr, ctx, kind, nv, np.float64, 48, 50 + nv, (1e-2, 1e-4, 1e-7), "mape", c=10.0, incremental=True)


def test_family_argument_checks(mdr, ctx):
    x = workloads.plain_level(seed=3, n=1000)
    rs = [mdr.refactor(ctx, upload([x]), 32) for _ in range(3)]
    rts = [mdr.Retriever(ctx, r) for r in rs]
    outs = [gpu_outputs([x]) for _ in range(3)]
    for kind, n in (("product", 1), ("product", 3), ("magnitude", 0)):
        with pytest.raises(mdr.MdrError) as ei:
            mdr.retrieve_qoi(kind, rts[:n], 1e-2, outs[:n], relative=True)
        assert ei.value.status == mdr.MDR_ERR_INVALID_ARG
    with pytest.raises(mdr.MdrError):
        mdr.retrieve_qoi("product", [rts[0], rts[0]], 1e-2, outs[:2], relative=True)
