"""GPU parity of the V_total QoI retrieval (Sec. 5.2, Alg. 3 with the MAPE, MA
and CP estimators) against the oracle's loop: same planes per variable, same
estimate (bit for bit), same number of rounds, same reconstructions; and the
paper's guarantee real error <= estimate <= tolerance."""
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


def _setup(mdr, ctx, seed, sizes, dtype=np.float32, B=32, m=4):
    rng = np.random.default_rng(seed)
    raw = [workloads.laplace_levels(sizes, 1.0, rng, dtype) for _ in range(3)]
    op = oracle.Params(group_planes=m)
    orc = [oracle.refactor(levels, B, op) for levels in raw]
    gpu = [mdr.refactor(ctx, upload(levels), B, mdr.default_params(group_planes=m)) for levels in raw]
    orig = [np.concatenate([a.astype(np.float64) for a in levels]) for levels in raw]
    vt = orig[0] ** 2 + orig[1] ** 2 + orig[2] ** 2
    return raw, orc, gpu, vt


def _check(mdr, raw, rts, outs3, info, ref, vt, tau):
    vals, ks, tprime, met, it = ref
    assert [rt.planes() for rt in rts] == ks, ([rt.planes() for rt in rts], ks)
    assert info["tau_est"] == tprime and info["iterations"] == it and info["met"] == int(met)
    got = []
    for c in range(3):
        g = np.concatenate([host(o).astype(np.float64) for o in outs3[c]])
        assert_same_bits(g, vals[c], ("component", c))
        got.append(g)
    real = np.abs(got[0] ** 2 + got[1] ** 2 + got[2] ** 2 - vt).max()
    assert real <= info["tau_est"]
    if met:
        assert info["tau_est"] <= tau


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_qoi_vtotal_matches_oracle(mdr, ctx, dtype):
    sizes = [8, 56, 448, 3584, 28672]
    raw, orc, gpu, vt = _setup(mdr, ctx, 4, sizes, dtype, B=32 if dtype == np.float32 else 48)
    rng_q = float(vt.max() - vt.min())
    for rel in (1e-1, 1e-3, 1e-5, 1e-9):
        tau = rel * rng_q
        say("qoi case dtype", dtype, "rel", rel)
        ref = oracle.retrieve_qoi_vtotal(orc, tau)
        rts = [mdr.Retriever(ctx, g) for g in gpu]
        outs3 = [gpu_outputs(levels) for levels in raw]
        info = mdr.retrieve_qoi_vtotal(*rts, tau, outs3)
        _check(mdr, raw, rts, outs3, info, ref, vt, tau)


def test_qoi_incremental_and_mape_threshold(mdr, ctx):
    sizes = [8, 56, 448, 3584]
    raw, orc, gpu, vt = _setup(mdr, ctx, 7, sizes)
    rng_q = float(vt.max() - vt.min())
    rts = [mdr.Retriever(ctx, g) for g in gpu]
    outs3 = [gpu_outputs(levels) for levels in raw]
    k_prev = None
    for rel in (1e-1, 1e-2, 1e-4):
        tau = rel * rng_q
        ref = oracle.retrieve_qoi_vtotal(orc, tau, k_in=k_prev)
        info = mdr.retrieve_qoi_vtotal(*rts, tau, outs3)
        _check(mdr, raw, rts, outs3, info, ref, vt, tau)
        k_prev = ref[1]
    for c_mape in (1.5, 2.0, 100.0):
        tau = 1e-3 * rng_q
        ref = oracle.retrieve_qoi_vtotal(orc, tau, c=c_mape)
        rts2 = [mdr.Retriever(ctx, g) for g in gpu]
        outs = [gpu_outputs(levels) for levels in raw]
        info = mdr.retrieve_qoi_vtotal(*rts2, tau, outs, mape_c=c_mape)
        _check(mdr, raw, rts2, outs, info, ref, vt, tau)


@pytest.mark.parametrize("estimator,decay", [("ma", 0.5), ("cp", 0.5), ("cp", 0.25), ("cp", 0.9)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_qoi_estimators_match_oracle(mdr, ctx, estimator, decay, dtype):
    """MA and CP (Sec. 5.2) against the oracle: same planes, estimate, rounds
    and reconstructions, fresh and incremental."""
    sizes = [8, 56, 448, 3584, 28672]
    raw, orc, gpu, vt = _setup(mdr, ctx, 11, sizes, dtype, B=32 if dtype == np.float32 else 48)
    rng_q = float(vt.max() - vt.min())
    rts = [mdr.Retriever(ctx, g) for g in gpu]
    outs3 = [gpu_outputs(levels) for levels in raw]
    k_prev = None
    for rel in (1e-1, 1e-3, 1e-5, 1e-9):
        tau = rel * rng_q
        say("qoi estimator", estimator, decay, dtype, "rel", rel)
        ref = oracle.retrieve_qoi_vtotal(orc, tau, estimator=estimator, decay=decay)
        fresh = [mdr.Retriever(ctx, g) for g in gpu]
        outs = [gpu_outputs(levels) for levels in raw]
        info = mdr.retrieve_qoi_vtotal(*fresh, tau, outs, estimator=estimator, cp_decay=decay)
        _check(mdr, raw, fresh, outs, info, ref, vt, tau)
        ref_inc = oracle.retrieve_qoi_vtotal(orc, tau, k_in=k_prev, estimator=estimator, decay=decay)
        info = mdr.retrieve_qoi_vtotal(*rts, tau, outs3, estimator=estimator, cp_decay=decay)
        _check(mdr, raw, rts, outs3, info, ref_inc, vt, tau)
        k_prev = ref_inc[1]


def test_qoi_cp_worst_point_ties(mdr, ctx):
    """Exact copies of the point that dominates every estimate, planted at three
    places of the finest level: CP must work on the first of them."""
    sizes = [8, 56, 448, 3584]
    rng = np.random.default_rng(12)
    raw = [workloads.laplace_levels(sizes, 1.0, rng, np.float32) for _ in range(3)]
    for c in range(3):
        big = np.float32(2.0 * max(float(np.abs(a).max()) for a in raw[c]))
        for at in (100, 1700, 3000):
            raw[c][-1][at] = -big if c == 1 else big
    op = oracle.Params()
    orc = [oracle.refactor(levels, 32, op) for levels in raw]
    gpu = [mdr.refactor(ctx, upload(levels), 32, mdr.default_params()) for levels in raw]
    orig = [np.concatenate([a.astype(np.float64) for a in levels]) for levels in raw]
    vt = orig[0] ** 2 + orig[1] ** 2 + orig[2] ** 2
    rng_q = float(vt.max() - vt.min())
    for rel in (1e-2, 1e-4, 1e-6):
        tau = rel * rng_q
        ref = oracle.retrieve_qoi_vtotal(orc, tau, estimator="cp")
        rts = [mdr.Retriever(ctx, g) for g in gpu]
        outs = [gpu_outputs(levels) for levels in raw]
        info = mdr.retrieve_qoi_vtotal(*rts, tau, outs, estimator="cp")
        _check(mdr, raw, rts, outs, info, ref, vt, tau)


def test_qoi_rejects_bad_estimator(mdr, ctx):
    a = mdr.refactor(ctx, upload([np.ones(100, np.float32)]), 32)
    rts = [mdr.Retriever(ctx, a) for _ in range(3)]
    outs = [gpu_outputs([np.ones(100, np.float32)]) for _ in range(3)]
    with pytest.raises(mdr.MdrError) as ei:
        mdr.retrieve_qoi_vtotal(*rts, 1.0, outs, estimator="cp", cp_decay=1.5)
    assert ei.value.status == mdr.MDR_ERR_INVALID_ARG


def test_qoi_rejects_mismatched_fields(mdr, ctx):
    a = mdr.refactor(ctx, upload([np.ones(100, np.float32)]), 32)
    b = mdr.refactor(ctx, upload([np.ones(101, np.float32)]), 32)
    ra, rb = mdr.Retriever(ctx, a), mdr.Retriever(ctx, b)
    outs = [gpu_outputs([np.ones(100, np.float32)]) for _ in range(3)]
    with pytest.raises(mdr.MdrError) as ei:
        mdr.retrieve_qoi_vtotal(ra, rb, ra, 1.0, outs)
    assert ei.value.status == mdr.MDR_ERR_INVALID_ARG
