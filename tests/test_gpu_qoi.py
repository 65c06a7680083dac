"""GPU parity of the V_total QoI retrieval (Sec. 5.2, Alg. 3 with MAPE) against
the oracle's loop: same planes per variable, same estimate (bit for bit), same
number of rounds, same reconstructions; and the paper's guarantee
real error <= estimate <= tolerance."""
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


def test_qoi_rejects_mismatched_fields(mdr, ctx):
    a = mdr.refactor(ctx, upload([np.ones(100, np.float32)]), 32)
    b = mdr.refactor(ctx, upload([np.ones(101, np.float32)]), 32)
    ra, rb = mdr.Retriever(ctx, a), mdr.Retriever(ctx, b)
    outs = [gpu_outputs([np.ones(100, np.float32)]) for _ in range(3)]
    with pytest.raises(mdr.MdrError) as ei:
        mdr.retrieve_qoi_vtotal(ra, rb, ra, 1.0, outs)
    assert ei.value.status == mdr.MDR_ERR_INVALID_ARG
