"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for bit.

Streams, methods, sizes, exponents, error tables and reconstructions are integer
or exact work, so the bar is equality of bytes everywhere."""
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


def run_case(mdr, ctx, levels_np, B, params, ks=None, check_streams=True):
    say("case: levels", [a.size for a in levels_np], "dtype", levels_np[0].dtype, "B", B,
        "m", params.group_planes, "force", params.force_method, "t_cr", params.t_cr_milli)
    dev = upload(levels_np)
    r = mdr.refactor(ctx, dev, B, params)
    orc = oracle.refactor(levels_np, B, to_oracle_params(params))
    compare_refactor(r, orc, check_streams)
    rt = mdr.Retriever(ctx, r)
    outs = gpu_outputs(levels_np)
    m = min(params.group_planes, B)
    if ks is None:
        ks = sorted(set([0, m, min(B, 2 * m), B]))
    for k in ks:
        kk = [k] * len(levels_np)
        rt.retrieve_planes(kk, outs)
        for l, ol in enumerate(orc):
            kl = max(min(B, (k + m - 1) // m * m), 0)
            ref = ol.reconstruct(kl)
            assert_same_bits(host(outs[l]), ref, ("level", l, "k", kl))
    return r, orc


# ------------------------------------------------------------------ single level, f32
@pytest.mark.parametrize("n", [1, 31, 32, 33, 1000, 8192, 8193, 70001, 1 << 16])
def test_plain_f32_ragged(mdr, ctx, n):
    x = workloads.plain_level(seed=n, n=n)
    run_case(mdr, ctx, [x], 32, mdr.default_params(group_planes=1), ks=[0, 1, 3, 10, 20, 32])


@pytest.mark.parametrize("m", [1, 3, 4, 32])
def test_group_sizes(mdr, ctx, m):
    x = workloads.plain_level(seed=10 + m, n=50000)
    run_case(mdr, ctx, [x], 32, mdr.default_params(group_planes=m))


@pytest.mark.parametrize("B", [1, 7, 16, 24, 31])
def test_fewer_planes(mdr, ctx, B):
    x = workloads.plain_level(seed=20 + B, n=40000)
    run_case(mdr, ctx, [x], B, mdr.default_params(group_planes=4))


@pytest.mark.parametrize("force", [0, 1, 2])
def test_forced_methods(mdr, ctx, force):
    x = workloads.plain_level(seed=30 + force, n=123457)
    run_case(mdr, ctx, [x], 32, mdr.default_params(group_planes=4, force_method=force))


@pytest.mark.parametrize("t_cr", [1000, 2000, 4000])
def test_ratio_thresholds(mdr, ctx, t_cr):
    x = workloads.plain_level(seed=40, n=200000)
    run_case(mdr, ctx, [x], 32, mdr.default_params(group_planes=4, t_cr_milli=t_cr))


@pytest.mark.parametrize("chunk,lmax", [(256, 8), (512, 10), (2048, 11), (4096, 12)])
def test_huffman_params(mdr, ctx, chunk, lmax):
    x = workloads.plain_level(seed=50, n=100000)
    run_case(mdr, ctx, [x], 32, mdr.default_params(group_planes=2, huf_chunk=chunk, huf_lmax=lmax,
                                                   force_method=2))


@pytest.mark.parametrize("chunk", [128, 768, 3840, 8192])
def test_huffman_chunk_not_power_of_two_rejected(mdr, ctx, chunk):
    x = workloads.plain_level(seed=51, n=10000)
    with pytest.raises(mdr.MdrError) as ei:
        mdr.refactor(ctx, upload([x]), 32, mdr.default_params(huf_chunk=chunk))
    assert ei.value.status == mdr.MDR_ERR_UNSUPPORTED


def test_special_values(mdr, ctx):
    rng = np.random.default_rng(3)
    x = rng.laplace(0, 1, 5000).astype(np.float32)
    x[:12] = [0.0, -0.0, 1e-45, -1e-45, 1.17e-38, 3e-39, -2.5e-42, np.finfo(np.float32).max,
              -np.finfo(np.float32).max, 2.0 ** -149, 0.5, -0.25]
    run_case(mdr, ctx, [x], 32, mdr.default_params(group_planes=4))
    sub = (rng.standard_normal(3000) * 1e-41).astype(np.float32)  # subnormal-only level
    run_case(mdr, ctx, [sub], 32, mdr.default_params(group_planes=4))
    run_case(mdr, ctx, [np.zeros(777, np.float32)], 32, mdr.default_params())
    run_case(mdr, ctx, [np.full(100000, -0.0, np.float32)], 32, mdr.default_params())
    big = np.array([1e30, -3e37, 1e-30, 2.0], np.float32)
    run_case(mdr, ctx, [big], 32, mdr.default_params(group_planes=1), ks=list(range(33)))


# ------------------------------------------------------------------ f64
@pytest.mark.parametrize("n,B", [(1, 64), (63, 64), (64, 64), (65, 64), (10000, 64), (33333, 40),
                                 (4097, 53)])
def test_f64(mdr, ctx, n, B):
    x = workloads.plain_level(seed=n + B, n=n, dtype=np.float64)
    run_case(mdr, ctx, [x], B, mdr.default_params(group_planes=4),
             ks=sorted(set(k for k in [0, 4, 16, 32, 48, B] if k <= B)))


def test_f64_special_and_forced(mdr, ctx):
    rng = np.random.default_rng(5)
    x = rng.laplace(0, 1, 20000)
    x[:8] = [0.0, -0.0, 5e-324, -1e-310, 1e-300, 1e300, -2.0 ** -1074, 0.75]
    for force in (0, 1, 2):
        run_case(mdr, ctx, [x], 64, mdr.default_params(group_planes=8, force_method=force))


# ------------------------------------------------------------------ multilevel, tolerance
def test_multilevel_tolerances_and_incremental(mdr, ctx):
    sizes = workloads.level_sizes((64, 64, 64), 6)
    rng = np.random.default_rng(2)
    levels = workloads.laplace_levels(sizes, 0.38, rng)
    params = mdr.default_params(group_planes=4)
    r, orc = run_case(mdr, ctx, levels, 32, params, ks=[0, 32])
    outs = gpu_outputs(levels)
    inc = mdr.Retriever(ctx, r)
    # 1e-13 and 0 lie below what every plane reaches (1e-9 near it): the
    # planner's shortcut to every plane must give the greedy's planes and bound
    for rel in [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-9, 1e-13, 0.0]:
        vals, k, bound, met = oracle.retrieve_to(orc, rel)
        fresh = mdr.Retriever(ctx, r)
        info = fresh.retrieve(rel, outs)
        assert fresh.planes() == k and info["bound"] == bound and info["met"] == int(met)
        for l in range(len(levels)):
            assert_same_bits(host(outs[l]), vals[l], ("fresh", rel, l))
        info2 = inc.retrieve(rel, outs)  # incremental from the previous tolerance
        assert inc.planes() == k and info2["bound"] == bound
        for l in range(len(levels)):
            assert_same_bits(host(outs[l]), vals[l], ("incremental", rel, l))


# ------------------------------------------------------------------ errors and container
def test_nonfinite_rejected(mdr, ctx):
    for bad in (np.nan, np.inf, -np.inf):
        x = np.ones(1000, np.float32)
        x[777] = bad
        with pytest.raises(mdr.MdrError) as ei:
            mdr.refactor(ctx, upload([x]), 32)
        assert ei.value.status == mdr.MDR_ERR_INVALID_ARG


def test_serialize_matches_oracle_and_roundtrips(mdr, ctx):
    sizes = [8, 56, 448, 3584, 28672]
    rng = np.random.default_rng(9)
    levels = workloads.laplace_levels(sizes, 1.0, rng)
    params = mdr.default_params(group_planes=4)
    r = mdr.refactor(ctx, upload(levels), 32, params)
    orc = oracle.refactor(levels, 32, to_oracle_params(params))
    blob = r.serialize()
    assert blob == oracle.serialize(orc, to_oracle_params(params))
    r2 = mdr.Refactored.deserialize(ctx, blob)
    assert r2.serialize() == blob
    compare_refactor(r2, orc)
    rt = mdr.Retriever(ctx, r2)
    outs = gpu_outputs(levels)
    rt.retrieve(1e-4, outs)
    vals, k, bound, met = oracle.retrieve_to(orc, 1e-4)
    for l in range(len(levels)):
        assert_same_bits(host(outs[l]), vals[l], ("deserialized", l))
    # corruption is detected before anything reaches the device
    for pos in (3, 50, 60, 200, len(blob) - 5):
        bad = bytearray(blob)
        bad[pos] ^= 0x10
        with pytest.raises(mdr.MdrError) as ei:
            mdr.Refactored.deserialize(ctx, bytes(bad))
        assert ei.value.status == mdr.MDR_ERR_CORRUPT_STREAM
    with pytest.raises(mdr.MdrError):
        mdr.Refactored.deserialize(ctx, blob[:-8])


def test_empty_level_and_run_twice_identical(mdr, ctx):
    levels = [np.zeros(0, np.float32), workloads.plain_level(1, 9999)]
    params = mdr.default_params(group_planes=4)
    run_case(mdr, ctx, levels, 32, params)
    for force in (1, 2):
        run_case(mdr, ctx, levels, 32, mdr.default_params(group_planes=4, force_method=force))
    # determinism: two refactors give the same serialized bytes
    a = mdr.refactor(ctx, upload(levels), 32, params).serialize()
    b = mdr.refactor(ctx, upload(levels), 32, params).serialize()
    assert a == b


@pytest.mark.parametrize("m", [1, 4])
def test_run_length_groups_in_one_pass(mdr, ctx, m):
    """Every run-length group of a retrieval decodes in one gather / scan /
    expand pass: groups of one run (constant planes), of long runs, and of
    words that change at every position, over several levels at once."""
    levels = [workloads.piecewise_constant_level(seed=90, n=70_000), workloads.ones_runs_level(seed=91, n=150_001),
              workloads.plain_level(seed=92, n=40_000)]
    run_case(mdr, ctx, levels, 32, mdr.default_params(group_planes=m, force_method=1), ks=[1, 4, 9, 32])
