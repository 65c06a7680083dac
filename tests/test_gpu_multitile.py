"""GPU parity where one encoder workgroup walks several tiles.

The encoder splits a pass's tiles (8192 values each) evenly over a target
number of workgroups, so large levels give each workgroup a contiguous range of
tiles.  Several pieces of state then live across tiles inside a workgroup: the
running maxima of the exact error keys (read without a barrier at the top of a
tile), the neighbour words that count run transitions at tile edges (fast and
general paths), and the staged rows of the general path.  These tests force
many tiles per workgroup by lowering the workgroup target, on inputs built to
stress each piece (long runs of ones in the significands, constant stretches
that cross tiles), and compare every table, method, stream and reconstruction
with the oracle (Alg. 1 in Sec. 3, Alg. 2 in Sec. 4.2).  The last two tests
run the 512^3 float32 field and one float64 slab of the 1024^3 field at full
size, with the launch shape the library picks by itself."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import (assert_same_bits, compare_refactor, gpu_outputs, host, say,
                      to_oracle_params, upload)

pytestmark = pytest.mark.gpu

TILE_VALUES = 8192


@pytest.fixture(scope="module")
def mdr():
    import paper_2505_00227_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mdr):
    c = mdr.Context(0)
    yield c
    c.set_launch(enc_target_wg=2304, stats_wg_values=65536, graphs=1)
    c.close()


def _tiles(levels):
    return sum(-(-a.size // TILE_VALUES) for a in levels)


def _check(mdr, ctx, levels, B, params, target, ks):
    ctx.set_launch(enc_target_wg=target, graphs=0)
    tiles = _tiles(levels)
    say("multitile case: sizes", [a.size for a in levels], levels[0].dtype, "B", B, "m",
        params.group_planes, "force", params.force_method, "target wg", target,
        "tiles per wg", -(-tiles // target))
    assert -(-tiles // target) > 1
    dev = upload(levels)
    r = mdr.refactor(ctx, dev, B, params)
    op = to_oracle_params(params)
    orc = oracle.refactor(levels, B, op)
    compare_refactor(r, orc)
    assert r.serialize() == oracle.serialize(orc, op)
    rt = mdr.Retriever(ctx, r)
    outs = gpu_outputs(levels)
    m = min(params.group_planes, B)
    for k in ks:
        kl = min(B, -(-k // m) * m)
        rt.retrieve_planes([kl] * len(levels), outs)
        for l, ol in enumerate(orc):
            assert_same_bits(host(outs[l]), ol.reconstruct(kl), ("level", l, "k", kl))


# the library takes at least 64 encoder workgroups, so the inputs grow instead:
# 8.4 M values over 64 workgroups is 17 tiles each, 1.2 M values over 100 is 2
@pytest.mark.parametrize("n,target", [(1_200_000, 100), (1_200_000, 64), (8_400_000, 64)])
def test_fast_path_f32_laplace(mdr, ctx, n, target):
    """B = 32, m = 4 (the encoder's register fast path)."""
    x = workloads.plain_level(seed=100 + target + n % 7, n=n)
    _check(mdr, ctx, [x], 32, mdr.default_params(group_planes=4), target, [4, 16, 32])


@pytest.mark.parametrize("n", [1_100_003, 8_000_001])
def test_fast_path_f32_runs_of_ones(mdr, ctx, n):
    x = workloads.ones_runs_level(seed=110 + n % 13, n=n)
    _check(mdr, ctx, [x], 32, mdr.default_params(group_planes=4), 64, [4, 12, 24, 32])


@pytest.mark.parametrize("force", [-1, 1, 2])
def test_fast_path_f32_constant_stretches(mdr, ctx, force):
    x = workloads.piecewise_constant_level(seed=120 + force, n=1_310_720 + 77)
    _check(mdr, ctx, [x], 32, mdr.default_params(group_planes=4, force_method=force), 64, [4, 32])


@pytest.mark.parametrize("m", [1, 3])
def test_general_path_f32(mdr, ctx, m):
    """Group sizes other than 4 take the encoder's general (LDS-staged) path."""
    x = workloads.plain_level(seed=130 + m, n=1_048_576 + 4099)
    _check(mdr, ctx, [x], 32, mdr.default_params(group_planes=m), 64, [1, 3, 9, 32])
    y = workloads.ones_runs_level(seed=135 + m, n=6_000_001)
    _check(mdr, ctx, [y], 32, mdr.default_params(group_planes=m), 64, [3, 15, 32])


def test_general_path_f32_rle_across_tiles(mdr, ctx):
    x = workloads.piecewise_constant_level(seed=140, n=1_048_576 + 12345)
    _check(mdr, ctx, [x], 32, mdr.default_params(group_planes=3, force_method=1), 64, [3, 32])
    _check(mdr, ctx, [x], 32, mdr.default_params(group_planes=1), 100, [1, 32])


def test_general_path_fewer_planes(mdr, ctx):
    x = workloads.ones_runs_level(seed=145, n=1_200_000)
    _check(mdr, ctx, [x], 27, mdr.default_params(group_planes=4), 64, [4, 20, 27])


@pytest.mark.parametrize("n", [2_100_000, 6_000_000])
def test_f64_multitile(mdr, ctx, n):
    """float64, B = 64: Laplace and runs of ones."""
    x = workloads.plain_level(seed=150 + n % 11, n=n, dtype=np.float64)
    _check(mdr, ctx, [x], 64, mdr.default_params(group_planes=4), 64, [4, 32, 64])
    y = workloads.ones_runs_level(seed=155 + n % 11, n=n + 3, dtype=np.float64)
    _check(mdr, ctx, [y], 64, mdr.default_params(group_planes=4), 64, [8, 40, 64])


def test_f64_multitile_constant_stretches(mdr, ctx):
    x = workloads.piecewise_constant_level(seed=160, n=2_097_152 + 5, dtype=np.float64)
    for force in (-1, 1):
        _check(mdr, ctx, [x], 64, mdr.default_params(group_planes=4, force_method=force), 64, [4, 64])


def test_multilevel_multitile(mdr, ctx):
    """Several levels in one pass, each level's tiles spread over workgroups."""
    sizes = workloads.level_sizes((160, 160, 160), 6)
    levels = workloads.laplace_levels(sizes, 0.7, np.random.default_rng(170))
    levels[-1][::997] = workloads.ones_runs_level(171, levels[-1][::997].size)
    _check(mdr, ctx, levels, 32, mdr.default_params(group_planes=4), 64, [4, 16, 32])


def _full_size_case(mdr, ctx, levels, B, rels):
    ctx.set_launch(enc_target_wg=2304, stats_wg_values=65536, graphs=1)
    say("full-size case:", len(levels), "levels,", sum(a.size for a in levels), "values,",
        levels[0].dtype, "tiles", _tiles(levels))
    params = mdr.default_params(group_planes=4)
    op = to_oracle_params(params)
    dev = upload(levels)
    r = mdr.refactor(ctx, dev, B, params)
    orc = oracle.refactor(levels, B, op)
    compare_refactor(r, orc)
    say("  streams and tables equal")
    outs = gpu_outputs(levels)
    inc = mdr.Retriever(ctx, r)
    for rel in rels:
        vals, k, bound, met = oracle.retrieve_to(orc, rel)
        fresh = mdr.Retriever(ctx, r)
        info = fresh.retrieve(rel, outs)
        assert fresh.planes() == k and info["bound"] == bound and info["met"] == int(met)
        for l in range(len(levels)):
            assert_same_bits(host(outs[l]), vals[l], ("fresh", rel, l))
        info = inc.retrieve(rel, outs)
        assert inc.planes() == k and info["bound"] == bound
        for l in range(len(levels)):
            assert_same_bits(host(outs[l]), vals[l], ("incremental", rel, l))
        say("  rel", rel, "planes", k, "equal")
        del vals


@pytest.mark.timeout(900)
def test_field512_f32_full_size(mdr, ctx):
    """The 512^3 float32 field (9 Laplace levels, seed 2, 2^27 values) at full
    size: every stream and table, and retrievals at 1e-1 .. 1e-6, fresh and
    incremental, bit for bit."""
    levels = workloads.field_levels(seed=2)
    _full_size_case(mdr, ctx, levels, 32, [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6])


@pytest.mark.timeout(900)
def test_chunk_f64_full_size(mdr, ctx):
    """One 32x1024x1024 float64 slab of the 1024^3 field (2^25 values, 9
    levels, B = 64) at full size, through to the all-planes retrieval."""
    levels = workloads.chunk_levels(seed=3, chunk=5)
    _full_size_case(mdr, ctx, levels, 64, [1e-3, 1e-9, 0.0])
