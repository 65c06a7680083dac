"""GPU parity of the Huffman decoders (Sec. 4.2's chunked codes): one thread a
chunk, and G = 4..64 lanes a chunk brought into step by resynchronisation.
Every lane count must give the oracle's reconstructions bit for bit, over
skewed, spread and single-symbol byte distributions, ragged last chunks,
chunks of 256..4096 symbols and code-length limits of 8..12 bits."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_same_bits, compare_refactor, gpu_outputs, host, say, to_oracle_params, upload

pytestmark = pytest.mark.gpu

LANES = [1, 4, 8, 16, 32, 64, 0]


@pytest.fixture(scope="module")
def mdr():
    import paper_2505_00227_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mdr):
    c = mdr.Context(0)
    yield c
    c.set_decode_lanes(0)
    c.close()


def _check(mdr, ctx, levels, B, params, ks):
    r = mdr.refactor(ctx, upload(levels), B, params)
    orc = oracle.refactor(levels, B, to_oracle_params(params))
    compare_refactor(r, orc)
    m = params.group_planes
    refs = {}
    for lanes in LANES:
        ctx.set_decode_lanes(lanes)
        rt = mdr.Retriever(ctx, r)
        outs = gpu_outputs(levels)
        for k in ks:
            say("huffman lanes", lanes, "levels", [a.size for a in levels], np.dtype(levels[0].dtype).name,
                "chunk", params.huf_chunk, "lmax", params.huf_lmax, "k", k)
            rt.retrieve_planes([k] * len(levels), outs)
            for l, ol in enumerate(orc):
                kl = min(B, (k + m - 1) // m * m)
                if (l, kl) not in refs:
                    refs[(l, kl)] = ol.reconstruct(kl)
                assert_same_bits(host(outs[l]), refs[(l, kl)], ("lanes", lanes, "level", l, "k", kl))
    ctx.set_decode_lanes(0)


@pytest.mark.parametrize("chunk,lmax", [(256, 12), (256, 8), (1024, 10), (4096, 12)])
def test_lanes_forced_huffman_f32(mdr, ctx, chunk, lmax):
    x = workloads.plain_level(seed=80 + lmax, n=300_000)  # a ragged last chunk for every chunk size
    p = mdr.default_params(group_planes=4, huf_chunk=chunk, huf_lmax=lmax, force_method=2)
    _check(mdr, ctx, [x], 32, p, [4, 12, 20, 32])


def test_lanes_selected_methods_multilevel(mdr, ctx):
    rng = np.random.default_rng(81)
    levels = workloads.laplace_levels([8, 56, 448, 3584, 28672, 229376], 1.0, rng)
    _check(mdr, ctx, levels, 32, mdr.default_params(group_planes=4), [0, 8, 16, 32])


def test_lanes_f64(mdr, ctx):
    x = workloads.plain_level(seed=82, n=70_001, dtype=np.float64)
    p = mdr.default_params(group_planes=8, force_method=2)
    _check(mdr, ctx, [x], 64, p, [8, 32, 64])


def test_lanes_runs_and_constant_pieces(mdr, ctx):
    """Planes of long runs and of one repeated byte: single-symbol and two-symbol
    codebooks, where every code is one bit long."""
    for x in (workloads.ones_runs_level(seed=83, n=200_000), workloads.piecewise_constant_level(seed=84, n=200_000)):
        _check(mdr, ctx, [x], 32, mdr.default_params(group_planes=2, force_method=2), [2, 10, 32])


def test_lanes_tiny_units(mdr, ctx):
    """Units of a few chunks and of less than one chunk."""
    for n in (1, 31, 2049, 8193):
        x = workloads.plain_level(seed=85 + n, n=n)
        _check(mdr, ctx, [x], 32, mdr.default_params(group_planes=1, force_method=2), [1, 5, 32])


def test_lanes_argument_check(mdr, ctx):
    for bad in (2, 3, 5, 128):
        with pytest.raises(mdr.MdrError) as ei:
            ctx.set_decode_lanes(bad)
        assert ei.value.status == mdr.MDR_ERR_INVALID_ARG
