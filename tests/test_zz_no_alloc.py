"""The allocation-free table entry point (mdr_l2_table_noalloc) against the
allocating one (mdr_l2_table): same kernels, fixed summation order, so the
squared-L2 tables must be equal bit for bit; two calls in a row, the second on
a smaller input, and the level limit of its fixed scratch."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdr():
    import paper_2505_00227_amd as m
    return m


def _tables(mdr, ctx, xs, B, noalloc):
    import torch
    dev = [torch.from_numpy(x).cuda() for x in xs]
    r = mdr.refactor(ctx, dev, B)
    if noalloc:
        r.l2_table_noalloc(dev)
    else:
        r.l2_table(dev)
    t = [r.l2(l) for l in range(len(xs))]
    r.close()
    return t


@pytest.mark.parametrize("dtype,B", [(np.float32, 32), (np.float64, 64)])
def test_noalloc_tables_equal_allocating_ones(mdr, dtype, B):
    ctx = mdr.Context(0)
    rng = np.random.default_rng(31)
    big = [rng.laplace(0, 2.0 ** -l, n).astype(dtype) for l, n in enumerate([0, 7, 1000, 1 << 20, 3_000_017])]
    small = [rng.laplace(0, 3.0, n).astype(dtype) for n in [5, 4099]]
    for name, xs in (("larger", big), ("smaller", small)):
        say("noalloc", np.dtype(dtype).name, name, [x.size for x in xs])
        want = _tables(mdr, ctx, xs, B, False)
        got = _tables(mdr, ctx, xs, B, True)
        assert got == want, name
    # a call whose levels all fit, then one with more levels than the scratch holds
    rng2 = np.random.default_rng(32)
    many = [rng2.laplace(0, 1, 33).astype(dtype) for _ in range(64)]
    assert _tables(mdr, ctx, many, B, True) == _tables(mdr, ctx, many, B, False)
    with pytest.raises(mdr.MdrError) as ei:
        _tables(mdr, ctx, many + [many[0]], B, True)
    assert ei.value.status == mdr.MDR_ERR_UNSUPPORTED
    ctx.close()
