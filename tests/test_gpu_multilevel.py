"""Multilevel decomposition on the GPU (the coefficient levels of Sec. 2/3):
decomposition and recomposition match the oracle bit for bit in float32 and
float64, on grids with ragged workgroups, non-dyadic edges, empty levels and
the 512^3 field at full size; and a field taken through decompose -> refactor
-> retrieve -> recompose lands within the requested max error."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import say
from oracle import multilevel as ml

pytestmark = pytest.mark.gpu

CASES = [((33, 17, 70), 3), ((1, 1, 1000), 5), ((65, 129, 257), 6), ((20, 31, 300), 4), ((3, 3, 3), 6),
         ((9, 8, 7), 0), ((2, 600, 5), 7), ((1, 1, 1), 2), ((40, 1, 513), 9),
         # rows of whole 16-byte vectors: the finest step takes the vector kernel
         ((7, 9, 68), 3), ((6, 5, 4), 2), ((33, 18, 1024), 4), ((1, 3, 8), 1)]


@pytest.fixture(scope="module")
def mdr():
    import paper_2505_00227_amd as m
    return m


def _bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


def _decompose_gpu(mdr, u, nsteps):
    import torch
    f = torch.from_numpy(u).cuda()
    out = torch.full((u.size,), float("nan"), dtype=f.dtype, device="cuda")  # every value must be written
    mdr.decompose(f, nsteps, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _recompose_gpu(mdr, coeffs, shape, nsteps):
    import torch
    c = torch.from_numpy(np.ascontiguousarray(coeffs)).cuda()
    out = torch.full(tuple(shape), float("nan"), dtype=c.dtype, device="cuda")
    mdr.recompose(c, nsteps, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape,nsteps", CASES)
def test_decompose_and_recompose_match_oracle(mdr, dtype, shape, nsteps):
    say("multilevel", np.dtype(dtype).name, shape, "nsteps", nsteps)
    u = workloads.smooth_field(11, shape, dtype)
    assert mdr.level_sizes(shape, nsteps) == ml.level_sizes(shape, nsteps)
    want = ml.concat(ml.decompose(u, nsteps))
    got = _decompose_gpu(mdr, u, nsteps)
    np.testing.assert_array_equal(_bits(got), _bits(want))
    # recomposition of arbitrary coefficients (not only a decomposition's)
    rng = np.random.default_rng(12)
    c = (want + rng.standard_normal(want.size) * 1e-3).astype(dtype)
    sizes = ml.level_sizes(shape, nsteps)
    ref = ml.recompose(np.split(c, np.cumsum(sizes)[:-1]), shape, nsteps)
    np.testing.assert_array_equal(_bits(_recompose_gpu(mdr, c, shape, nsteps)), _bits(ref))


def test_special_values_pass_through(mdr):
    shape, nsteps = (17, 9, 33), 3
    u = workloads.smooth_field(13, shape, np.float32)
    u[3, 4, 5] = np.inf
    u[8, 2, 31] = np.nan
    u[0, 0, 1] = -0.0
    u[16, 8, 32] = np.float32(1e-40)  # subnormal: not flushed
    want = ml.concat(ml.decompose(u, nsteps))
    np.testing.assert_array_equal(_bits(_decompose_gpu(mdr, u, nsteps)), _bits(want))


def test_unaligned_field_takes_the_general_step(mdr):
    import torch
    shape, nsteps = (9, 10, 64), 3
    u = workloads.smooth_field(15, shape, np.float32)
    buf = torch.zeros(u.size + 1, dtype=torch.float32, device="cuda")
    buf[1:] = torch.from_numpy(u.ravel()).cuda()
    field = buf[1:].view(shape)  # 4 bytes past a 16-byte boundary
    out = torch.full((u.size,), float("nan"), dtype=torch.float32, device="cuda")
    mdr.decompose(field, nsteps, out)
    want = ml.concat(ml.decompose(u, nsteps))
    np.testing.assert_array_equal(_bits(out.cpu().numpy()), _bits(want))
    back = torch.zeros(u.size + 1, dtype=torch.float32, device="cuda")
    mdr.recompose(out, nsteps, back[1:].view(shape))
    np.testing.assert_array_equal(_bits(back[1:].cpu().numpy()), _bits(ml.recompose(ml.decompose(u, nsteps), shape, nsteps).ravel()))


def test_bad_buffers_are_rejected(mdr):
    import torch
    shape = (9, 10, 64)
    n = 9 * 10 * 64
    field = torch.zeros(shape, dtype=torch.float32, device="cuda")
    short = torch.zeros(n - 1, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        mdr.decompose(field, 3, short)                     # size
    with pytest.raises(ValueError):
        mdr.decompose(field, 3, torch.zeros(n, dtype=torch.float32))  # host tensor
    with pytest.raises(ValueError):
        mdr.decompose(field, 3, torch.zeros(2 * n, dtype=torch.float32, device="cuda")[::2])  # strided
    # through the C ABI: a host buffer, and a device buffer too small for the grid
    import ctypes as C
    host = torch.zeros(n, dtype=torch.float32).numpy()
    st = mdr.mdr_decompose(mdr.MDR_F32, C.c_void_p(field.data_ptr()), 9, 10, 64, 3,
                           C.c_void_p(host.ctypes.data), None)
    assert st == mdr.MDR_ERR_INVALID_ARG and b"device memory" in mdr.mdr_last_error()
    small = torch.cuda.caching_allocator_alloc(1 << 10)  # its own small block
    try:
        st = mdr.mdr_recompose(mdr.MDR_F32, C.c_void_p(small), 90, 100, 640, 3,
                               C.c_void_p(field.data_ptr()), None)
        assert st == mdr.MDR_ERR_INVALID_ARG
    finally:
        torch.cuda.caching_allocator_delete(small)


def test_full_size_field(mdr):
    shape, nsteps = (512, 512, 512), 8
    say("multilevel full size", shape)
    u = workloads.smooth_field(2, shape, np.float32)
    want = ml.decompose(u, nsteps)
    got = _decompose_gpu(mdr, u, nsteps)
    np.testing.assert_array_equal(_bits(got), _bits(ml.concat(want)))
    back = _recompose_gpu(mdr, got, shape, nsteps)
    np.testing.assert_array_equal(_bits(back), _bits(ml.recompose(want, shape, nsteps)))


@pytest.mark.parametrize("dtype,rel", [(np.float32, 1e-2), (np.float32, 1e-4), (np.float64, 1e-7)])
def test_field_through_the_path_meets_tolerance(mdr, orc, dtype, rel):
    import torch
    shape, nsteps, B = (65, 97, 132), 5, 32 if dtype == np.float32 else 64
    say("multilevel path", np.dtype(dtype).name, "rel", rel)
    u = workloads.smooth_field(14, shape, dtype)
    tol = rel * float(u.max() - u.min())
    sizes = ml.level_sizes(shape, nsteps)
    ctx = mdr.Context(0)
    coeffs = torch.empty(u.size, dtype=torch.float32 if dtype == np.float32 else torch.float64, device="cuda")
    mdr.decompose(torch.from_numpy(u).cuda(), nsteps, coeffs)
    levels = list(torch.split(coeffs, sizes))
    r = mdr.refactor(ctx, levels, B)
    rt = mdr.Retriever(ctx, r)
    outs = [torch.empty_like(x) for x in levels]
    info = rt.retrieve(tol, outs, relative=False)
    assert info["bound"] <= tol
    field = torch.empty(shape, dtype=coeffs.dtype, device="cuda")
    mdr.recompose(torch.cat(outs), nsteps, field)
    got = field.cpu().numpy()
    # the oracle's chain gives the same field bit for bit
    olv = orc.refactor(ml.decompose(u, nsteps), B)
    rec, k, bound, ok = orc.retrieve_to(olv, tol, relative=False)
    assert ok and list(k) == list(rt.planes())
    want = ml.recompose(rec, shape, nsteps)
    np.testing.assert_array_equal(_bits(got), _bits(want))
    # field max error: the levels' bound plus recomposition rounding
    slack = 4 * nsteps * np.finfo(dtype).eps * float(np.abs(u).max())
    assert np.abs(got.astype(np.float64) - u).max() <= tol + slack
    rt.close()
    r.close()
    ctx.close()
