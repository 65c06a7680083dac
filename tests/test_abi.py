"""CPU checks of the C-ABI boundary: the library loads, exports every function
that include/mdr.h declares, the binding exposes them under the same names, and
host-side argument validation answers without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mdr_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["mdr_refactor", "mdr_retrieve", "mdr_retrieve_planes", "mdr_serialize",
                 "mdr_deserialize", "mdr_retriever_create", "mdr_context_create"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2505_00227_amd as mdr
    lib = C.CDLL(mdr.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert hasattr(mdr, name), name  # the binding keeps the C names


def test_host_side_validation_without_gpu():
    import paper_2505_00227_amd as mdr
    p = mdr.default_params()
    assert (p.group_planes, p.t_cr_milli, p.t_s_bytes, p.huf_chunk, p.huf_lmax, p.force_method) == \
        (4, 2000, 4096, 256, 12, -1)
    out = C.c_void_p()
    views = (mdr.mdr_level_view * 1)()
    st = mdr.mdr_refactor(None, views, 1, mdr.MDR_F32, 32, None, None, C.byref(out))
    assert st == mdr.MDR_ERR_INVALID_ARG and out.value is None
    assert b"ctx" in mdr.mdr_last_error()
    used = C.c_uint64()
    assert mdr.mdr_serialize(None, None, 0, C.byref(used)) == mdr.MDR_ERR_INVALID_ARG
    assert mdr.mdr_deserialize(None, None, 0, C.byref(out)) == mdr.MDR_ERR_INVALID_ARG
    assert mdr.version().startswith("mdr")


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib.util
    import shutil
    pkg = tmp_path / "paper_2505_00227_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_2505_00227_amd", "__init__.py"), pkg / "__init__.py")
    spec = importlib.util.spec_from_file_location("mdr_nolib", pkg / "__init__.py")
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


def test_ablation_host_side_without_gpu():
    import paper_2505_00227_amd as mdr
    assert [mdr.ablation_plane_words("locality", n) for n in (0, 1, 32, 33)] == [0, 1, 1, 2]
    assert [mdr.ablation_plane_words("regblock", n) for n in (0, 1, 2048, 2049)] == [0, 64, 64, 128]
    assert mdr.mdr_ablation_plane_words(9, 100) == 0
    assert mdr.mdr_ablation_encode(9, None, 100, None, None) == mdr.MDR_ERR_INVALID_ARG
    assert mdr.mdr_ablation_encode(0, None, 0, None, None) == mdr.MDR_OK  # nothing to do
    assert mdr.mdr_ablation_decode(4, None, 10, None, None) == mdr.MDR_ERR_INVALID_ARG


def test_qoi_estimator_validation_without_gpu():
    import paper_2505_00227_amd as mdr
    prm = mdr.mdr_qoi_params()
    prm.estimator = 7
    info = mdr.mdr_qoi_info()
    st = mdr.mdr_retrieve_qoi_vtotal_with(None, None, None, mdr.MDR_ABS, 1.0, C.byref(prm), None, None, None,
                                          None, C.byref(info))
    assert st == mdr.MDR_ERR_INVALID_ARG and b"estimator" in mdr.mdr_last_error()
    prm.estimator = mdr.MDR_QOI_CP
    prm.cp_decay = 1.0
    st = mdr.mdr_retrieve_qoi_vtotal_with(None, None, None, mdr.MDR_ABS, 1.0, C.byref(prm), None, None, None,
                                          None, C.byref(info))
    assert st == mdr.MDR_ERR_INVALID_ARG and b"cp_decay" in mdr.mdr_last_error()


def test_multilevel_host_side_without_gpu():
    import paper_2505_00227_amd as mdr
    from oracle import multilevel as ml
    for shape, nsteps in [((512, 512, 512), 8), ((7, 10, 13), 3), ((1, 1, 6), 2), ((0, 4, 4), 1),
                          ((3, 3, 3), 30), ((32, 1024, 1024), 8)]:
        assert mdr.level_sizes(shape, nsteps) == ml.level_sizes(shape, nsteps), (shape, nsteps)
    sizes = (C.c_uint64 * 32)()
    assert mdr.mdr_level_sizes(4, 4, 4, 31, sizes) == mdr.MDR_ERR_INVALID_ARG
    assert mdr.mdr_level_sizes(4, 4, 4, 2, None) == mdr.MDR_ERR_INVALID_ARG
    fake, other = C.c_void_p(1 << 20), C.c_void_p(1 << 30)
    for fn in (mdr.mdr_decompose, mdr.mdr_recompose):
        assert fn(mdr.MDR_F32, fake, 4, 4, 4, 31, other, None) == mdr.MDR_ERR_INVALID_ARG
        assert fn(mdr.MDR_F32, fake, 70000, 4, 4, 2, other, None) == mdr.MDR_ERR_UNSUPPORTED
        assert fn(mdr.MDR_F32, fake, 4, 70000, 4, 2, other, None) == mdr.MDR_ERR_UNSUPPORTED
        assert fn(7, fake, 4, 4, 4, 2, other, None) == mdr.MDR_ERR_INVALID_ARG
        assert fn(mdr.MDR_F32, None, 4, 4, 4, 2, other, None) == mdr.MDR_ERR_INVALID_ARG
        assert fn(mdr.MDR_F64, C.c_void_p((1 << 20) + 4), 4, 4, 4, 2, other, None) == mdr.MDR_ERR_INVALID_ARG
        # 64 values of 4 bytes from 1 MiB overlap a buffer starting 128 bytes later
        assert fn(mdr.MDR_F32, fake, 4, 4, 4, 2, C.c_void_p((1 << 20) + 128), None) == mdr.MDR_ERR_INVALID_ARG
        assert b"overlap" in mdr.mdr_last_error()
        assert fn(mdr.MDR_F32, None, 0, 4, 4, 2, None, None) == mdr.MDR_OK  # empty grid: no-op
