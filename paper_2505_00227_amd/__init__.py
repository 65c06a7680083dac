"""Python binding of libmdr: bitplane refactor / progressive retrieve on MI355X.

Argument marshalling only: every step of the path runs in the HIP kernels of
``libmdr.so`` behind the C ABI declared in ``include/mdr.h``.  The raw ABI
functions are exposed under their C names (``mdr_refactor``, ``mdr_retrieve``,
...); ``Context`` / ``Refactored`` / ``Retriever`` wrap the handles for torch
tensors (device memory and streams come from PyTorch).

Importing fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

# torch ships its own HIP runtime whose SONAME equals the system one
# (libamdhip64.so.7).  Loading torch first makes libmdr.so bind to that same
# runtime, so one process has one HIP runtime: torch's tensors, streams and
# synchronizations and this library's launches share queues and state.
import torch  # noqa: E402,F401  (must precede the CDLL below)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdr.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libmdr.so is not built; run `python paper_2505_00227_amd/build.py` "
        "(or __graft_entry__.build()) first")

_lib = C.CDLL(LIB_PATH)

# ---------------------------------------------------------------- ABI types
MDR_OK, MDR_ERR_INVALID_ARG, MDR_ERR_UNSUPPORTED, MDR_ERR_OUT_OF_MEMORY = 0, 1, 2, 3
MDR_ERR_HIP, MDR_ERR_CORRUPT_STREAM, MDR_ERR_BUSY = 4, 5, 6
MDR_F32, MDR_F64 = 0, 1
MDR_DC, MDR_RLE, MDR_HUF, MDR_PLACEHOLDER = 0, 1, 2, 3
MDR_ABS, MDR_REL, MDR_L2 = 0, 1, 2
MDR_MAX_PLANES = 64
STAGES = ["stats", "encode", "select", "lossless", "assemble", "huf_decode", "rle_decode",
          "reconstruct"]
STATUS_NAMES = {0: "MDR_OK", 1: "MDR_ERR_INVALID_ARG", 2: "MDR_ERR_UNSUPPORTED",
                3: "MDR_ERR_OUT_OF_MEMORY", 4: "MDR_ERR_HIP", 5: "MDR_ERR_CORRUPT_STREAM",
                6: "MDR_ERR_BUSY"}


class mdr_codec_params(C.Structure):
    _fields_ = [("group_planes", C.c_uint32), ("t_cr_milli", C.c_uint32),
                ("t_s_bytes", C.c_uint64), ("huf_chunk", C.c_uint32), ("huf_lmax", C.c_uint32),
                ("force_method", C.c_int32)]


class mdr_level_view(C.Structure):
    _fields_ = [("data", C.c_void_p), ("n", C.c_uint64)]


class mdr_qoi_params(C.Structure):
    _fields_ = [("estimator", C.c_int32), ("pad", C.c_uint32), ("mape_c", C.c_double), ("cp_decay", C.c_double)]


MDR_QOI_MAPE, MDR_QOI_MA, MDR_QOI_CP = 0, 1, 2
QOI_ESTIMATORS = {"mape": MDR_QOI_MAPE, "ma": MDR_QOI_MA, "cp": MDR_QOI_CP}
QOI_FAMILIES = {"sumsq": 0, "magnitude": 1, "product": 2}


class mdr_qoi_info(C.Structure):
    _fields_ = [("tau_abs", C.c_double), ("tau_est", C.c_double), ("eps", C.c_double * 3),
                ("bytes_fetched", C.c_uint64), ("iterations", C.c_uint32), ("met", C.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["eps"] = list(self.eps)
        return d


class mdr_retrieve_info(C.Structure):
    _fields_ = [("tol_abs", C.c_double), ("bound", C.c_double), ("bytes_fetched", C.c_uint64),
                ("bytes_held", C.c_uint64), ("groups_fetched", C.c_uint32), ("met", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class mdr_request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("field", C.c_uint32 * 3), ("bound", C.c_int32),
                ("tol", C.c_double), ("mape_c", C.c_double), ("parent", C.c_uint64),
                ("tag", C.c_uint64)]


class mdr_completion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("tag", C.c_uint64), ("status", C.c_int32), ("met", C.c_int32),
                ("tol_abs", C.c_double), ("bound", C.c_double), ("bytes_fetched", C.c_uint64),
                ("iterations", C.c_uint32), ("pad", C.c_uint32), ("t_submit_ms", C.c_double),
                ("t_start_ms", C.c_double), ("t_done_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class mdr_server_info(C.Structure):
    _fields_ = [("pending", C.c_uint32), ("active", C.c_uint32), ("completed_unreleased", C.c_uint32),
                ("pad", C.c_uint32), ("steps", C.c_uint64), ("step_requests", C.c_uint64),
                ("hbm_in_use", C.c_uint64), ("hbm_budget", C.c_uint64), ("hbm_held", C.c_uint64)]


class mdr_launch_shape(C.Structure):
    _fields_ = [("enc_target_wg", C.c_uint32), ("stats_wg_values", C.c_uint32),
                ("select_threads", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class mdr_tune_result(C.Structure):
    _fields_ = [("best", mdr_launch_shape), ("dflt", mdr_launch_shape), ("best_ms", C.c_double),
                ("default_ms", C.c_double), ("candidates", C.c_uint32), ("value_bucket", C.c_uint32),
                ("level_bucket", C.c_uint32)]

    def as_dict(self):
        return {"best": self.best.as_dict(), "default": self.dflt.as_dict(), "best_ms": self.best_ms,
                "default_ms": self.default_ms, "candidates": self.candidates,
                "value_bucket": self.value_bucket, "level_bucket": self.level_bucket}


class mdr_pipeline_info(C.Structure):
    _fields_ = [("wall_ms", C.c_double), ("h2d_ms", C.c_double), ("compute_ms", C.c_double),
                ("d2h_ms", C.c_double), ("h2d_bytes", C.c_uint64), ("d2h_bytes", C.c_uint64),
                ("stream_bytes", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


MDR_REQ_FIELD, MDR_REQ_QOI_VTOTAL = 0, 1

_vp, _u32, _u64, _i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32
_P = C.POINTER
_SIGS = {
    "mdr_version": ([], C.c_char_p),
    "mdr_last_error": ([], C.c_char_p),
    "mdr_codec_params_default": ([_P(mdr_codec_params)], C.c_int),
    "mdr_context_create": ([C.c_int, _P(_vp)], C.c_int),
    "mdr_context_destroy": ([_vp], None),
    "mdr_context_set_timing": ([_vp, C.c_int], C.c_int),
    "mdr_context_timing": ([_vp, _P(C.c_double), _P(_u64), C.c_int], C.c_int),
    "mdr_refactor": ([_vp, _P(mdr_level_view), _u32, C.c_int, _u32, _P(mdr_codec_params), _vp,
                      _P(_vp)], C.c_int),
    "mdr_context_set_launch": ([_vp, _u32, _u32, C.c_int], C.c_int),
    "mdr_context_set_decode_lanes": ([_vp, _u32], C.c_int),
    "mdr_refactor_batch": ([_vp, _P(_P(mdr_level_view)), _P(_u32), _u32, C.c_int, _u32,
                            _P(mdr_codec_params), _vp, _P(_vp)], C.c_int),
    "mdr_refactored_destroy": ([_vp], None),
    "mdr_refactored_shape": ([_vp, _P(_u32), _P(C.c_int), _P(_u32), _P(mdr_codec_params)], C.c_int),
    "mdr_refactored_info": ([_vp, _u32, _P(_i32), _P(_u64), _P(C.c_double), _P(C.c_double),
                             _P(C.c_double)], C.c_int),
    "mdr_refactored_stream": ([_vp, _u32, _i32, _P(_vp), _P(_u64), _P(C.c_int)], C.c_int),
    "mdr_serialize": ([_vp, _vp, _u64, _P(_u64)], C.c_int),
    "mdr_deserialize": ([_vp, _vp, _u64, _P(_vp)], C.c_int),
    "mdr_retriever_create": ([_vp, _vp, _P(_vp)], C.c_int),
    "mdr_retriever_destroy": ([_vp], None),
    "mdr_retrieve": ([_vp, C.c_int, C.c_double, _P(_vp), _vp, _P(mdr_retrieve_info)], C.c_int),
    "mdr_retrieve_planes": ([_vp, _P(_u32), _P(_vp), _vp, _P(mdr_retrieve_info)], C.c_int),
    "mdr_retriever_planes": ([_vp, _P(_u32)], C.c_int),
    "mdr_retrieve_batch": ([_P(_vp), _u32, C.c_int, _P(C.c_double), _P(_P(_vp)), _vp,
                            _P(mdr_retrieve_info)], C.c_int),
    "mdr_retrieve_qoi_vtotal": ([_vp, _vp, _vp, C.c_int, C.c_double, C.c_double, _P(_vp), _P(_vp),
                                 _P(_vp), _vp, _P(mdr_qoi_info)], C.c_int),
    "mdr_retrieve_qoi_vtotal_with": ([_vp, _vp, _vp, C.c_int, C.c_double, _P(mdr_qoi_params), _P(_vp),
                                      _P(_vp), _P(_vp), _vp, _P(mdr_qoi_info)], C.c_int),
    "mdr_l2_table": ([_vp, _P(mdr_level_view), _u32, _vp], C.c_int),
    "mdr_l2_table_noalloc": ([_vp, _P(mdr_level_view), _u32, _vp], C.c_int),
    "mdr_refactored_l2": ([_vp, _u32, _P(C.c_double)], C.c_int),
    "mdr_level_sizes": ([_u64, _u64, _u64, _u32, _P(_u64)], C.c_int),
    "mdr_decompose": ([C.c_int, _vp, _u64, _u64, _u64, _u32, _vp, _vp], C.c_int),
    "mdr_recompose": ([C.c_int, _vp, _u64, _u64, _u64, _u32, _vp, _vp], C.c_int),
    "mdr_ablation_plane_words": ([C.c_int32, _u64], _u64),
    "mdr_ablation_encode": ([C.c_int32, _vp, _u64, _vp, _vp], C.c_int),
    "mdr_ablation_decode": ([C.c_int32, _vp, _u64, _vp, _vp], C.c_int),
    "mdr_pipeline_create": ([_vp, _u32, _P(_u64), _u32, C.c_int, _u32, _P(mdr_codec_params), _P(_vp)],
                            C.c_int),
    "mdr_pipeline_refactor": ([_vp, _vp, C.c_int, _P(mdr_pipeline_info)], C.c_int),
    "mdr_pipeline_retrieve": ([_vp, C.c_int, C.c_double, _vp, C.c_int, _P(mdr_pipeline_info)], C.c_int),
    "mdr_pipeline_chunk": ([_vp, _u32, _vp, _P(_vp)], C.c_int),
    "mdr_pipeline_destroy": ([_vp], None),
    "mdr_server_create": ([_vp, _u64, _u32, _P(_vp)], C.c_int),
    "mdr_server_add_field": ([_vp, _vp, _P(_u32)], C.c_int),
    "mdr_server_submit": ([_vp, _P(mdr_request), _P(_u64)], C.c_int),
    "mdr_server_poll": ([_vp, _P(mdr_completion), _u32, _P(_u32)], C.c_int),
    "mdr_server_output": ([_vp, _u64, _u32, _u32, _P(_vp), _P(_u64)], C.c_int),
    "mdr_server_release": ([_vp, _u64], C.c_int),
    "mdr_server_stats": ([_vp, _P(mdr_server_info)], C.c_int),
    "mdr_server_destroy": ([_vp], None),
    "mdr_context_set_select_threads": ([_vp, _u32], C.c_int),
    "mdr_retrieve_qoi": ([C.c_int, _P(_vp), _u32, C.c_int, C.c_double, _P(mdr_qoi_params), _P(_P(_vp)), _vp,
                          _P(mdr_qoi_info)], C.c_int),
    "mdr_autotune_refactor": ([_vp, _P(_P(mdr_level_view)), _P(_u32), _u32, C.c_int, _u32,
                               _P(mdr_codec_params), _vp, _u32, C.c_int, _P(mdr_tune_result)], C.c_int),
    "mdr_tune_save": ([_vp, C.c_char_p], C.c_int),
    "mdr_tune_load": ([_vp, C.c_char_p], C.c_int),
    "mdr_tune_entries": ([_vp, _P(_u32)], C.c_int),
    "mdr_tune_entry": ([_vp, _u32, _P(_u32), _P(mdr_launch_shape)], C.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res
    globals()[_name] = _f


class MdrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def _check(st: int) -> None:
    if st != MDR_OK:
        raise MdrError(st, _lib.mdr_last_error().decode(errors="replace"))


def version() -> str:
    return _lib.mdr_version().decode()


def default_params(**overrides) -> mdr_codec_params:
    p = mdr_codec_params()
    _check(_lib.mdr_codec_params_default(C.byref(p)))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- HIP copies for inspection
_hip = None


def _hip_lib():
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so.7")  # resolves to the runtime already loaded
        _hip.hipMemcpy.argtypes = [_vp, _vp, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipDeviceSynchronize.restype = C.c_int
    return _hip


def device_bytes(ptr: int, n: int) -> bytes:
    """Copy n bytes of device memory to the host (synchronizes the device)."""
    if n == 0:
        return b""
    h = _hip_lib()
    if h.hipDeviceSynchronize() != 0:
        raise RuntimeError("hipDeviceSynchronize failed")
    buf = C.create_string_buffer(n)
    if h.hipMemcpy(C.cast(buf, _vp), C.c_void_p(ptr), n, 2) != 0:  # hipMemcpyDeviceToHost
        raise RuntimeError("hipMemcpy failed")
    return buf.raw


# ---------------------------------------------------------------- handles
class Context:
    """One HIP device and its reusable workspaces (mdr_context)."""

    def __init__(self, device: int = 0):
        h = _vp()
        _check(_lib.mdr_context_create(device, C.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            # at interpreter exit the module may already be torn down:
            # the process releases everything then
            if _lib is not None:
                _lib.mdr_context_destroy(self.handle)
            self.handle = None

    def set_timing(self, enable: bool = True) -> None:
        _check(_lib.mdr_context_set_timing(self.handle, 1 if enable else 0))

    def timing(self, reset: bool = True) -> dict:
        """{stage: (milliseconds, launches)} of the kernels timed since the last reset."""
        ms = (C.c_double * len(STAGES))()
        n = (_u64 * len(STAGES))()
        _check(_lib.mdr_context_timing(self.handle, ms, n, 1 if reset else 0))
        return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}

    def set_launch(self, enc_target_wg: int = 0, stats_wg_values: int = 0, graphs: int = -1) -> None:
        """Refactor launch shape (0 / -1 leave a knob unchanged); see mdr_context_set_launch."""
        _check(_lib.mdr_context_set_launch(self.handle, int(enc_target_wg), int(stats_wg_values),
                                           int(graphs)))

    def set_decode_lanes(self, lanes: int) -> None:
        """Lanes a Huffman chunk is decoded by (0 = per launch, 1, 4..64)."""
        _check(_lib.mdr_context_set_decode_lanes(self.handle, int(lanes)))

    def set_select_threads(self, threads: int) -> None:
        """Workgroup size of the selection kernel (256, 512 or 1024; 0: by the pass's unit count)."""
        _check(_lib.mdr_context_set_select_threads(self.handle, int(threads)))

    def autotune(self, variables, nplanes: int, params: mdr_codec_params | None = None, reps: int = 2,
                 force: bool = False, stream=None) -> dict:
        """mdr_autotune_refactor over these variables (lists of device tensors)."""
        dt = _dtype_code(variables[0][0])
        keep = [_views(levels, dt)[0] for levels in variables]
        vp = (_P(mdr_level_view) * len(keep))(*[C.cast(v, _P(mdr_level_view)) for v in keep])
        nl = (_u32 * len(keep))(*[len(levels) for levels in variables])
        res = mdr_tune_result()
        _check(_lib.mdr_autotune_refactor(self.handle, vp, nl, len(keep), dt, nplanes,
                                          C.byref(params) if params is not None else None,
                                          _stream_ptr(stream), int(reps), 1 if force else 0, C.byref(res)))
        return res.as_dict()

    def tune_save(self, path: str) -> None:
        _check(_lib.mdr_tune_save(self.handle, path.encode()))

    def tune_load(self, path: str) -> None:
        _check(_lib.mdr_tune_load(self.handle, path.encode()))

    def tune_table(self) -> list:
        n = _u32()
        _check(_lib.mdr_tune_entries(self.handle, C.byref(n)))
        out = []
        for i in range(n.value):
            key = (_u32 * 5)()
            sh = mdr_launch_shape()
            _check(_lib.mdr_tune_entry(self.handle, i, key, C.byref(sh)))
            out.append({"key": list(key), "shape": sh.as_dict()})
        return out

    def __del__(self):
        self.close()


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return MDR_F32
    if t.dtype == torch.float64:
        return MDR_F64
    raise TypeError("levels must be float32 or float64 tensors")


class Refactored:
    """Refactored variable (mdr_refactored): plane streams + error tables on the device."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle
        nl, dt, B = _u32(), C.c_int(), _u32()
        prm = mdr_codec_params()
        _check(_lib.mdr_refactored_shape(handle, C.byref(nl), C.byref(dt), C.byref(B), C.byref(prm)))
        self.nlevels, self.dtype, self.nplanes, self.params = nl.value, dt.value, B.value, prm

    def close(self):
        if getattr(self, "handle", None):
            if _lib is not None:
                _lib.mdr_refactored_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    def l2_table(self, levels, stream=None) -> None:
        """mdr_l2_table: squared-L2 per-plane tables from the levels this was refactored from."""
        views, _ = _views(levels, self.dtype)
        _check(_lib.mdr_l2_table(self.handle, views, len(levels), _stream_ptr(stream)))

    def l2_table_noalloc(self, levels, stream=None) -> None:
        """mdr_l2_table_noalloc: the same tables through the library's fixed scratch (no device allocation)."""
        views, _ = _views(levels, self.dtype)
        _check(_lib.mdr_l2_table_noalloc(self.handle, views, len(levels), _stream_ptr(stream)))

    def l2(self, level: int):
        """mdr_refactored_l2: the level's squared-L2 table (nplanes + 1 values)."""
        out = (C.c_double * (self.nplanes + 1))()
        _check(_lib.mdr_refactored_l2(self.handle, level, out))
        return list(out)

    def info(self, level: int) -> dict:
        e, n = _i32(), _u64()
        lo, hi = C.c_double(), C.c_double()
        E = (C.c_double * (self.nplanes + 1))()
        _check(_lib.mdr_refactored_info(self.handle, level, C.byref(e), C.byref(n), C.byref(lo),
                                        C.byref(hi), E))
        return {"e": e.value, "n": n.value, "vmin": lo.value, "vmax": hi.value, "E": list(E)}

    def stream(self, level: int, stream: int):
        """(device pointer, bytes, method) of stream -1 (sign) or plane 0..nplanes-1."""
        p, nb, meth = _vp(), _u64(), C.c_int()
        _check(_lib.mdr_refactored_stream(self.handle, level, stream, C.byref(p), C.byref(nb),
                                          C.byref(meth)))
        return (p.value or 0), nb.value, meth.value

    def stream_bytes(self, level: int, stream: int) -> bytes:
        p, nb, _ = self.stream(level, stream)
        return device_bytes(p, nb)

    def serialize(self) -> bytes:
        used = _u64()
        _check(_lib.mdr_serialize(self.handle, None, 0, C.byref(used)))
        buf = C.create_string_buffer(used.value)
        _check(_lib.mdr_serialize(self.handle, C.cast(buf, _vp), used.value, C.byref(used)))
        return buf.raw[:used.value]

    @classmethod
    def deserialize(cls, ctx: Context, blob: bytes) -> "Refactored":
        h = _vp()
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _check(_lib.mdr_deserialize(ctx.handle, C.cast(buf, _vp), len(blob), C.byref(h)))
        return cls(ctx, h)


def _views(levels, dt=None):
    if not levels:
        raise ValueError("no levels")
    dt = _dtype_code(levels[0]) if dt is None else dt
    views = (mdr_level_view * len(levels))()
    for i, t in enumerate(levels):
        if _dtype_code(t) != dt or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("levels must be contiguous device tensors of one dtype")
        views[i].data = t.data_ptr() if t.numel() else None
        views[i].n = t.numel()
    return views, dt


def refactor(ctx: Context, levels, nplanes: int, params: mdr_codec_params | None = None,
             stream=None) -> Refactored:
    """mdr_refactor on a list of contiguous device tensors (one per level, coarsest first)."""
    views, dt = _views(levels)
    h = _vp()
    _check(_lib.mdr_refactor(ctx.handle, views, len(levels), dt, nplanes,
                             C.byref(params) if params is not None else None,
                             _stream_ptr(stream), C.byref(h)))
    return Refactored(ctx, h)


class BatchViews:
    """The marshalled level views of a batch of variables (each a list of
    contiguous device tensors of one dtype), built once for passes repeated on
    the same tensors; it holds the tensors, so they stay allocated."""

    def __init__(self, variables):
        if not variables:
            raise ValueError("no variables")
        self.variables = [list(v) for v in variables]
        self.dt = _dtype_code(self.variables[0][0])
        self._keep = [_views(levels, self.dt)[0] for levels in self.variables]
        self.vp = (_P(mdr_level_view) * len(self._keep))(*[C.cast(v, _P(mdr_level_view)) for v in self._keep])
        self.nl = (_u32 * len(self._keep))(*[len(levels) for levels in self.variables])
        self.n = len(self._keep)


class BatchOutputs:
    """The marshalled output pointers of a batch retrieval (per variable, one
    device tensor per level), built once for retrievals repeated into the
    same tensors; it holds the tensors."""

    def __init__(self, outs_per_var):
        self.outs = [list(o) for o in outs_per_var]
        self._keep = [Retriever._outs(o) for o in self.outs]
        self.op = (_P(_vp) * len(self._keep))(*[C.cast(o, _P(_vp)) for o in self._keep])
        self.n = len(self._keep)


def refactor_batch(ctx: Context, variables, nplanes: int, params: mdr_codec_params | None = None,
                   stream=None) -> list:
    """mdr_refactor_batch: one pass over every level of every variable (each a
    list of contiguous device tensors of one dtype, or a BatchViews of them);
    returns one Refactored each."""
    bv = variables if isinstance(variables, BatchViews) else BatchViews(variables)
    hs = (_vp * bv.n)()
    _check(_lib.mdr_refactor_batch(ctx.handle, bv.vp, bv.nl, bv.n, bv.dt, nplanes,
                                   C.byref(params) if params is not None else None,
                                   _stream_ptr(stream), hs))
    return [Refactored(ctx, _vp(h)) for h in hs]


class Retriever:
    """Progressive / incremental retrieval state of one refactored variable (mdr_retriever)."""

    def __init__(self, ctx: Context, r: Refactored):
        h = _vp()
        _check(_lib.mdr_retriever_create(ctx.handle, r.handle, C.byref(h)))
        self.ctx, self.r, self.handle = ctx, r, h

    def close(self):
        if getattr(self, "handle", None):
            if _lib is not None:
                _lib.mdr_retriever_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    @staticmethod
    def _outs(outs):
        arr = (_vp * len(outs))()
        for i, t in enumerate(outs):
            arr[i] = t.data_ptr() if t.numel() else None
        return arr

    def retrieve(self, tol: float, outs, relative: bool = True, stream=None) -> dict:
        info = mdr_retrieve_info()
        _check(_lib.mdr_retrieve(self.handle, MDR_REL if relative else MDR_ABS, float(tol),
                                 self._outs(outs), _stream_ptr(stream), C.byref(info)))
        return info.as_dict()

    def retrieve_l2(self, tol: float, outs, stream=None) -> dict:
        """mdr_retrieve with MDR_L2: L2 norm of the coefficient error <= tol."""
        info = mdr_retrieve_info()
        _check(_lib.mdr_retrieve(self.handle, MDR_L2, float(tol), self._outs(outs), _stream_ptr(stream),
                                 C.byref(info)))
        return info.as_dict()

    def retrieve_planes(self, k, outs, stream=None) -> dict:
        kk = (_u32 * len(k))(*[int(v) for v in k])
        info = mdr_retrieve_info()
        _check(_lib.mdr_retrieve_planes(self.handle, kk, self._outs(outs), _stream_ptr(stream),
                                        C.byref(info)))
        return info.as_dict()

    def planes(self):
        k = (_u32 * self.r.nlevels)()
        _check(_lib.mdr_retriever_planes(self.handle, k))
        return list(k)


def retrieve_batch(rts, tols, outs_per_var, relative: bool = True, stream=None) -> list:
    """mdr_retrieve_batch: retriever i to tols[i], writing outs_per_var[i] (per
    level; or a BatchOutputs of them)."""
    n = len(rts)
    hs = (_vp * n)(*[r.handle.value for r in rts])
    tl = (C.c_double * n)(*[float(t) for t in tols])
    bo = outs_per_var if isinstance(outs_per_var, BatchOutputs) else BatchOutputs(outs_per_var)
    if bo.n != n:
        raise ValueError("one output list per retriever")
    infos = (mdr_retrieve_info * n)()
    _check(_lib.mdr_retrieve_batch(hs, n, MDR_REL if relative else MDR_ABS, tl, bo.op,
                                   _stream_ptr(stream), infos))
    return [i.as_dict() for i in infos]


def retrieve_qoi_vtotal(rx: Retriever, ry: Retriever, rz: Retriever, tau: float, outs3,
                        relative: bool = False, mape_c: float = 10.0, stream=None,
                        estimator: str = "mape", cp_decay: float = 0.5) -> dict:
    """mdr_retrieve_qoi_vtotal_with: refine vx, vy, vz until the V_total bound
    meets tau; estimator "mape" (threshold mape_c), "ma" or "cp" (factor cp_decay)."""
    info = mdr_qoi_info()
    prm = mdr_qoi_params()
    prm.estimator = QOI_ESTIMATORS[estimator]
    prm.mape_c = float(mape_c)
    prm.cp_decay = float(cp_decay)
    o = [Retriever._outs(outs) for outs in outs3]
    _check(_lib.mdr_retrieve_qoi_vtotal_with(rx.handle, ry.handle, rz.handle,
                                             MDR_REL if relative else MDR_ABS, float(tau), C.byref(prm),
                                             o[0], o[1], o[2], _stream_ptr(stream), C.byref(info)))
    return info.as_dict()


def retrieve_qoi(family: str, rts, tau: float, outs, relative: bool = False, mape_c: float = 10.0,
                 stream=None, estimator: str = "mape", cp_decay: float = 0.5) -> dict:
    """mdr_retrieve_qoi: refine the retrievers until the family's bound
    ("sumsq" of 1-3 variables, "magnitude" of 1-3, "product" of 2) meets tau."""
    info = mdr_qoi_info()
    prm = mdr_qoi_params()
    prm.estimator = QOI_ESTIMATORS[estimator]
    prm.mape_c = float(mape_c)
    prm.cp_decay = float(cp_decay)
    n = len(rts)
    hs = (_vp * n)(*[r.handle.value for r in rts])
    keep = [Retriever._outs(o) for o in outs]
    op = (_P(_vp) * n)(*[C.cast(o, _P(_vp)) for o in keep])
    _check(_lib.mdr_retrieve_qoi(QOI_FAMILIES[family], hs, n, MDR_REL if relative else MDR_ABS, float(tau),
                                 C.byref(prm), op, _stream_ptr(stream), C.byref(info)))
    return info.as_dict()


# ---------------------------------------------------------------- encoder-design ablation
ABLATION_DESIGNS = {"locality": 0, "ballot": 1, "shift": 2, "butterfly": 3, "regblock": 4}


def ablation_plane_words(design: str, n: int) -> int:
    """mdr_ablation_plane_words: 32-bit words per plane for n values."""
    return int(_lib.mdr_ablation_plane_words(ABLATION_DESIGNS[design], int(n)))


def ablation_encode(design: str, x, planes, stream=None) -> None:
    """mdr_ablation_encode: x (n uint32-sized elements, device) -> planes [32][words] (device)."""
    _check(_lib.mdr_ablation_encode(ABLATION_DESIGNS[design], C.c_void_p(x.data_ptr()), x.numel(),
                                    C.c_void_p(planes.data_ptr()), _stream_ptr(stream)))


def ablation_decode(design: str, planes, out, stream=None) -> None:
    """mdr_ablation_decode: planes (device) -> out (n uint32-sized elements, device)."""
    _check(_lib.mdr_ablation_decode(ABLATION_DESIGNS[design], C.c_void_p(planes.data_ptr()), out.numel(),
                                    C.c_void_p(out.data_ptr()), _stream_ptr(stream)))


# ---------------------------------------------------------------- multilevel decomposition
def level_sizes(shape, nsteps: int):
    """mdr_level_sizes: values per level (coarsest first) of an n0 x n1 x n2 grid."""
    out = (_u64 * (int(nsteps) + 1))()
    _check(_lib.mdr_level_sizes(int(shape[0]), int(shape[1]), int(shape[2]), int(nsteps), out))
    return [int(v) for v in out]


def _ml_dtype(t) -> int:
    if t.dtype == torch.float32:
        return MDR_F32
    if t.dtype == torch.float64:
        return MDR_F64
    raise TypeError("multilevel decomposition takes float32 or float64 tensors")


def _ml_check(field, coeffs, what: str) -> None:
    if field.dim() != 3 or not field.is_contiguous() or not coeffs.is_contiguous() \
            or coeffs.dtype != field.dtype or coeffs.numel() != field.numel():
        raise ValueError(what + ": contiguous 3-D field and a contiguous coefficient buffer of the same size and dtype")
    if not (field.is_cuda and coeffs.is_cuda):
        raise ValueError(what + ": field and coefficients must be device tensors")


def decompose(field, nsteps: int, coeffs, stream=None) -> None:
    """mdr_decompose: field (contiguous n0 x n1 x n2 device tensor) -> coeffs
    (its levels concatenated, coarsest first)."""
    _ml_check(field, coeffs, "decompose")
    n0, n1, n2 = field.shape
    _check(_lib.mdr_decompose(_ml_dtype(field), C.c_void_p(field.data_ptr()), n0, n1, n2, int(nsteps),
                              C.c_void_p(coeffs.data_ptr()), _stream_ptr(stream)))


def recompose(coeffs, nsteps: int, field, stream=None) -> None:
    """mdr_recompose: concatenated levels -> field (contiguous n0 x n1 x n2 device tensor)."""
    _ml_check(field, coeffs, "recompose")
    n0, n1, n2 = field.shape
    _check(_lib.mdr_recompose(_ml_dtype(field), C.c_void_p(coeffs.data_ptr()), n0, n1, n2, int(nsteps),
                              C.c_void_p(field.data_ptr()), _stream_ptr(stream)))


class Server:
    """Retrieval server (mdr_server): resident fields, continuous batching on an
    engine thread, admission by HBM budget."""

    def __init__(self, ctx: Context, hbm_budget: int, max_slots: int = 64):
        h = _vp()
        _check(_lib.mdr_server_create(ctx.handle, int(hbm_budget), int(max_slots), C.byref(h)))
        self.ctx, self.handle, self.fields = ctx, h, []

    def close(self):
        if getattr(self, "handle", None):
            if _lib is not None:
                _lib.mdr_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    def add_field(self, r: Refactored) -> int:
        fid = _u32()
        _check(_lib.mdr_server_add_field(self.handle, r.handle, C.byref(fid)))
        self.fields.append(r)  # keep the field alive as long as the server
        return fid.value

    def submit(self, kind: int, fields, tol: float, relative: bool = True, parent: int = 0,
               tag: int = 0, mape_c: float = 10.0) -> int:
        q = mdr_request()
        q.kind = kind
        fl = list(fields) + [0] * (3 - len(fields))
        for i in range(3):
            q.field[i] = int(fl[i])
        q.bound = MDR_REL if relative else MDR_ABS
        q.tol = float(tol)
        q.mape_c = float(mape_c)
        q.parent = int(parent)
        q.tag = int(tag)
        t = _u64()
        _check(_lib.mdr_server_submit(self.handle, C.byref(q), C.byref(t)))
        return t.value

    def poll(self, cap: int = 256) -> list:
        buf = (mdr_completion * cap)()
        n = _u32()
        _check(_lib.mdr_server_poll(self.handle, buf, cap, C.byref(n)))
        return [buf[i].as_dict() for i in range(n.value)]

    def output(self, ticket: int, comp: int, level: int):
        """(device pointer, values) of one output level of a completed request."""
        p, n = _vp(), _u64()
        _check(_lib.mdr_server_output(self.handle, int(ticket), int(comp), int(level), C.byref(p),
                                      C.byref(n)))
        return (p.value or 0), n.value

    def release(self, ticket: int) -> None:
        _check(_lib.mdr_server_release(self.handle, int(ticket)))

    def stats(self) -> dict:
        i = mdr_server_info()
        _check(_lib.mdr_server_stats(self.handle, C.byref(i)))
        return {f: getattr(i, f) for f, _ in i._fields_ if f != "pad"}


class Pipeline:
    """Chunked H2D / refactor / D2H pipeline over a field in host memory (mdr_pipeline)."""

    def __init__(self, ctx: Context, nchunks: int, level_sizes, dtype, nplanes: int,
                 params: mdr_codec_params | None = None):
        import torch
        dt = MDR_F64 if dtype in (torch.float64, "f64") else MDR_F32
        sz = (_u64 * len(level_sizes))(*[int(n) for n in level_sizes])
        h = _vp()
        _check(_lib.mdr_pipeline_create(ctx.handle, int(nchunks), sz, len(level_sizes), dt, int(nplanes),
                                        C.byref(params) if params is not None else None, C.byref(h)))
        self.ctx, self.handle = ctx, h

    def close(self):
        if getattr(self, "handle", None):
            if _lib is not None:
                _lib.mdr_pipeline_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    def refactor(self, host_values, overlap: bool = True) -> dict:
        """host_values: a (pinned) CPU tensor holding every chunk, levels concatenated."""
        info = mdr_pipeline_info()
        _check(_lib.mdr_pipeline_refactor(self.handle, C.c_void_p(host_values.data_ptr()),
                                          1 if overlap else 0, C.byref(info)))
        return info.as_dict()

    def retrieve(self, tol: float, host_out, relative: bool = True, overlap: bool = True) -> dict:
        info = mdr_pipeline_info()
        _check(_lib.mdr_pipeline_retrieve(self.handle, MDR_REL if relative else MDR_ABS, float(tol),
                                          C.c_void_p(host_out.data_ptr()), 1 if overlap else 0,
                                          C.byref(info)))
        return info.as_dict()

    def chunk(self, c: int) -> Refactored:
        h = _vp()
        _check(_lib.mdr_pipeline_chunk(self.handle, int(c), self.ctx.handle, C.byref(h)))
        return Refactored(self.ctx, h)
