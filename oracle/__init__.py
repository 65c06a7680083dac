"""Plain CPU oracle for HP-MDR's bitplane + lossless path (arXiv 2505.00227).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_2505_00227_amd``) never imports it, and the two share no code.

The arithmetic lives in ``mdr_oracle.c`` (plain C, one value / one bit at a
time); this module only marshals numpy arrays through ctypes.  The QoI loop of
Sec. 5.2 (Alg. 3 with the MAPE estimator) is written here in Python on top of
the C planner and bound, because it is control flow, not arithmetic.  The
multilevel decomposition that produces the levels from a field is in
``multilevel.py`` (numpy, in the field's own dtype).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdr_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

F32, F64 = 0, 1
DC, RLE, HUF, PLACEHOLDER = 0, 1, 2, 3
METHOD_NAMES = {DC: "DC", RLE: "RLE", HUF: "HUF", PLACEHOLDER: "PLACEHOLDER"}
OK, EINVAL, EUNSUP, ENOMEM, ECORRUPT = 0, 1, 2, 3, 5


class OracleError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__(f"oracle error {code} {what}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        u64, u32, i32, vp = C.c_uint64, C.c_uint32, C.c_int32, C.c_void_p
        dp = C.POINTER(C.c_double)
        L.orc_stats.argtypes = [vp, u64, C.c_int, C.POINTER(i32), dp, dp, dp]
        L.orc_fixed_point.argtypes = [vp, u64, C.c_int, i32, u32, vp, vp]
        L.orc_fixed_point.restype = None
        L.orc_plane_bytes.argtypes = [u64, u32]
        L.orc_plane_bytes.restype = u64
        L.orc_bitplanes.argtypes = [vp, vp, u64, u32, u32, vp]
        L.orc_bitplanes.restype = None
        L.orc_error_table.argtypes = [vp, vp, u64, C.c_int, i32, u32, vp]
        L.orc_error_table.restype = None
        L.orc_huffman_lengths.argtypes = [vp, u32, vp]
        L.orc_huffman_codes.argtypes = [vp, vp]
        L.orc_huffman_codes.restype = None
        L.orc_huffman_estimate.argtypes = [vp, vp, u64, u32]
        L.orc_huffman_estimate.restype = u64
        L.orc_huffman_encoded_size.argtypes = [vp, u64, u32, u32]
        L.orc_huffman_encoded_size.restype = u64
        L.orc_huffman_encode.argtypes = [vp, u64, u32, u32, vp, u64, C.POINTER(u64)]
        L.orc_huffman_decode.argtypes = [vp, u64, u32, vp, u64]
        L.orc_rle_runs.argtypes = [vp, u64, u32]
        L.orc_rle_runs.restype = u64
        L.orc_rle_estimate.argtypes = [u64, u32]
        L.orc_rle_estimate.restype = u64
        L.orc_rle_encode.argtypes = [vp, u64, u32, vp, u64, C.POINTER(u64)]
        L.orc_rle_decode.argtypes = [vp, u64, u32, vp, u64]
        L.orc_select.argtypes = [u64, u64, u64, C.POINTER(_Params)]
        L.orc_crc32.argtypes = [vp, u64]
        L.orc_crc32.restype = u32
        L.orc_refactor_level.argtypes = [vp, u64, C.c_int, u32, C.POINTER(_Params), C.POINTER(vp)]
        L.orc_level_free.argtypes = [vp]
        L.orc_level_free.restype = None
        L.orc_level_info.argtypes = [vp, C.POINTER(u64), C.POINTER(i32), dp, dp, dp, vp]
        L.orc_level_stream.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(u64),
                                       C.POINTER(C.POINTER(C.c_uint8)), C.POINTER(u64),
                                       C.POINTER(u64)]
        L.orc_level_rows.argtypes = [vp, C.POINTER(u64)]
        L.orc_level_rows.restype = C.POINTER(C.c_uint8)
        L.orc_reconstruct.argtypes = [vp, u32, vp]
        L.orc_plan.argtypes = [u32, u32, u32, vp, vp, C.c_double, vp, vp, dp]
        L.orc_plan_one_step.argtypes = [u32, u32, u32, vp, vp, vp]
        L.orc_qoi_vtotal_tau.argtypes = [u64, vp, vp, vp, vp]
        L.orc_qoi_vtotal_tau.restype = C.c_double
        L.orc_abl_planes.argtypes = [C.c_int, vp, u64, vp, u64]
        L.orc_abl_planes.restype = None
        L.orc_qoi_vtotal_argmax.argtypes = [u64, vp, vp, vp, vp]
        L.orc_qoi_vtotal_argmax.restype = u64
        L.orc_serialize.argtypes = [vp, u32, C.POINTER(_Params), vp, u64, C.POINTER(u64)]
        L.orc_qoi_score_max.argtypes = [C.c_int, u32, u64, vp, vp, vp, vp, C.POINTER(u64)]
        L.orc_qoi_score_max.restype = C.c_double
        L.orc_qoi_estimate.argtypes = [C.c_int, u32, C.c_double, vp]
        L.orc_qoi_estimate.restype = C.c_double
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_get_threads.restype = C.c_int
        _lib = L
    return _lib


class _Params(C.Structure):
    _fields_ = [("group_planes", C.c_uint32), ("t_cr_milli", C.c_uint32), ("t_s", C.c_uint64),
                ("huf_chunk", C.c_uint32), ("huf_lmax", C.c_uint32), ("force_method", C.c_int32)]


@dataclass
class Params:
    """Codec parameters (Alg. 2): m, T_cr, T_s, Huffman chunking, forced method."""
    group_planes: int = 4
    t_cr_milli: int = 2000
    t_s: int = 4096
    huf_chunk: int = 256
    huf_lmax: int = 12
    force_method: int = -1

    def c(self) -> _Params:
        return _Params(self.group_planes, self.t_cr_milli, self.t_s, self.huf_chunk,
                       self.huf_lmax, self.force_method)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _dtype_code(x: np.ndarray) -> int:
    if x.dtype == np.float32:
        return F32
    if x.dtype == np.float64:
        return F64
    raise TypeError(x.dtype)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


# ---------------------------------------------------------------- step functions
def stats(x: np.ndarray):
    x = np.ascontiguousarray(x)
    e = C.c_int32()
    lo, hi, am = C.c_double(), C.c_double(), C.c_double()
    st = lib().orc_stats(_ptr(x), x.size, _dtype_code(x), C.byref(e), C.byref(lo), C.byref(hi),
                         C.byref(am))
    if st:
        raise OracleError(st, "stats")
    return e.value, lo.value, hi.value, am.value


def fixed_point(x: np.ndarray, e: int, B: int):
    x = np.ascontiguousarray(x)
    mag = np.zeros(x.size, np.uint64)
    sign = np.zeros(x.size, np.uint8)
    lib().orc_fixed_point(_ptr(x), x.size, _dtype_code(x), e, B, _ptr(mag), _ptr(sign))
    return mag, sign


def plane_bytes(n: int, W: int) -> int:
    return int(lib().orc_plane_bytes(n, W))


def ablation_planes(x: np.ndarray, interleaved: bool) -> np.ndarray:
    """Sec. 3's experiment: 32-bit words -> [32][words] planes (plane p = bit
    31-p); block layout, or the register block's interleaved one."""
    x = np.ascontiguousarray(x, np.uint32)
    n = x.size
    words = (n + 2047) // 2048 * 64 if interleaved else (n + 31) // 32
    planes = np.zeros((32, words), np.uint32)
    lib().orc_abl_planes(1 if interleaved else 0, _ptr(x), n, _ptr(planes), words)
    return planes


def bitplanes(mag: np.ndarray, sign: np.ndarray, B: int, W: int) -> np.ndarray:
    """Rows [B+1, plane_bytes]: row 0 = sign plane, row 1+p = plane p (bit B-1-p)."""
    mag = np.ascontiguousarray(mag, np.uint64)
    sign = np.ascontiguousarray(sign, np.uint8)
    pb = plane_bytes(mag.size, W)
    rows = np.zeros((B + 1, pb), np.uint8)
    lib().orc_bitplanes(_ptr(mag), _ptr(sign), mag.size, B, W, _ptr(rows))
    return rows


def error_table(x: np.ndarray, mag: np.ndarray, e: int, B: int) -> np.ndarray:
    x = np.ascontiguousarray(x)
    mag = np.ascontiguousarray(mag, np.uint64)
    E = np.zeros(B + 1, np.float64)
    lib().orc_error_table(_ptr(x), _ptr(mag), x.size, _dtype_code(x), e, B, _ptr(E))
    return E


def huffman_lengths(freq, lmax: int = 12) -> np.ndarray:
    f = np.ascontiguousarray(freq, np.uint64)
    assert f.size == 256
    ln = np.zeros(256, np.uint8)
    st = lib().orc_huffman_lengths(_ptr(f), lmax, _ptr(ln))
    if st:
        raise OracleError(st, "huffman_lengths")
    return ln


def huffman_codes(lengths) -> np.ndarray:
    ln = np.ascontiguousarray(lengths, np.uint8)
    codes = np.zeros(256, np.uint32)
    lib().orc_huffman_codes(_ptr(ln), _ptr(codes))
    return codes


def huffman_estimate(freq, lengths, S: int, chunk: int) -> int:
    f = np.ascontiguousarray(freq, np.uint64)
    ln = np.ascontiguousarray(lengths, np.uint8)
    return int(lib().orc_huffman_estimate(_ptr(f), _ptr(ln), S, chunk))


def huffman_encode(g: bytes, chunk: int = 1024, lmax: int = 12) -> bytes:
    a = np.frombuffer(bytes(g), np.uint8) if len(g) else np.zeros(1, np.uint8)
    S = len(g)
    cap = int(lib().orc_huffman_encoded_size(_ptr(a), S, chunk, lmax))
    out = np.zeros(max(cap, 1), np.uint8)
    used = C.c_uint64()
    st = lib().orc_huffman_encode(_ptr(a), S, chunk, lmax, _ptr(out), cap, C.byref(used))
    if st:
        raise OracleError(st, "huffman_encode")
    return out[:used.value].tobytes()


def huffman_decode(p: bytes, S: int, chunk: int = 1024) -> bytes:
    a = np.frombuffer(bytes(p), np.uint8)
    g = np.zeros(max(S, 1), np.uint8)
    st = lib().orc_huffman_decode(_ptr(a), len(p), chunk, _ptr(g), S)
    if st:
        raise OracleError(st, "huffman_decode")
    return g[:S].tobytes()


def rle_runs(g: bytes, wbytes: int) -> int:
    a = np.frombuffer(bytes(g), np.uint8) if len(g) else np.zeros(1, np.uint8)
    return int(lib().orc_rle_runs(_ptr(a), len(g), wbytes))


def rle_estimate(nruns: int, wbytes: int) -> int:
    return int(lib().orc_rle_estimate(nruns, wbytes))


def rle_encode(g: bytes, wbytes: int) -> bytes:
    a = np.frombuffer(bytes(g), np.uint8) if len(g) else np.zeros(1, np.uint8)
    cap = rle_estimate(rle_runs(g, wbytes), wbytes)
    out = np.zeros(cap, np.uint8)
    used = C.c_uint64()
    st = lib().orc_rle_encode(_ptr(a), len(g), wbytes, _ptr(out), cap, C.byref(used))
    if st:
        raise OracleError(st, "rle_encode")
    return out[:used.value].tobytes()


def rle_decode(p: bytes, S: int, wbytes: int) -> bytes:
    a = np.frombuffer(bytes(p), np.uint8)
    g = np.zeros(max(S, 1), np.uint8)
    st = lib().orc_rle_decode(_ptr(a), len(p), wbytes, _ptr(g), S)
    if st:
        raise OracleError(st, "rle_decode")
    return g[:S].tobytes()


def select(S: int, est_huf: int, est_rle: int, params: Params) -> int:
    p = params.c()
    return int(lib().orc_select(S, est_huf, est_rle, C.byref(p)))


def crc32(b: bytes) -> int:
    a = np.frombuffer(bytes(b), np.uint8) if len(b) else np.zeros(1, np.uint8)
    return int(lib().orc_crc32(_ptr(a), len(b)))


# ---------------------------------------------------------------- one level
class Level:
    """One refactored level produced by the oracle."""

    def __init__(self, x: np.ndarray, B: int, params: Params | None = None):
        self.params = params or Params()
        x = np.ascontiguousarray(x)
        self.dtype = x.dtype
        self.B = B
        self.W = 32 if x.dtype == np.float32 else 64
        h = C.c_void_p()
        p = self.params.c()
        st = lib().orc_refactor_level(_ptr(x) if x.size else None, x.size, _dtype_code(x), B,
                                      C.byref(p), C.byref(h))
        if st:
            raise OracleError(st, "refactor_level")
        self._h = h
        n, e = C.c_uint64(), C.c_int32()
        lo, hi, am = C.c_double(), C.c_double(), C.c_double()
        E = np.zeros(B + 1, np.float64)
        lib().orc_level_info(h, C.byref(n), C.byref(e), C.byref(lo), C.byref(hi), C.byref(am),
                             _ptr(E))
        self.n, self.e = n.value, e.value
        self.vmin, self.vmax, self.vmaxabs = lo.value, hi.value, am.value
        self.E = E
        self.streams = []  # index 0 = sign, 1+p = plane p: (method, payload bytes)
        self.est_huf, self.est_rle = [], []
        for s in range(-1, B):
            meth, nb = C.c_int32(), C.c_uint64()
            eh, er = C.c_uint64(), C.c_uint64()
            dptr = C.POINTER(C.c_uint8)()
            lib().orc_level_stream(h, s, C.byref(meth), C.byref(nb), C.byref(dptr), C.byref(eh),
                                   C.byref(er))
            data = C.string_at(dptr, nb.value) if nb.value else b""
            self.streams.append((meth.value, data))
            self.est_huf.append(eh.value)
            self.est_rle.append(er.value)
        pb = C.c_uint64()
        rp = lib().orc_level_rows(h, C.byref(pb))
        self.plane_bytes = pb.value
        self.rows = np.ctypeslib.as_array(rp, shape=((B + 1) * pb.value,)).copy().reshape(
            B + 1, pb.value) if pb.value else np.zeros((B + 1, 0), np.uint8)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_level_free(h)
            self._h = None

    @property
    def m(self) -> int:
        return min(self.params.group_planes, self.B)

    def unit_bytes(self) -> np.ndarray:
        """Stream sizes in table order (sign, plane 0..B-1); placeholders are 0."""
        return np.array([len(d) if m != PLACEHOLDER else 0 for m, d in self.streams], np.uint64)

    def reconstruct(self, k: int) -> np.ndarray:
        out = np.zeros(self.n, self.dtype)
        st = lib().orc_reconstruct(self._h, k, _ptr(out) if self.n else None)
        if st:
            raise OracleError(st, "reconstruct")
        return out


def refactor(levels, B: int, params: Params | None = None):
    """Refactor a variable given as a list of coefficient levels (coarsest first)."""
    return [Level(x, B, params) for x in levels]


def serialize(levels, params: Params | None = None) -> bytes:
    params = params or levels[0].params
    arr = (C.c_void_p * len(levels))(*[lv._h.value for lv in levels])
    p = params.c()
    used = C.c_uint64()
    lib().orc_serialize(arr, len(levels), C.byref(p), None, 0, C.byref(used))
    out = np.zeros(used.value, np.uint8)
    st = lib().orc_serialize(arr, len(levels), C.byref(p), _ptr(out), used.value, C.byref(used))
    if st:
        raise OracleError(st, "serialize")
    return out.tobytes()


# ---------------------------------------------------------------- planner
def variable_range(levels) -> float:
    """max - min over every coefficient of the variable (for relative bounds)."""
    nonempty = [lv for lv in levels if lv.n]
    if not nonempty:
        return 0.0
    lo = min(lv.vmin for lv in nonempty)
    hi = max(lv.vmax for lv in nonempty)
    return float(hi) - float(lo)


def _E_matrix(levels):
    return np.ascontiguousarray(np.stack([lv.E for lv in levels]), np.float64)


def _U_matrix(levels):
    return np.ascontiguousarray(np.stack([lv.unit_bytes() for lv in levels]), np.uint64)


def plan(levels, tol_abs: float, k_in=None):
    """Greedy tolerance -> planes per level; returns (k list, bound)."""
    L = len(levels)
    B, m = levels[0].B, levels[0].m
    kin = np.zeros(L, np.uint32) if k_in is None else np.ascontiguousarray(k_in, np.uint32)
    kout = np.zeros(L, np.uint32)
    bound = C.c_double()
    E, U = _E_matrix(levels), _U_matrix(levels)
    lib().orc_plan(L, B, m, _ptr(E), _ptr(U), float(tol_abs), _ptr(kin), _ptr(kout),
                   C.byref(bound))
    return [int(v) for v in kout], bound.value


def plan_one_step(levels, k):
    kk = np.ascontiguousarray(k, np.uint32).copy()
    E, U = _E_matrix(levels), _U_matrix(levels)
    moved = lib().orc_plan_one_step(len(levels), levels[0].B, levels[0].m, _ptr(E), _ptr(U),
                                    _ptr(kk))
    return [int(v) for v in kk], bool(moved)


def bound_of(levels, k) -> float:
    s = 0.0
    for lv, kl in zip(levels, k):
        s += float(lv.E[kl])
    return s


def retrieve(levels, k):
    """Reconstruct every level from its first k[l] planes."""
    return [lv.reconstruct(int(kl)) for lv, kl in zip(levels, k)]


def l2_table(x: np.ndarray, lv: "Level") -> np.ndarray:
    """Squared L2 error of a level after k planes, k = 0..B (an MDR option the
    paper does not use; it controls L-infinity error throughout): E2[k] =
    sum_i (x_i - xhat_i^(k))^2, with xhat^(k) the oracle's own k-plane
    reconstruction, each square rounded once in fp64 and the sum exactly
    rounded (math.fsum)."""
    x64 = np.asarray(x, np.float64)
    out = np.zeros(lv.B + 1, np.float64)
    for k in range(lv.B + 1):
        r = x64 - lv.reconstruct(k).astype(np.float64)
        out[k] = math.fsum((r * r).tolist())
    return out


def plan_l2(levels, tables, tol: float, k_in=None):
    """The greedy planner of `plan` run on squared-L2 tables against tol^2."""
    L = len(levels)
    B, m = levels[0].B, levels[0].m
    kin = np.zeros(L, np.uint32) if k_in is None else np.ascontiguousarray(k_in, np.uint32)
    kout = np.zeros(L, np.uint32)
    bound = C.c_double()
    E2 = np.ascontiguousarray(np.stack([np.asarray(t, np.float64) for t in tables]))
    lib().orc_plan(L, B, m, _ptr(E2), _ptr(_U_matrix(levels)), tol * tol, _ptr(kin), _ptr(kout),
                   C.byref(bound))
    return [int(v) for v in kout], bound.value


def retrieve_to(levels, tol: float, relative: bool = True, k_in=None):
    tol_abs = tol * variable_range(levels) if relative else tol
    k, bound = plan(levels, tol_abs, k_in)
    return retrieve(levels, k), k, bound, bound <= tol_abs


# ---------------------------------------------------------------- QoI (Alg. 3 + MAPE)
def qoi_tau(vx: np.ndarray, vy: np.ndarray, vz: np.ndarray, eps) -> float:
    a = [np.ascontiguousarray(v, np.float64) for v in (vx, vy, vz)]
    e = np.ascontiguousarray(eps, np.float64)
    return float(lib().orc_qoi_vtotal_tau(a[0].size, _ptr(a[0]), _ptr(a[1]), _ptr(a[2]), _ptr(e)))


def qoi_initial_eps(vars3, tau: float):
    """Reading of Alg. 3's initial bounds: eps_c = (tau / Q_max) * range_c, with
    Q_max = sum_c max(|min_c|, |max_c|)^2 (the largest V_total the ranges allow)."""
    qmax = 0.0
    for levels in vars3:
        nonempty = [lv for lv in levels if lv.n]
        lo = min((lv.vmin for lv in nonempty), default=0.0)
        hi = max((lv.vmax for lv in nonempty), default=0.0)
        a = max(abs(lo), abs(hi))
        qmax = qmax + a * a
    if qmax == 0.0:
        return [0.0, 0.0, 0.0]
    return [(tau / qmax) * variable_range(levels) for levels in vars3]


def qoi_argmax(vx: np.ndarray, vy: np.ndarray, vz: np.ndarray, eps) -> int:
    """First point (level-concatenated order) with the largest V_total estimate."""
    a = [np.ascontiguousarray(v, np.float64) for v in (vx, vy, vz)]
    e = np.ascontiguousarray(eps, np.float64)
    return int(lib().orc_qoi_vtotal_argmax(a[0].size, _ptr(a[0]), _ptr(a[1]), _ptr(a[2]), _ptr(e)))


QOI_INFLATE = 1.0 + 2.0 ** -40


def cp_bounds(v, eps, tau: float, decay: float = 0.5, max_steps: int = 2200):
    """The CP estimator's host step (Sec. 5.2), reading: at the point with the
    largest estimate, whose current values are v = (|vx|, |vy|, |vz|), every
    bound is multiplied by `decay` until that point's estimate, evaluated as the
    global one (same order, same inflation), is within tau."""
    e = [float(x) for x in eps]

    def est(e):
        s = 0.0
        for c in range(3):
            s = s + e[c] * ((2.0 * v[c]) + e[c])
        return s * QOI_INFLATE

    steps = 0
    while est(e) > tau and steps < max_steps:
        e = [x * decay for x in e]
        steps += 1
    return e


def retrieve_qoi_vtotal(vars3, tau: float, c: float = 10.0, k_in=None, max_iter: int = 10000,
                        estimator: str = "mape", decay: float = 0.5):
    """Alg. 3 (Sec. 5.2): returns (values per var, k per var, tau', met, iterations).

    Each iteration recomposes the three variables from the planes held (identity
    recomposition: values are the level-concatenated coefficients), evaluates
    tau' = (1+2^-40) max_p sum_c eps_c (2|v_c| + eps_c), and stops when tau' <= tau.
    Otherwise the next bounds come from the estimator:
      "mape": with p = tau'/tau, if p > c every eps_c <- eps_c / p and each
              variable is re-planned;
      "ma":   nothing but the step below (minimal augmentation);
      "cp":   the bounds `cp_bounds` gives at the point with the largest
              estimate, each variable re-planned to them;
    and if that adds nothing, one greedy step per variable (one more merged
    group)."""
    assert estimator in ("mape", "ma", "cp")
    ks = [list(k_in[i]) if k_in is not None else [0] * len(v) for i, v in enumerate(vars3)]
    eps0 = qoi_initial_eps(vars3, tau)
    for i, levels in enumerate(vars3):
        ks[i], _ = plan(levels, eps0[i], ks[i])
    it = 0
    while True:
        it += 1
        vals = [np.concatenate([a.astype(np.float64) for a in retrieve(levels, ks[i])])
                for i, levels in enumerate(vars3)]
        eps = [bound_of(levels, ks[i]) for i, levels in enumerate(vars3)]
        tprime = qoi_tau(vals[0], vals[1], vals[2], eps)
        full = all(all(k == levels[0].B for k in ks[i]) for i, levels in enumerate(vars3))
        if tprime <= tau or full or it >= max_iter:
            return vals, ks, tprime, tprime <= tau, it
        target = None
        if estimator == "mape":
            p = tprime / tau if tau > 0 else math.inf
            if p > c:
                target = [e / p for e in eps]
        elif estimator == "cp":
            at = qoi_argmax(vals[0], vals[1], vals[2], eps)
            target = cp_bounds([abs(float(vals[ci][at])) for ci in range(3)], eps, tau, decay)
        moved = False
        if target is not None:
            for i, levels in enumerate(vars3):
                knew, _ = plan(levels, target[i], ks[i])
                moved = moved or knew != ks[i]
                ks[i] = knew
        if not moved:
            for i, levels in enumerate(vars3):
                ks[i], _ = plan_one_step(levels, ks[i])


# ---------------------------------------------------------------- QoI families (Sec. 5.2)
QOI_KINDS = {"sumsq": 0, "magnitude": 1, "product": 2}


def _qoi_nvars_ok(kind: str, nvars: int) -> bool:
    return (kind == "product" and nvars == 2) or (kind in ("sumsq", "magnitude") and 1 <= nvars <= 3)


def qoi_score_max(kind: str, vals, eps):
    """(max_p r(p), first point attaining it) for the family's score r (see
    orc_qoi_score_max in mdr_oracle.c); vals: one float64 array per variable."""
    a = [np.ascontiguousarray(v, np.float64) for v in vals]
    while len(a) < 3:
        a.append(a[0])
    e = np.zeros(3, np.float64)
    e[:len(eps)] = eps
    at = C.c_uint64()
    m = lib().orc_qoi_score_max(QOI_KINDS[kind], len(vals), a[0].size, _ptr(a[0]), _ptr(a[1]), _ptr(a[2]),
                                _ptr(e), C.byref(at))
    return float(m), int(at.value)


def qoi_estimate(kind: str, nvars: int, score_max: float, eps) -> float:
    e = np.zeros(3, np.float64)
    e[:len(eps)] = eps
    return float(lib().orc_qoi_estimate(QOI_KINDS[kind], nvars, float(score_max), _ptr(e)))


def _abs_max(levels) -> float:
    nonempty = [lv for lv in levels if lv.n]
    lo = min((lv.vmin for lv in nonempty), default=0.0)
    hi = max((lv.vmax for lv in nonempty), default=0.0)
    return max(abs(lo), abs(hi))


def qoi_scale(kind: str, vars_) -> float:
    """The family's value scale (relative tolerances multiply it): sum of squares:
    Q_max = sum_c A_c^2 with A_c = max(|min_c|, |max_c|); magnitude: sqrt(Q_max);
    product: A_0 A_1 (the largest values the ranges allow)."""
    A = [_abs_max(levels) for levels in vars_]
    if kind == "product":
        return A[0] * A[1]
    q = 0.0
    for a in A:
        q = q + a * a
    return q if kind == "sumsq" else math.sqrt(q)


def qoi_initial_bounds(kind: str, vars_, tau: float):
    """Reading of Alg. 3's initial bounds per family.  Sum of squares: the
    V_total reading, eps_c = (tau / Q_max) range_c.  Magnitude: tau / sqrt(n),
    the largest equal bounds its value-free estimate sqrt(sum eps^2) accepts.
    Product: eps_0 = tau / (2 A_1), eps_1 = tau / (2 A_0), the first-order terms
    of its bound splitting tau evenly (infinite when the other factor is 0)."""
    if kind == "sumsq":
        q = qoi_scale("sumsq", vars_)
        if q == 0.0:
            return [0.0] * len(vars_)
        return [(tau / q) * variable_range(levels) for levels in vars_]
    if kind == "magnitude":
        return [tau / math.sqrt(len(vars_))] * len(vars_)
    A = [_abs_max(levels) for levels in vars_]
    return [tau / (2.0 * A[1]) if A[1] > 0 else math.inf, tau / (2.0 * A[0]) if A[0] > 0 else math.inf]


def qoi_point_estimate(kind: str, point_vals, eps) -> float:
    """The estimate at one point (values as given), evaluated as tau' is."""
    m, _ = qoi_score_max(kind, [np.array([v], np.float64) for v in point_vals], eps)
    return qoi_estimate(kind, len(point_vals), m, eps)


def retrieve_qoi(kind: str, vars_, tau: float, c: float = 10.0, k_in=None, max_iter: int = 10000,
                 estimator: str = "mape", decay: float = 0.5):
    """Alg. 3 (Sec. 5.2) for a QoI family: returns (values per var, k per var,
    tau', met, iterations).  The same loop as retrieve_qoi_vtotal: plan each
    variable to its initial bound; then reconstruct, take eps_c = the bound of
    the planes held, tau' = the family's estimate; stop when tau' <= tau or
    every plane is held; else next bounds from the estimator (MAPE: eps_c / p
    when p = tau'/tau > c; CP: at the point with the largest score, every bound
    times `decay` until that point's estimate is within tau; MA: none) with
    one more merged group per variable when they add nothing."""
    assert estimator in ("mape", "ma", "cp") and _qoi_nvars_ok(kind, len(vars_))
    nv = len(vars_)
    ks = [list(k_in[i]) if k_in is not None else [0] * len(v) for i, v in enumerate(vars_)]
    eps0 = qoi_initial_bounds(kind, vars_, tau)
    for i, levels in enumerate(vars_):
        ks[i], _ = plan(levels, eps0[i], ks[i])
    it = 0
    while True:
        it += 1
        vals = [np.concatenate([a.astype(np.float64) for a in retrieve(levels, ks[i])])
                for i, levels in enumerate(vars_)]
        eps = [bound_of(levels, ks[i]) for i, levels in enumerate(vars_)]
        score, at = qoi_score_max(kind, vals, eps)
        tprime = qoi_estimate(kind, nv, score, eps)
        full = all(all(k == levels[0].B for k in ks[i]) for i, levels in enumerate(vars_))
        if tprime <= tau or full or it >= max_iter:
            return vals, ks, tprime, tprime <= tau, it
        target = None
        if estimator == "mape":
            p = tprime / tau if tau > 0 else math.inf
            if p > c:
                target = [e / p for e in eps]
        elif estimator == "cp":
            pv = [float(vals[i][at]) for i in range(nv)]
            e = [float(x) for x in eps]
            steps = 0
            while qoi_point_estimate(kind, pv, e) > tau and steps < 2200:
                e = [x * decay for x in e]
                steps += 1
            target = e
        moved = False
        if target is not None:
            for i, levels in enumerate(vars_):
                knew, _ = plan(levels, target[i], ks[i])
                moved = moved or knew != ks[i]
                ks[i] = knew
        if not moved:
            for i, levels in enumerate(vars_):
                ks[i], _ = plan_one_step(levels, ks[i])
