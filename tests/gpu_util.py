"""Helpers for the GPU parity tests: run the same seeded input through the HIP
path (via the C ABI) and through the oracle, and compare what must be equal."""
import sys

import numpy as np

import oracle


def to_oracle_params(p) -> "oracle.Params":
    return oracle.Params(group_planes=p.group_planes, t_cr_milli=p.t_cr_milli, t_s=p.t_s_bytes,
                         huf_chunk=p.huf_chunk, huf_lmax=p.huf_lmax, force_method=p.force_method)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def upload(levels_np):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in levels_np]


def compare_refactor(r, orc_levels, check_streams=True):
    """e, n, min, max, exact error tables, and every stream (method + bytes)."""
    import paper_2505_00227_amd as mdr
    B = r.nplanes
    for l, ol in enumerate(orc_levels):
        inf = r.info(l)
        assert inf["n"] == ol.n, (l, inf["n"], ol.n)
        assert inf["e"] == ol.e, (l, inf["e"], ol.e)
        if ol.n:
            assert inf["vmin"] == ol.vmin and inf["vmax"] == ol.vmax, (l, inf, ol.vmin, ol.vmax)
        E = np.array(inf["E"])
        bad = np.nonzero(E != ol.E)[0]
        assert bad.size == 0, ("error table", l, bad[:5], E[bad[:5]], ol.E[bad[:5]])
        if not check_streams:
            continue
        for s in range(-1, B):
            ptr, nb, meth = r.stream(l, s)
            om, od = ol.streams[s + 1]
            assert meth == om, ("method", l, s, meth, om, ol.est_huf[s + 1], ol.est_rle[s + 1])
            assert nb == len(od), ("bytes", l, s, meth, nb, len(od))
            if nb:
                got = mdr.device_bytes(ptr, nb)
                if got != od:
                    a = np.frombuffer(got, np.uint8)
                    b = np.frombuffer(od, np.uint8)
                    i = int(np.nonzero(a != b)[0][0])
                    raise AssertionError(("payload", l, s, meth, "first diff at byte", i,
                                          a[i:i + 8].tolist(), b[i:i + 8].tolist()))


def gpu_outputs(levels_np):
    import torch
    return [torch.empty(a.size, dtype=torch.float32 if a.dtype == np.float32 else torch.float64,
                        device="cuda") for a in levels_np]


def host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def assert_same_bits(got: np.ndarray, ref: np.ndarray, what=""):
    if got.tobytes() != ref.tobytes():
        gb = got.view(np.uint32 if got.dtype == np.float32 else np.uint64)
        rb = ref.view(np.uint32 if ref.dtype == np.float32 else np.uint64)
        i = int(np.nonzero(gb != rb)[0][0])
        raise AssertionError((what, "first diff at", i, got[i], ref[i], hex(int(gb[i])), hex(int(rb[i]))))
