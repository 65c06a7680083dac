"""Pins for the oracle's lossless stage (Sec. 4): Huffman, RLE, direct copy, the
hybrid selection of Alg. 2, CRC-32 and the container."""
import heapq
import itertools
import json
import os
import zlib

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def kraft(lengths):
    from fractions import Fraction
    return sum(Fraction(1, 2 ** int(L)) for L in lengths if L)


def heap_huffman_cost(freq):
    """Textbook Huffman (heapq) total cost sum f*L; unique for any tie-breaking."""
    h = [int(f) for f in freq if f]
    if len(h) == 1:
        return h[0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a = heapq.heappop(h)
        b = heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


def brute_optimal_cost(freq):
    """Minimum sum f*L over all length vectors with Kraft sum exactly 1 (<= 6 symbols)."""
    from fractions import Fraction
    f = [int(v) for v in freq if v]
    best = None
    for ls in itertools.product(range(1, len(f)), repeat=len(f)):
        if sum(Fraction(1, 2 ** L) for L in ls) == 1:
            c = sum(a * b for a, b in zip(f, ls))
            best = c if best is None else min(best, c)
    return best


# ------------------------------------------------------------------ Huffman
def test_golden_huffman(orc):
    g = json.load(open(os.path.join(GOLD, "toy_huffman.json")))
    freq = np.zeros(256, np.uint64)
    for s, c in g["counts"].items():
        freq[int(s)] = c
    ln = orc.huffman_lengths(freq, 12)
    assert {s: int(ln[int(s)]) for s in g["lengths"]} == g["lengths"]
    codes = orc.huffman_codes(ln)
    assert {s: int(codes[int(s)]) for s in g["codes"]} == g["codes"]
    p = orc.huffman_encode(bytes(g["message"]), 1024, 12)
    assert len(p) == g["payload_total_bytes"]
    words = np.frombuffer(p[8 + 256 + 8:], "<u4").tolist()
    assert words == g["payload_words"]
    assert orc.huffman_decode(p, len(g["message"]), 1024) == bytes(g["message"])


def test_huffman_kraft_and_optimality(orc):
    rng = np.random.default_rng(3)
    for trial in range(200):
        nsym = int(rng.integers(1, 257))
        freq = np.zeros(256, np.uint64)
        syms = rng.choice(256, nsym, replace=False)
        freq[syms] = rng.integers(1, 1000, nsym)
        ln = orc.huffman_lengths(freq, 24)
        assert kraft(ln) == 1
        assert all((ln > 0) == (freq > 0)) or nsym == 1
        if nsym > 1:
            assert int((freq * ln.astype(np.uint64)).sum()) == heap_huffman_cost(freq)
    for trial in range(40):
        nsym = int(rng.integers(2, 7))
        freq = np.zeros(256, np.uint64)
        freq[rng.choice(256, nsym, replace=False)] = rng.integers(1, 50, nsym)
        ln = orc.huffman_lengths(freq, 24)
        assert int((freq * ln.astype(np.uint64)).sum()) == brute_optimal_cost(freq)


def test_huffman_single_symbol_phantom(orc):
    for s in (0, 7, 255):
        freq = np.zeros(256, np.uint64)
        freq[s] = 1000
        ln = orc.huffman_lengths(freq, 12)
        assert ln[s] == 1 and kraft(ln) == 1 and int((ln > 0).sum()) == 2
        msg = bytes([s]) * 3000
        p = orc.huffman_encode(msg, 1024, 12)
        assert orc.huffman_decode(p, len(msg), 1024) == msg


def test_huffman_length_limit_fibonacci(orc):
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    freq = np.zeros(256, np.uint64)
    freq[:40] = fib
    unlimited = orc.huffman_lengths(freq, 24)
    assert unlimited.max() > 12  # the limit must bite
    for lmax in (8, 10, 12, 16):
        ln = orc.huffman_lengths(freq, lmax)
        assert ln.max() <= lmax and kraft(ln) == 1
        # a heavier symbol never gets a longer code
        order = np.argsort(freq[:40], kind="stable")
        assert all(ln[order[i]] >= ln[order[i + 1]] for i in range(39))
    # random skewed counts that exceed the limit keep Kraft equality and the code count
    rng = np.random.default_rng(12)
    for _ in range(50):
        f = np.zeros(256, np.uint64)
        k = int(rng.integers(20, 257))
        f[rng.choice(256, k, replace=False)] = (2.0 ** rng.uniform(0, 30, k)).astype(np.uint64) + 1
        ln = orc.huffman_lengths(f, 10)
        assert ln.max() <= 10 and kraft(ln) == 1 and int((ln > 0).sum()) == k
    msg = np.repeat(np.arange(40, dtype=np.uint8), [min(f, 500) for f in fib]).tobytes()
    for lmax in (9, 12):
        p = orc.huffman_encode(msg, 333, lmax)
        assert orc.huffman_decode(p, len(msg), 333) == msg


def test_huffman_roundtrip_and_prefix_free(orc):
    rng = np.random.default_rng(9)
    for n, chunk in [(0, 1024), (1, 1024), (1023, 1024), (1025, 1024), (5000, 100), (70000, 1024)]:
        msg = np.minimum(rng.geometric(0.3, n), 255).astype(np.uint8).tobytes()
        p = orc.huffman_encode(msg, chunk, 12)
        assert orc.huffman_decode(p, n, chunk) == msg
        freq = np.bincount(np.frombuffer(msg, np.uint8), minlength=256).astype(np.uint64)
        if n:
            ln = orc.huffman_lengths(freq, 12)
            codes = orc.huffman_codes(ln)
            words = [format(int(codes[s]), "0%db" % ln[s]) for s in range(256) if ln[s]]
            for a, b in itertools.permutations(words, 2):
                assert not b.startswith(a)
            assert len(p) >= orc.huffman_estimate(freq, ln, n, chunk)
            assert len(p) <= orc.huffman_estimate(freq, ln, n, chunk) + 4 * ((n + chunk - 1) // chunk)


# ------------------------------------------------------------------ RLE
@pytest.mark.parametrize("wb", [4, 8])
def test_rle_runs_closed_form_and_roundtrip(orc, wb):
    rng = np.random.default_rng(wb)
    for n in (0, 1, 2, 17, 1000):
        w = rng.integers(0, 3, n).astype(np.uint32 if wb == 4 else np.uint64)
        w = np.repeat(w, rng.integers(1, 9, n)) if n else w
        g = w.tobytes()
        runs = orc.rle_runs(g, wb)
        assert runs == (0 if w.size == 0 else 1 + int(np.count_nonzero(np.diff(w))))
        p = orc.rle_encode(g, wb)
        assert len(p) == orc.rle_estimate(runs, wb) == 8 + runs * (wb + 4)
        assert orc.rle_decode(p, len(g), wb) == g


def test_rle_rejects_corruption(orc):
    g = np.array([5, 5, 5, 7], np.uint32).tobytes()
    p = bytearray(orc.rle_encode(g, 4))
    p[8 + 8] = 9  # first run length 3 -> 9: overruns the group
    with pytest.raises(orc.OracleError):
        orc.rle_decode(bytes(p), len(g), 4)


# ------------------------------------------------------------------ Alg. 2 selection
def test_selection_decision_table(orc):
    P = orc.Params
    d = P()  # T_s = 4096, T_cr = 2.0
    # small groups are always copied
    assert orc.select(4096, 1, 1, d) == orc.DC
    # Huffman first when its ratio clears T_cr, RLE second, else DC
    assert orc.select(10000, 4999, 1, d) == orc.HUF
    assert orc.select(10000, 5000, 4999, d) == orc.RLE
    assert orc.select(10000, 5000, 5000, d) == orc.DC
    # thresholds 1.0 and 4.0
    assert orc.select(10000, 9999, 10 ** 6, P(t_cr_milli=1000)) == orc.HUF
    assert orc.select(10000, 2500, 2499, P(t_cr_milli=4000)) == orc.RLE
    # forced method
    assert orc.select(10, 10 ** 9, 10 ** 9, P(force_method=orc.RLE)) == orc.RLE


def test_selection_on_hand_built_groups(orc):
    """End to end on levels whose planes have a known shape."""
    B = 8
    n = 65536
    # all-zero level: every plane is zero bytes -> Huffman (ratio ~ 8)
    lv = orc.Level(np.zeros(n, np.float32), B, orc.Params(group_planes=4))
    assert [m for m, _ in lv.streams] == [orc.HUF, orc.HUF, 3, 3, 3, orc.HUF, 3, 3, 3]
    # random bits in every plane: incompressible -> DC
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, n).astype(np.float32)
    lv = orc.Level(x, B, orc.Params(group_planes=4))
    assert [m for m, _ in lv.streams][0] == orc.DC and lv.streams[1][0] == orc.DC
    # sparse level: long runs of identical words -> Huffman first, RLE when forced by T_cr
    y = np.zeros(n, np.float32)
    y[::4096] = 1.0
    lv = orc.Level(y, B, orc.Params(group_planes=4))
    assert lv.streams[1][0] == orc.HUF
    est_h, est_r = lv.est_huf[1], lv.est_rle[1]
    S = 4 * (n // 8)
    assert est_r < est_h  # runs beat 1 bit per byte here
    t_between = int(1000 * S / est_h) + 1  # Huffman fails, RLE still clears it
    lv = orc.Level(y, B, orc.Params(group_planes=4, t_cr_milli=t_between))
    assert lv.streams[1][0] == orc.RLE
    # tiny level: S <= T_s -> DC
    lv = orc.Level(np.zeros(100, np.float32), B)
    assert all(m in (orc.DC, 3) for m, _ in lv.streams)


def test_all_methods_roundtrip_through_levels(orc):
    rng = np.random.default_rng(2)
    x = rng.laplace(0, 1, 40000).astype(np.float32)
    for fm in (orc.DC, orc.RLE, orc.HUF):
        lv = orc.Level(x, 32, orc.Params(group_planes=4, force_method=fm))
        assert all(m in (fm, 3) for m, _ in lv.streams)
        ref = orc.Level(x, 32, orc.Params(group_planes=4, force_method=orc.DC))
        for k in (0, 4, 12, 32):
            assert lv.reconstruct(k).tobytes() == ref.reconstruct(k).tobytes()


# ------------------------------------------------------------------ CRC + container
def test_crc32_matches_zlib(orc):
    rng = np.random.default_rng(4)
    for n in (0, 1, 9, 1000):
        b = rng.integers(0, 256, n, dtype=np.uint8).tobytes()
        assert orc.crc32(b) == zlib.crc32(b)
    assert orc.crc32(b"123456789") == 0xCBF43926


def test_container_layout(orc):
    rng = np.random.default_rng(8)
    levels = [rng.laplace(0, 2.0 ** -l, s).astype(np.float32) for l, s in enumerate([8, 56, 448])]
    P = orc.Params(group_planes=4)
    lv = orc.refactor(levels, 32, P)
    blob = orc.serialize(lv, P)
    assert blob[:4] == b"MDR1" and blob[4] == 1 and blob[5] == 0 and blob[6] == 32 and blob[7] == 4
    assert int.from_bytes(blob[40:48], "little") == len(blob)
    assert int.from_bytes(blob[48:52], "little") == zlib.crc32(blob[:48])
    pos = 56
    for L in lv:
        assert int.from_bytes(blob[pos:pos + 8], "little") == L.n
        assert int.from_bytes(blob[pos + 8:pos + 12], "little", signed=True) == L.e
        E = np.frombuffer(blob[pos + 40:pos + 40 + 8 * 33], "<f8")
        assert (E == L.E).all()
        tab = pos + 40 + 8 * 33
        sizes = []
        for s in range(33):
            ent = blob[tab + 16 * s:tab + 16 * s + 16]
            meth, crc, nb = ent[0], int.from_bytes(ent[4:8], "little"), int.from_bytes(ent[8:], "little")
            assert meth == L.streams[s][0] and nb == len(L.streams[s][1])
            assert crc == zlib.crc32(L.streams[s][1])
            sizes.append(nb)
        rec_end = tab + 16 * 33
        assert int.from_bytes(blob[rec_end:rec_end + 4], "little") == zlib.crc32(blob[pos:rec_end])
        pos = rec_end + 8
        for s, nb in enumerate(sizes):
            assert blob[pos:pos + nb] == L.streams[s][1]
            pos += (nb + 7) // 8 * 8
    assert pos == len(blob)
