"""Pins for the oracle's bitplane steps (Sec. 3, Alg. 1) and its error table.

Each check reaches the expected value by a route other than the oracle's own
formula: exhaustive search, bit strings of exact rationals, numpy's frexp, a
hand-computed fixture, or an invariant the mathematics fixes.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def frac(v) -> Fraction:
    return Fraction(float(v))


def exp_bruteforce(vals) -> int:
    """Smallest e with |x| < 2^e for every x (search), 0 if all zero."""
    nz = [abs(frac(v)) for v in vals if v != 0]
    if not nz:
        return 0
    a = max(nz)
    e = -1200
    while not a < Fraction(2) ** e:
        e += 1
    return e


def mag_search(v, e, B) -> int:
    """Largest integer m with m * 2^(e-B) <= |v|, by binary search on exact rationals."""
    a = abs(frac(v))
    unit = Fraction(2) ** (e - B)
    lo, hi = 0, 1 << B
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if mid * unit <= a:
            lo = mid
        else:
            hi = mid - 1
    return lo


def bits_msb_first(a: Fraction, e: int, B: int) -> str:
    """Binary digits of a/2^e (a < 2^e) after the point, first B of them, by doubling."""
    y = a / Fraction(2) ** e
    out = []
    for _ in range(B):
        y *= 2
        if y >= 1:
            out.append("1")
            y -= 1
        else:
            out.append("0")
    return "".join(out)


def trunc_multiple(a: Fraction, step: Fraction) -> Fraction:
    """Largest multiple of step not above a, by search from the binary expansion."""
    q = 0
    # grow then refine (no floor() of the ratio: a search)
    hi = 1
    while hi * step <= a:
        hi *= 2
    lo = 0
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if mid * step <= a:
            lo = mid
        else:
            hi = mid - 1
    q = lo
    return q * step


# ------------------------------------------------------------------ golden toy
def test_golden_toy_alg1(orc):
    g = json.load(open(os.path.join(GOLD, "toy_alg1.json")))
    x = np.array(g["x"], np.float32)
    B = g["B"]
    e, vmin, vmax, vmaxabs = orc.stats(x)
    assert e == g["e"]
    mag, sign = orc.fixed_point(x, e, B)
    assert mag.tolist() == g["magnitudes"]
    assert sign.tolist() == g["signs"]
    rows = orc.bitplanes(mag, sign, B, 32)
    words = rows.view("<u4")[:, 0].tolist()
    pw = g["plane_words"]
    assert words == [pw["sign"], pw["p0_bit3"], pw["p1_bit2"], pw["p2_bit1"], pw["p3_bit0"]]
    E = orc.error_table(x, mag, e, B)
    assert E.tolist() == g["error_table"]
    lv = orc.Level(x, B, orc.Params(force_method=orc.DC))
    for k, ref in g["reconstruct"].items():
        y = lv.reconstruct(int(k))
        assert y.tolist() == ref
        assert np.signbit(y).tolist() == np.signbit(np.array(ref)).tolist() or int(k) == 0


# ------------------------------------------------------------------ exponent
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_exponent_matches_numpy_frexp(orc, dt):
    rng = np.random.default_rng(7)
    for scale in [1e-300, 1e-40, 1e-3, 1.0, 3.0, 1e5, 1e30, 1e300]:
        if dt == np.float32 and (scale < 1e-44 or scale > 1e37):
            continue
        x = (rng.standard_normal(257) * scale).astype(dt)
        e, lo, hi, am = orc.stats(x)
        assert e == int(np.frexp(np.abs(x).max())[1])
        assert e == exp_bruteforce(x)
        assert am == float(np.abs(x).max()) and lo == float(x.min()) and hi == float(x.max())


def test_exponent_special_cases(orc):
    assert orc.stats(np.zeros(5, np.float32))[0] == 0
    assert orc.stats(np.array([-0.0, 0.0], np.float32))[1:] == (0.0, 0.0, 0.0)
    sub = np.array([1e-45, -3e-44, 0.0], np.float32)  # subnormal-only level
    assert orc.stats(sub)[0] == int(np.frexp(np.float32(3e-44))[1]) == exp_bruteforce(sub)
    for bad in [np.nan, np.inf, -np.inf]:
        with pytest.raises(orc.OracleError):
            orc.stats(np.array([1.0, bad], np.float32))


# ------------------------------------------------------------------ fixed point
@pytest.mark.parametrize("dt,B", [(np.float32, 32), (np.float32, 17), (np.float64, 64),
                                  (np.float64, 40), (np.float32, 1)])
def test_fixed_point_matches_search(orc, dt, B):
    rng = np.random.default_rng(B)
    x = (rng.laplace(0, 1, 300) * 10.0 ** rng.integers(-5, 5, 300)).astype(dt)
    x[:3] = [0.0, -0.0, np.finfo(dt).tiny / 8]
    e = orc.stats(x)[0]
    mag, sign = orc.fixed_point(x, e, B)
    for i in range(x.size):
        assert int(mag[i]) == mag_search(x[i], e, B)
        assert int(mag[i]) == int(bits_msb_first(abs(frac(x[i])), e, B) or "0", 2)
        assert sign[i] == (1 if math.copysign(1.0, float(x[i])) < 0 else 0)


def test_fixed_point_special_values(orc):
    for dt, B in [(np.float32, 32), (np.float64, 64), (np.float32, 8)]:
        # |x| = 2^(e-1) gives exactly 2^(B-1)
        x = np.array([0.5, -0.25, 0.375], dt)
        e = orc.stats(x)[0]
        assert e == 0
        mag, sign = orc.fixed_point(x, e, B)
        assert int(mag[0]) == 1 << (B - 1)
        assert sign.tolist() == [0, 1, 0]
    # largest finite value and subnormals keep exactness
    x = np.array([np.finfo(np.float32).max, 1e-45], np.float32)
    e = orc.stats(x)[0]
    mag, _ = orc.fixed_point(x, e, 32)
    assert int(mag[0]) == mag_search(x[0], e, 32) and int(mag[1]) == 0
    sub = np.array([1e-45, 2.5e-44, -7e-45], np.float32)
    e = orc.stats(sub)[0]
    mag, sign = orc.fixed_point(sub, e, 32)
    assert [int(m) for m in mag] == [mag_search(v, e, 32) for v in sub]
    assert sign.tolist() == [0, 0, 1]


# ------------------------------------------------------------------ planes (Alg. 1)
def literal_alg1(mag, sign, B, W):
    """Alg. 1 transcribed on bit strings: for b = B-1 down to 0, bit (m >> b) & 1 of
    every value, written to a plane as a little-endian bit string."""
    n = len(mag)
    nb = (n + W - 1) // W * (W // 8)

    def flush(bits):
        s = "".join(bits) + "0" * (nb * 8 - len(bits))
        return bytes(int(s[8 * j:8 * j + 8][::-1], 2) for j in range(nb))

    rows = [flush(["1" if s else "0" for s in sign])]
    for b in range(B - 1, -1, -1):
        rows.append(flush([format(int(m), "0%db" % max(B, 1))[B - 1 - b] for m in mag]))
    return rows


@pytest.mark.parametrize("n,B,W", [(1, 32, 32), (31, 32, 32), (33, 32, 32), (100, 5, 32),
                                   (64, 64, 64), (65, 64, 64), (127, 13, 64), (1000, 32, 32)])
def test_planes_literal(orc, n, B, W):
    rng = np.random.default_rng(n * 7 + B)
    mag = rng.integers(0, 1 << B, n, dtype=np.uint64) if B < 64 else \
        rng.integers(0, 1 << 63, n, dtype=np.uint64) * 2 + rng.integers(0, 2, n, dtype=np.uint64)
    sign = rng.integers(0, 2, n).astype(np.uint8)
    rows = orc.bitplanes(mag, sign, B, W)
    ref = literal_alg1(mag, sign, B, W)
    assert rows.shape == (B + 1, len(ref[0]))
    for r in range(B + 1):
        assert rows[r].tobytes() == ref[r], r
    # invertibility: reassembling the planes gives every magnitude and sign back
    bits = np.unpackbits(rows, axis=1, bitorder="little")[:, :n].astype(np.uint64)
    back = np.zeros(n, np.uint64)
    for p in range(B):
        back |= bits[1 + p] << np.uint64(B - 1 - p)
    assert (back == mag).all() and (bits[0] == sign).all()
    # padding beyond n is zero
    assert not np.unpackbits(rows, axis=1, bitorder="little")[:, n:].any()


# ------------------------------------------------------------------ exhaustive tiny
def test_exhaustive_tiny_levels(orc):
    """All 16^3 magnitude patterns of 3 values with B = 4 (plus sign patterns and a
    sub-fixed-point tail on some values): exponent, magnitudes, planes, error table
    and every reconstruction, each checked against exact rationals."""
    B = 4
    for code in range(16 ** 3):
        ms = [(code >> (4 * j)) & 15 for j in range(3)]
        signs = [(code >> j) & 1 for j in range(3)]
        tail = [0.0, 1.0 / 128, 0.0][code % 3]
        vals = [(-1 if s else 1) * (m / 16.0 + (tail if m else 0.0)) for m, s in zip(ms, signs)]
        x = np.array(vals, np.float32)
        e = orc.stats(x)[0]
        assert e == exp_bruteforce(x)
        mag, sign = orc.fixed_point(x, e, B)
        ex = [mag_search(v, e, B) for v in x]
        assert [int(v) for v in mag] == ex
        E = orc.error_table(x, mag, e, B)
        for k in range(B + 1):
            step = Fraction(2) ** (e - k)
            errs = [abs(frac(v)) - trunc_multiple(abs(frac(v)), step) for v in x]
            assert Fraction(float(E[k])) == max(errs), (vals, k)
        if code % 61 == 0:
            lv = orc.Level(x, B, orc.Params(force_method=orc.DC))
            for k in range(B + 1):
                y = lv.reconstruct(k)
                step = Fraction(2) ** (e - k)
                for v, yy in zip(x, y):
                    if k == 0:
                        assert yy == 0.0 and not np.signbit(yy)
                        continue
                    t = trunc_multiple(abs(frac(v)), step)
                    assert Fraction(float(abs(yy))) == t
                    assert np.signbit(yy) == np.signbit(v)


# ------------------------------------------------------------------ error table
@pytest.mark.parametrize("dt,B", [(np.float32, 32), (np.float32, 12), (np.float64, 64),
                                  (np.float64, 30)])
def test_error_table_invariants(orc, dt, B):
    rng = np.random.default_rng(B + 3)
    x = rng.laplace(0, 3.0, 5000).astype(dt)
    x[:4] = [0.0, -0.0, np.finfo(dt).tiny / 4, -np.finfo(dt).tiny]
    lv = orc.Level(x, B, orc.Params(force_method=orc.DC))
    E, e = lv.E, lv.e
    assert E[0] == np.abs(x).max()
    assert all(E[k + 1] <= E[k] for k in range(B))
    for k in range(B + 1):
        assert E[k] < 2.0 ** (e - k)
        assert float(dt(E[k])) == E[k]  # exactly representable in the input type
        y = lv.reconstruct(k).astype(np.float64)
        err = np.abs(x.astype(np.float64) - y)
        assert err.max() <= E[k]
        assert err.max() == E[k]  # the table is the attained maximum
    # Fraction spot check on a sample of values for a few k
    for k in (1, B // 2, B):
        step = Fraction(2) ** (e - k)
        best = max(abs(frac(v)) - trunc_multiple(abs(frac(v)), step) for v in x[:200])
        assert Fraction(float(E[k])) >= best


@pytest.mark.parametrize("dt,B", [(np.float32, 32), (np.float64, 64), (np.float32, 20)])
def test_lossless_when_on_fixed_point_grid(orc, dt, B):
    """Values that are multiples of 2^(e-B) come back bit-exact with all planes."""
    rng = np.random.default_rng(11)
    bits = min(B, 24 if dt == np.float32 else 53)
    m = rng.integers(0, 1 << (bits - 1), 3000).astype(np.float64)
    m[0] = (1 << (bits - 1))  # fixes e
    x = (m * 2.0 ** (-bits + 3) * np.where(rng.random(3000) < 0.5, -1, 1)).astype(dt)
    x[5] = -0.0
    lv = orc.Level(x, B, orc.Params(group_planes=4))
    y = lv.reconstruct(B)
    assert y.tobytes() == x.tobytes()
    assert lv.E[B] == 0.0


def test_bound_after_k_planes(orc):
    """The bound named for the method: |x - xhat^(k)| <= E[k] <= 2^(e-k)."""
    rng = np.random.default_rng(5)
    for n in (1, 31, 32, 33, 1000):
        x = rng.laplace(0, 1, n).astype(np.float32)
        lv = orc.Level(x, 32, orc.Params(group_planes=1))
        for k in range(33):
            y = lv.reconstruct(k).astype(np.float64)
            assert np.abs(x - y).max() <= lv.E[k] <= 2.0 ** (lv.e - k)


def test_ablation_layouts(orc):
    """Sec. 3's encoding experiment (32-bit words -> 32 planes): single bits land
    where each layout says; the block layout equals the magnitude rows of the
    refactor path's bitplanes; the register block's interleaved layout is the
    block layout of the input reordered region by region."""
    rng = np.random.default_rng(9)
    for n in (1, 31, 33, 2047, 2049, 5000):
        for _ in range(5):
            x = np.zeros(n, np.uint32)
            i, b = int(rng.integers(0, n)), int(rng.integers(0, 32))
            x[i] = np.uint32(1) << np.uint32(b)
            blk = orc.ablation_planes(x, False)
            assert blk.sum(dtype=np.uint64) == 1 << (i % 32) and blk[31 - b, i // 32] == 1 << (i % 32)
            itl = orc.ablation_planes(x, True)
            r, o = divmod(i, 2048)
            assert itl.sum(dtype=np.uint64) == 1 << (o // 64)
            assert itl[31 - b, 64 * r + o % 64] == 1 << (o // 64)
        x = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
        blk = orc.ablation_planes(x, False)
        rows = orc.bitplanes(x.astype(np.uint64), np.zeros(n, np.uint8), 32, 32)
        words = rows[1:].copy().view(np.uint32)
        assert np.array_equal(words, blk)
        regions = (n + 2047) // 2048
        xp = np.zeros(regions * 2048, np.uint32)
        xp[:n] = x
        y = xp.reshape(regions, 32, 64).transpose(0, 2, 1).reshape(-1)  # y[32(64r+l)+k] = x[2048r+l+64k]
        assert np.array_equal(orc.ablation_planes(y, False), orc.ablation_planes(x, True))
