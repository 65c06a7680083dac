"""Pins of the oracle's squared-L2 per-plane table (the MDR option of an L2
error table beside the L-infinity one) and of L2-driven planning: the k = 0
closed form, exact rational sums on tiny inputs, the sandwich between the
L-infinity table (computed by other code) squared and n times it, monotonicity,
exact representation, and the planner's guarantee."""
from fractions import Fraction

import numpy as np
import pytest


def _level(orc, x, B):
    lv = orc.refactor([x], B)[0]
    return lv, orc.l2_table(x, lv)


@pytest.mark.parametrize("dtype,B", [(np.float32, 32), (np.float64, 64), (np.float32, 12)])
def test_first_entry_is_the_sum_of_squares(orc, dtype, B):
    x = np.random.default_rng(1).laplace(0, 1, 5000).astype(dtype)
    lv, E2 = _level(orc, x, B)
    x64 = x.astype(np.float64)
    assert E2[0] == pytest.approx(float(np.sum(x64 * x64)), rel=1e-12)


@pytest.mark.parametrize("B", [3, 7, 32])
def test_exact_rationals_on_tiny_inputs(orc, B):
    rng = np.random.default_rng(2)
    x = (rng.integers(-2 ** 12, 2 ** 12, 9) / 2.0 ** 7).astype(np.float32)
    lv, E2 = _level(orc, x, B)
    e = lv.e
    for k in range(B + 1):
        s = Fraction(0)
        for v in x.tolist():
            a = Fraction(abs(v))
            q = Fraction(2) ** (k - e)
            xh = Fraction(int(a * q)) / q   # top k bits of the aligned magnitude
            s += (a - xh) ** 2
        # each square rounded once in fp64, the sum exactly rounded
        assert abs(Fraction(E2[k]) - s) <= Fraction(len(x)) * Fraction(2) ** -52 * s, k


@pytest.mark.parametrize("dtype,B", [(np.float32, 32), (np.float64, 64)])
def test_sandwich_by_the_linf_table_and_monotone(orc, dtype, B):
    x = np.random.default_rng(3).laplace(0, 3, 4000).astype(dtype)
    lv, E2 = _level(orc, x, B)
    n = x.size
    for k in range(B + 1):
        lo, hi = lv.E[k] ** 2, n * lv.E[k] ** 2
        assert lo * (1 - 1e-12) <= E2[k] <= hi * (1 + 1e-12) or (lv.E[k] == 0 and E2[k] == 0), k
    assert np.all(np.diff(E2) <= 0)


def test_exactly_representable_values_vanish_at_full_precision(orc):
    x = np.random.default_rng(4).integers(-1000, 1000, 3000).astype(np.float32)
    lv, E2 = _level(orc, x, 32)
    assert E2[32] == 0.0 and E2[0] > 0


def test_l2_plan_meets_the_squared_bound(orc):
    rng = np.random.default_rng(5)
    xs = [rng.laplace(0, 2.0 ** -l, 2000 * (l + 1)).astype(np.float32) for l in range(4)]
    levels = orc.refactor(xs, 32)
    tables = [orc.l2_table(x, lv) for x, lv in zip(xs, levels)]
    total = float(np.sqrt(sum(t[0] for t in tables)))
    for rel in (1e-1, 1e-3, 1e-6):
        tol = rel * total
        k, bound = orc.plan_l2(levels, tables, tol)
        assert bound == pytest.approx(sum(t[kk] for t, kk in zip(tables, k)), rel=1e-15)
        assert bound <= tol * tol
        # the field of reconstructions really is within tol in L2
        err2 = sum(float(np.sum((x.astype(np.float64) - lv.reconstruct(kk).astype(np.float64)) ** 2))
                   for x, lv, kk in zip(xs, levels, k))
        assert err2 <= tol * tol * (1 + 1e-9)
