"""Pins for the oracle's planner (tolerance -> planes) and the V_total QoI loop
(Sec. 5.2, Alg. 3 with MAPE)."""
import itertools
import math

import numpy as np
import pytest

import workloads


def test_single_level_greedy_is_smallest_k(orc):
    """One level: the greedy reduces to the smallest group-aligned k with E[k] <= tol."""
    rng = np.random.default_rng(1)
    x = rng.laplace(0, 1, 20000).astype(np.float32)
    for m in (1, 3, 4):
        lv = orc.Level(x, 32, orc.Params(group_planes=m))
        ks = sorted(set([min(32, g * m) for g in range(0, 32 // m + 2)]))
        for tol in [10.0, 1.0, 1e-1, 1e-3, 1e-6, 1e-9, 0.0]:
            k, bound = orc.plan([lv], tol)
            brute = next((kk for kk in ks if lv.E[kk] <= tol), 32)
            assert k == [brute] and bound == lv.E[brute]


def test_multilevel_greedy_meets_bound_bruteforce(orc):
    """Tiny cases: enumerate every k-vector; the greedy's choice meets the bound
    whenever some choice does, and only stops early when the bound is met."""
    rng = np.random.default_rng(2)
    sizes = [8, 56, 448]
    levels = [rng.laplace(0, 2.0 ** -l, s).astype(np.float32) for l, s in enumerate(sizes)]
    lv = orc.refactor(levels, 8, orc.Params(group_planes=2, force_method=orc.DC))
    grid = [0, 2, 4, 6, 8]
    bounds = {kv: sum(float(L.E[k]) for L, k in zip(lv, kv)) for kv in itertools.product(grid, repeat=3)}
    for tol in [1.0, 0.3, 0.1, 0.03, 0.01, 0.003, 1e-4, 0.0]:
        k, bound = orc.plan(lv, tol)
        assert tuple(k) in bounds and bound == bounds[tuple(k)]
        feasible = any(b <= tol for b in bounds.values())
        assert (bound <= tol) == feasible
    # the greedy's step sequence does not depend on tol (only where it stops), so
    # planning on from an earlier result equals planning from scratch
    for t1, t2 in [(0.3, 0.03), (0.1, 0.003), (0.03, 1e-4)]:
        k1, _ = orc.plan(lv, t1)
        assert orc.plan(lv, t2, k1) == orc.plan(lv, t2)


def test_bound_is_conservative_on_reconstruction(orc):
    rng = np.random.default_rng(3)
    levels = workloads.laplace_levels([8, 56, 448, 3584], b0=1.0, rng=rng)
    lv = orc.refactor(levels, 32, orc.Params(group_planes=4))
    rng_v = orc.variable_range(lv)
    for rel in (1e-1, 1e-3, 1e-6):
        vals, k, bound, met = orc.retrieve_to(lv, rel)
        assert met
        err = max(float(np.abs(v.astype(np.float64) - x).max()) for v, x in zip(vals, levels))
        assert err <= bound <= rel * rng_v


def test_qoi_vtotal_guarantee(orc):
    """The paper's QoI check: max real V_total error <= estimate <= requested."""
    rng = np.random.default_rng(4)
    sizes = [8, 56, 448, 3584]
    raw = [workloads.laplace_levels(sizes, 1.0, rng) for _ in range(3)]
    vars3 = [orc.refactor(levels, 32, orc.Params()) for levels in raw]
    orig = [np.concatenate([a.astype(np.float64) for a in levels]) for levels in raw]
    vt = orig[0] ** 2 + orig[1] ** 2 + orig[2] ** 2
    rng_q = float(vt.max() - vt.min())
    for rel in (1e-1, 1e-3, 1e-5):
        tau = rel * rng_q
        vals, ks, tprime, met, it = orc.retrieve_qoi_vtotal(vars3, tau)
        assert met and tprime <= tau
        real = np.abs(vals[0] ** 2 + vals[1] ** 2 + vals[2] ** 2 - vt).max()
        assert real <= tprime


def test_qoi_argmax_first_of_ties_bruteforce(orc):
    """The CP estimator's point: the first index with the largest estimate,
    checked by brute force in plain Python floats on small inputs with planted
    ties (the maximum copied to earlier and later positions)."""
    rng = np.random.default_rng(5)
    for trial in range(20):
        n = int(rng.integers(1, 300))
        v = [rng.laplace(0, 1, n) for _ in range(3)]
        eps = [float(x) for x in rng.uniform(1e-4, 1e-1, 3)]
        if n > 3:
            src = int(rng.integers(0, n))
            for dst in rng.choice(n, 2, replace=False):
                for c in range(3):
                    v[c][dst] = -v[c][src] if trial % 2 else v[c][src]  # |.| ties
        best, at = -1.0, n
        for i in range(n):
            s = 0.0
            for c in range(3):
                s = s + eps[c] * ((2.0 * abs(float(v[c][i]))) + eps[c])
            if s > best:
                best, at = s, i
        assert orc.qoi_argmax(v[0], v[1], v[2], eps) == at
        assert orc.qoi_tau(v[0], v[1], v[2], eps) == best * (1.0 + 2.0 ** -40)


def test_cp_bounds_take_the_fewest_decays(orc):
    """The CP step stops at the first multiple of the decay that brings the
    worst point's estimate within tau (one decay fewer would not)."""
    rng = np.random.default_rng(6)
    for _ in range(50):
        v = [abs(float(x)) for x in rng.laplace(0, 4, 3)]
        eps = [float(x) for x in rng.uniform(1e-3, 1.0, 3)]
        tau = float(10 ** rng.uniform(-8, 0))
        decay = float(rng.choice([0.5, 0.25, 0.9]))
        e = orc.cp_bounds(v, eps, tau, decay)

        def est(b):
            return sum(b[c] * (2 * v[c] + b[c]) for c in range(3)) * (1 + 2.0 ** -40)

        ratio = e[0] / eps[0]
        steps = round(math.log(ratio) / math.log(decay)) if ratio > 0 else None
        assert steps is not None and steps >= 0
        assert est(e) <= tau
        if steps > 0:
            back = [x / decay for x in e]
            assert est(back) > tau


@pytest.mark.parametrize("estimator,c", [("mape", 10.0), ("mape", 2.0), ("ma", 10.0), ("cp", 10.0)])
def test_qoi_estimators_guarantee(orc, estimator, c):
    """Every estimator of Sec. 5.2 ends with max real V_total error <= estimate
    <= requested tolerance (the paper's check), and MA is MAPE that never takes
    the proportional step (an infinite threshold)."""
    rng = np.random.default_rng(7)
    sizes = [8, 56, 448, 3584]
    raw = [workloads.laplace_levels(sizes, 1.0 + 0.5 * i, rng) for i in range(3)]
    vars3 = [orc.refactor(levels, 32, orc.Params()) for levels in raw]
    orig = [np.concatenate([a.astype(np.float64) for a in levels]) for levels in raw]
    vt = orig[0] ** 2 + orig[1] ** 2 + orig[2] ** 2
    rng_q = float(vt.max() - vt.min())
    for rel in (1e-1, 1e-2, 1e-4, 1e-6):
        tau = rel * rng_q
        vals, ks, tprime, met, it = orc.retrieve_qoi_vtotal(vars3, tau, c=c, estimator=estimator)
        assert met and tprime <= tau
        real = np.abs(vals[0] ** 2 + vals[1] ** 2 + vals[2] ** 2 - vt).max()
        assert real <= tprime
        if estimator == "ma":
            same = orc.retrieve_qoi_vtotal(vars3, tau, c=math.inf, estimator="mape")
            assert same[1] == ks and same[2] == tprime and same[4] == it


def _ones_level(orc, vals):
    """One level of float32 values, 8 planes, one plane per group."""
    return orc.refactor([np.array(vals, np.float32)], 8, orc.Params(group_planes=1))


def test_qoi_initial_bound_and_mape_step_by_hand(orc):
    """Alg. 3 traced by hand on three variables whose error tables are known in
    closed form.  Each variable is one level of two values +-a, a = 1 - 2^-8
    (eight ones below the binary point), so e = 0 and after k planes the tail
    is E[k] = 2^-k - 2^-8 and the value held is 1 - 2^-k.

    Initial bound (Sec. 5.2): eps_c = (tau / Q_max) * range_c with
    Q_max = sum_c max|v_c|^2 = 3a^2 and range_c = 2a, so eps = 2 tau / (3a);
    at tau = 1/16 that is 0.041830...; E[4] = 15/256 is above it and
    E[5] = 7/256 below, so every variable starts at k = 5 (the reading
    eps = tau would give k = 4; tau / Q_max or tau * max|v| / Q_max, k = 6).

    First estimate: tau' = 3 * E[5] * (2 (1 - 2^-5) + E[5]) = 10563/65536
    (exact in binary), times the 1 + 2^-40 rounding cover.  p = tau'/tau =
    2.579 > c = 2, so MAPE sets eps <- E[5] / p = 0.010604: E[6] = 3/256 is
    above it, E[7] = 1/256 below, so k = 7 and tau' = 3 * 509 / 65536 <= tau:
    done after two estimates.  Dividing by p is what reaches k = 7: eps * p
    adds no plane and neither does skipping the step (p < c read the other way
    round); both fall back to one more plane (k = 6, tau' = 4563/65536 > tau)
    and need a third estimate, which is what MA (c = infinity) does."""
    a = 1.0 - 2.0 ** -8
    vars3 = [_ones_level(orc, [a, -a]) for _ in range(3)]
    for lv in vars3:
        assert list(lv[0].E) == [a] + [2.0 ** -k - 2.0 ** -8 for k in range(1, 9)]
    tau = 1.0 / 16
    for e in orc.qoi_initial_eps(vars3, tau):
        assert abs(e - 2.0 * tau / (3.0 * a)) <= 4e-16 * e
    inflate = 1.0 + 2.0 ** -40
    vals, ks, tp, met, it = orc.retrieve_qoi_vtotal(vars3, tau, c=2.0, max_iter=1)
    assert ks == [[5], [5], [5]] and it == 1 and not met
    assert tp == (10563.0 / 65536.0) * inflate
    vals, ks, tp, met, it = orc.retrieve_qoi_vtotal(vars3, tau, c=2.0)
    assert ks == [[7], [7], [7]] and it == 2 and met
    assert tp == (3.0 * 509.0 / 65536.0) * inflate
    # minimal augmentation takes one plane per round: 5 -> 6 -> 7
    vals, ks, tp, met, it = orc.retrieve_qoi_vtotal(vars3, tau, c=math.inf)
    assert ks == [[7], [7], [7]] and it == 3 and met
    vals, ks, tp, met, it = orc.retrieve_qoi_vtotal(vars3, tau, c=math.inf, max_iter=2)
    assert ks == [[6], [6], [6]] and tp == (4563.0 / 65536.0) * inflate


def test_qoi_initial_bound_scales_with_each_range(orc):
    """Uneven variables: +-a, {a/2, 0} and +-a/4 (a = 1 - 2^-8; exponents 0,
    -1, -2, so E_x[k] = 2^-k - 2^-8, E_y[k] = 2^-(k+1) - 2^-9,
    E_z[k] = 2^-(k+2) - 2^-10).  Q_max = a^2 (1 + 1/4 + 1/16) = 21 a^2 / 16 and
    the ranges are 2a, a/2, a/2, so at tau = 1/16 the initial bounds are
    2/(21a) = 0.0956 and 1/(42a) = 0.0239 (twice).  The smallest k under them:
    x: E[3] = 0.121 > 0.0956 >= E[4] = 0.0586, so 4; y: E[4] = 0.0293 > 0.0239
    >= E[5] = 0.0137, so 5; z: E[3] = 0.0303 > 0.0239 >= E[4] = 0.0146, so 4."""
    a = 1.0 - 2.0 ** -8
    vars3 = [_ones_level(orc, [a, -a]), _ones_level(orc, [a / 2, 0.0]), _ones_level(orc, [-a / 4, a / 4])]
    eps = orc.qoi_initial_eps(vars3, 1.0 / 16)
    for got, want in zip(eps, [2.0 / (21.0 * a), 1.0 / (42.0 * a), 1.0 / (42.0 * a)]):
        assert abs(got - want) <= 4e-16 * want
    vals, ks, tp, met, it = orc.retrieve_qoi_vtotal(vars3, 1.0 / 16, c=2.0, max_iter=1)
    assert ks == [[4], [5], [4]]
