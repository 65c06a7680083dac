"""Pins for the oracle's planner (tolerance -> planes) and the V_total QoI loop
(Sec. 5.2, Alg. 3 with MAPE)."""
import itertools

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
