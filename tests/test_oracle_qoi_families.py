"""Pins for the oracle's QoI families beyond V_total (Sec. 5.2's error control
for derived quantities): sum of squares of 1..3 variables, the magnitude
sqrt(sum of squares), and the product of two variables.  Each family's
pointwise estimate is checked at hand-computed points (where the bound is
attained, or by a closed form), against sampled perturbations inside the
bounds, and the retrieval loop against the paper's invariant real <= tau' <=
tau and hand-derived initial plans."""
import math

import numpy as np
import pytest

import workloads

INFL = 1.0 + 2.0 ** -40


def test_product_estimate_is_attained_at_a_corner(orc):
    # vhat = (3, -2), eps = (1/2, 1/4): 3/4 + 1 + 1/8 = 15/8, reached by
    # (3.5)(-2.25) = -7.875 against -6
    m, at = orc.qoi_score_max("product", [np.array([3.0]), np.array([-2.0])], [0.5, 0.25])
    assert m == 1.875 and at == 0
    assert orc.qoi_estimate("product", 2, m, [0.5, 0.25]) == 1.875 * INFL
    assert abs(3.5 * -2.25 - (3.0 * -2.0)) == 1.875


def test_sum_of_squares_one_variable(orc):
    # |v^2 - 9| for v in [2.5, 3.5]: largest at 3.5, 12.25 - 9 = 3.25 = eps (2|vhat| + eps)
    m, _ = orc.qoi_score_max("sumsq", [np.array([-3.0])], [0.5])
    assert m == 3.25 and orc.qoi_estimate("sumsq", 1, m, [0.5]) == 3.25 * INFL


def test_magnitude_estimate_closed_forms(orc):
    # perpendicular error: vhat = (0, 32, 0), eps = (1/2, 0, 0): D = 1/4, Shat =
    # 1024, D^2 / Shat = 2^-14 < A = 1/4, so tau' = 2^-7; the real worst is
    # sqrt(1024.25) - 32 = 0.0039...
    v = [np.array([0.0]), np.array([32.0]), np.array([0.0])]
    m, _ = orc.qoi_score_max("magnitude", v, [0.5, 0.0, 0.0])
    assert m == 2.0 ** -14
    assert orc.qoi_estimate("magnitude", 3, m, [0.5, 0.0, 0.0]) == 2.0 ** -7 * INFL
    assert math.sqrt(1024.25) - 32.0 <= 2.0 ** -7
    # parallel error: vhat = (3, 4, 0), eps = (1/2, 1/2, 0): D = 7.5, D^2 / Shat =
    # 2.25 > A = 1/2, so tau' = sqrt(1/2); the real worst is sqrt(32.5) - 5
    v = [np.array([3.0]), np.array([4.0]), np.array([0.0])]
    m, _ = orc.qoi_score_max("magnitude", v, [0.5, 0.5, 0.0])
    assert m == 2.25
    assert orc.qoi_estimate("magnitude", 3, m, [0.5, 0.5, 0.0]) == math.sqrt(0.5) * INFL
    assert math.sqrt(32.5) - 5.0 <= math.sqrt(0.5)
    # at the origin the ratio is infinite and the estimate is sqrt(A) = the real worst
    v = [np.array([0.0]), np.array([0.0])]
    m, _ = orc.qoi_score_max("magnitude", v, [0.25, 0.0])
    assert m == math.inf and orc.qoi_estimate("magnitude", 2, m, [0.25, 0.0]) == 0.25 * INFL


@pytest.mark.parametrize("kind,nv", [("sumsq", 1), ("sumsq", 2), ("sumsq", 3), ("magnitude", 1),
                                     ("magnitude", 2), ("magnitude", 3), ("product", 2)])
def test_estimates_bound_sampled_perturbations(orc, kind, nv):
    """At random points and bounds, the QoI of any perturbation inside the
    bounds (corners, and uniform samples) differs from the reconstruction's by
    at most the point estimate."""
    from fractions import Fraction as Fr
    rng = np.random.default_rng(11 + nv + 7 * len(kind))

    def err(v, vh):
        # the QoI difference, exact in rationals (for the magnitude: the exact
        # difference of the squares over the sum of the two roots, relative
        # error ~1e-16, far below the estimate's 2^-40 cover)
        v = [Fr(x) for x in v]
        vh = [Fr(x) for x in vh]
        if kind == "product":
            return abs(v[0] * v[1] - vh[0] * vh[1])
        d = sum(x * x for x in v) - sum(x * x for x in vh)
        if kind == "sumsq":
            return abs(d)
        den = math.sqrt(float(sum(x * x for x in v))) + math.sqrt(float(sum(x * x for x in vh)))
        return Fr(abs(float(d)) / den) if den > 0 else Fr(0)

    for trial in range(300):
        vh = [float(x) for x in rng.laplace(0, 2, nv) * (rng.random(nv) < 0.8)]
        eps = [float(x) for x in rng.uniform(0, 1, nv) * (10.0 ** rng.integers(-3, 1))]
        est = orc.qoi_point_estimate(kind, vh, eps)
        pts = [[Fr(vh[c]) + Fr(eps[c]) * (ix[c] - 1) for c in range(nv)] for ix in np.ndindex(*(3,) * nv)]
        pts += [[Fr(vh[c]) + Fr(eps[c]) * Fr(float(u)) for c, u in enumerate(rng.uniform(-1, 1, nv))]
                for _ in range(20)]
        worst = max(err(p, vh) for p in pts)
        assert worst <= Fr(est), (kind, vh, eps, float(worst), est)


def _ones_level(orc, vals):
    return orc.refactor([np.array(vals, np.float32)], 8, orc.Params(group_planes=1))


def test_initial_bounds_by_hand(orc):
    """Variables of two values +-a, a = 1 - 2^-8, so E[k] = 2^-k - 2^-8 (as in
    the V_total pin).  Product at tau = 1/16: eps = tau / (2a) = 0.0314, between
    E[5] = 0.0273 and E[4] = 0.0586, so k = 5 (tau / a or tau alone would give
    4).  Magnitude of two variables at tau = 3/32: eps = tau / sqrt(2) = 0.0663
    >= E[4], so k = 4 (tau / 2 or tau / 3 would give 5); then tau' = sqrt(A) =
    sqrt(2) 15/256 = 0.0829 <= tau, since D^2 / Shat = 0.0292 exceeds A =
    450/65536: one round."""
    a = 1.0 - 2.0 ** -8
    two = [_ones_level(orc, [a, -a]) for _ in range(2)]
    e = orc.qoi_initial_bounds("product", two, 1.0 / 16)
    assert e == [1.0 / 16 / (2.0 * a)] * 2
    vals, ks, tp, met, it = orc.retrieve_qoi("product", two, 1.0 / 16, max_iter=1)
    assert ks == [[5], [5]]
    # (1 - 2^-5) 7/256 twice plus (7/256)^2 = 3521/65536
    assert tp == (3521.0 / 65536.0) * INFL and met
    vals, ks, tp, met, it = orc.retrieve_qoi("magnitude", two, 3.0 / 32)
    assert ks == [[4], [4]] and it == 1 and met
    assert tp == math.sqrt(450.0 / 65536.0) * INFL


@pytest.mark.parametrize("kind,nv", [("sumsq", 1), ("sumsq", 2), ("magnitude", 3), ("magnitude", 1),
                                     ("product", 2)])
@pytest.mark.parametrize("estimator", ["mape", "ma", "cp"])
def test_loop_guarantee(orc, kind, nv, estimator):
    """The paper's check for every family and estimator: the real QoI error of
    the reconstruction (from the originals) <= tau' <= tau."""
    rng = np.random.default_rng(21 + nv)
    sizes = [8, 56, 448, 3584]
    raw = [workloads.laplace_levels(sizes, 1.0 + 0.5 * i, rng) for i in range(nv)]
    vs = [orc.refactor(levels, 32, orc.Params()) for levels in raw]
    orig = [np.concatenate([a.astype(np.float64) for a in levels]) for levels in raw]

    def qoi(v):
        if kind == "product":
            return v[0] * v[1]
        s = sum(x * x for x in v)
        return np.sqrt(s) if kind == "magnitude" else s

    q = qoi(orig)
    scale = orc.qoi_scale(kind, vs)
    for rel in (1e-1, 1e-3, 1e-5):
        tau = rel * scale
        vals, ks, tp, met, it = orc.retrieve_qoi(kind, vs, tau, c=2.0, estimator=estimator)
        assert met and tp <= tau
        real = float(np.abs(qoi(vals) - q).max())
        assert real <= tp, (rel, real, tp)


def test_sum_of_squares_of_three_is_vtotal(orc):
    """The family with three variables is V_total: same planes, estimate and
    rounds as the V_total loop, for every estimator."""
    rng = np.random.default_rng(31)
    raw = [workloads.laplace_levels([8, 56, 448], 1.0, rng) for _ in range(3)]
    vs = [orc.refactor(levels, 32, orc.Params()) for levels in raw]
    for est in ("mape", "ma", "cp"):
        for rel in (1e-2, 1e-4):
            tau = rel * orc.qoi_scale("sumsq", vs)
            a = orc.retrieve_qoi("sumsq", vs, tau, c=2.0, estimator=est)
            b = orc.retrieve_qoi_vtotal(vs, tau, c=2.0, estimator=est)
            assert a[1] == b[1] and a[2] == b[2] and a[4] == b[4]
