"""Pins of the oracle's multilevel decomposition (hierarchical multilinear
interpolation, the reading of the prior-work decomposition of Sec. 2/3).

Each check ties the oracle to something other than itself: the hat-function
basis written out from its definition, closed forms for linear and quadratic
fields, a hand-derived 1D case with the right-boundary rule, node counts by
brute force, and the max-error bound of a convex interpolation.
"""
import itertools

import numpy as np
import pytest

from oracle import multilevel as ml


def _level_of(idx, nsteps):
    """Brute force: the step at which a node first appears (nsteps = coarsest)."""
    j = 0
    while j < nsteps and all(i % (2 << j) == 0 for i in idx):
        j += 1
    return j


@pytest.mark.parametrize("shape,nsteps", [((9, 5, 17), 2), ((7, 10, 13), 3), ((1, 1, 6), 2),
                                          ((4, 4, 4), 5), ((0, 3, 3), 1), ((16, 16, 16), 4)])
def test_level_sizes_by_brute_force(shape, nsteps):
    counts = [0] * (nsteps + 1)
    for idx in itertools.product(*(range(n) for n in shape)):
        counts[nsteps - _level_of(idx, nsteps)] += 1
    assert ml.level_sizes(shape, nsteps) == counts
    u = np.random.default_rng(0).standard_normal(shape)
    assert [len(c) for c in ml.decompose(u, nsteps)] == counts


def test_level_sizes_dyadic_cube():
    # 512^3 in 8 steps: 8 coarsest nodes, then each level 7/8 of what remains
    s = ml.level_sizes((512, 512, 512), 8)
    assert s == [8] + [7 * 8 ** l for l in range(1, 9)]
    assert sum(s) == 512 ** 3


def _hat_basis(shape, nsteps):
    """Columns: each level's nodes (coarsest first, row-major on their grid) as
    tensor-product hat functions of half-width = the stride of their grid."""
    pts = np.array(list(itertools.product(*(range(n) for n in shape))), dtype=np.float64)
    cols = []
    for l in range(nsteps + 1):
        h = 1 << (nsteps - l) if l else 1 << nsteps
        g = [range(0, n, h) for n in shape]
        for p in itertools.product(*g):
            if l and _level_of(p, nsteps) != nsteps - l:
                continue
            w = np.ones(len(pts))
            for d in range(3):
                w *= np.maximum(0.0, 1.0 - np.abs(pts[:, d] - p[d]) / h)
            cols.append(w)
    return np.stack(cols, axis=1)


def test_recompose_is_hat_function_expansion():
    # n - 1 a multiple of 2^nsteps on every axis: no boundary extrapolation
    shape, nsteps = (9, 5, 17), 2
    A = _hat_basis(shape, nsteps)
    sizes = ml.level_sizes(shape, nsteps)
    assert A.shape == (np.prod(shape), sum(sizes))
    rng = np.random.default_rng(1)
    c = rng.integers(-64, 64, sum(sizes)).astype(np.float64) / 8
    levels = np.split(c, np.cumsum(sizes)[:-1])
    u = ml.recompose(levels, shape, nsteps)
    np.testing.assert_array_equal(u.ravel(), A @ c)
    # and the decomposition inverts it
    back = ml.concat(ml.decompose(u, nsteps))
    np.testing.assert_array_equal(back, c)


def test_one_dimensional_right_boundary_by_hand():
    u = np.array([3.0, 5.0, -1.0, 4.0, 2.0, 7.0]).reshape(1, 1, 6)
    lv = ml.decompose(u, 2)
    x = u.ravel()
    np.testing.assert_array_equal(lv[0], [x[0], x[4]])
    np.testing.assert_array_equal(lv[1], [x[2] - (x[0] + x[4]) / 2])
    np.testing.assert_array_equal(lv[2], [x[1] - (x[0] + x[2]) / 2, x[3] - (x[2] + x[4]) / 2, x[5] - x[4]])
    np.testing.assert_array_equal(ml.recompose(lv, u.shape, 2), u)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_multilinear_field_has_zero_detail(dtype):
    shape, nsteps = (17, 9, 33), 3
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64) for n in shape), indexing="ij")
    u = (3 + 2 * x - y + 0.5 * z + 0.25 * x * y - 0.125 * y * z + x * z / 16 + x * y * z / 32).astype(dtype)
    lv = ml.decompose(u, nsteps)
    for l in range(1, nsteps + 1):
        assert not np.any(lv[l]), l


def test_quadratic_field_detail_closed_form():
    # u = x^2 + y^2 + z^2: a node with m odd axes at stride h gets -m h^2
    shape, nsteps = (9, 17, 33), 3
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64) for n in shape), indexing="ij")
    lv = ml.decompose(x * x + y * y + z * z, nsteps)
    for l in range(1, nsteps + 1):
        h = 1 << (nsteps - l)
        dims = ml.grid_dims(shape, h)
        a = np.stack(np.meshgrid(*(np.arange(m) for m in dims), indexing="ij"))
        nodd = (a % 2).sum(axis=0)
        want = (-(h * h) * nodd)[nodd > 0]
        np.testing.assert_array_equal(lv[l], want)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape,nsteps", [((7, 10, 13), 3), ((12, 1, 20), 4), ((5, 6, 7), 0), ((3, 3, 3), 6)])
def test_round_trip_exact_on_small_integers(dtype, shape, nsteps):
    u = np.random.default_rng(2).integers(-500, 500, shape).astype(dtype)
    lv = ml.decompose(u, nsteps)
    assert all(x.dtype == dtype for x in lv)
    np.testing.assert_array_equal(ml.recompose(lv, shape, nsteps), u)


def test_float32_coefficients_within_rounding_of_float64():
    shape, nsteps = (20, 33, 40), 4
    u = np.random.default_rng(3).standard_normal(shape).astype(np.float32)
    c32 = ml.concat(ml.decompose(u, nsteps)).astype(np.float64)
    c64 = ml.concat(ml.decompose(u.astype(np.float64), nsteps))
    M = float(np.abs(u).max())
    # three nested means and one subtraction, each rounding once
    assert np.abs(c32 - c64).max() <= 8 * 2.0 ** -24 * M


def test_field_error_bounded_by_sum_of_level_errors():
    shape, nsteps = (13, 21, 18), 3
    rng = np.random.default_rng(4)
    u = rng.standard_normal(shape)
    lv = ml.decompose(u, nsteps)
    eps = [10.0 ** -(l + 1) for l in range(nsteps + 1)]
    worst = 0.0
    for trial in range(4):
        pert = [x + rng.choice([-1.0, 1.0], x.size) * e * (1 if trial % 2 else rng.random(x.size))
                for x, e in zip(lv, eps)]
        err = np.abs(ml.recompose(pert, shape, nsteps) - u).max()
        assert err <= sum(eps) * (1 + 1e-9), (trial, err)
        worst = max(worst, err)
    # same-sign perturbations of every level reach the bound at some node
    same = [x + e for x, e in zip(lv, eps)]
    assert np.abs(ml.recompose(same, shape, nsteps) - u).max() == pytest.approx(sum(eps), rel=1e-9)
