"""Multilevel decomposition and recomposition of a 3D field: the oracle side.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and ``bench.py``'s ``cpu_baseline`` leg, never by the product library.

The method (Sec. 2 and Sec. 3) takes its input as the coefficient levels of a
multilevel decomposition that earlier work supplies; the paper does not spell
that decomposition out.  Reading taken here: the hierarchical multilinear
interpolation decomposition, i.e. the interpolation step of MGARD's
decomposition without its L2-projection correction.  Nodes live on a row-major
n0 x n1 x n2 grid (n2 fastest).  With ``nsteps`` coarsening steps, step j
(j = 0 finest) works on the grid of stride h = 2^j; the nodes of that grid
that are not on the stride-2h grid get the coefficient

    c = u - P(u on the stride-2h grid),

where P refines along x (axis 2), then y, then z: a node halfway between two
coarse nodes takes the mean (a + b) * 0.5 of them, and a node past the last
coarse node of its line (possible when n - 1 is not a multiple of 2h) takes
that last node's value.  The coarsest level holds the raw values on the
stride-2^nsteps grid.  Levels are ordered coarsest first; within a level the
nodes keep the row-major order of their stride-h grid.  Because every P is a
convex combination, the recomposed field's max error is at most the sum over
levels of each level's max coefficient error (plus rounding).

Arithmetic runs in the field's own dtype, so that float32 coefficients here
are the float32 coefficients the bitplane encoder receives; numpy evaluates
each operation on its own, with no fused multiply-add.
"""
from __future__ import annotations

import numpy as np


def grid_dims(shape, h: int):
    """Nodes per axis of the stride-h grid (0 for an empty axis)."""
    return tuple(0 if n == 0 else (n - 1) // h + 1 for n in shape)


def level_sizes(shape, nsteps: int):
    """Values per level, coarsest first (nsteps + 1 entries)."""
    def count(h):
        d = grid_dims(shape, h)
        return int(d[0]) * int(d[1]) * int(d[2])
    sizes = [count(1 << nsteps)]
    for j in range(nsteps - 1, -1, -1):
        sizes.append(count(1 << j) - count(1 << (j + 1)))
    return sizes


def _refine(c: np.ndarray, axis: int, m: int) -> np.ndarray:
    """Values on a line of m stride-h nodes from the ceil(m/2) stride-2h nodes."""
    c = np.moveaxis(c, axis, 0)
    out = np.empty((m,) + c.shape[1:], dtype=c.dtype)
    out[0::2] = c
    nodd = m // 2
    if nodd:
        half = c.dtype.type(0.5)
        inner = min(nodd, c.shape[0] - 1)   # odd nodes with a coarse node on each side
        odd = np.empty((nodd,) + c.shape[1:], dtype=c.dtype)
        odd[:inner] = (c[:inner] + c[1:inner + 1]) * half
        odd[inner:] = c[inner:nodd]         # past the last coarse node: its value
        out[1::2] = odd
    return np.moveaxis(out, 0, axis)


def _predict(coarse: np.ndarray, dims) -> np.ndarray:
    p = _refine(coarse, 2, dims[2])
    p = _refine(p, 1, dims[1])
    return _refine(p, 0, dims[0])


def _new_nodes(dims) -> np.ndarray:
    """Mask of the stride-h nodes that are not on the stride-2h grid."""
    ev = [np.arange(m) % 2 == 0 for m in dims]
    return ~(ev[0][:, None, None] & ev[1][None, :, None] & ev[2][None, None, :])


def decompose(u: np.ndarray, nsteps: int):
    """Field -> list of coefficient levels (coarsest first), in u's dtype."""
    u = np.asarray(u)
    assert u.ndim == 3 and u.dtype in (np.float32, np.float64)
    fine_first = []
    for j in range(nsteps):
        h = 1 << j
        U = u[::h, ::h, ::h]
        dims = U.shape
        P = _predict(U[::2, ::2, ::2], dims)
        fine_first.append((U - P)[_new_nodes(dims)])
    H = 1 << nsteps
    return [np.ascontiguousarray(u[::H, ::H, ::H]).ravel()] + fine_first[::-1]


def recompose(levels, shape, nsteps: int, dtype=None) -> np.ndarray:
    """Coefficient levels (coarsest first) -> field."""
    dtype = np.dtype(dtype or levels[0].dtype)
    u = np.zeros(shape, dtype=dtype)
    H = 1 << nsteps
    u[::H, ::H, ::H] = np.asarray(levels[0], dtype=dtype).reshape(grid_dims(shape, H))
    for l, j in enumerate(range(nsteps - 1, -1, -1), start=1):
        h = 1 << j
        dims = grid_dims(shape, h)
        if 0 in dims:
            continue
        P = _predict(u[::2 * h, ::2 * h, ::2 * h], dims)
        mask = _new_nodes(dims)
        V = P.copy()
        V[mask] = np.asarray(levels[l], dtype=dtype) + P[mask]
        u[::h, ::h, ::h] = V
    return u


def concat(levels) -> np.ndarray:
    """Levels as one array, coarsest first (the device layout)."""
    return np.concatenate([np.asarray(x).ravel() for x in levels])
