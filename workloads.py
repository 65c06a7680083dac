"""Seeded synthetic inputs for the refactor / retrieve path.

This module holds no arithmetic of the method: it only draws coefficient
levels with the shapes, sizes and value distributions of the evaluation
workloads, so that the oracle and the GPU path can be fed the same buffers.

The paper's datasets (NYX, LETKF, Miranda, Hurricane ISABEL, JHTDB; Sec. 6.1,
Table 1) are not available; these generators stand in for them:

* for the refactor/retrieve workloads a "field" is represented by its
  coefficient levels directly (smooth_field materialises the field itself for
  the multilevel decomposition): level sizes follow the 3D
  dyadic coarsening rule (each finer level holds the points added by halving
  the grid spacing, i.e. 7/8 of the remaining points for power-of-two edges);
* coefficients of level l (l = 0 coarsest) are Laplace(0, b0 * 2^-l), drawn in
  float64 and rounded to the working type;
* b0 is the standard deviation of a smooth field made of 16 random-phase
  sinusoids (integer wavevectors in [1, 8]^3, amplitude 1/|k|) plus Gaussian
  noise of 1% of the signal's standard deviation.  On a periodic grid the
  sinusoids are orthogonal, so that deviation has a closed form (used here
  instead of materialising the 512^3 or 1024^3 field; b0 only sets units).
"""
from __future__ import annotations

import math

import numpy as np


def level_sizes(edges, nlevels: int):
    """Points per coefficient level for a grid with the given edge lengths.

    level 0 = prod ceil(E_d / 2^(L-1)); level l >= 1 adds
    prod ceil(E_d / 2^(L-1-l)) - prod ceil(E_d / 2^(L-l)) points."""
    def pts(shift):
        p = 1
        for e in edges:
            p *= -(-e // (1 << shift))
        return p

    sizes = [pts(nlevels - 1)]
    for l in range(1, nlevels):
        sizes.append(pts(nlevels - 1 - l) - pts(nlevels - l))
    return sizes


def smooth_field_std(seed: int, n_modes: int = 16, noise: float = 0.01) -> float:
    """Standard deviation of sum_j a_j sin(2 pi k_j . x / N + phi_j) + noise on a
    periodic grid (closed form: each distinct wavevector contributes |sum a e^{i phi}|^2 / 2)."""
    rng = np.random.default_rng(seed)
    ks = rng.integers(1, 9, size=(n_modes, 3))
    phases = rng.uniform(0.0, 2.0 * math.pi, n_modes)
    amp = {}
    for k, ph in zip(map(tuple, ks), phases):
        a = 1.0 / math.sqrt(sum(int(c) * int(c) for c in k))
        amp[k] = amp.get(k, 0j) + a * complex(math.cos(ph), math.sin(ph))
    var = sum(abs(v) ** 2 / 2.0 for v in amp.values())
    return math.sqrt(var * (1.0 + noise * noise))


def smooth_field(seed: int, shape, dtype=np.float32, n_modes: int = 16, noise: float = 0.01) -> np.ndarray:
    """The smooth field itself, for the multilevel decomposition: the 16
    random-phase sinusoids of smooth_field_std (the same draws, phases along
    each axis scaled by that axis' length) plus Gaussian noise of 1% of the
    signal's standard deviation; evaluated in float64, then rounded to dtype."""
    return smooth_field_tensor(seed, shape, "cpu", n_modes, noise).numpy().astype(dtype)


def smooth_field_tensor(seed: int, shape, device, n_modes: int = 16, noise: float = 0.01):
    """smooth_field as a float64 torch tensor evaluated on `device` (the sines
    may differ in the last bits between devices)."""
    import torch
    rng = np.random.default_rng(seed)
    ks = rng.integers(1, 9, size=(n_modes, 3))
    phases = rng.uniform(0.0, 2.0 * math.pi, n_modes)
    axes = [torch.arange(n, dtype=torch.float64, device=device) * (2.0 * math.pi / max(n, 1)) for n in shape]
    u = torch.zeros(tuple(shape), dtype=torch.float64, device=device)
    for k, ph in zip(ks, phases):
        a = 1.0 / math.sqrt(sum(int(c) * int(c) for c in k))
        ang = (axes[0] * int(k[0]))[:, None, None] + (axes[1] * int(k[1]))[None, :, None] \
            + (axes[2] * int(k[2]) + float(ph))[None, None, :]
        u += a * torch.sin(ang)
    sd = smooth_field_std(seed, n_modes, 0.0)
    u += torch.from_numpy(rng.standard_normal(tuple(shape))).to(device) * (noise * sd)
    return u


def laplace_levels(sizes, b0: float, rng: np.random.Generator, dtype=np.float32):
    """Coefficient levels l = 0.. with Laplace(0, b0 * 2^-l) values (f64 draw, then cast)."""
    return [rng.laplace(0.0, b0 * 2.0 ** (-l), int(s)).astype(dtype) for l, s in enumerate(sizes)]


# ---------------------------------------------------------------- named workloads
def plain_level(seed: int = 1, n: int = 1 << 20, dtype=np.float32):
    """One level of n Laplace(0, 1) coefficients (32 planes, blocks of 32)."""
    rng = np.random.default_rng(seed)
    return rng.laplace(0.0, 1.0, n).astype(dtype)


def field_levels(seed: int, edge: int = 512, nlevels: int = 9, dtype=np.float32):
    """Coefficient levels standing in for an edge^3 smooth field."""
    b0 = smooth_field_std(seed)
    rng = np.random.default_rng(seed)
    return laplace_levels(level_sizes((edge, edge, edge), nlevels), b0, rng, dtype)


def chunk_level_sizes(slab: int = 32, edge: int = 1024, nlevels: int = 9):
    """Levels of one slab (slab x edge x edge) processed as its own sub-domain."""
    return level_sizes((slab, edge, edge), nlevels)


def chunk_levels(seed: int, chunk: int, slab: int = 32, edge: int = 1024, nlevels: int = 9,
                 dtype=np.float64):
    """Coefficient levels of slab `chunk` of an edge^3 float64 field."""
    b0 = smooth_field_std(seed)
    rng = np.random.default_rng([seed, chunk])
    return laplace_levels(chunk_level_sizes(slab, edge, nlevels), b0, rng, dtype)


def batch_variables(seed: int = 4, nvars: int = 256, nlevels: int = 5, lo: int = 16, hi: int = 256,
                    dtype=np.float32, max_vars=None):
    """Variables of uneven size: cube edge ~ U{lo..hi}, nlevels Laplace levels, b0 = 1."""
    rng = np.random.default_rng(seed)
    edges = rng.integers(lo, hi + 1, nvars)
    out = []
    for v, e in enumerate(edges):
        if max_vars is not None and v >= max_vars:
            break
        out.append(laplace_levels(level_sizes((int(e),) * 3, nlevels), 1.0, rng, dtype))
    return [int(e) for e in edges], out


def batch_edges(seed: int = 4, nvars: int = 256, lo: int = 16, hi: int = 256):
    return [int(e) for e in np.random.default_rng(seed).integers(lo, hi + 1, nvars)]


def serving_requests(seed: int = 58, n: int = 10000, nfields: int = 8, rate: float = 1.0,
                     tol_lo: float = 1e-7, tol_hi: float = 1e-1, qoi_frac: float = 0.5,
                     incr_frac: float = 0.3):
    """Poisson arrivals (rate per second) of retrieval requests.

    Each request: arrival time, kind ('raw' on a uniform field or 'qoi' V_total on
    fields 0..2), relative tolerance log-uniform in [tol_lo, tol_hi], and for a
    fraction of them the id of an earlier session they refine (tolerance tightened)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    t = np.cumsum(gaps)
    kinds = np.where(rng.random(n) < qoi_frac, "qoi", "raw")
    fields = rng.integers(0, nfields, n)
    tols = np.exp(rng.uniform(math.log(tol_lo), math.log(tol_hi), n))
    incr = rng.random(n) < incr_frac
    reqs = []
    for i in range(n):
        parent = None
        if incr[i] and i > 0:
            parent = int(rng.integers(0, i))
        reqs.append({"id": i, "t": float(t[i]), "kind": str(kinds[i]), "field": int(fields[i]),
                     "tol": float(tols[i]), "parent": parent})
    return reqs


def ones_runs_level(seed: int, n: int, dtype=np.float32):
    """Stress input for the exact error table: values whose significands are
    runs of ones (2^a - 1) at varied positions, with run lengths that grow along
    the array, so that every cut's largest tail keeps being raised by later
    values; a third of the values are Laplace(0, 1) noise."""
    rng = np.random.default_rng(seed)
    p = 24 if dtype == np.float32 else 53
    frac = np.arange(n, dtype=np.float64) / max(n, 1)
    a = np.clip(1 + np.floor(frac * (p - 1)) + rng.integers(-2, 3, n), 1, p).astype(np.int64)
    sig = np.ldexp(1.0, a) - 1.0                      # exact: a <= 53 ones
    q = rng.integers(-40, 2, n) - a                  # the run's top bit below 2^2
    x = np.ldexp(sig, q) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    noise = rng.random(n) < 1.0 / 3.0
    x[noise] = rng.laplace(0.0, 1.0, int(noise.sum()))
    return x.astype(dtype)


def piecewise_constant_level(seed: int, n: int, dtype=np.float32):
    """Stress input for run-length statistics: constant stretches of 1..40000
    values (zero, or one Laplace draw), so that equal plane words run across
    many encoder tiles and workgroup ranges."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, np.float64)
    i = 0
    while i < n:
        run = int(rng.integers(1, 40001))
        out[i:i + run] = 0.0 if rng.random() < 0.3 else rng.laplace(0.0, 1.0)
        i += run
    return out.astype(dtype)
