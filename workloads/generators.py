"""Seeded synthetic point sets shaped like the paper's workloads.

This module is shared by the oracle side and the GPU side of every test and
benchmark, so it holds no distance arithmetic of the self-join: it only draws
points. Every array is float64, shape (n, d), C-contiguous.

The paper evaluates uniform and exponential synthetic sets (Section IV-A,
Table I) but states neither their range nor the exponential rate; the recipes
below fix them: uniform in [0,1]^d, exponential with rate 40 per coordinate
clipped to [0,1] (explicit inverse CDF, so the draw does not depend on numpy's
ziggurat sampler), and a Gaussian mixture for the high-dimensional precision
workload (Box-Muller on uniforms, again to stay independent of numpy's normal
sampler). All draws come from numpy's PCG64 (`default_rng`).
"""
from __future__ import annotations

import numpy as np


def _rng(seed) -> np.random.Generator:
    return np.random.default_rng(seed)


def uniform(n: int, d: int, seed=0) -> np.ndarray:
    """n points uniform in [0,1)^d."""
    return np.ascontiguousarray(_rng(seed).random((n, d)), dtype=np.float64)


def exponential(n: int, d: int, lam: float = 40.0, seed=0) -> np.ndarray:
    """n points, each coordinate i.i.d. exponential(rate=lam), clipped to 1."""
    u = _rng(seed).random((n, d))
    x = -np.log1p(-u) / lam
    np.minimum(x, 1.0, out=x)
    return np.ascontiguousarray(x, dtype=np.float64)


def gaussian_mixture(n: int, d: int, clusters: int = 100, sigma: float = 0.02,
                     seed=0) -> np.ndarray:
    """n points from `clusters` isotropic Gaussians (std `sigma` per coordinate)
    whose centres are uniform in [0,1)^d; labels uniform over the clusters."""
    rng = _rng(seed)
    centres = rng.random((clusters, d))
    labels = rng.integers(0, clusters, n)
    out = np.empty((n, d), dtype=np.float64)
    # Box-Muller, written out so the normal draw is pinned to the uniform stream.
    step = 1 << 20
    for s in range(0, n, step):
        e = min(n, s + step)
        u1 = rng.random((e - s, d))
        u2 = rng.random((e - s, d))
        z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
        out[s:e] = centres[labels[s:e]] + sigma * z
    return out


def lattice(L: int, d: int, h: float = 2.0 ** -6) -> np.ndarray:
    """All points of the integer lattice {0..L-1}^d scaled by h (h a power of
    two keeps every coordinate difference and square exact in float64)."""
    axes = [np.arange(L, dtype=np.float64) * h] * d
    grid = np.meshgrid(*axes, indexing="ij")
    return np.ascontiguousarray(np.stack([g.ravel() for g in grid], axis=1))


def make(dist: str, n: int, d: int, seed=0) -> np.ndarray:
    """Dispatch by distribution name: 'uniform', 'expo', 'gmm'."""
    if dist == "uniform":
        return uniform(n, d, seed)
    if dist == "expo":
        return exponential(n, d, 40.0, seed)
    if dist == "gmm":
        return gaussian_mixture(n, d, 100, 0.02, seed)
    raise ValueError(f"unknown distribution {dist!r}")


def batch_problems(count: int = 256, seed: int = 0,
                   n_lo: float = 1e3, n_hi: float = 2e5,
                   dims=(2, 3, 4, 8, 16)):
    """Parameters of the batched workload: per problem (n_b, d_b); n is
    log-uniform in [n_lo, n_hi], d uniform over `dims`. Problem b's points are
    then drawn with `uniform(n_b, d_b, seed=[seed, b])`."""
    rng = _rng(seed)
    n = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), count))).astype(np.int64)
    d = rng.choice(np.asarray(dims, dtype=np.int64), count)
    return [(int(a), int(b)) for a, b in zip(n, d)]
