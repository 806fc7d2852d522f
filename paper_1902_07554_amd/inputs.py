"""Seeded synthetic point-set generators.

These generators are the only code shared between the CPU oracle's tests and
the GPU path: they produce the input point sets and hold none of the method's
arithmetic.  All arrays are float64, row-major (n, D), and end with a random
permutation so that input order carries no spatial locality.

Distributions follow the paper's evaluation inputs (Section "Evaluation"):
points uniform in the unit cube, normally distributed around a centre, and
"bubbles" (several Gaussian clusters with centres uniform in the unit cube).
The paper prints no bubble parameters; the recipe below (64 centres, sigma
log-uniform in [0.01, 0.05], Dirichlet(1) weights, 5 % uniform background,
no clipping) is this project's reading and is documented with the workloads.
"""
from __future__ import annotations

import math

import numpy as np


def uniform(n: int, dim: int, seed: int = 1) -> np.ndarray:
    """n points i.i.d. uniform in [0,1)^dim."""
    rng = np.random.default_rng(seed)
    return rng.random((n, dim))


def normal(n: int, dim: int, seed: int = 1) -> np.ndarray:
    """n points i.i.d. N(0, I_dim)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, dim))


def bubbles(n: int, dim: int = 3, seed: int = 1, clusters: int = 64,
            sigma_lo: float = 0.01, sigma_hi: float = 0.05,
            background: float = 0.05) -> np.ndarray:
    """Gaussian clusters ("bubbles") plus a uniform background.

    Centres ~ U[0,1)^dim, sigma_j log-uniform in [sigma_lo, sigma_hi],
    weights ~ Dirichlet(1,...,1), cluster sizes ~ Multinomial, points =
    centre + sigma * N(0, I) without clipping, plus floor(background*n)
    points uniform in [0,1)^dim; finally a random permutation.
    """
    rng = np.random.default_rng(seed)
    nb = int(math.floor(background * n))
    centres = rng.random((clusters, dim))
    sig = np.exp(rng.uniform(math.log(sigma_lo), math.log(sigma_hi), clusters))
    w = rng.dirichlet(np.ones(clusters))
    counts = rng.multinomial(n - nb, w)
    lab = np.repeat(np.arange(clusters), counts)
    pts = centres[lab] + sig[lab, None] * rng.standard_normal((n - nb, dim))
    pts = np.concatenate([pts, rng.random((nb, dim))], axis=0)
    return pts[rng.permutation(n)]


def make(dist: str, n: int, dim: int, seed: int = 1) -> np.ndarray:
    if dist == "uniform":
        return uniform(n, dim, seed)
    if dist == "normal":
        return normal(n, dim, seed)
    if dist == "bubbles":
        return bubbles(n, dim, seed)
    raise ValueError(f"unknown distribution {dist!r}")


def lattice(side: int, dim: int, seed: int = 1, scale: float = 1.0) -> np.ndarray:
    """Integer grid points (highly degenerate: co-circular / co-spherical
    groups everywhere), randomly permuted.  Exercises tie-breaking."""
    rng = np.random.default_rng(seed)
    axes = [np.arange(side, dtype=np.float64) * scale] * dim
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, dim)
    return g[rng.permutation(len(g))]


def jittered_lattice(side: int, dim: int, rel: float, seed: int = 1) -> np.ndarray:
    """Integer grid points, each coordinate moved by a uniform offset of at
    most `rel` grid steps, randomly permuted: near-ties everywhere, at a
    chosen distance from exact degeneracy."""
    rng = np.random.default_rng(seed)
    g = lattice(side, dim, seed=seed)
    return g + rel * rng.uniform(-1.0, 1.0, g.shape)


def batch_sets(num_sets: int = 4096, lo: int = 64, hi: int = 65536,
               dim: int = 2, seed: int = 1):
    """Independent point sets with sizes log-uniform in [lo, hi]; each set is
    uniform in [0,1)^dim or N(0, I) by a fair coin.  Returns (points, offsets)
    with points concatenated set after set and offsets of length num_sets+1."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), num_sets))).astype(np.int64)
    kinds = rng.integers(0, 2, num_sets)
    parts = []
    for s, kd in zip(sizes, kinds):
        if kd == 0:
            parts.append(rng.random((int(s), dim)))
        else:
            parts.append(rng.standard_normal((int(s), dim)))
    offsets = np.zeros(num_sets + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    return np.concatenate(parts, axis=0), offsets


def serve_stream(rate: float = 200.0, duration: float = 60.0, lo: int = 1000,
                 hi: int = 1_000_000, dim: int = 3, seed: int = 1):
    """Poisson arrival stream of triangulation jobs.  Returns a list of
    (arrival_time_s, n, kind, job_seed) with kind in {"uniform", "bubbles"};
    the points of a job are drawn lazily with make(kind, n, dim, job_seed)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        n = int(np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi)))))
        kind = "uniform" if rng.integers(0, 2) == 0 else "bubbles"
        jobs.append((t, n, kind, int(rng.integers(1, 2**31 - 1))))
    return jobs
