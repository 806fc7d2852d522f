"""Seeded near-degenerate predicate queries (test input only, no predicate
arithmetic): point tuples whose orientation or in-sphere determinant is
zero or nearly zero, so that a floating-point filter with a wrong error
bound would certify a wrong sign.

Each generator returns an array of queries, (q, D+1, D) for orientation and
(q, D+2, D) for in-sphere (the last row is the query point):
  * exact ties built on small integer lattices (spheres through integer
    points of equal norm, hyperplanes through lattice points), then one
    coordinate offset by a relative 2^-k, k in [20, 60];
  * the same configurations scaled by 2^s (s in [-80, 80]) and translated,
    which moves the offsets into and out of the FP32 filter's band;
  * a query point within a relative 2^-40 .. 2^-75 of a vertex, so that
    FP32 intermediates of the in-sphere determinant underflow;
  * plain random tuples.
"""
from __future__ import annotations

import numpy as np

# integer vectors of equal squared norm (used as sphere directions)
_SPHERE2 = [(5, 0), (3, 4), (4, 3), (0, 5)]                 # norm^2 25
_SPHERE3 = [(3, 2, 6), (2, 3, 6), (6, 2, 3), (2, 6, 3), (3, 6, 2), (6, 3, 2),
            (7, 0, 0), (0, 7, 0), (0, 0, 7)]                # norm^2 49


def _sphere_dirs(dim, rng, count):
    base = _SPHERE2 if dim == 2 else _SPHERE3
    out = []
    seen = set()
    while len(out) < count:
        v = np.array(base[rng.integers(len(base))], dtype=np.float64)
        v = v[rng.permutation(dim)] * np.where(rng.random(dim) < 0.5, -1.0, 1.0)
        t = tuple(v)
        if t not in seen:
            seen.add(t)
            out.append(v)
    return np.array(out)


def insphere_queries(dim: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    out = np.empty((count, dim + 2, dim))
    for t in range(count):
        kind = t % 4
        if kind == 3:
            out[t] = rng.random((dim + 2, dim))
            continue
        c = rng.integers(-3, 4, dim).astype(np.float64)
        q = c + _sphere_dirs(dim, rng, dim + 2)
        # perturb the query point by a relative 2^-k along one axis
        k = int(rng.integers(20, 61))
        ax = int(rng.integers(dim))
        q[-1, ax] += float(rng.choice([-1.0, 0.0, 1.0])) * 7.0 * 2.0 ** -k
        if kind == 1:
            s = float(2.0 ** int(rng.integers(-80, 81)))
            q = q * s + rng.integers(-4, 5, dim) * s * 0.25
        if kind == 2:
            # query next to a vertex: tiny differences, underflowing FP32 products
            j = int(rng.integers(dim + 1))
            e = float(2.0 ** -int(rng.integers(40, 76)))
            q[-1] = q[j] + e * rng.integers(-3, 4, dim)
            if not np.any(q[-1] != q[j]):
                q[-1, 0] += e
        out[t] = q
    return out


def orient_queries(dim: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    out = np.empty((count, dim + 1, dim))
    for t in range(count):
        kind = t % 3
        if kind == 2:
            out[t] = rng.random((dim + 1, dim))
            continue
        base = rng.integers(-8, 9, (dim, dim)).astype(np.float64)
        w = rng.integers(-3, 4, dim).astype(np.float64)
        # last point: an integer affine combination of the others (on their hyperplane)
        last = base[0] + sum(w[i] * (base[i] - base[0]) for i in range(1, dim))
        p = np.vstack([base, last])
        k = int(rng.integers(20, 61))
        p[-1, int(rng.integers(dim))] += float(rng.choice([-1.0, 0.0, 1.0])) * 2.0 ** -k * 5.0
        if kind == 1:
            s = float(2.0 ** int(rng.integers(-80, 81)))
            p = p * s + rng.integers(-4, 5, dim) * s * 0.25
        out[t] = p
    return out
