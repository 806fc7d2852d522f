"""Independent exact references used to pin the oracle (pure Python).

Determinants are evaluated with fractions.Fraction by the Leibniz formula,
and the perturbed lifting as a polynomial in eps: entry |p_i|^2 of the
height column becomes |p_i|^2 + eps^(r_i), r_i = 1 + rank of point i's key.
The sign of the perturbed determinant is the sign of its lowest-order
nonzero coefficient (eps -> 0+).  Nothing here shares code with the oracle.
"""
from __future__ import annotations

import itertools
from fractions import Fraction


def _perm_sign(p):
    s = 1
    p = list(p)
    for i in range(len(p)):
        while p[i] != i:
            j = p[i]
            p[i], p[j] = p[j], p[i]
            s = -s
    return s


def det(M):
    n = len(M)
    tot = Fraction(0)
    for p in itertools.permutations(range(n)):
        t = Fraction(_perm_sign(p))
        for i in range(n):
            t *= M[i][p[i]]
            if t == 0:
                break
        tot += t
    return tot


def sgn(x) -> int:
    return (x > 0) - (x < 0)


def orient1(pts) -> int:
    """sign det [p_i 1]"""
    M = [[Fraction(float(c)) for c in p] + [Fraction(1)] for p in pts]
    return sgn(det(M))


def _poly_mul(a, b):
    r = {}
    for da, ca in a.items():
        for db, cb in b.items():
            r[da + db] = r.get(da + db, 0) + ca * cb
    return {d: c for d, c in r.items() if c != 0}


def _poly_add(a, b):
    r = dict(a)
    for d, c in b.items():
        r[d] = r.get(d, 0) + c
    return {d: c for d, c in r.items() if c != 0}


def insphere_poly(pts, keys=None):
    """det [p_i, h_i, 1] with h_i = |p_i|^2 (+ eps^(1+rank(key_i))) as a
    polynomial {degree: Fraction}."""
    n = len(pts)
    if keys is not None:
        order = sorted(range(n), key=lambda i: keys[i])
        rank = {i: r for r, i in enumerate(order)}
    M = []
    for i, p in enumerate(pts):
        row = [{0: Fraction(float(c))} for c in p]
        h = {0: sum(Fraction(float(c)) ** 2 for c in p)}
        if keys is not None:
            h = _poly_add(h, {1 + rank[i]: Fraction(1)})
        row.append(h)
        row.append({0: Fraction(1)})
        M.append([{d: c for d, c in e.items() if c != 0} for e in row])
    tot = {}
    for perm in itertools.permutations(range(n)):
        t = {0: Fraction(_perm_sign(perm))}
        for i in range(n):
            t = _poly_mul(t, M[i][perm[i]])
            if not t:
                break
        tot = _poly_add(tot, t)
    return tot


def insphere_sign(pts, keys=None) -> int:
    poly = insphere_poly(pts, keys)
    if not poly:
        return 0
    return sgn(poly[min(poly)])
