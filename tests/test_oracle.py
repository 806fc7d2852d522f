"""Pins of the CPU oracle against references other than itself.

* predicates vs exact Fraction determinants (Leibniz formula);
* the perturbed lifting vs the lowest-order coefficient of the determinant
  as a polynomial in eps (tests/exact_ref.py);
* DT(P) vs brute force: no point strictly inside any circumsphere under the
  perturbed predicate, simplices tile the convex hull (volume, facet
  pairing), Euler relation, 2D triangle count 2n-2-h;
* DT(P) vs scipy.spatial.Delaunay (Qhull) on random inputs in general
  position;
* independence of input order and of the point labels' positions.
"""
import math

import numpy as np
import pytest
from scipy.spatial import ConvexHull, Delaunay

import oracle
from paper_1902_07554_amd import inputs
from tests import exact_ref as X

rng = np.random.default_rng(12345)


# ---------------------------------------------------------------- predicates
@pytest.mark.parametrize("dim", [2, 3])
def test_orient_random_and_near_degenerate(dim):
    for t in range(300):
        p = rng.random((dim + 1, dim))
        if t % 3 == 1:   # nearly degenerate: last point on the hyperplane + tiny offset
            w = rng.random(dim)
            w /= w.sum()
            p[-1] = w @ p[:-1] if dim == 2 else (w[:, None] * p[:-1]).sum(0)
            p[-1, 0] += (rng.random() - 0.5) * 1e-15
        if t % 3 == 2:   # exactly degenerate on a dyadic lattice
            p = rng.integers(0, 4, (dim + 1, dim)).astype(float) / 4
            p[-1] = p[0] + (p[1] - p[0]) * 2
        assert oracle.orient(p) == X.orient1(p)


@pytest.mark.parametrize("dim", [2, 3])
def test_insphere_random_and_near_degenerate(dim):
    for t in range(200):
        p = rng.random((dim + 2, dim))
        if t % 2 == 1:
            # co-spherical: points on a sphere with dyadic coordinates
            c = rng.integers(-2, 3, dim).astype(float)
            cand = []
            r = np.array([3.0, 4.0, 0.0][:dim]) if dim == 2 else np.array([2.0, 3.0, 6.0])
            for s in rng.permutation(64)[: dim + 2]:
                v = np.array(r)
                rng.shuffle(v)
                v *= np.where(rng.random(dim) < 0.5, -1.0, 1.0)
                cand.append(c + v)
            p = np.array(cand)
            p[-1, 0] += [0.0, 2.0 ** -40, -(2.0 ** -40)][t % 3]
        assert oracle.insphere(p) == X.insphere_sign(p), p


@pytest.mark.parametrize("dim", [2, 3])
def test_perturbation_matches_eps_polynomial(dim):
    """Degenerate (co-circular / co-spherical / co-linear) configurations:
    the perturbed sign is that of the lowest-order eps coefficient."""
    pts2 = [np.array([[1, 0], [0, 1], [-1, 0], [0, -1]], float),      # co-circular
            np.array([[0, 0], [1, 0], [2, 0], [1, 1]], float),         # three co-linear
            np.array([[0, 0], [2, 0], [2, 2], [0, 2]], float)]
    pts3 = [np.array([[1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, 1]], float),
            np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [0, 0, 1]], float),
            np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [2, 2, 0]], float),
            np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1], [1, 1, -1]], float)]
    cases = pts2 if dim == 2 else pts3
    checked = 0
    for p in cases:
        for keys in map(list, __import__("itertools").permutations(range(dim + 2))):
            k = np.array(keys, dtype=np.int64) * 7 + 3
            want = X.insphere_sign(p, list(k))
            got = oracle.insphere(p, k)
            assert got == want, (p, k, got, want)
            checked += 1
    assert checked >= 3 * 24


@pytest.mark.parametrize("dim", [2, 3])
def test_predicates_in_the_filter_band(dim):
    """Near-ties with relative offsets 2^-20 .. 2^-60, scaled by 2^-80 ..
    2^80, and query points next to a vertex: the floating-point filters must
    hand every case they cannot certify to the exact stage."""
    from tests import near_ties
    for q in near_ties.insphere_queries(dim, 160, seed=31 + dim):
        assert oracle.insphere(q) == X.insphere_sign(q), q
    for q in near_ties.orient_queries(dim, 160, seed=41 + dim):
        assert oracle.orient(q) == X.orient1(q), q


# ----------------------------------------------------------------- DT checks
def _conflict_ref(pts, ids, simplex, q):
    """Brute-force perturbed conflict test with exact Fraction arithmetic."""
    P = [pts[i] for i in simplex] + [pts[q]]
    keys = [ids[i] for i in simplex] + [ids[q]]
    o = X.orient1(P[:-1])
    s = X.insphere_sign(P) or X.insphere_sign(P, keys)
    return s != 0 and s == o


def _check_empty(p, ids, simp):
    pos = {int(g): i for i, g in enumerate(ids)}
    for s in simp:
        loc = [pos[int(g)] for g in s]
        for q in range(len(p)):
            if q in loc:
                continue
            assert not _conflict_ref(p, ids, loc, q), (s, q)


def _check_tiling(p, simp_loc):
    dim = p.shape[1]
    vol = sum(abs(np.linalg.det(p[s[1:]] - p[s[0]])) for s in simp_loc) / math.factorial(dim)
    assert vol == pytest.approx(ConvexHull(p).volume, rel=1e-9)
    facets = {}
    for s in simp_loc:
        for j in range(dim + 1):
            f = tuple(sorted(np.delete(s, j)))
            facets[f] = facets.get(f, 0) + 1
    assert max(facets.values()) <= 2
    for s in simp_loc:   # no flat simplices
        assert X.orient1(p[s]) != 0


@pytest.mark.parametrize("dim,n", [(2, 40), (3, 22)])
def test_dt_brute_force_random(dim, n):
    p = inputs.uniform(n, dim, seed=7)
    ids = np.arange(n)
    simp = oracle.delaunay(p, ids)
    _check_empty(p, ids, simp)
    _check_tiling(p, simp)


@pytest.mark.parametrize("side,dim", [(5, 2), (3, 3)])
def test_dt_brute_force_lattice(side, dim):
    """Highly degenerate input: the perturbed DT is a proper triangulation
    of the hull in which no point conflicts with any simplex."""
    p = inputs.lattice(side, dim, seed=3)
    ids = rng.permutation(len(p)) * 3 + 1   # ids need not equal positions
    simp = oracle.delaunay(p, ids)
    _check_empty(p, ids, simp)
    pos = {int(g): i for i, g in enumerate(ids)}
    loc = np.array([[pos[int(g)] for g in s] for s in simp])
    _check_tiling(p, loc)


def test_dt_2d_count_formula():
    for side in (4, 9, 16):
        p = inputs.lattice(side, 2, seed=side)
        simp = oracle.delaunay(p)
        assert len(simp) == 2 * len(p) - 2 - 4 * (side - 1)
    p = inputs.uniform(3000, 2, seed=9)
    h = len(ConvexHull(p).vertices)
    assert len(oracle.delaunay(p)) == 2 * 3000 - 2 - h


def test_dt_3d_euler():
    p = inputs.uniform(2000, 3, seed=4)
    simp = oracle.delaunay(p)
    edges = {tuple(sorted((a, b))) for s in simp for a in s for b in s if a < b}
    faces = {tuple(sorted(np.delete(s, j))) for s in simp for j in range(4)}
    assert len(p) - len(edges) + len(faces) - len(simp) == 1


@pytest.mark.parametrize("dim,n,dist", [(2, 5000, "uniform"), (3, 5000, "uniform"),
                                        (3, 5000, "bubbles"), (2, 3000, "normal")])
def test_dt_matches_qhull(dim, n, dist):
    p = inputs.make(dist, n, dim, seed=11)
    assert np.array_equal(oracle.delaunay(p), oracle.canonical(Delaunay(p).simplices))


def test_dt_order_and_label_independence():
    p = inputs.lattice(6, 3, seed=1)
    ids = np.arange(len(p)) * 5 + 2
    a = oracle.delaunay(p, ids)
    perm = rng.permutation(len(p))
    assert np.array_equal(a, oracle.delaunay(p[perm], ids[perm]))


def test_dt_errors():
    with pytest.raises(oracle.OracleError) as e:
        oracle.delaunay(np.array([[0, 0], [1, 1], [2, 2], [3, 3.0]]))
    assert e.value.status == oracle.DEGENERATE
    with pytest.raises(oracle.OracleError) as e:
        oracle.delaunay(np.array([[0, 0], [1, 0], [0, 1], [1, 0.0]]))
    assert e.value.status == oracle.DUPLICATE
    with pytest.raises(oracle.OracleError) as e:
        oracle.delaunay(np.array([[0, 0], [1, 0], [0, np.nan]]))
    assert e.value.status == oracle.NONFINITE
