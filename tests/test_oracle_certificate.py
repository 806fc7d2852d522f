"""Pins of the oracle's Delaunay certificate (oracle.certify), which checks
claimed triangulations too large for the plain oracle run.

It must accept the oracle's own DT (which is pinned against Qhull and brute
force in test_oracle.py) and reject each kind of mistake a triangulation
can carry: a flipped facet (a valid triangulation that is not Delaunay), a
missing simplex, a repeated simplex, an unused point, an out-of-range or
repeated index.  Hull facets and the volume are compared with Qhull's
convex hull, and the Euler characteristic is that of a ball."""
import numpy as np
import pytest
from scipy.spatial import ConvexHull

import oracle
from paper_1902_07554_amd import inputs


def _hull(p):
    h = ConvexHull(p)
    return h.simplices, h.volume


def _orient(p, rows):
    v = p[rows]
    a = v[:, 1:, :] - v[:, :1, :]
    return np.sign(np.linalg.det(a))


@pytest.mark.parametrize("dim,dist,n", [(2, "uniform", 3000), (3, "uniform", 3000),
                                        (3, "bubbles", 4000), (2, "normal", 2500)])
def test_accepts_the_delaunay_triangulation(dim, dist, n):
    p = inputs.make(dist, n, dim, seed=7)
    rows = oracle.delaunay(p)
    cert = oracle.certify(p, rows)
    hs, hv = _hull(p)
    assert oracle.certificate_ok(cert, hs, hv) == []
    assert cert["hull"] == len(hs)
    # vertex order inside rows and row order do not matter
    rng = np.random.default_rng(1)
    shuffled = rng.permuted(rows, axis=1)[rng.permutation(len(rows))]
    c2 = oracle.certify(p, shuffled)
    assert oracle.certificate_ok(c2, hs, hv) == []


def test_accepts_degenerate_input_under_the_perturbation():
    """A lattice: every empty-sphere test is a tie, decided by the
    perturbation; the certificate uses the same one."""
    p = inputs.lattice(6, 3, seed=3)
    rows = oracle.delaunay(p)
    cert = oracle.certify(p, rows)
    for f in ("bad_rows", "flat", "over_shared", "same_side", "not_local", "unused"):
        assert cert[f] == 0, f
    assert abs(cert["volume"] - ConvexHull(p).volume) < 1e-9 * cert["volume"]
    # the same rows under the reversed perturbation order are not Delaunay
    rev = oracle.certify(p, rows, ids=np.arange(len(p))[::-1].copy())
    assert rev["not_local"] > 0


def test_rejects_a_2d_edge_flip():
    p = inputs.uniform(500, 2, seed=2)
    rows = oracle.delaunay(p)
    nb = oracle.neighbors(rows)
    hs, hv = _hull(p)
    # an interior edge whose quadrilateral is convex: flip it
    for i in range(len(rows)):
        for j in range(3):
            k = nb[i, j]
            if k < 0:
                continue
            a = rows[i, j]
            e = [x for x in rows[i] if x != a]
            b = [x for x in rows[k] if x not in e][0]
            t1, t2 = np.array([[a, b, e[0]]]), np.array([[a, b, e[1]]])
            if _orient(p, t1)[0] * _orient(p, t2)[0] < 0:
                bad = np.concatenate([np.delete(rows, [i, k], axis=0), t1, t2])
                cert = oracle.certify(p, bad)
                assert cert["not_local"] >= 1
                assert cert["over_shared"] == 0 and cert["same_side"] == 0
                assert oracle.certificate_ok(cert, hs, hv) == ["not_local"]
                return
    raise AssertionError("no convex quadrilateral found")


def test_rejects_a_3d_two_three_flip():
    p = inputs.uniform(400, 3, seed=5)
    rows = oracle.delaunay(p)
    nb = oracle.neighbors(rows)
    hs, hv = _hull(p)
    for i in range(len(rows)):
        for j in range(4):
            k = nb[i, j]
            if k < 0:
                continue
            d = rows[i, j]
            f = [x for x in rows[i] if x != d]
            e = [x for x in rows[k] if x not in f][0]
            new = np.array([[d, e, f[0], f[1]], [d, e, f[1], f[2]], [d, e, f[2], f[0]]])
            s = _orient(p, new)
            if np.all(s == s[0]) and s[0] != 0:
                bad = np.concatenate([np.delete(rows, [i, k], axis=0), new])
                cert = oracle.certify(p, bad)
                assert cert["not_local"] >= 1
                assert oracle.certificate_ok(cert, hs, hv) == ["not_local"]
                return
    raise AssertionError("no convex pair found")


@pytest.mark.parametrize("dim", [2, 3])
def test_rejects_missing_repeated_and_invalid_rows(dim):
    p = inputs.uniform(800, dim, seed=9)
    rows = oracle.delaunay(p)
    hs, hv = _hull(p)
    # a missing interior simplex: its facets become one-sided
    nb = oracle.neighbors(rows)
    inner = int(np.nonzero((nb >= 0).all(axis=1))[0][0])
    cert = oracle.certify(p, np.delete(rows, inner, axis=0))
    assert set(oracle.certificate_ok(cert, hs, hv)) >= {"hull_facets", "volume"}
    # a repeated simplex
    cert = oracle.certify(p, np.concatenate([rows, rows[:1]]))
    assert cert["over_shared"] > 0
    assert "volume" in oracle.certificate_ok(cert, hs, hv)
    # an index out of range, and a row with a repeated index
    bad = rows.copy()
    bad[0, 0] = len(p)
    assert oracle.certify(p, bad)["bad_rows"] == 1
    bad = rows.copy()
    bad[1, 1] = bad[1, 0]
    assert oracle.certify(p, bad)["bad_rows"] == 1


def test_rejects_an_unused_point():
    """Leaving a point out of an otherwise valid Delaunay triangulation of
    the rest: every condition but 'unused' holds when the point is inside
    the hull (it is then in some circumsphere, so not_local may hold too;
    what must fail is 'unused')."""
    p = inputs.uniform(600, 3, seed=4)
    inner = int(np.argmin(np.abs(p - 0.5).max(axis=1)))
    keep = np.delete(np.arange(len(p)), inner)
    rows = oracle.delaunay(p[keep], keep)
    cert = oracle.certify(p, rows)
    assert cert["unused"] == 1
    hs, hv = _hull(p)
    assert "unused" in oracle.certificate_ok(cert, hs, hv)
