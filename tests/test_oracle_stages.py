"""Pins of the oracle's per-stage references (sample, graph, nearest sample,
buckets, kd divide, merge, quality metrics) against brute force, published
test vectors and closed forms."""
import numpy as np
import pytest

import oracle
from paper_1902_07554_amd import inputs
from tests import exact_ref as X


def test_splitmix64_published_vectors():
    # SplitMix64 seeded with 0 yields 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
    # 0x06C45D188009454F (Steele, Lea, Flood 2014 reference generator): the
    # k-th output is the finaliser applied to k * golden-gamma.
    g = 0x9E3779B97F4A7C15
    xs = np.array([0, g, (2 * g) & ((1 << 64) - 1)], dtype=np.uint64)
    got = [int(v) for v in oracle.splitmix64(xs)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_sample_ids_brute_force():
    n, seed = 3000, 17
    eta = oracle.sample_size(n, 0.01, 3)
    assert eta == 30
    got = oracle.sample_ids(n, eta, seed)
    M = (1 << 64) - 1

    def mix(z):
        z = (z + 0x9E3779B97F4A7C15) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)
    keys = [(mix(seed ^ ((i * 0x9E3779B97F4A7C15) & M)), i) for i in range(n)]
    want = sorted(i for _, i in sorted(keys)[:eta])
    assert list(got) == want
    assert len(set(got)) == eta


def test_sample_size_rules():
    assert oracle.sample_size(10000, 0.01, 2) == 100
    assert oracle.sample_size(1048576, 0.005, 3) == 5243       # 5242.88
    assert oracle.sample_size(4194304, 0.005, 3) == 20972      # 20971.52
    assert oracle.sample_size(4194304, 0.0, 3) == 2048          # sqrt(n)
    assert oracle.sample_size(10, 0.01, 3) == 5                 # at least D+2


def test_graph_edges_and_weights():
    p = np.array([[0, 0], [1, 0], [0, 1], [1, 1.0]])
    simp = np.array([[0, 1, 2], [1, 2, 3]])
    e = oracle.graph_edges(simp)
    assert e.tolist() == [[0, 1], [0, 2], [1, 2], [1, 3], [2, 3]]
    w = oracle.edge_weights(p, e, "log")
    d = np.array([1, 1, np.sqrt(2), 1, 1]) / np.sqrt(2)
    assert np.allclose(w, -np.log(d))
    assert np.allclose(oracle.edge_weights(p, e, "inverse"), 1 / d)
    assert np.allclose(oracle.edge_weights(p, e, "linear"), 1 - d)
    assert np.allclose(oracle.edge_weights(p, e, "const"), 1)


def test_nearest_sample_brute_force_with_ties():
    r = np.random.default_rng(3)
    s = r.random((40, 3))
    sid = np.arange(40) * 2 + 1
    # ties: a point equidistant from two samples (mirror images)
    s[5] = [0.5 - 2.0 ** -10, 0.5, 0.5]
    s[9] = [0.5 + 2.0 ** -10, 0.5, 0.5]
    pts = np.concatenate([r.random((300, 3)), [[0.5, 0.5, 0.5]]])
    got = oracle.nearest_sample(pts, s, sid)
    for i, q in enumerate(pts):
        best = None
        for j in range(40):
            d = ((q[0] - s[j, 0]) * (q[0] - s[j, 0]) + (q[1] - s[j, 1]) * (q[1] - s[j, 1])) \
                + (q[2] - s[j, 2]) * (q[2] - s[j, 2])
            key = (d, sid[j])
            if best is None or key < best[0]:
                best = (key, j)
        assert got[i] == best[1]
    assert got[-1] == 5


def test_buckets_are_the_partitions():
    pid = np.array([2, 0, 1, 0, 2, 1, 0])
    b = oracle.buckets(pid, 4)
    assert [x.tolist() for x in b] == [[1, 3, 6], [2, 5], [0, 4], []]


def test_kd_divide_boxes():
    p = inputs.uniform(1000, 3, seed=2)
    pid = oracle.kd_divide(p, 8)
    cnt = np.bincount(pid, minlength=8)
    assert cnt.max() - cnt.min() <= 1
    # first split on x: blocks 0-3 left of blocks 4-7; then y; then z
    assert p[pid < 4, 0].max() <= p[pid >= 4, 0].min()
    for h in (0, 4):
        a, b = pid >= h, pid < h + 4
        lo = a & b & (pid < h + 2)
        hi = a & b & (pid >= h + 2)
        assert p[lo, 1].max() <= p[hi, 1].min()
    for b in range(0, 8, 2):
        assert p[pid == b, 2].max() <= p[pid == b + 1, 2].min()


def test_quality_metrics_closed_forms():
    s = np.array([10, 12, 8, 10])
    assert np.allclose(oracle.deviation(s), [0, 0.2, -0.2, 0])
    assert oracle.coeff_variation(s) == pytest.approx(np.sqrt(8 / 3) / 10)
    assert oracle.overtriangulation(100, 10, 5) == pytest.approx(1.15)
    e = np.array([[0, 1], [1, 2], [2, 3]])
    assert oracle.cut_weight(e, np.array([1.0, 2.0, 4.0]), np.array([0, 0, 1, 1])) == 2.0
    assert oracle.balanced(np.array([0, 0, 1, 1, 1]), 2, 0.05) is True
    assert oracle.balanced(np.array([0, 1, 1, 1, 1]), 2, 0.05) is False


# ------------------------------------------------------ Algorithm 1 merge pin
def _hull_facets(simp):
    cnt = {}
    apex = {}
    for s in simp:
        for j in range(len(s)):
            f = tuple(sorted(np.delete(s, j)))
            cnt[f] = cnt.get(f, 0) + 1
            apex[f] = s[j]
    return [(f, apex[f]) for f, c in cnt.items() if c == 1]


def _border_sets(p, pid, k, all_hull):
    """T_i = DT(P_i); B = finite simplices whose circumsphere contains a
    point of another partition (exact perturbed test); hull cells flagged if
    their outer half-space holds such a point (or all of them)."""
    n = len(p)
    ids = np.arange(n)
    parts, flags, vb = [], [], set()
    for i in range(k):
        mine = ids[pid == i]
        other = ids[pid != i]
        t = oracle.delaunay(p[mine], mine)
        f = np.zeros(len(t), bool)
        for r, s in enumerate(t):
            o = X.orient1(p[s])
            for q in other:
                keys = list(s) + [q]
                P = [p[v] for v in s] + [p[q]]
                sg = X.insphere_sign(P) or X.insphere_sign(P, keys)
                if sg == o:
                    f[r] = True
                    break
        parts.append(t)
        flags.append(f)
        for s in t[f]:
            vb.update(int(v) for v in s)
        for fac, ap in _hull_facets(t):
            if all_hull:
                vb.update(int(v) for v in fac)
                continue
            oa = X.orient1([p[v] for v in fac] + [p[ap]])
            for q in other:
                if X.orient1([p[v] for v in fac] + [p[q]]) == -oa:
                    vb.update(int(v) for v in fac)
                    break
    return parts, flags, np.array(sorted(vb))


@pytest.mark.parametrize("all_hull", [False, True])
@pytest.mark.parametrize("divide", ["kd", "sample"])
def test_merge_reproduces_dt_2d(divide, all_hull):
    n, k = 120, 4
    p = inputs.uniform(n, 2, seed=21)
    if divide == "kd":
        pid = oracle.kd_divide(p, k)
    else:
        sid = oracle.sample_ids(n, 12, seed=1)
        pid = oracle.nearest_sample(p, p[sid], sid) % k
    parts, flags, vb = _border_sets(p, pid, k, all_hull)
    tb = oracle.delaunay(p[vb], vb)
    got = oracle.merge(parts, flags, tb, pid)
    assert np.array_equal(got, oracle.delaunay(p))


def test_merge_reproduces_dt_3d():
    n, k = 60, 4
    p = inputs.bubbles(n, 3, seed=5)
    pid = oracle.kd_divide(p, k)
    parts, flags, vb = _border_sets(p, pid, k, all_hull=True)
    tb = oracle.delaunay(p[vb], vb)
    assert np.array_equal(oracle.merge(parts, flags, tb, pid), oracle.delaunay(p))


@pytest.mark.parametrize("dim", [2, 3])
def test_neighbors_pins(dim):
    """Neighbours of DT(P): symmetric, sharing exactly D vertices; the
    facets without a neighbour are the convex hull's facets (Qhull)."""
    from scipy.spatial import ConvexHull
    p = inputs.uniform(300, dim, seed=6)
    rows = oracle.delaunay(p)
    nb = oracle.neighbors(rows)
    m, w = rows.shape
    for i in range(m):
        for j in range(w):
            k = nb[i, j]
            if k < 0:
                continue
            assert i in nb[k]
            shared = set(rows[i]) & set(rows[k])
            assert len(shared) == dim and rows[i, j] not in shared
    hull = ConvexHull(p)
    assert (nb < 0).sum() == len(hull.simplices)
    hull_facets = {tuple(sorted(f)) for f in hull.simplices}
    got = {tuple(sorted(int(rows[i, r]) for r in range(w) if r != j))
           for i, j in zip(*np.nonzero(nb < 0))}
    assert got == hull_facets
