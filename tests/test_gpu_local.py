"""GPU parity of the batched local triangulation (the kernels behind the
partial, sample and border triangulations): the simplex sets equal the CPU
oracle's bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1902_07554_amd import inputs

pytestmark = pytest.mark.gpu


def _rows(res):
    return oracle.canonical(res.rows())


@pytest.mark.parametrize("dim,n,dist", [(2, 3000, "uniform"), (3, 3000, "uniform"),
                                        (2, 20000, "normal"), (3, 20000, "bubbles"),
                                        (3, 60000, "uniform")])
def test_direct_matches_oracle(dtlib, dim, n, dist):
    p = inputs.make(dist, n, dim, seed=3)
    print(f"[direct] dim={dim} n={n} dist={dist}", flush=True)
    res = dtlib.triangulate(p, k=1)
    got = _rows(res)
    want = oracle.delaunay(p)
    assert got.shape == want.shape
    assert np.array_equal(got, want)


@pytest.mark.parametrize("side,dim", [(24, 2), (7, 3)])
def test_direct_lattice_matches_oracle(dtlib, side, dim):
    """Degenerate input: every tie is decided by the perturbation."""
    p = inputs.lattice(side, dim, seed=5)
    print(f"[lattice] side={side} dim={dim}", flush=True)
    got = _rows(dtlib.triangulate(p, k=1))
    assert np.array_equal(got, oracle.delaunay(p))


@pytest.mark.parametrize("dim", [2, 3])
def test_batch_matches_oracle_per_set(dtlib, dim):
    rng = np.random.default_rng(9)
    sizes = rng.integers(dim + 1, 400, 40)
    sizes[3] = 1        # too small: no simplices
    offsets = np.concatenate([[0], np.cumsum(sizes)])
    pts = rng.random((offsets[-1], dim))
    ids = rng.permutation(offsets[-1]).astype(np.int64) * 3 + 7
    print(f"[batch] dim={dim} sets={len(sizes)} n={offsets[-1]}", flush=True)
    res = dtlib.batch_triangulate(pts, offsets, ids=ids)
    rows = res.rows()
    so = res.set_offsets(len(sizes))
    for s in range(len(sizes)):
        got = oracle.canonical(rows[so[s]:so[s + 1]])
        a, b = offsets[s], offsets[s + 1]
        if b - a < dim + 1:
            assert len(got) == 0
            continue
        want = oracle.delaunay(pts[a:b], ids[a:b])
        assert np.array_equal(got, want), s


def test_error_paths(dtlib):
    with pytest.raises(dtlib.DTError) as e:
        dtlib.triangulate(np.array([[0, 0], [1, 0], [0, 1], [1, 0.0]]))
    assert e.value.status == dtlib.DT_E_DUPLICATE
    with pytest.raises(dtlib.DTError) as e:
        dtlib.triangulate(np.array([[0, 0], [1, 0], [0, np.inf]]))
    assert e.value.status == dtlib.DT_E_NONFINITE
    with pytest.raises(dtlib.DTError) as e:
        dtlib.triangulate(np.array([[0, 0], [1, 1], [2, 2], [3, 3.0]]))
    assert e.value.status == dtlib.DT_E_DEGENERATE
    with pytest.raises(dtlib.DTError) as e:
        dtlib.triangulate(np.zeros((5, 4)))
    assert e.value.status == dtlib.DT_E_INVALID_ARG
    # level step outside 9..32 eighths
    for bad in (8, 33):
        with pytest.raises(dtlib.DTError) as e:
            dtlib.triangulate(np.array([[0, 0], [1, 0], [0, 1.0]]), grow_num=bad)
        assert e.value.status == dtlib.DT_E_INVALID_ARG


def test_autotuned_batch_is_identical(dtlib):
    """Launch tunables change timing only: the autotuned batch, the default
    batch and extreme tunables give the same simplices, equal to the
    oracle's on sampled sets."""
    pts, offsets = inputs.batch_sets(96, 64, 8192, dim=2, seed=4)
    print(f"[autotune] sets=96 n={offsets[-1]}", flush=True)
    tuned = dtlib.batch_autotune(pts, offsets, sample_points=60000)
    assert set(tuned) == {"start_active", "grow_div", "cand_blocks", "grow_num"}
    assert 9 <= tuned["grow_num"] <= 32
    # a second call of the same size class comes from the cache
    assert dtlib.batch_autotune(pts, offsets, sample_points=60000) == tuned
    a = dtlib.batch_triangulate(pts, offsets, **tuned)
    b = dtlib.batch_triangulate(pts, offsets)
    c = dtlib.batch_triangulate(pts, offsets, start_active=16, grow_div=64, cand_blocks=1,
                                grow_num=32)
    ra, rb, rc = a.rows(), b.rows(), c.rows()
    soa, sob, soc = a.set_offsets(96), b.set_offsets(96), c.set_offsets(96)
    for s in range(96):
        x = oracle.canonical(ra[soa[s]:soa[s + 1]])
        assert np.array_equal(x, oracle.canonical(rb[sob[s]:sob[s + 1]])), s
        assert np.array_equal(x, oracle.canonical(rc[soc[s]:soc[s + 1]])), s
        if s % 16 == 0:
            a, b = offsets[s], offsets[s + 1]   # rows carry global point indices
            assert np.array_equal(x, oracle.delaunay(pts[a:b], np.arange(a, b))), s


def test_batch_allows_same_point_in_different_sets(dtlib):
    """Sets are independent: a point repeated in another set is no duplicate."""
    p = inputs.make("uniform", 300, 3, seed=8)
    pts = np.concatenate([p, p[::-1]])
    res = dtlib.batch_triangulate(pts, [0, 300, 600])
    rows, so = res.rows(), res.set_offsets(2)
    want = oracle.delaunay(p)
    assert np.array_equal(oracle.canonical(rows[so[0]:so[1]]), want)
    assert len(rows[so[1]:so[2]]) == len(want)
    dup = pts.copy()
    dup[400] = dup[420]
    with pytest.raises(dtlib.DTError) as e:
        dtlib.batch_triangulate(dup, [0, 300, 600])
    assert e.value.status == dtlib.DT_E_DUPLICATE


@pytest.mark.parametrize("dim,n,dist", [(2, 20000, "normal"), (3, 30000, "bubbles"),
                                        (3, 8 ** 3, "lattice")])
def test_fp32_filter_matches_oracle(dtlib, dim, n, dist):
    """FP32 filtered predicates (with FP64 and exact fallbacks) decide every
    sign exactly: the simplex set is the oracle's, and on a lattice the
    exact stage is reached."""
    p = inputs.lattice(8, 3, seed=6) if dist == "lattice" else inputs.make(dist, n, dim, seed=12)
    print(f"[fp32] dim={dim} n={len(p)} dist={dist}", flush=True)
    res = dtlib.triangulate(p, k=1, precision="fp32")
    assert np.array_equal(_rows(res), oracle.delaunay(p))
    pred = res.stats()["pred"]
    ins = pred["insphere3d" if dim == 3 else "insphere2d"]
    assert ins["calls"] > 0
    assert ins["calls"] == ins["fp32"] + ins["fp64"] + ins["exact"]
    if dist == "lattice":
        assert ins["exact"] > 0


@pytest.mark.parametrize("dim,side,rel,k", [(3, 9, 2.0 ** -20, 1), (3, 9, 2.0 ** -33, 1),
                                            (3, 9, 2.0 ** -45, 1), (2, 40, 2.0 ** -30, 1),
                                            (3, 12, 2.0 ** -28, 8), (2, 50, 2.0 ** -40, 4)])
def test_fp32_filter_on_jittered_lattices(dtlib, dim, side, rel, k):
    """Lattices moved by relative 2^-20 .. 2^-45: every in-sphere test is a
    near-tie inside or just outside the FP32 filter's band; the FP32 mode
    must still give the oracle's simplex set, directly and divided."""
    p = inputs.jittered_lattice(side, dim, rel, seed=3)
    print(f"[fp32] jittered lattice dim={dim} side={side} rel=2^{np.log2(rel):.0f} k={k}",
          flush=True)
    res = dtlib.triangulate(p, k=k, sample_rate=0.05, precision="fp32")
    assert np.array_equal(_rows(res), oracle.delaunay(p))
    ins = res.stats()["pred"]["insphere3d" if dim == 3 else "insphere2d"]
    assert ins["fp64"] + ins["exact"] > 0


def _sphere_and_centre(n, dim, seed, jitter=1e-4):
    """n points within a relative `jitter` of the unit sphere (circle) and
    its centre, randomly permuted: inserted after a few percent of the
    sphere points, the centre's conflict region holds almost every cell."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, dim))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    v *= 1.0 + jitter * rng.uniform(-1.0, 1.0, (n, 1))
    p = np.concatenate([v, np.zeros((1, dim))])
    return p[rng.permutation(len(p))]


def _circles_and_centres(count, n, seed):
    """`count` circles of n points each (radius 1, centres 4 apart on a
    line) and their centres, randomly permuted: each centre inserted after
    a fifth of its circle's points has a conflict region of more than 8,300
    triangles."""
    rng = np.random.default_rng(seed)
    parts = []
    for c in range(count):
        t = rng.uniform(0.0, 2.0 * np.pi, n)
        ring = np.stack([np.cos(t), np.sin(t)], 1) + [4.0 * c, 0.0]
        parts += [ring, [[4.0 * c, 0.0]]]
    p = np.concatenate(parts)
    return p[rng.permutation(len(p))]


@pytest.mark.parametrize("dim,n,precision", [(3, 100_000, "fp64"), (2, 12_000, "fp32")])
def test_cavity_larger_than_the_candidate_lists(dtlib, dim, n, precision):
    """A cavity of more cells than a candidate's list and its extension
    chunk hold (192 + 8192 in 3D, 96 + 8192 in 2D) is inserted through the
    pool-sized list: the result is the oracle's DT."""
    p = _sphere_and_centre(n, dim, seed=5) if dim == 3 else _circles_and_centres(10, n, seed=5)
    print(f"[large cavity] dim={dim} n={len(p)}", flush=True)
    res = dtlib.triangulate(p, k=1, precision=precision)
    st = res.stats()
    assert st["large_cavities"] >= 1
    assert np.array_equal(_rows(res), oracle.delaunay(p))


@pytest.mark.parametrize("dim,k", [(2, 1), (3, 1), (3, 8)])
def test_neighbors_match_oracle(dtlib, dim, k):
    """dt_result_neighbors equals the facet-sharing definition on the rows
    the library returns."""
    p = inputs.make("bubbles" if dim == 3 else "normal", 6000, dim, seed=5)
    print(f"[neighbors] dim={dim} k={k}", flush=True)
    res = dtlib.triangulate(p, k=k, sample_rate=0.05, sort_output=1)
    rows = res.rows()
    assert np.array_equal(rows, oracle.delaunay(p))
    assert np.array_equal(res.neighbors(), oracle.neighbors(rows))


def test_neighbors_stay_inside_each_set(dtlib):
    """Batch rows of different sets never pair, even with equal labels."""
    a = inputs.make("uniform", 400, 2, seed=1)
    b = inputs.make("normal", 300, 2, seed=2)
    pts = np.concatenate([a, b])
    ids = np.concatenate([np.arange(400), np.arange(300)]).astype(np.int64)
    res = dtlib.batch_triangulate(pts, [0, 400, 700], ids=ids)
    rows, so, nb = res.rows(), res.set_offsets(2), res.neighbors()
    for s in range(2):
        lo, hi = so[s], so[s + 1]
        want = oracle.neighbors(rows[lo:hi])
        got = nb[lo:hi].astype(np.int64)
        got[got >= 0] -= lo
        assert np.array_equal(got, want)


@pytest.mark.parametrize("dim,kind,n,prec", [
    (3, "bubbles", 120_000, "fp32"),
    (3, "uniform", 100_000, "fp64"),
    (2, "normal", 150_000, "fp32"),
    (2, "lattice", 67_600, "fp64"),     # 260 x 260: every tie perturbed
    (3, "jittered", 68_921, "fp32"),    # 41^3, moved by 2^-30 grid steps
])
def test_single_set_seeded_by_gift_wrap(dtlib, dim, kind, n, prec):
    """A single set of at least 65,536 points starts from the gift-wrapped
    triangulation of its first points in insertion order (neighbour links by
    facet matching, a hull cell per hull facet) and inserts the rest in
    parallel rounds: the oracle's simplices, as when it starts from one
    simplex."""
    if kind == "lattice":
        p = inputs.lattice(round(n ** (1.0 / dim)), dim, seed=6)
    elif kind == "jittered":
        p = inputs.jittered_lattice(round(n ** (1.0 / dim)), dim, 2.0 ** -30, seed=6)
    else:
        p = inputs.make(kind, n, dim, seed=6)
    print(f"[seed] dim={dim} kind={kind} n={len(p)} {prec}", flush=True)
    res = dtlib.triangulate(p, k=1, precision=prec)
    assert res.stats()["seeded_sets"] == 1
    got = _rows(res)
    assert np.array_equal(got, oracle.delaunay(p))
    ref = dtlib.triangulate(p, k=1, precision=prec, gift_wrap=-1)
    assert ref.stats()["seeded_sets"] == 0
    assert np.array_equal(_rows(ref), got)


@pytest.mark.parametrize("dim,prec", [(3, "fp32"), (3, "fp64"), (2, "fp32")])
def test_batch_sets_seeded_by_gift_wrap(dtlib, dim, prec):
    """Every set of a batched run with at least 8192 points starts from the
    gift-wrapped triangulation of its points below a common priority
    threshold (all sets wrapped together); smaller sets start from one
    simplex.  Each set's simplices are the oracle's, and the same as when
    every set starts from one simplex.  The sets mix distributions, a
    lattice (every tie perturbed) and a lattice moved by 2^-30 steps."""
    side = 24 if dim == 3 else 110
    sets = [inputs.make("bubbles", 15_000, dim, seed=11),
            inputs.make("uniform", 9_000, dim, seed=12),
            inputs.make("normal", 600, dim, seed=13),          # small: one simplex
            inputs.lattice(side, dim, seed=14),
            inputs.jittered_lattice(side - 2, dim, 2.0 ** -30, seed=15),
            inputs.make("uniform", 3_000, dim, seed=16),       # small: one simplex
            inputs.make("normal", 20_000, dim, seed=17)]
    sizes = [len(x) for x in sets]
    offsets = np.concatenate([[0], np.cumsum(sizes)])
    pts = np.concatenate(sets)
    ids = np.concatenate([np.arange(n) for n in sizes]).astype(np.int64)
    print(f"[seed-sets] dim={dim} {prec} sizes={sizes}", flush=True)
    res = dtlib.batch_triangulate(pts, offsets, ids=ids, precision=prec)
    assert res.stats()["seeded_sets"] == sum(1 for n in sizes if n >= 8192)
    ref = dtlib.batch_triangulate(pts, offsets, ids=ids, precision=prec, gift_wrap=-1)
    assert ref.stats()["seeded_sets"] == 0
    rows, so = res.rows(), res.set_offsets(len(sizes))
    rrows, rso = ref.rows(), ref.set_offsets(len(sizes))
    for s in range(len(sizes)):
        got = oracle.canonical(rows[so[s]:so[s + 1]])
        want = oracle.delaunay(sets[s])
        assert np.array_equal(got, want), s
        assert np.array_equal(oracle.canonical(rrows[rso[s]:rso[s + 1]]), got), s


def _thin(n, seed):
    """Points on a segment in the plane, up to the rounding of y = 1/4 + t/2
    (a valid input: distinct, not all collinear in floating point, with
    extremely thin triangles and cavities of thousands of cells)."""
    t = np.random.default_rng(seed).random(n)
    return np.stack([t, 0.25 + 0.5 * t], axis=1)


def test_thin_sets_seeded_and_unseeded(dtlib):
    """Nearly collinear sets, whose new points conflict with thousands of
    triangles around one vertex: a batch with such a set among others, with
    and without the gift-wrapped seeds, gives the oracle's triangles per
    set; a single set of 70,000 such points (large enough for its own seed)
    gives the same rows seeded and not, every interior edge locally
    Delaunay under the oracle's exact predicate and every point a vertex
    (the hull of such a set is beyond Qhull's precision, so the hull is not
    compared)."""
    sets = [inputs.make("normal", 10_000, 2, seed=32), _thin(9000, 31),
            inputs.make("uniform", 12_000, 2, seed=33)]
    sizes = [len(x) for x in sets]
    offsets = np.concatenate([[0], np.cumsum(sizes)])
    pts = np.concatenate(sets)
    ids = np.concatenate([np.arange(n) for n in sizes]).astype(np.int64)
    print(f"[thin] batch sizes={sizes}", flush=True)
    for gw, seeded in ((0, 3), (-1, 0)):
        res = dtlib.batch_triangulate(pts, offsets, ids=ids, gift_wrap=gw)
        assert res.stats()["seeded_sets"] == seeded
        rows, so = res.rows(), res.set_offsets(len(sizes))
        for s in range(len(sizes)):
            got = oracle.canonical(rows[so[s]:so[s + 1]])
            assert np.array_equal(got, oracle.delaunay(sets[s])), (gw, s)
    p = _thin(70_000, 41)
    print("[thin] single set n=70000", flush=True)
    a = _rows(dtlib.triangulate(p, k=1))
    b = _rows(dtlib.triangulate(p, k=1, gift_wrap=-1))
    assert np.array_equal(a, b)
    cert = oracle.certify(p, a)
    assert [f for f in ("bad_rows", "flat", "over_shared", "same_side", "not_local", "unused")
            if cert[f]] == []
    assert len(p) - cert["edges"] + cert["m"] == 1      # Euler: a triangulated disk


def test_nearly_planar_3d_set(dtlib):
    """3D points on a plane up to rounding (slivers everywhere, thousands
    of tetrahedra around an edge in one cavity): the oracle's tetrahedra,
    alone and batched with a seeded set, with and without gift wrapping."""
    xy = np.random.default_rng(51).random((6000, 2))
    p = np.stack([xy[:, 0], xy[:, 1], 0.3 + 0.2 * xy[:, 0] - 0.1 * xy[:, 1]], axis=1)
    want = oracle.delaunay(p)
    off = np.array([0, 6000, 15000])
    q = np.concatenate([p, inputs.make("uniform", 9000, 3, seed=52)])
    print("[thin] nearly planar 3D n=6000", flush=True)
    for gw in (0, -1):
        assert np.array_equal(_rows(dtlib.triangulate(p, k=1, gift_wrap=gw)), want), gw
        r = dtlib.batch_triangulate(q, off, gift_wrap=gw)
        so = r.set_offsets(2)
        assert np.array_equal(oracle.canonical(r.rows()[so[0]:so[1]]), want), gw

