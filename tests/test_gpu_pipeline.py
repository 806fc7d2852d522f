"""GPU parity of the whole divide-and-conquer path (Algorithm 1 with the
sample divide of Algorithm 2, and with the cyclic kd divide) against the CPU
oracle: every deterministic stage element by element, the partition by its
balance bound, the border by its soundness property, and the final simplex
set bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1902_07554_amd import inputs

pytestmark = pytest.mark.gpu


def _check_buckets(order, pid, k):
    """Algorithm 2's partitions as buckets: `order` is a permutation of the
    points, grouped by partition in partition order, and bucket i holds
    exactly P_i (the order inside a bucket is free)."""
    n = len(pid)
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.all(np.diff(pid[order]) >= 0)
    off = np.concatenate([[0], np.cumsum(np.bincount(pid, minlength=k))])
    for i, members in enumerate(oracle.buckets(pid, k)):
        assert np.array_equal(np.sort(order[off[i]:off[i + 1]]), members), f"bucket {i}"


def _check_graph(res, p, sid, part, k, weight, st):
    """Algorithm 2's weighted graph (the sample DT's edges, Table "weights")
    and the partition's cut weight (Section "Partitioning Quality") against
    the oracle, given the same sample triangulation."""
    edges = res.stage("graph").astype(np.int64)
    w = res.stage("weights")
    want = oracle.graph_edges(oracle.canonical(res.stage("sample_dt")))
    assert np.array_equal(edges, want), "sample-graph edges"
    ww = oracle.edge_weights(p, want, kind=weight)
    np.testing.assert_allclose(w, ww, rtol=1e-12, atol=1e-12)
    part_of = np.full(len(p), -1, dtype=np.int64)
    part_of[sid] = part
    cut = oracle.cut_weight(want, ww, part_of)
    assert st["cut_weight"] == pytest.approx(cut, rel=1e-9, abs=1e-9)


def _check_metrics(st, pid, k, n, eta, nvb, loc_flag, n_tb):
    """Section "Partitioning Quality": deviation, c_v, o_DT and the border
    sizes, from the oracle's formulas on the stage arrays."""
    sizes = np.bincount(pid, minlength=k)
    assert st["max_dev"] == pytest.approx(float(oracle.deviation(sizes).max()), rel=1e-12, abs=1e-12)
    assert st["cv"] == pytest.approx(oracle.coeff_variation(sizes), rel=1e-12, abs=1e-12)
    assert st["max_part"] == sizes.max() and st["min_part"] == sizes.min()
    assert st["o_dt"] == pytest.approx(oracle.overtriangulation(n, eta, nvb), rel=1e-15)
    assert st["border_simplices"] == int(loc_flag.sum())
    assert st["local_simplices"] == len(loc_flag)
    assert st["tb_simplices"] == n_tb


def _stage_checks(dtlib, p, k, rate, seed, divide, border="region", weight="log", eps=0.05,
                  grid_cell=1.0):
    n, dim = p.shape
    res = dtlib.triangulate(p, k=k, sample_rate=rate, divide=divide, seed=seed, keep_stages=1,
                            border=border, weight=weight, eps=eps, grid_cell=grid_cell)
    ids = np.arange(n)
    full = oracle.delaunay(p)
    got = oracle.canonical(res.rows())
    assert np.array_equal(got, full), "merged simplex set differs from the oracle"
    pid = res.stage("pid").astype(np.int64)
    st = res.stats()
    eta = 0
    if divide == "sample":
        eta = oracle.sample_size(n, rate, dim)
        sid = res.stage("sample")
        assert np.array_equal(sid, oracle.sample_ids(n, eta, seed))
        assert np.array_equal(oracle.canonical(res.stage("sample_dt")), oracle.delaunay(p[sid], sid))
        part = res.stage("part").astype(np.int64)
        assert oracle.balanced(part, k, eps)
        near = oracle.nearest_sample(p, p[sid], sid)
        assert np.array_equal(res.stage("nearest"), near)
        assert np.array_equal(pid, part[near])
        _check_graph(res, p, sid, part, k, weight, st)
    else:
        assert np.array_equal(pid, oracle.kd_divide(p, k))
    _check_buckets(res.stage("order").astype(np.int64), pid, k)
    loc = res.stage("local")
    rows, flag = oracle.canonical(loc[:, :-1]), None
    # per-partition triangulations and border soundness
    order = np.lexsort(np.sort(loc[:, :-1], axis=1).T[::-1])
    loc = loc[order]
    flag = loc[:, -1].astype(bool)
    srows = np.sort(loc[:, :-1], axis=1)
    fullset = {tuple(r) for r in full}
    for i in range(k):
        mine = ids[pid == i]
        sel = pid[srows[:, 0]] == i
        if len(mine) < dim + 1:
            assert not sel.any()
            continue
        want = oracle.delaunay(p[mine], mine)
        assert np.array_equal(oracle.canonical(srows[sel]), want), f"T_{i}"
        for r, f in zip(srows[sel], flag[sel]):
            if tuple(r) not in fullset:
                assert f, "a simplex of T_i outside DT(P) was not flagged"
    vb = res.stage("border_v")
    assert set(np.unique(srows[flag])) <= set(vb.tolist())
    tb = oracle.delaunay(p[vb], vb)
    assert np.array_equal(oracle.canonical(res.stage("border_dt")), tb)
    assert st["border_vertices"] == len(vb)
    assert st["num_simplices"] == len(full)
    _check_metrics(st, pid, k, n, eta, len(vb), flag, len(tb))
    return res


@pytest.mark.parametrize("divide,border", [("sample", "region"), ("kd", "region"),
                                           ("sample", "grid"), ("sample", "bbox"),
                                           ("sample", "exact"), ("kd", "exact"),
                                           ("sample", "refined"), ("kd", "refined")])
def test_config_2d_10k(dtlib, divide, border):
    """2D, n = 10,000 uniform, sample 1 % (100 points), k = 4."""
    p = inputs.uniform(10_000, 2, seed=1)
    print(f"[pipeline] 2d 10k {divide} {border}", flush=True)
    _stage_checks(dtlib, p, 4, 0.01, 1, divide, border)


@pytest.mark.parametrize("divide,dist,k,border", [
    ("sample", "uniform", 16, "region"), ("kd", "uniform", 16, "region"),
    ("sample", "bubbles", 32, "region"), ("kd", "bubbles", 32, "region"),
    ("sample", "normal", 8, "region"), ("sample", "bubbles", 32, "grid"),
    ("kd", "uniform", 16, "grid"), ("sample", "bubbles", 32, "bbox"),
    ("sample", "bubbles", 32, "exact"), ("kd", "uniform", 16, "exact"),
    ("sample", "bubbles", 32, "refined")])
def test_3d_stages(dtlib, divide, dist, k, border):
    p = inputs.make(dist, 20_000, 3, seed=4)
    print(f"[pipeline] 3d 20k {dist} {divide} k={k} border={border}", flush=True)
    _stage_checks(dtlib, p, k, 0.01, 3, divide, border)


@pytest.mark.parametrize("weight,eps,grid_cell,border", [
    ("const", 0.05, 1.0, "region"), ("inverse", 0.05, 1.0, "region"),
    ("linear", 0.05, 1.0, "region"), ("log", 0.03, 1.0, "region"), ("log", 0.3, 1.0, "region"),
    ("log", 0.05, 0.5, "grid"), ("log", 0.05, 2.0, "grid"), ("inverse", 0.3, 2.0, "grid")])
def test_weights_balance_and_grid_sizes(dtlib, weight, eps, grid_cell, border):
    """Table "weights" (constant, inverse, linear next to log), the balance
    bound at eps 0.03 and 0.3, and the grid test at c_G = 1/2 and 2
    (Section "Grid-based Intersection Test"): every stage against the
    oracle, the final set bit for bit."""
    p = inputs.make("bubbles", 20_000, 3, seed=21)
    print(f"[pipeline] weight={weight} eps={eps} c_G={grid_cell} border={border}", flush=True)
    _stage_checks(dtlib, p, 16, 0.02, 5, "sample", border, weight=weight, eps=eps,
                  grid_cell=grid_cell)


def test_partition_is_deterministic_and_cuts_less_than_its_start(dtlib):
    """The partitioner is not KaHIP, whose output is not reproducible; its
    own pins: the same blocks on every run, and label propagation never
    raises the cut of its starting blocks (the kd split of the sample)."""
    p = inputs.make("bubbles", 40_000, 3, seed=3)
    a = dtlib.triangulate(p, k=16, sample_rate=0.02, keep_stages=1)
    b = dtlib.triangulate(p, k=16, sample_rate=0.02, keep_stages=1)
    assert np.array_equal(a.stage("part"), b.stage("part"))
    assert np.array_equal(a.stage("pid"), b.stage("pid"))
    sid = a.stage("sample")
    edges = a.stage("graph").astype(np.int64)
    w = a.stage("weights")
    start = np.full(len(p), -1, dtype=np.int64)
    start[sid] = oracle.kd_divide(p[sid], 16)
    assert a.stats()["cut_weight"] <= oracle.cut_weight(edges, w, start) + 1e-9


def test_pair_exchanges_under_a_strict_bound(dtlib):
    """At eight samples per block the 5 % bound leaves no room (the 4M
    clustered workload's setting, eta = 2048 and k = 256), so only pair
    exchanges can change the kd start.  With them the blocks stay within
    the bound and the same on every run, the cut is no larger than with
    moves alone or at the start, and the simplex set is the oracle's
    whichever partition is used (Algorithm 1 does not depend on it)."""
    p = inputs.make("bubbles", 40_000, 3, seed=5)
    k, rate = 64, 512 / 40_000
    print(f"[pipeline] pair exchanges k={k} eta=512", flush=True)
    on = dtlib.triangulate(p, k=k, sample_rate=rate, keep_stages=1)
    again = dtlib.triangulate(p, k=k, sample_rate=rate, keep_stages=1)
    off = dtlib.triangulate(p, k=k, sample_rate=rate, keep_stages=1, refine_swaps=-1)
    assert on.stats()["eta"] == 512
    part_on = on.stage("part")
    assert np.array_equal(part_on, again.stage("part"))
    sid = on.stage("sample")
    full = np.full(len(p), -1, dtype=np.int64)
    full[sid] = part_on
    assert oracle.balanced(part_on, k, 0.05)
    assert np.bincount(part_on, minlength=k).max() == 8
    edges = on.stage("graph").astype(np.int64)
    w = on.stage("weights")
    start = np.full(len(p), -1, dtype=np.int64)
    start[sid] = oracle.kd_divide(p[sid], k)
    assert np.array_equal(start[sid], off.stage("part"))   # nothing moves without exchanges
    cut_on = oracle.cut_weight(edges, w, full)
    assert on.stats()["cut_weight"] == pytest.approx(cut_on, rel=1e-9, abs=1e-9)
    assert cut_on <= oracle.cut_weight(edges, w, start) + 1e-9
    assert not np.array_equal(part_on, off.stage("part"))
    want = oracle.canonical(oracle.delaunay(p))
    for r in (on, off):
        assert np.array_equal(oracle.canonical(r.rows()), want)


@pytest.mark.parametrize("dim,side,k", [(2, 60, 4), (3, 12, 8)])
def test_lattice_through_pipeline(dtlib, dim, side, k):
    """Degenerate input: ties everywhere, also across partition borders."""
    p = inputs.lattice(side, dim, seed=2)
    print(f"[pipeline] lattice dim={dim} side={side}", flush=True)
    want = oracle.delaunay(p)
    for divide in ("sample", "kd"):
        for border in ("region", "grid"):
            res = dtlib.triangulate(p, k=k, sample_rate=0.02, divide=divide, border=border)
            assert np.array_equal(oracle.canonical(res.rows()), want), (divide, border)


def test_kd_divide_selection_and_ties(dtlib):
    """The kd divide's median split, found by selection, equals the split of
    a full (coordinate, id) sort: at a size with many points per histogram
    bin, and on columns of equal x coordinates whose median bin is too large
    for the in-LDS sort (that level is split by the sorting path)."""
    p = inputs.make("bubbles", 300_000, 3, seed=4)
    res = dtlib.triangulate(p, k=64, divide="kd", keep_stages=1)
    assert np.array_equal(res.stage("pid").astype(np.int64), oracle.kd_divide(p, 64))
    rng = np.random.default_rng(6)
    q = np.stack([rng.integers(0, 8, 40_000).astype(np.float64), rng.random(40_000)], 1)
    q = np.unique(q, axis=0)
    res = dtlib.triangulate(q, k=16, divide="kd", keep_stages=1)
    assert np.array_equal(res.stage("pid").astype(np.int64), oracle.kd_divide(q, 16))


def test_independent_of_division(dtlib):
    """DT(P) does not depend on the division: k, divide and seed vary."""
    p = inputs.bubbles(30_000, 3, seed=8)
    base = oracle.canonical(dtlib.triangulate(p, k=1).rows())
    for k, divide, seed in [(2, "sample", 1), (16, "sample", 5), (64, "sample", 9),
                            (16, "kd", 1), (64, "kd", 1)]:
        print(f"[independence] k={k} {divide} seed={seed}", flush=True)
        got = oracle.canonical(dtlib.triangulate(p, k=k, sample_rate=0.01, divide=divide,
                                                 seed=seed).rows())
        assert np.array_equal(got, base), (k, divide, seed)
    assert np.array_equal(base, oracle.delaunay(p))


def test_small_and_edge_inputs(dtlib):
    # partitions may be tiny or degenerate; the result must still be DT(P)
    rng = np.random.default_rng(3)
    p = rng.random((60, 3))
    res = dtlib.triangulate(p, k=8, sample_rate=0.2)
    assert np.array_equal(oracle.canonical(res.rows()), oracle.delaunay(p))
    # collinear clusters inside a 2D set
    q = np.concatenate([rng.random((200, 2)), np.stack([np.linspace(0, 1, 50), np.full(50, 0.5)], 1)])
    q = np.unique(q, axis=0)
    res = dtlib.triangulate(q, k=4, sample_rate=0.1, divide="sample")
    assert np.array_equal(oracle.canonical(res.rows()), oracle.delaunay(q))
    with pytest.raises(dtlib.DTError) as e:
        dtlib.triangulate(p, k=3, divide="kd")       # kd needs a power of two
    assert e.value.status == dtlib.DT_E_INVALID_ARG
    with pytest.raises(dtlib.DTError) as e:
        dtlib.triangulate(p, k=40, sample_rate=0.1)   # k > eta
    assert e.value.status == dtlib.DT_E_INVALID_ARG


def test_border_primitives_order(dtlib):
    """Section "Geometric Primitives": the exact test flags the fewest
    simplices, the bounding-box test the most; every primitive gives the
    same triangulation."""
    p = inputs.make("bubbles", 20_000, 3, seed=9)
    print("[pipeline] border primitives", flush=True)
    nb, rows = {}, {}
    for border in ("exact", "refined", "region", "grid", "bbox"):
        res = dtlib.triangulate(p, k=16, sample_rate=0.01, border=border, sort_output=1)
        nb[border] = res.stats()["border_simplices"]
        rows[border] = res.rows()
    for border in ("refined", "region", "grid", "bbox"):
        assert np.array_equal(rows[border], rows["exact"])
        assert nb["exact"] <= nb[border]
    assert nb["refined"] == nb["exact"] and nb["refined"] <= nb["region"]
    assert nb["region"] <= nb["bbox"] and nb["grid"] <= nb["bbox"]


@pytest.mark.parametrize("dist,want", [("uniform", 1), ("bubbles", 0)])
def test_auto_divide(dtlib, dist, want):
    """The adaptive divide picks kd for evenly spread input and the sample
    divide for clustered input; either way the result is the DT."""
    p = inputs.make(dist, 30_000, 3, seed=2)
    print(f"[pipeline] auto divide {dist}", flush=True)
    res = dtlib.triangulate(p, k=16, sample_rate=0.02, divide="auto", sort_output=1)
    st = res.stats()
    assert st["divide_used"] == want, st["divide_stat"]
    assert np.array_equal(res.rows(), oracle.delaunay(p))


@pytest.mark.parametrize("dim,dist,n,k,divide,border", [
    (2, "uniform", 10_000, 4, "kd", "region"), (2, "normal", 10_000, 8, "sample", "region"),
    (3, "bubbles", 20_000, 8, "kd", "region"), (3, "bubbles", 20_000, 16, "sample", "region"),
    (3, "uniform", 20_000, 2, "sample", "region"), (3, "bubbles", 20_000, 16, "sample", "grid"),
    (3, "uniform", 20_000, 8, "kd", "grid"), (2, "uniform", 12_000, 32, "sample", "region")])
def test_recursive_bisection(dtlib, dim, dist, n, k, divide, border):
    """Section "Recursive Bisection": log2 k levels of 2-way division (kd:
    cyclic median split; sample: per block a new sample, its Delaunay
    graph cut in two, nearest-sample assignment) and k-1 merges (region or
    grid test) give DT(P) as well; every level halves every block."""
    p = inputs.make(dist, n, dim, seed=11)
    print(f"[pipeline] recursive {dim}d {dist} k={k} {divide} {border}", flush=True)
    res = dtlib.triangulate(p, k=k, sample_rate=0.02, divide=divide, recursive=1, sort_output=1,
                            border=border, keep_stages=1)
    assert np.array_equal(res.rows(), oracle.delaunay(p))
    st = res.stats()
    assert st["num_simplices"] == len(res.rows())
    assert st["border_vertices"] > 0
    leaf = res.stage("pid").astype(np.int64)
    assert leaf.min() >= 0 and leaf.max() < k
    if divide == "kd":
        assert np.array_equal(leaf, oracle.kd_divide(p, k))
    else:
        # the samples of all levels, and a split of every block at every level
        levels = int(np.log2(k))
        assert st["eta"] >= oracle.sample_size(n, 0.02, dim) + (levels - 1)
        for l in range(1, levels + 1):
            blocks = np.bincount(leaf >> (levels - l), minlength=1 << l)
            assert (blocks > 0).all(), (l, blocks)
        assert st["o_dt"] == pytest.approx((n + st["eta"] + st["border_vertices"]) / n)


@pytest.mark.parametrize("dim,dist,n,rate,prec", [
    (3, "bubbles", 200_000, 0.0, "fp32"),      # eta = sqrt(n) = 447
    (3, "uniform", 400_000, 0.02, "fp64"),     # eta = 8000
    (3, "bubbles", 600_000, 0.05, "fp32"),     # eta = 30000: 16-bit keys, the grid
    (2, "normal", 100_000, 0.05, "fp32"),      # eta = 5000
    (3, "lattice", 8000, 0.25, "fp64"),        # co-spherical and coplanar samples
    (2, "lattice", 4900, 0.3, "fp32"),
    (3, "jittered", 8000, 0.25, "fp32"),       # near-ties at 2^-30 grid steps
])
def test_sample_triangulation_gift_wrapped(dtlib, dim, dist, n, rate, prec):
    """The sample's Delaunay triangulation by gift wrapping (one facet
    search per simplex facet, level by level from an empty seed simplex;
    samples of more than 2048 points searched through a grid of their
    cells) equals the oracle's DT of the sample, and the whole run gives the
    same simplices as with the sample inserted in parallel rounds."""
    if dist == "lattice":
        p = inputs.lattice(round(n ** (1.0 / dim)), dim, seed=4)
    elif dist == "jittered":
        p = inputs.jittered_lattice(round(n ** (1.0 / dim)), dim, 2.0 ** -30, seed=4)
    else:
        p = inputs.make(dist, n, dim, seed=4)
    print(f"[wrap] dim={dim} dist={dist} n={len(p)} rate={rate} {prec}", flush=True)
    res = dtlib.triangulate(p, k=16, sample_rate=rate, keep_stages=1, precision=prec)
    st = res.stats()
    assert st["wrap_levels"] > 0
    sid = res.stage("sample").astype(np.int64)
    assert np.array_equal(oracle.canonical(res.stage("sample_dt")), oracle.delaunay(p[sid], sid))
    ref = dtlib.triangulate(p, k=16, sample_rate=rate, precision=prec, gift_wrap=-1)
    assert ref.stats()["wrap_levels"] == 0
    assert np.array_equal(oracle.canonical(res.rows()), oracle.canonical(ref.rows()))
