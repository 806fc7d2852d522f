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


def _stage_checks(dtlib, p, k, rate, seed, divide, border="region"):
    n, dim = p.shape
    res = dtlib.triangulate(p, k=k, sample_rate=rate, divide=divide, seed=seed, keep_stages=1,
                            border=border)
    ids = np.arange(n)
    full = oracle.delaunay(p)
    got = oracle.canonical(res.rows())
    assert np.array_equal(got, full), "merged simplex set differs from the oracle"
    pid = res.stage("pid").astype(np.int64)
    if divide == "sample":
        eta = oracle.sample_size(n, rate, dim)
        sid = res.stage("sample")
        assert np.array_equal(sid, oracle.sample_ids(n, eta, seed))
        assert np.array_equal(oracle.canonical(res.stage("sample_dt")), oracle.delaunay(p[sid], sid))
        part = res.stage("part").astype(np.int64)
        assert oracle.balanced(part, k, 0.05)
        near = oracle.nearest_sample(p, p[sid], sid)
        assert np.array_equal(res.stage("nearest"), near)
        assert np.array_equal(pid, part[near])
    else:
        assert np.array_equal(pid, oracle.kd_divide(p, k))
    assert np.array_equal(res.stage("order"), oracle.bucket_order(pid, p))
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
    assert np.array_equal(oracle.canonical(res.stage("border_dt")), oracle.delaunay(p[vb], vb))
    st = res.stats()
    assert st["border_vertices"] == len(vb)
    assert st["num_simplices"] == len(full)
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


@pytest.mark.parametrize("dim,dist,n,k,divide", [
    (2, "uniform", 10_000, 4, "kd"), (2, "normal", 10_000, 8, "sample"),
    (3, "bubbles", 20_000, 8, "kd"), (3, "bubbles", 20_000, 16, "sample"),
    (3, "uniform", 20_000, 2, "sample")])
def test_recursive_bisection(dtlib, dim, dist, n, k, divide):
    """Section "Recursive Bisection": log2 k levels of 2-way division and
    k-1 merges give DT(P) as well."""
    p = inputs.make(dist, n, dim, seed=11)
    print(f"[pipeline] recursive {dim}d {dist} k={k} {divide}", flush=True)
    res = dtlib.triangulate(p, k=k, sample_rate=0.02, divide=divide, recursive=1, sort_output=1)
    assert np.array_equal(res.rows(), oracle.delaunay(p))
    st = res.stats()
    assert st["num_simplices"] == len(res.rows())
    assert st["border_vertices"] > 0
