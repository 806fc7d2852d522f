"""Serving: jobs submitted to the continuous-batching server give exactly
the triangulation each gives on its own (and the CPU oracle's), whatever
they were batched with; admission follows arrival order under the memory
budget; bad jobs fail alone."""
import time

import numpy as np
import pytest

import oracle
from paper_1902_07554_amd import inputs

pytestmark = pytest.mark.gpu


def _mix(seed):
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(24):
        dim = 2 if i % 3 else 3
        n = int(rng.integers(dim + 1, 3000))
        dist = ("uniform", "normal", "bubbles")[i % 3]
        jobs.append((inputs.make(dist, n, dim, seed=100 + i), 1, 0.0))
    jobs.append((inputs.make("bubbles", 30000, 3, seed=7), 8, 0.0))   # divide and conquer
    jobs.append((inputs.lattice(9, 2, seed=2), 1, 0.0))               # every tie perturbed
    return jobs


def test_server_mix_matches_standalone_and_oracle(dtlib):
    jobs = _mix(4)
    print(f"[server] jobs={len(jobs)}", flush=True)
    srv = dtlib.Server(1 << 34, sort_output=1)
    try:
        tickets = [srv.submit(p, k=k, sample_rate=r) for p, k, r in jobs]
        got = [srv.wait(t).rows() for t in tickets]
        times = [srv.times(t) for t in tickets]
    finally:
        srv.close()
    for i, ((p, k, r), rows) in enumerate(zip(jobs, got)):
        alone = dtlib.triangulate(p, k=k, sample_rate=r, sort_output=1).rows()
        assert np.array_equal(rows, alone), i
        if len(p) <= 3000 or i == len(jobs) - 1:
            assert np.array_equal(oracle.canonical(rows), oracle.delaunay(p)), i
    for t in times:
        assert t[0] <= t[1] <= t[2]


def test_server_large_jobs_match_standalone(dtlib):
    """Jobs of the served workload's largest sizes: two of 1M points
    (batched with small jobs as independent sets) and one of 2.2M points
    (above the batching limit: its own k-way divide-and-conquer), each
    identical to dt_triangulate on it alone with its k."""
    jobs = [(inputs.make("bubbles", 1_000_000, 3, seed=31), 64),
            (inputs.make("uniform", 5_000, 3, seed=32), 1),
            (inputs.make("uniform", 1_000_000, 3, seed=33), 64),
            (inputs.make("bubbles", 40_000, 3, seed=34), 2),
            (inputs.make("uniform", 2_200_000, 3, seed=35), 128)]
    print("[server] large jobs", flush=True)
    srv = dtlib.Server(64 << 30)
    try:
        tickets = [srv.submit(p, k=k) for p, k in jobs]
        got = [oracle.canonical(srv.wait(t).rows()) for t in tickets]
    finally:
        srv.close()
    for i, ((p, k), rows) in enumerate(zip(jobs, got)):
        alone = oracle.canonical(dtlib.triangulate(p, k=k, precision="fp64").rows())
        assert np.array_equal(rows, alone), i
    assert np.array_equal(got[1], oracle.delaunay(jobs[1][0]))


def test_server_fifo_admission_under_budget(dtlib):
    """A budget of about one job: admission times follow ticket order and
    every job still finishes."""
    pts = [inputs.make("uniform", 20000, 3, seed=s) for s in range(6)]
    # one 3D job of 20000 points is estimated below 160 MB
    srv = dtlib.Server(160 << 20)
    try:
        tickets = [srv.submit(p) for p in pts]
        res = [srv.wait(t) for t in tickets]
        times = [srv.times(t) for t in tickets]
    finally:
        srv.close()
    adm = [t[1] for t in times]
    assert adm == sorted(adm)
    for p, r in zip(pts[:2], res[:2]):
        assert np.array_equal(oracle.canonical(r.rows()), oracle.delaunay(p))


def test_server_errors_are_per_job(dtlib):
    good = inputs.make("uniform", 500, 2, seed=1)
    dup = good.copy()
    dup[10] = dup[20]
    line = np.stack([np.arange(50.0), 2.0 * np.arange(50.0)], 1)   # collinear
    srv = dtlib.Server(1 << 32)
    try:
        tg = srv.submit(good)
        td = srv.submit(dup)
        tl = srv.submit(line)
        tg2 = srv.submit(good[::-1].copy())
        with pytest.raises(dtlib.DTError) as e:
            srv.wait(td)
        assert e.value.status == dtlib.DT_E_DUPLICATE
        with pytest.raises(dtlib.DTError) as e:
            srv.wait(tl)
        assert e.value.status == dtlib.DT_E_DEGENERATE
        a = srv.wait(tg).rows()
        b = srv.wait(tg2).rows()
        # a result is handed out once
        with pytest.raises(dtlib.DTError):
            srv.wait(tg)
        # too few points, and a budget that cannot hold the job
        with pytest.raises(dtlib.DTError) as e:
            srv.submit(good[:2])
        assert e.value.status == dtlib.DT_E_DEGENERATE
    finally:
        srv.close()
    assert np.array_equal(oracle.canonical(a), oracle.delaunay(good))
    assert np.array_equal(oracle.canonical(b), oracle.delaunay(good[::-1].copy()))
    small = dtlib.Server(1 << 20)
    try:
        with pytest.raises(dtlib.DTError) as e:
            small.submit(good)
        assert e.value.status == dtlib.DT_E_NOMEM
    finally:
        small.close()


def test_server_poll_until_done(dtlib):
    p = inputs.make("normal", 5000, 3, seed=3)
    srv = dtlib.Server(1 << 32)
    try:
        t = srv.submit(p)
        deadline = time.time() + 60
        r = None
        while r is None and time.time() < deadline:
            r = srv.poll(t)
            time.sleep(0.001)
        assert r is not None
    finally:
        srv.close()
    assert np.array_equal(oracle.canonical(r.rows()), oracle.delaunay(p))


def test_release_cached_memory(dtlib):
    """The blocks kept between calls go back to the driver; a later call
    allocates afresh and gives the same simplices."""
    import torch
    p = inputs.make("bubbles", 300_000, 3, seed=2)
    dp = torch.from_numpy(p).cuda()
    print("[release] first run", flush=True)
    a = oracle.canonical(dtlib.triangulate(dp, k=16, precision="fp32").rows())
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    dtlib.release_cached_memory()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 > free0
    print("[release] second run", flush=True)
    b = oracle.canonical(dtlib.triangulate(dp, k=16, precision="fp32").rows())
    assert np.array_equal(a, b)
    dtlib.release_cached_memory()
