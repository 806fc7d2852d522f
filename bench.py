#!/usr/bin/env python3
"""Benchmark of the sample-based divide-and-conquer Delaunay triangulation.

One step = one full triangulation (every stage of the path: sample, sample
DT, partition, nearest-sample assignment, bucket scatter, local DTs, border
test, border DT, merge) of one synthetic point set already resident in HBM.

Default workload: 3D, n = 4,194,304 "bubbles" points (64 Gaussian clusters,
sigma log-uniform in [0.01, 0.05], Dirichlet(1) weights, 5 % uniform
background, seed 1), k = 256 partitions, sample size sqrt(n) = 2048 (the
paper's default),
FP32-filtered predicates with FP64 and exact fallbacks.  The metric is
Mpoints/s with the sample divide; the kd median-split divide runs on the
same input for comparison, with balance and border sizes for both.

The same line carries the two patterns: a batching leg (4096 independent
2D sets, sizes log-uniform in [64, 65536], one batched run with autotuned
tunables against one launch per set) and a serving leg (a Poisson stream of
3D jobs, n log-uniform in [1e3, 1e6], half uniform half bubbles, for
--serve-seconds at --serve-rate jobs/s: Mpoints/s and p50/p99 latency from
arrival to result).

Prints one JSON line (rank 0).  `--gpus N` with N > 1 is not supported: the
build targets one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (distribution, n, dim, k, sample rate, precision)
    # sample size: the paper's default sqrt(n) (rate 0); the workload fixes only k
    "bubbles-3d-4M-k256": ("bubbles", 4_194_304, 3, 256, 0.0, "fp32"),
    "uniform-3d-1M-k64": ("uniform", 1_048_576, 3, 64, 0.005, "fp64"),
    "uniform-2d-10k-k4": ("uniform", 10_000, 2, 4, 0.01, "fp64"),
}

# Bytes per unit of work.  Two figures per kernel:
#   algorithmic bytes -- what the method itself must move (the per-unit
#     figures of the measurement plan), the basis of the roofline fraction;
#   work bytes -- the records the kernel gathers for the work it actually
#     does (losing searches and repeated tests included), reported beside.
PT = 32          # point record: x, y, z, id (double4)
CELL = 16        # cell vertex record (uint4); neighbours another 16


def simplices_per_point(dim: int) -> float:
    """Simplices per point of a random Delaunay triangulation: about 6.77
    in 3D (uniform points in the cube), 2 in 2D."""
    return 6.77 if dim == 3 else 2.0


def inserted_points(st: dict) -> int:
    """Points inserted by all local-DT runs of a step: the local sets, the
    sample (sample divide, unless it was gift-wrapped) and the border set."""
    if st.get("k", 1) <= 1:
        return int(st["n"])
    sample = 0 if st.get("wrap_levels", 0) else st["eta"]
    return int(st["n"] + sample + st["border_vertices"])


def alg_bytes(name: str, st: dict, dim: int) -> float:
    """Algorithmic bytes of one step for a kernel (0 when the kernel has no
    figure of its own).  The local DT's figure (its output: per point the
    simplices it adds, D+1 vertex and D+1 neighbour words of 4 bytes each)
    belongs to the four insertion kernels together and is attributed to the
    cavity search, the one that bounds them."""
    n = st["n"]
    v = dim + 1
    if name == "k4_cavity":
        return inserted_points(st) * simplices_per_point(dim) * 8 * v
    if name == "assign":        # read the coordinates, write the block (1 byte)
        return n * (8 * dim + 1)
    if name == "bucket":        # read coordinates and block, write coordinates and id
        return n * (8 * dim + 1 + 8 * dim + 4)
    if name == "border":        # per local simplex: its vertex words and its flag
        return st["local_simplices"] * (4 * v + 1)
    if name == "merge":         # read T_i simplices + flags, write DT(P), hash B, probe T_B
        return (st["local_simplices"] * (4 * v + 1) + st["num_simplices"] * 4 * v
                + st["border_simplices"] * (4 * v + 4) + st["tb_simplices"] * 4 * v)
    return 0.0


def work_bytes(name: str, st: dict, dim: int) -> float:
    """Bytes gathered for the work a kernel actually did in one step."""
    pred = st["pred"]
    o = pred["orient3d" if dim == 3 else "orient2d"]["calls"]
    ins = pred["insphere3d" if dim == 3 else "insphere2d"]["calls"]
    v = dim + 1
    n = st["n"]
    if name == "k4_cavity":     # per in-sphere test: cell vertices + neighbours + claim + D+1 points
        return ins * (2 * CELL + 8 + v * PT)
    if name == "k4_pick":       # per walk step (about D+1 orientation tests): cell + D+1 points
        return (o / v) * (2 * CELL + v * PT)
    if name == "k4_select":     # per candidate: its cell's bid and links, three rings of bids
        r1, r2, r3 = v, v * dim, v * dim * dim     # cells one, two and three facet-hops away
        return st["candidates"] * (8 + CELL + r1 * (8 + CELL) + r2 * (8 + CELL) + r3 * 8)
    if name == "k4_insert":     # per cavity cell: vertices, neighbours, two claim words
        return st["cavity_cells"] * (2 * CELL + 16)
    if name == "assign":        # per point: read the point, write block and nearest sample
        return n * (PT + 8)
    if name == "bucket":        # per point: read pid, write order, read + write the point
        return n * (4 + 4 + 2 * PT)
    if name == "border":        # per local simplex: vertices, D+1 points, flag
        return st["local_simplices"] * (CELL + v * PT + 1)
    if name == "merge":         # per simplex of T_i and T_B: vertices, keys, flag, row
        return (st["local_simplices"] + st["tb_simplices"]) * (CELL + v * PT + 1 + 4 * v)
    return 0.0


def sig(x: float, digits: int = 4) -> float:
    """x rounded to `digits` significant digits."""
    return float(f"{x:.{digits}g}")


def roofline_object(dom: str, per_step: dict, st: dict, dim: int, workload: str) -> dict:
    """Roofline of the dominant kernel: algorithmic bytes per launch over
    the average launch duration (HIP events on the launch stream), against
    the HBM peak; measured HBM traffic per launch from the committed counter
    summary; and the work behind it (tests per inserted point, rounds,
    candidates against winners)."""
    launches = per_step[dom]["launches"]
    a = alg_bytes(dom, st, dim) / launches
    w = work_bytes(dom, st, dim) / launches
    avg_s = per_step[dom]["ms"] / 1000.0 / launches
    achieved = a / avg_s / 1e9 if avg_s > 0 else 0.0
    traffic = measured_traffic(dom, workload)
    ins = inserted_points(st)
    pred = st["pred"]
    return {"bound": "hbm", "kernel": dom, "achieved": sig(achieved), "peak": 8000.0,
            "unit": "GB/s", "frac": sig(achieved / 8000.0),
            "traffic": round(traffic) if traffic is not None else None,
            "algorithmic_bytes_per_launch": round(a),
            "algorithmic_rule": ("inserted points x simplices per point x (D+1) x 8 B"
                                 if dom == "k4_cavity" else "per-unit figure x units"),
            "work_bytes_per_launch": round(w),
            "avg_launch_us": round(avg_s * 1e6, 2), "launches_per_step": launches,
            "ms_per_step": round(per_step[dom]["ms"], 3),
            "inserted_points": ins,
            "insphere_tests_per_inserted_point":
                round(pred["insphere3d" if dim == 3 else "insphere2d"]["calls"] / ins, 2),
            "orient_tests_per_inserted_point":
                round(pred["orient3d" if dim == 3 else "orient2d"]["calls"] / ins, 2),
            "rounds": st["rounds"], "candidates": st["candidates"], "winners": ins,
            "kernel_source": kernel_source_hash()}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(points, sample_n: int) -> dict:
    """The CPU oracle (single-threaded Bowyer-Watson, exact predicates) on
    the first `sample_n` points of the same input."""
    import oracle
    sub = points[:sample_n]
    t0 = time.perf_counter()
    simp = oracle.delaunay(sub)
    dt = time.perf_counter() - t0
    return {"value": round(sample_n / dt / 1e6, 4), "unit": "Mpoints/s", "cores": 1,
            "kind": "oracle", "seconds": round(dt, 2), "simplices": int(len(simp)),
            "cpu": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"first {sample_n} points of the same input (same generator and seed)"}


def run(binding, pts, steps: int, warmup: int, k: int, rate: float, **opts):
    """Warm-up steps, then `steps` timed steps; then one more step with
    kernel timing on (HIP events around every timed launch, on the launch
    stream), outside the timed region, for the per-kernel table."""
    import torch
    res = None
    for _ in range(warmup):
        res = binding.triangulate(pts, k=k, sample_rate=rate, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = binding.triangulate(pts, k=k, sample_rate=rate, **opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = binding.triangulate(pts, k=k, sample_rate=rate, profile=1, **opts)
    pst = prof.stats()
    kern = {name: dict(v) for name, v in pst["kern"].items()}
    return res, (t1 - t0) * 1000.0 / steps, kern, pst


def kernel_source_hash() -> str:
    """Hash of the sources the insertion kernels are built from (a traffic
    measurement is valid only for the kernels it was taken on)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("dt_k4.hip", "dt_pred.hpp", "dt_common.hpp", "dt_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1902_07554_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by the same
    counters on a copy kernel of known size), or None when there is no
    summary or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                a, b = line.split(":", 1)
                kv[a.strip()] = b.strip()
    try:
        if kv.get("source_sha256") != kernel_source_hash():
            return None
        fetch = float(kv["fetch_kib_per_dispatch"]) * 1024 * float(kv["copy_fetch_factor"])
        write = float(kv["write_kib_per_dispatch"]) * 1024 * float(kv["copy_write_factor"])
        return fetch + write
    except (KeyError, ValueError):
        return None


def bench_copy(args) -> dict:
    """Calibration for the HBM counters: a plain device copy of 1 GiB."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / 3
    return {"metric": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
            "GB/s": round(2 * nbytes / dt / 1e9, 1)}


def bench_batch(args) -> dict:
    """Batching pattern: 4096 independent 2D sets, sizes log-uniform in
    [64, 65536], each uniform or N(0, I) (seed 1); one batched run with
    autotuned launch tunables vs one launch per set."""
    import torch
    from paper_1902_07554_amd import binding, inputs
    host, offsets = inputs.batch_sets(4096, 64, 65536, dim=2, seed=1)
    n = int(offsets[-1])
    pts = torch.from_numpy(host).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tuned = binding.batch_autotune(pts, offsets)
    tune_s = time.perf_counter() - t0

    def timed(**o):
        res = None
        for _ in range(args.warmup):
            res = binding.batch_triangulate(pts, offsets, **o)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.steps):
            res = binding.batch_triangulate(pts, offsets, **o)
        torch.cuda.synchronize()
        return res, (time.perf_counter() - a) * 1000.0 / args.steps

    res, ms = timed(**tuned)
    _, ms_def = timed()
    # one launch per set on every 8th set (512 sets, same size mix)
    sub = list(range(0, 4096, 8))
    so = res.set_offsets(4096)
    sub_n = int(sum(offsets[s + 1] - offsets[s] for s in sub))
    for s in sub[:8]:
        binding.triangulate(pts[offsets[s]:offsets[s + 1]], k=1)
    torch.cuda.synchronize()
    a = time.perf_counter()
    counts_equal = True
    for s in sub:
        r = binding.triangulate(pts[offsets[s]:offsets[s + 1]], k=1)
        counts_equal &= (r.count == so[s + 1] - so[s])
    torch.cuda.synchronize()
    per_set_s = time.perf_counter() - a
    per_set = sub_n / per_set_s / 1e6
    value = n / (ms / 1000.0) / 1e6
    return {
        "metric": "Mpoints/s batched 2D DT, one batched run vs one launch per set",
        "value": round(value, 4), "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch-2d-4096-sets", "sets": 4096, "n": n,
                   "sizes": "log-uniform [64, 65536]", "dim": 2, "precision": "fp64"},
        "simplices": res.count, "autotuned": tuned, "autotune_s": round(tune_s, 3),
        "default_tunables_ms": round(ms_def, 3),
        "per_set_launches": {"sets": len(sub), "points": sub_n, "seconds": round(per_set_s, 3),
                             "Mpoints_per_s": round(per_set, 4),
                             "simplex_counts_equal": bool(counts_equal)},
        "batched_vs_per_set": round(value / per_set, 3),
    }


def bench_serve(args) -> dict:
    """Serving pattern: Poisson stream of 3D jobs (mean rate --serve-rate per
    second over --serve-seconds), n log-uniform in [1e3, 1e6], half uniform
    half bubbles; k = max(1, n / 16384) rounded to a power of two; HBM
    budget --serve-budget-gib (192 GiB of the 288 by default).  Latency =
    arrival to result ready."""
    import math
    import threading
    import numpy as np
    import torch
    from paper_1902_07554_amd import binding, inputs
    jobs = inputs.serve_stream(args.serve_rate, args.serve_seconds, 1000, 1_000_000, 3, seed=1)
    data = [inputs.make(kind, n, 3, seed=js) for _, n, kind, js in jobs]
    ks = [1 << max(0, round(math.log2(max(1.0, n / 16384)))) for _, n, _, _ in jobs]
    torch.cuda.synchronize()
    srv = binding.Server(int(args.serve_budget_gib) << 30)
    tickets = [None] * len(jobs)
    t0 = time.perf_counter()

    def submitter():
        for i, (at, n, kind, js) in enumerate(jobs):
            d = at - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            tickets[i] = srv.submit(data[i], k=ks[i])

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    # jobs whose result is also computed alone afterwards (identity check)
    rng = np.random.default_rng(7)
    small = [i for i, (_, n, _, _) in enumerate(jobs) if n <= 200_000]
    check = set(rng.choice(small, size=min(8, len(small)), replace=False).tolist()) if small else set()
    kept = {}
    lat, total = [], 0
    for i, t in enumerate(tickets):
        r = srv.wait(t)
        total += jobs[i][1]
        tt = srv.times(t)
        lat.append(tt[2] - tt[0])
        if i in check:
            kept[i] = r.rows()
        del r
    wall = time.perf_counter() - t0
    srv.close()

    def canon(rows):
        rows = np.sort(rows.astype(np.int64), axis=1)
        return rows[np.lexsort(rows.T[::-1])]

    identical = all(np.array_equal(canon(kept[i]),
                                   canon(binding.triangulate(data[i], k=ks[i]).rows()))
                    for i in sorted(kept))
    lat = np.array(lat) * 1000.0
    return {
        "metric": "Mpoints/s and p50/p99 latency of a served Poisson stream of 3D DT jobs",
        "value": round(total / wall / 1e6, 4), "unit": "Mpoints/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": round(wall * 1000.0, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "serve-3d-poisson", "rate_per_s": args.serve_rate,
                   "seconds": args.serve_seconds, "jobs": len(jobs), "points": total,
                   "n": "log-uniform [1e3, 1e6]", "kinds": "uniform / bubbles",
                   "hbm_budget_GiB": args.serve_budget_gib, "offered_Mpoints_per_s":
                       round(total / args.serve_seconds / 1e6, 3)},
        "p50_ms": round(float(np.percentile(lat, 50)), 2),
        "p99_ms": round(float(np.percentile(lat, 99)), 2),
        "max_ms": round(float(lat.max()), 2),
        "alone_vs_mix": {"jobs_checked": len(kept), "identical": bool(identical)},
    }


def bench_sweep(args) -> dict:
    """Primitive, sample-size and weight sweeps (border size vs runtime) on
    3D bubbles, n = 1,048,576, k = 64, FP32 filter, and the same for the kd
    divide's primitives."""
    import torch
    from paper_1902_07554_amd import binding, inputs
    n, k = 1_048_576, 64
    pts = torch.from_numpy(inputs.make("bubbles", n, 3, seed=1)).to("cuda")
    binding.triangulate(pts, k=k, precision="fp32")
    rows = []

    def one(kk=k, **o):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = binding.triangulate(pts, k=kk, precision="fp32", **o)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) * 1000.0
        st = r.stats()
        row = dict(o, k=kk)
        row.update(ms=round(dt, 2), eta=st["eta"], border_vertices=st["border_vertices"],
                   border_simplices=st["border_simplices"], tb_simplices=st["tb_simplices"],
                   o_dt=round(st["o_dt"], 4), cv=round(st["cv"], 4),
                   border_ms=round(st["stage_ms"]["border"], 2),
                   border_dt_ms=round(st["stage_ms"]["border_dt"], 2),
                   divide_used=st["divide_used"])
        rows.append(row)

    for rate in (0.0, 0.005, 0.01, 0.02):
        for border, cell in (("region", 1.0), ("grid", 0.5), ("grid", 1.0), ("grid", 2.0),
                             ("bbox", 1.0), ("exact", 1.0)):
            one(divide="sample", sample_rate=rate, border=border, grid_cell=cell)
    for w in ("const", "inverse", "linear"):
        one(divide="sample", sample_rate=0.005, weight=w)
    for border, cell in (("region", 1.0), ("grid", 1.0), ("bbox", 1.0), ("exact", 1.0)):
        one(divide="kd", border=border, grid_cell=cell)
    # recursive bisection (log2 k levels, k-1 merges with the grid test)
    one(divide="kd", recursive=1)
    one(divide="sample", sample_rate=0.0, recursive=1)
    one(divide="auto", sample_rate=0.0)
    # the logarithmic sample size (eta = log2 n = 20) needs k <= eta: at k = 16, beside the
    # square-root sample and the kd divide at the same k
    for rate in (math.log2(n) / n, 0.0):
        one(kk=16, divide="sample", sample_rate=rate)
    one(kk=16, divide="kd")
    return {"metric": "border size and runtime by primitive, sample size and weight",
            "config": {"workload": "bubbles-3d-1M-k64", "n": n, "k": k, "precision": "fp32"},
            "runs": rows}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="bubbles-3d-4M-k256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-kd", action="store_true", help="skip the kd-divide comparison")
    ap.add_argument("--no-direct", action="store_true",
                    help="skip the comparison with the whole input as one set (k = 1)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batching leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--cpu-sample", type=int, default=1_500_000,
                    help="points of the CPU-oracle baseline sample (0 = skip)")
    ap.add_argument("--mode", default="dt", choices=["dt", "batch", "serve", "copy", "sweep"],
                    help="dt: the headline triangulation; batch / serve: the patterns")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-budget-gib", type=int, default=192,
                    help="HBM budget of the server (GiB)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; the benchmark runs on one GPU "
              "(sharding over several GPUs is a design, not built)", file=sys.stderr)
        return 2
    if args.mode == "batch":
        print(json.dumps(bench_batch(args)), flush=True)
        return 0
    if args.mode == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return 0
    if args.mode == "copy":
        print(json.dumps(bench_copy(args)), flush=True)
        return 0
    if args.mode == "sweep":
        print(json.dumps(bench_sweep(args)), flush=True)
        return 0

    import torch
    from paper_1902_07554_amd import binding, inputs

    dist, n, dim, k, rate, prec = WORKLOADS[args.workload]
    host = inputs.make(dist, n, dim, seed=1)
    pts = torch.from_numpy(host).to("cuda")
    torch.cuda.synchronize()

    res, ms, kern, pst = run(binding, pts, args.steps, args.warmup, k, rate, precision=prec,
                             divide="sample")
    st = res.stats()
    value = n / (ms / 1000.0) / 1e6

    # dominant kernel of the timed region: achieved algorithmic bytes / time
    per_step = {name: {"ms": v["ms"], "launches": v["launches"]}
                for name, v in kern.items() if v["launches"]}
    dom = max(per_step, key=lambda x: per_step[x]["ms"])
    roofline = roofline_object(dom, per_step, pst, dim, args.workload)
    kernels = {}
    for name, v in per_step.items():
        sec = v["ms"] / 1000.0
        a, w = alg_bytes(name, pst, dim), work_bytes(name, pst, dim)
        kernels[name] = {"ms": round(v["ms"], 3), "launches": v["launches"],
                         "alg_GB/s": round(a / sec / 1e9, 2) if sec > 0 and a else None,
                         "work_GB/s": round(w / sec / 1e9, 2) if sec > 0 else None}
    k4_ms = sum(per_step[x]["ms"] for x in ("k4_pick", "k4_select", "k4_cavity", "k4_insert")
                if x in per_step)
    kernels["k4_all_four"] = {"ms": round(k4_ms, 3),
                              "alg_GB/s": round(alg_bytes("k4_cavity", pst, dim) / (k4_ms / 1000.0)
                                                / 1e9, 2) if k4_ms > 0 else None}

    def summary(s):
        return {"border_vertices": s["border_vertices"], "border_simplices": s["border_simplices"],
                "tb_simplices": s["tb_simplices"], "o_dt": round(s["o_dt"], 4),
                "cv": round(s["cv"], 4), "max_dev": round(s["max_dev"], 4),
                "cut_weight": round(s["cut_weight"], 2), "rounds": s["rounds"],
                "stage_ms": {a: round(b, 2) for a, b in s["stage_ms"].items() if b}}

    line = {
        "metric": "Mpoints/s DT (3D, 4M pts) sample- vs kd-divide; border size; p50/p99 latency",
        "value": round(value, 4),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "distribution": dist, "n": n, "dim": dim, "k": k,
                   "sample_rate": rate, "eta": st["eta"], "divide": "sample",
                   "precision": prec, "border": "region"},
        "simplices": res.count,
        "sample_divide": summary(st),
        "predicates": st["pred"],
        "roofline": roofline,
        "kernels": kernels,
    }
    if not args.no_kd:
        kres, kms, _, _ = run(binding, pts, args.steps, args.warmup, k, rate, precision=prec,
                           divide="kd")
        kst = kres.stats()
        line["kd_divide"] = dict(value=round(n / (kms / 1000.0) / 1e6, 4), ms_per_step=round(kms, 3),
                                 **summary(kst))
        line["sample_vs_kd_speedup"] = round(kms / ms, 4)
        line["kd_simplex_count_equal"] = bool(kres.count == res.count)
        del kres
    if not args.no_kd and k != 16:
        # context: both divides at the paper's own k = 16 (its runtime
        # experiments use k = t = 16)
        r16, ms16, _, _ = run(binding, pts, args.steps, args.warmup, 16, rate, precision=prec,
                              divide="sample")
        k16, kms16, _, _ = run(binding, pts, args.steps, args.warmup, 16, rate, precision=prec,
                               divide="kd")
        line["k16"] = {"sample_ms_per_step": round(ms16, 3), "kd_ms_per_step": round(kms16, 3),
                       "sample_vs_kd_speedup": round(kms16 / ms16, 4),
                       "border_vertices": {"sample": r16.stats()["border_vertices"],
                                           "kd": k16.stats()["border_vertices"]},
                       "simplex_counts_equal": bool(r16.count == k16.count == res.count)}
        del r16, k16
    if not args.no_direct:
        # context, not the method: the same input triangulated as one set
        dres, dms, _, _ = run(binding, pts, args.steps, args.warmup, 1, 0.0, precision=prec)
        line["direct_k1"] = {"value": round(n / (dms / 1000.0) / 1e6, 4),
                             "ms_per_step": round(dms, 3), "rounds": dres.stats()["rounds"],
                             "simplex_count_equal": bool(dres.count == res.count)}
        del dres
    if args.cpu_sample > 0:
        line["cpu_baseline"] = cpu_baseline(host, min(args.cpu_sample, n))
    del pts, res

    def fresh():
        # each pattern leg starts without the blocks the previous legs left
        # in the library's cache
        binding.release_cached_memory()
        torch.cuda.empty_cache()

    if not args.no_batch:
        fresh()
        b = bench_batch(args)
        line["batch"] = {k2: b[k2] for k2 in ("value", "unit", "ms_per_step", "config",
                                               "autotuned", "default_tunables_ms",
                                               "per_set_launches", "batched_vs_per_set")}
    if not args.no_serve:
        fresh()
        v = bench_serve(args)
        line["serve"] = {k2: v[k2] for k2 in ("value", "unit", "p50_ms", "p99_ms", "max_ms",
                                               "ms_per_step", "config", "alone_vs_mix")}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
