"""Host logic of bench.py (CPU): the one-GPU contract, the algorithmic byte
counts behind the roofline object, and the rule that a traffic summary is
used only for the kernel sources it was measured on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _stats(ins=0, orient=0, cand=0, cav=0, n=0, local=0, tb=0, k=1, eta=0, vb=0, m=0, b=0):
    return {"rounds": 0, "pred": {"orient3d": {"calls": orient}, "insphere3d": {"calls": ins},
                     "orient2d": {"calls": orient}, "insphere2d": {"calls": ins}},
            "candidates": cand, "cavity_cells": cav, "n": n, "k": k, "eta": eta,
            "border_vertices": vb, "local_simplices": local, "tb_simplices": tb,
            "num_simplices": m, "border_simplices": b}


def test_algorithmic_bytes_per_unit():
    # local DT: per inserted point (local sets + sample + border set), 6.77
    # simplices of 4 vertex and 4 neighbour words of 4 bytes in 3D
    st = _stats(n=1000, k=8, eta=30, vb=200)
    assert bench.inserted_points(st) == 1230
    # a gift-wrapped sample is not inserted
    assert bench.inserted_points(dict(st, wrap_levels=25)) == 1200
    assert bench.alg_bytes("k4_cavity", st, 3) == pytest.approx(1230 * 6.77 * 32)
    assert bench.alg_bytes("k4_cavity", _stats(n=1000), 2) == pytest.approx(1000 * 2 * 24)
    # assign 25 B, scatter 53 B per point in 3D (17 and 37 in 2D)
    assert bench.alg_bytes("assign", _stats(n=5), 3) == 5 * 25
    assert bench.alg_bytes("bucket", _stats(n=5), 3) == 5 * 53
    assert bench.alg_bytes("assign", _stats(n=5), 2) == 5 * 17
    assert bench.alg_bytes("bucket", _stats(n=5), 2) == 5 * 37
    # merge: read T_i rows and flags, write DT(P), hash B, probe T_B
    assert bench.alg_bytes("merge", _stats(local=10, m=8, b=3, tb=4), 3) == \
        10 * 17 + 8 * 16 + 3 * 20 + 4 * 16
    assert bench.alg_bytes("k4_pick", _stats(n=5), 3) == 0.0


def test_work_bytes_per_unit():
    # cavity search, 3D: vertices 16 + links 16 + claim 8 + four 32-byte points
    assert bench.work_bytes("k4_cavity", _stats(ins=1000), 3) == 1000 * 168
    assert bench.work_bytes("k4_cavity", _stats(ins=1000), 2) == 1000 * (16 + 16 + 8 + 3 * 32)
    assert bench.work_bytes("k4_pick", _stats(orient=400), 3) == 100 * (32 + 4 * 32)
    assert bench.work_bytes("k4_select", _stats(cand=10), 3) == 10 * 696
    assert bench.work_bytes("k4_insert", _stats(cav=7), 3) == 7 * 48
    assert bench.work_bytes("assign", _stats(n=5), 3) == 5 * 40
    assert bench.work_bytes("bucket", _stats(n=5), 3) == 5 * 72
    assert bench.work_bytes("border", _stats(local=3), 3) == 3 * 145
    assert bench.work_bytes("merge", _stats(local=3, tb=2), 3) == 5 * 161
    assert bench.work_bytes("unknown", _stats(), 3) == 0.0


def test_roofline_object_follows_the_rule():
    st = _stats(n=4000, k=8, eta=60, vb=900, ins=90000, orient=40000, cand=7000)
    per_step = {"k4_cavity": {"ms": 20.0, "launches": 100}}
    r = bench.roofline_object("k4_cavity", per_step, st, 3, "none")
    a = 4960 * 6.77 * 32 / 100
    assert r["algorithmic_bytes_per_launch"] == round(a)
    assert r["achieved"] == pytest.approx(a / 200e-6 / 1e9, rel=1e-2)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-2)
    assert r["winners"] == 4960 and r["traffic"] is None


def test_traffic_is_used_only_for_the_measured_sources(monkeypatch):
    path = os.path.join(ROOT, "profiles", "k4_cavity_bubbles-3d-4M-k256_traffic.txt")
    if not os.path.exists(path):
        pytest.skip("no traffic summary committed")
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            a, b = line.split(":", 1)
            kv[a.strip()] = b.strip()
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: kv["source_sha256"])
    t = bench.measured_traffic("k4_cavity", "bubbles-3d-4M-k256")
    want = (float(kv["fetch_kib_per_dispatch"]) * 1024 * float(kv["copy_fetch_factor"])
            + float(kv["write_kib_per_dispatch"]) * 1024 * float(kv["copy_write_factor"]))
    assert t == pytest.approx(want) and t > 0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("k4_cavity", "bubbles-3d-4M-k256") is None
    assert bench.measured_traffic("k4_cavity", "no-such-workload") is None

