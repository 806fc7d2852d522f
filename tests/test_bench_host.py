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


def _stats(ins=0, orient=0, cand=0, cav=0, n=0, local=0, tb=0):
    return {"pred": {"orient3d": {"calls": orient}, "insphere3d": {"calls": ins},
                     "orient2d": {"calls": orient}, "insphere2d": {"calls": ins}},
            "candidates": cand, "cavity_cells": cav, "n": n,
            "local_simplices": local, "tb_simplices": tb}


def test_kernel_bytes_per_unit():
    # cavity search, 3D: vertices 16 + links 16 + claim 8 + four 32-byte points
    assert bench.kernel_bytes("k4_cavity", _stats(ins=1000), 3) == 1000 * 168
    # 2D: three points
    assert bench.kernel_bytes("k4_cavity", _stats(ins=1000), 2) == 1000 * (16 + 16 + 8 + 3 * 32)
    # walk: one step per D+1 orientation tests, a cell and D+1 points each
    assert bench.kernel_bytes("k4_pick", _stats(orient=400), 3) == 100 * (32 + 4 * 32)
    # selection: three rings of bids around a candidate's cell
    assert bench.kernel_bytes("k4_select", _stats(cand=10), 3) == 10 * 696
    assert bench.kernel_bytes("k4_insert", _stats(cav=7), 3) == 7 * 48
    assert bench.kernel_bytes("assign", _stats(n=5), 3) == 5 * 40
    assert bench.kernel_bytes("bucket", _stats(n=5), 3) == 5 * 72
    assert bench.kernel_bytes("border", _stats(local=3), 3) == 3 * 145
    assert bench.kernel_bytes("merge", _stats(local=3, tb=2), 3) == 5 * 161
    assert bench.kernel_bytes("unknown", _stats(), 3) == 0.0


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

