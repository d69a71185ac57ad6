"""Host logic of bench.py (CPU only): the one-GPU guard, the algorithmic byte
count of a chain launch, the lookup of measured traffic in profile summaries
(guarded by the kernel's source hash), and the stencil pair count."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_alg_bytes_formula():
    st = {"stencils": 10, "candidates": 100, "attempts": [3, 4, 5], "accepts": [1, 2, 0]}
    # 10 stencils x 27 counters x 4 B + 100 candidates x 28 B + (3 + 5) picked records x 32 B
    # + 3 accepted moves x 72 B
    assert bench.alg_bytes(st, 27) == 10 * 27 * 4 + 100 * 28 + 8 * 32 + 3 * 72


def test_resident_alg_bytes_formula():
    # 500 records read, 480 records and entries written back, 64 counters cleared and counted
    assert bench.resident_alg_bytes(500, 480, 64) == 500 * 32 + 480 * 64 + 64 * 8


def test_measured_traffic_lookup(tmp_path, monkeypatch):
    os.makedirs(tmp_path / "profiles")
    rec = {"kernel": "k_chain_spec", "launch": [8, 0], "workload": "w", "moves_per_launch": 1000,
           "fetch_kib": 100.0, "write_kib": 10.0, "fetch_scale": 2.0, "write_scale": 1.0,
           "alg_bytes": 100000.0, "source_hash": "abc"}
    (tmp_path / "profiles" / "k.md").write_text("text\n<!-- traffic %s -->\n" % json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k: "abc")
    traffic, src, ratio = bench.measured_traffic("k_chain_spec", (8, 0), "w", 2000)
    measured = (100.0 * 2.0 + 10.0 * 1.0) * 1024.0
    assert traffic == pytest.approx(measured * 2)            # per move x the moves of this launch
    assert src == os.path.join("profiles", "k.md")
    assert ratio == pytest.approx(measured / 100000.0)
    assert bench.measured_traffic("k_chain_spec", (4, 0), "w", 2000) == (None, None, None)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k: "changed")
    assert bench.measured_traffic("k_chain_spec", (8, 0), "w", 2000) == (None, None, None)


def test_stencil_candidates_brute_force():
    rng = np.random.default_rng(1)
    count = rng.integers(0, 5, (4, 5, 6))
    got = bench.stencil_candidates(count, [3, 3, 3])
    want = 0
    Z, Y, X = count.shape
    for z in range(Z):
        for y in range(Y):
            for x in range(X):
                s = 0
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            s += count[(z + dz) % Z, (y + dy) % Y, (x + dx) % X]
                want += count[z, y, x] * s
    assert got == want
