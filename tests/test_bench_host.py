"""Host logic of bench.py (no GPU): the one-GPU contract, the kernel source
hash behind the traffic table, and the ingestion of rocprofv3 counter runs."""
from __future__ import annotations

import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr and r.stdout == ""


def test_source_hash_ignores_comments_only():
    code = "int f(int a) { return a + 1; } // one\n/* two\n three */ int g;\n"
    assert bench.code_only(code) == bench.code_only("int f(int a) {\n  return a + 1;\n}\n// other\nint g;")
    assert bench.code_only(code) != bench.code_only(code.replace("a + 1", "a + 2"))
    assert len(bench.source_sha()) == 16


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_counter_ingestion_scales_by_the_calibration(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    kname = "void fof::(anonymous namespace)::k_gather(fof::Plan)"
    fill = "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float> >(int)"
    copy = "__amd_rocclr_copyBuffer"
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    # the copy of a 1024 KiB buffer reads FETCH_SIZE 512 (factor 2), the fill writes 1024 (factor 1)
    _write(str(tmp_path / "fetch" / "run_counter_collection.csv"), hdr,
           [[copy, "FETCH_SIZE", 512], [kname, "FETCH_SIZE", 100], [kname, "FETCH_SIZE", 300]])
    _write(str(tmp_path / "write" / "run_counter_collection.csv"), hdr,
           [[fill, "WRITE_SIZE", 1024], [kname, "WRITE_SIZE", 50]])
    _write(str(tmp_path / "trace" / "run_kernel_stats.csv"), ["Name", "Calls", "AverageNs"],
           [[kname, 4, 1000.0], [copy, 1, 10.0]])
    table = bench.ingest_counters(str(tmp_path), "batched256")
    d = json.load(open(out))["batched256"]
    assert d["fetch_factor"] == 2.0 and d["write_factor"] == 1.0 and d["source_sha"] == bench.source_sha()
    g = d["kernels"]["k_gather"]
    assert g["calls"] == 4 and g["bytes_per_launch"] == (200 * 2.0 + 50 * 1.0) * 1024.0
    assert "`k_gather`" in table
    assert bench.measured_traffic("k_gather", "batched256") == g["bytes_per_launch"]
    assert bench.measured_traffic("k_gather", "clustered256") is None      # another workload's counters
    bench.ingest_counters(str(tmp_path), "clustered256")                   # entries of workloads side by side
    both = json.load(open(out))
    assert set(both) == {"batched256", "clustered256"}
    # counters taken on other kernel sources are not reported
    both["batched256"]["source_sha"] = "0" * 16
    json.dump(both, open(out, "w"))
    assert bench.measured_traffic("k_gather", "batched256") is None
    assert bench.measured_traffic("k_gather", "clustered256") == g["bytes_per_launch"]


def test_ingestion_needs_the_calibration_runs(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    _write(str(tmp_path / "fetch" / "run_counter_collection.csv"), hdr, [["x", "FETCH_SIZE", 1]])
    _write(str(tmp_path / "write" / "run_counter_collection.csv"), hdr, [["x", "WRITE_SIZE", 1]])
    _write(str(tmp_path / "trace" / "run_kernel_stats.csv"), ["Name", "Calls", "AverageNs"], [["x", 1, 1.0]])
    with pytest.raises(SystemExit):
        bench.ingest_counters(str(tmp_path), "batched256")
    assert not (tmp_path / "traffic.json").exists()


def test_roofline_and_kernel_table_from_times_and_statistics():
    class W:
        n = 1000
        name = "toy"
    st = {"n_cells": 5000, "queued_links": 300, "pair_tests": 10 ** 6, "sparse_pair_tests": 2 * 10 ** 5}
    kern = {"k_link_dense": (0.5, 3), "k_gather": (0.01, 3), "k_link_sparse": (0.2, 3)}
    r = bench.roofline_of(kern, W, st, 100, "toy")
    assert r["kernel"] == "k_link_dense" and r["bound"] == "alu"
    assert r["pair_tests_per_launch"] == 8 * 10 ** 5
    assert abs(r["achieved"] - 8 * 10 ** 5 * 8 / 0.5e-3 / 1e12) < 1e-12
    assert abs(r["frac"] - r["achieved"] / 157.3) < 1e-15 and r["traffic"] is None
    t = bench.kernel_table(kern, W, st, 100)
    assert t["k_gather"]["GB/s"] == round(1000 * 20 / 0.01e-3 / 1e9, 1) and "GB/s" not in t["k_link_dense"]
    kern = {"k_gather": (0.5, 1), "k_link_dense": (0.1, 1)}
    r = bench.roofline_of(kern, W, st, 100, "toy")
    assert r["bound"] == "hbm" and r["bytes_per_launch"] == 1000 * 20


def test_exactness_compares_every_output():
    import numpy as np
    a = (np.arange(5), np.ones(5), np.array([3]))
    assert bench.same(a, (np.arange(5), np.ones(5), np.array([3])))
    assert not bench.same(a, (np.arange(5), np.ones(5), np.array([4])))        # group counts differ
    assert not bench.same(a, (np.arange(5), np.zeros(5), np.array([3])))       # sizes differ


def test_sq_summary_per_wave(tmp_path):
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    k = "void fof::(anonymous namespace)::k_link_dense<false, false, false>(fof::Plan)"
    _write(str(tmp_path / "a" / "run_counter_collection.csv"), hdr,
           [[k, "SQ_WAVES", 100], [k, "SQ_INSTS_VALU", 5000], [k, "SQ_WAVE_CYCLES", 1000], [k, "SQ_WAVES", 100],
            [k, "SQ_INSTS_VALU", 7000], [k, "SQ_WAVE_CYCLES", 1000]])
    _write(str(tmp_path / "b" / "run_counter_collection.csv"), hdr, [[k, "SQ_WAIT_ANY", 700]])
    t = bench.summarize_sq([str(tmp_path / "a"), str(tmp_path / "b")])
    row = [l for l in t.splitlines() if "k_link_dense" in l][0]
    cells = [c.strip() for c in row.split("|")]
    assert cells[2] == "100" and cells[3] == "60" and cells[-2] == "0.70"
