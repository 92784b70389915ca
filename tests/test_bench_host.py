"""Host-side logic of bench.py (no GPU): the kernel-source hash that decides
whether committed counter summaries still describe the built kernel, and the
reading of those summaries."""
from __future__ import annotations

import os
import shutil

import bench


def _copy_sources(tmp_path):
    for rel in bench.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, rel), dst)


def _hash_at(root, kernel="batch_step<0>"):
    old = bench.ROOT
    try:
        bench.ROOT = str(root)
        return bench.kernel_sources_sha256(kernel)
    finally:
        bench.ROOT = old


def test_hash_ignores_comments_but_not_code(tmp_path):
    _copy_sources(tmp_path)
    h0 = _hash_at(tmp_path)
    w0 = _hash_at(tmp_path, "weighted_run<0>")
    assert w0 != h0
    hip = tmp_path / "paper_2008_05718_amd/csrc/bc_batched.hip"
    text = hip.read_text()
    hip.write_text("// a new comment line\n" + text.replace("\n", "\n  ", 3) + "\n/* trailing\n block */\n")
    assert _hash_at(tmp_path) == h0
    hip.write_text(text.replace("constexpr int kUnroll = BC_UNROLL;", "constexpr int kUnroll = BC_UNROLL + 0;"))
    assert _hash_at(tmp_path) != h0
    # a kernel's hash covers its own sources only
    assert _hash_at(tmp_path, "weighted_run<0>") == w0
    dev = tmp_path / "paper_2008_05718_amd/csrc/bc_dev.h"
    dev.write_text(dev.read_text() + "\nconstexpr int kUnusedHere = 1;\n")
    assert _hash_at(tmp_path, "weighted_run<1>") != w0


def test_summaries_are_read_only_for_their_sources():
    # a summary's traffic is used while its recorded hash is the current one
    # and ignored (null in the bench line) once the kernel sources change
    import re
    tags = {"batch_step_u64": "batch_step<0>", "batch_step_f64": "batch_step<1>", "block_run_u64": "block_run<0>",
            "weighted_run_u64": "weighted_run<0>", "weighted_run_f64": "weighted_run<1>"}
    found = 0
    for name in os.listdir(os.path.join(bench.ROOT, "profiles")):
        m = re.match(r"((?:batch_step|block_run|weighted_run)_[uf]64)_(\w+)\.md$", name)
        if not m:
            continue
        found += 1
        kernel = tags[m.group(1)]
        text = open(os.path.join(bench.ROOT, "profiles", name)).read()
        rec = re.search(r"- kernel_sources_sha256: (\w+)", text).group(1)
        t = bench.measured_traffic(kernel, m.group(2))
        cur = bench.kernel_sources_sha256(kernel)
        assert (t is not None and t > 0) if rec == cur else t is None, name
    assert found >= 1
    assert bench.measured_traffic("batch_step<0>", "no_such_workload") is None


def _write_csv(path, header, rows):
    import csv
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_profile_summary_reduces_rocprof_csvs(tmp_path):
    # fixture shaped like rocprofv3 output: a kernel trace with stats, one
    # FETCH_SIZE and one WRITE_SIZE counter run, and the copy calibration
    import argparse
    import json
    K = "void bcx::batch_step<0>(bcx::BatchArgs)"
    _write_csv(tmp_path / "kt/h/1_kernel_stats.csv",
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"],
               [[K, 5, 5000, 1000, 90.0, 900, 1100, 1.0], ["fill_u64", 2, 100, 50, 10.0, 40, 60, 1.0]])
    # 5 dispatches; the last 4 are the timed step: 1000 ns each, two at a time
    starts = [0, 10000, 10000, 11000, 11000]
    _write_csv(tmp_path / "kt/h/1_kernel_trace.csv",
               ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"],
               [["KERNEL_DISPATCH", i + 1, K, t, t + 1000] for i, t in enumerate(starts)])
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    _write_csv(tmp_path / "f/h/1_counter_collection.csv", hdr,
               [[i + 1, K, "FETCH_SIZE", 999999 if i == 0 else 100.0] for i in range(5)])
    _write_csv(tmp_path / "w/h/1_counter_collection.csv", hdr,
               [[i + 1, K, "WRITE_SIZE", 50.0] for i in range(5)])
    _write_csv(tmp_path / "cf/h/1_counter_collection.csv", hdr, [[1, "copy", "FETCH_SIZE", 524288.0]])
    _write_csv(tmp_path / "cw/h/1_counter_collection.csv", hdr, [[1, "copy", "WRITE_SIZE", 1048576.0]])
    line = {"value": 1.0, "roofline": {"launches": 4, "kernel": "batch_step<0>", "algo_bytes_per_launch": 1e5,
                                       "avg_launch_us": 0.5, "achieved": 1.0, "frac": 0.1, "peak": 8000.0}}
    (tmp_path / "bench.log").write_text("noise\n" + json.dumps(line) + "\n")
    args = argparse.Namespace(kernel="batch_step<0>", workload="fixture", bench_json=str(tmp_path / "bench.log"),
                              command=["cmd a", "cmd b"], trace_dir=str(tmp_path / "kt"),
                              fetch_dir=str(tmp_path / "f"), write_dir=str(tmp_path / "w"),
                              cal_fetch_dir=str(tmp_path / "cf"), cal_write_dir=str(tmp_path / "cw"))
    text = bench.profile_summary(args)
    # factors: a 1 GiB copy reads as 524288 KiB of FETCH_SIZE (x2) and 1048576 KiB of WRITE_SIZE (x1)
    want = 100.0 * 1024 * 2.0 + 50.0 * 1024 * 1.0
    assert f"- traffic_bytes_per_launch: {want:.0f}" in text
    assert "- avg_launch_us_trace: 1.000" in text
    assert "- launches_in_flight: 2.000" in text
    assert "cmd a" in text and f"- kernel_sources_sha256: {bench.kernel_sources_sha256('batch_step<0>')}" in text
    # read back the way the bench line reads it
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "batch_step_u64_fixture.md").write_text(text)
    old = bench.ROOT
    try:
        _copy_sources(tmp_path)
        bench.ROOT = str(tmp_path)
        assert bench.measured_traffic("batch_step<0>", "fixture") == want
    finally:
        bench.ROOT = old
