"""Benchmark: exact Brandes BC throughput (GTEPS = m x sources / s) on one MI355X.

One step = one complete BC run (forward + backward for every source, all
levels, scores summed) over the workload's source list, through libbc's C ABI.
The default workload is R-MAT scale 22 (4,194,304 vertices, edge factor 16,
16,384 sources).  Inputs are resident in HBM before the timed region
(bc_graph_create is timed separately).  The batched engine (64 sources per
traversal) with the learned level policy is the headline value; beside it,
on the same workload: the same engine with the direction-optimising
heuristic (its scores must be bitwise equal), the plain per-source engine on
a prefix of the source list, and the CPU oracle (one core, and one thread
per host core) on a bounded sample.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload rmat22] [--gpus 1]
    python bench.py --summarize-profile ...   (reduce rocprofv3 output to a profile summary)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BC GTEPS (m x sources / s) on 1 MI355X, batched+learned vs plain; % HBM peak"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TUNE_SOURCES = 2048  # autotuner sample: the first sources of the list (untimed)
# autotuner results for the benchmark workloads on this GPU model, written by
# `bench.py --tune-cache-out` on an MI355X; a hit skips the timing runs
TUNE_CACHE = os.path.join(ROOT, "paper_2008_05718_amd", "tune_cache.json")
_COMMON_SOURCES = ["paper_2008_05718_amd/csrc/bc_common.h", "paper_2008_05718_amd/csrc/bc_dev.h",
                   "paper_2008_05718_amd/build.py"]
# the sources each step kernel is compiled from (its counters per launch
# depend on these and on the workload, not on the host driver)
KERNEL_FILES = {
    "batch_step": ["paper_2008_05718_amd/csrc/bc_batched.hip"] + _COMMON_SOURCES,
    "block_run": ["paper_2008_05718_amd/csrc/bc_batched.hip"] + _COMMON_SOURCES,
    "weighted_run": ["paper_2008_05718_amd/csrc/bc_weighted.hip"] + _COMMON_SOURCES,
    "wbatch_run": ["paper_2008_05718_amd/csrc/bc_wbatch.hip", "paper_2008_05718_amd/csrc/bc_wbatch.h"]
    + _COMMON_SOURCES,
}
KERNEL_SOURCES = sorted({f for v in KERNEL_FILES.values() for f in v})


def _code_only(text: str) -> str:
    """C/C++ source without comments and with whitespace collapsed."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_sources_sha256(kernel: str = "batch_step<0>") -> str:
    """Hash of the sources a step kernel is built from (``kernel`` as in the
    bench line, e.g. "batch_step<0>"); comments and whitespace of the HIP
    sources are ignored, so an edit of comments only keeps the recorded
    counters valid."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_FILES[kernel.split("<")[0]]:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            text = f.read()
        if rel.endswith((".hip", ".h")):
            text = _code_only(text)
        h.update(text.encode())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE and WRITE_SIZE, each scaled by its
    copy-kernel calibration), or None when there is none or the kernel
    sources changed since the counters were taken."""
    tag = {"batch_step<0>": "batch_step_u64", "batch_step<1>": "batch_step_f64", "block_run<0>": "block_run_u64",
           "weighted_run<0>": "weighted_run_u64", "weighted_run<1>": "weighted_run_f64",
           "wbatch_run<0>": "wbatch_run_u64", "wbatch_run<1>": "wbatch_run_f64"}.get(kernel)
    path = os.path.join(ROOT, "profiles", f"{tag}_{workload}.md")
    if tag is None or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                key, _, val = line[2:].partition(":")
                vals[key.strip()] = val.strip().strip("`")
    try:
        if vals.get("kernel_sources_sha256") != kernel_sources_sha256(kernel):
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ------------------------------------------------------- profile summaries
def _csv_rows(directory, suffix):
    """Rows of every rocprofv3 CSV file under ``directory`` whose name ends in
    ``suffix`` (e.g. "kernel_stats.csv"), as dicts with lower-case keys."""
    import csv
    rows = []
    for dirpath, _, files in os.walk(directory):
        for fn in sorted(files):
            if fn.endswith(suffix):
                with open(os.path.join(dirpath, fn), newline="") as f:
                    for r in csv.DictReader(f):
                        rows.append({(k or "").strip().lower(): (v or "").strip() for k, v in r.items()})
    return rows


def _kernel_match(name: str, kernel: str) -> bool:
    """'batch_step<0>' matches 'void bcx::batch_step<0>(bcx::BatchArgs)'."""
    return kernel in name.replace(" ", "")


def _counter_per_dispatch(directory, counter, kernel):
    """{dispatch id: value} of one counter for the dispatches of a kernel."""
    out = {}
    for r in _csv_rows(directory, "counter_collection.csv"):
        if r.get("counter_name") != counter or not _kernel_match(r.get("kernel_name", ""), kernel):
            continue
        d = int(r.get("dispatch_id") or r.get("correlation_id") or len(out))
        out[d] = out.get(d, 0.0) + float(r["counter_value"])
    return out


def _copy_factor(directory, counter, copy_bytes):
    """Bytes one KiB of ``counter`` stands for, from a plain device copy of
    ``copy_bytes`` bytes (the largest dispatch in the calibration run)."""
    best = 0.0
    for r in _csv_rows(directory, "counter_collection.csv"):
        if r.get("counter_name") == counter:
            best = max(best, float(r["counter_value"]))
    return (copy_bytes / (best * 1024.0)) if best > 0 else None, best


def profile_summary(args) -> str:
    """Reduce a rocprofv3 kernel trace (--trace-dir, run with --kernel-trace
    --stats) and two counter runs (--fetch-dir with FETCH_SIZE, --write-dir
    with WRITE_SIZE, in KiB per dispatch) of the same bench command, plus the
    same counters for a 1 GiB device copy (--cal-fetch-dir, --cal-write-dir),
    to the summary bench.py reads back (measured_traffic).  Only the last
    ``launches`` dispatches of the kernel (the timed step, from the bench
    line given with --bench-json) enter the averages."""
    kernel = args.kernel
    bench = {}
    if args.bench_json:
        with open(args.bench_json) as f:
            for line in f:
                line = line.strip()
                if line.startswith("{") and '"roofline"' in line:
                    bench = json.loads(line)
    roof = bench.get("roofline") or {}
    n_timed = int(roof.get("launches") or 0)
    lines = [f"# {kernel} on {args.workload}", ""]
    if args.command:
        lines += ["## Commands (from the repository root, after `cd /tmp && export TMPDIR=/tmp` and back)", "", "```"]
        lines += list(args.command)
        lines += ["```", ""]
    stats = [r for r in _csv_rows(args.trace_dir, "kernel_stats.csv")] if args.trace_dir else []
    if stats:
        lines += ["## Kernel trace (top kernels)", "", "| kernel | calls | total ns | average ns | % |",
                  "|---|---:|---:|---:|---:|"]
        for r in sorted(stats, key=lambda r: -float(r.get("totaldurationns", 0) or 0))[:6]:
            lines.append(f"| `{r.get('name', '')[:70]}` | {r.get('calls')} | {r.get('totaldurationns')} | "
                         f"{float(r.get('averagens', 0) or 0):.0f} | {float(r.get('percentage', 0) or 0):.2f} |")
        lines.append("")
    trace = [r for r in _csv_rows(args.trace_dir, "kernel_trace.csv")
             if _kernel_match(r.get("kernel_name", ""), kernel)] if args.trace_dir else []
    avg_us = inflight = None
    if trace:
        trace.sort(key=lambda r: int(r["start_timestamp"]))
        tail = trace[-n_timed:] if n_timed else trace
        dur = [int(r["end_timestamp"]) - int(r["start_timestamp"]) for r in tail]
        span = max(int(r["end_timestamp"]) for r in tail) - min(int(r["start_timestamp"]) for r in tail)
        avg_us = sum(dur) / len(dur) / 1e3
        inflight = sum(dur) / max(span, 1)
        lines += [f"Timed step only (the last {len(tail)} dispatches of {kernel}): average duration "
                  f"{avg_us:.1f} us, {len(tail)} dispatches within {span / 1e6:.1f} ms, i.e. on average "
                  f"{inflight:.2f} dispatches in flight; duration / in flight = {avg_us / inflight:.1f} us of "
                  f"device time per dispatch.", ""]
    traffic = None
    if args.fetch_dir and args.write_dir and args.cal_fetch_dir and args.cal_write_dir:
        fetch = _counter_per_dispatch(args.fetch_dir, "FETCH_SIZE", kernel)
        write = _counter_per_dispatch(args.write_dir, "WRITE_SIZE", kernel)
        ff, fraw = _copy_factor(args.cal_fetch_dir, "FETCH_SIZE", 1 << 30)
        wf, wraw = _copy_factor(args.cal_write_dir, "WRITE_SIZE", 1 << 30)
        fk = [fetch[d] for d in sorted(fetch)][-n_timed:] if n_timed else list(fetch.values())
        wk = [write[d] for d in sorted(write)][-n_timed:] if n_timed else list(write.values())
        if fk and wk and ff and wf:
            f_kib = sum(fk) / len(fk)
            w_kib = sum(wk) / len(wk)
            traffic = f_kib * 1024 * ff + w_kib * 1024 * wf
            algo = float(roof.get("algo_bytes_per_launch") or 0)
            lines += ["## Counters per dispatch (the timed step's dispatches; the counter pass serialises them)", "",
                      "| counter | dispatches | KiB per dispatch | 1 GiB copy reads as | factor | bytes per dispatch |",
                      "|---|---:|---:|---:|---:|---:|",
                      f"| FETCH_SIZE | {len(fk)} | {f_kib:.0f} | {fraw:.0f} KiB | {ff:.3f} | {f_kib * 1024 * ff:.4g} |",
                      f"| WRITE_SIZE | {len(wk)} | {w_kib:.0f} | {wraw:.0f} KiB | {wf:.3f} | {w_kib * 1024 * wf:.4g} |",
                      "",
                      f"Counted traffic per dispatch: {traffic / 1e6:.1f} MB; algorithmic bytes per dispatch "
                      f"(bench line of the same command): {algo / 1e6:.1f} MB; ratio "
                      f"{traffic / algo if algo else float('nan'):.2f}.  These counters see the requests "
                      f"between the L2 caches and the memory fabric, so reads served by the Infinity Cache "
                      f"are included: an upper bound on HBM bytes, not a measurement of them.", ""]
    if roof:
        lines += [f"Bench line of the profiled command: {bench.get('value')} GTEPS, {roof.get('launches')} "
                  f"dispatches of {roof.get('kernel')}, {roof.get('avg_launch_us')} us of device time per "
                  f"dispatch (HIP events), algorithmic {roof.get('achieved')} GB/s = {roof.get('frac')} of "
                  f"{roof.get('peak')}.", ""]
    lines += ["## Values read by bench.py", "", f"- kernel: {kernel}", f"- workload: {args.workload}"]
    if avg_us is not None:
        lines += [f"- avg_launch_us_trace: {avg_us:.3f}", f"- launches_in_flight: {inflight:.3f}"]
    if traffic is not None:
        lines.append(f"- traffic_bytes_per_launch: {traffic:.0f}")
    lines.append(f"- kernel_sources_sha256: {kernel_sources_sha256(kernel)}")
    return "\n".join(lines) + "\n"


def traversed_edges(g, srcs) -> float:
    """Work of a run in edges x sources: the edge count of each source's own
    graph (a block-diagonal union counts only the block the source is in)."""
    off = getattr(g, "vtx_offsets", None)
    if off is None or len(off) <= 2:
        return float(g.m) * len(srcs)
    off = np.asarray(off, dtype=np.int64)
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    m_g = (rp[off[1:]] - rp[off[:-1]]) // 2
    gi = np.searchsorted(off, np.asarray(srcs, dtype=np.int64), side="right") - 1
    return float(m_g[gi].sum())


def _cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, os.cpu_count() or 1, avail


def cpu_baseline(g, srcs, workload, seconds):
    """The oracle as it stands on the host: first one source at a time on one
    core for about half the budget, then one contiguous slice of sources per
    host thread (at most 16: the host share of one GPU) for about the other
    half.  Sources are taken from the front of the workload's list."""
    import oracle
    oracle.build(force=False)
    model, ncpu, avail = _cpu_info()
    threads = max(1, min(16, avail))
    k = 0
    t = time.perf_counter()
    while (time.perf_counter() - t < seconds / 2 or k == 0) and k < len(srcs):
        oracle.bc(g, srcs[k:k + 1])
        k += 1
    el1 = time.perf_counter() - t
    one = traversed_edges(g, srcs[:k]) / el1 / 1e9
    # all threads: rounds of `threads` sources (one per thread) while time remains
    per = el1 / k
    rounds = max(1, int((seconds / 2) / max(per, 1e-9)))
    lo = k
    hi = min(len(srcs), lo + threads * rounds)
    if hi <= lo:
        lo, hi = 0, min(len(srcs), threads)
    t = time.perf_counter()
    oracle.bc_sliced(g, srcs[lo:hi], threads=threads)
    elp = time.perf_counter() - t
    many = traversed_edges(g, srcs[lo:hi]) / elp / 1e9
    log(f"[bench] oracle: 1 core {k} sources in {el1:.1f}s -> {one:.4f} GTEPS; {threads} threads {hi - lo} "
        f"sources in {elp:.1f}s -> {many:.4f} GTEPS ({model}, {ncpu} CPUs, {avail} usable)")
    return {"value": round(many, 6), "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "sample": f"sources {lo}..{hi - 1} of the {len(srcs)} of {workload}, one contiguous slice per host "
                      f"thread (single-threaded C oracle per slice, partial scores added in slice order)",
            "single_core": {"value": round(one, 6), "unit": "GTEPS", "cores": 1,
                            "sample": f"first {k} sources of {workload}, one at a time"},
            "cpu_model": model, "nproc": ncpu, "usable_cpus": avail}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--policy", default="auto", choices=["auto", "heuristic", "mlp", "tpv", "wpv", "pull"])
    ap.add_argument("--heuristic-steps", type=int, default=2,
                    help="timed steps of the heuristic-policy leg (0 = skip it)")
    ap.add_argument("--plain-sources", type=int, default=1024,
                    help="sources (a prefix of the list) for the plain-engine leg (0 = the full list)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the oracle CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2008_05718_amd", "policy_weights.npy"))
    ap.add_argument("--sources", type=int, default=0, help="use only the first N sources (profiling runs)")
    ap.add_argument("--no-graphs", action="store_true", help="launch level steps one by one")
    ap.add_argument("--grid", type=int, default=0, help="workgroups per step launch (0 = library default)")
    ap.add_argument("--no-blocks", action="store_true", help="never use the block engine (small graphs)")
    ap.add_argument("--lanes-per-entry", type=float, default=0.0,
                    help="entry-by-source summation threshold of the batched engine (0 = library default, <0 = off)")
    ap.add_argument("--no-tune", action="store_true",
                    help=f"skip bc_autotune (default: tune on the first {TUNE_SOURCES} sources)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE, help="tune cache file to load (if it exists)")
    ap.add_argument("--tune-cache-out", help="write the process's tune cache here after tuning")
    ap.add_argument("--retune", action="store_true", help="tune even when the cache holds a result")
    ap.add_argument("--weighted-lanes", type=int, default=0, choices=[0, 1, 16],
                    help="graphs with arc weights: sources per workgroup (0 = library default, 16)")
    ap.add_argument("--policy-margin", type=float, default=0.0,
                    help="learned policy: log2 gain needed to override the rule (0 = library default, <0 = none)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes 3 times (counter calibration)")
    ap.add_argument("--summarize-profile", action="store_true",
                    help="only reduce rocprofv3 output directories to a profile summary (see profile_summary)")
    ap.add_argument("--trace-dir"), ap.add_argument("--fetch-dir"), ap.add_argument("--write-dir")
    ap.add_argument("--cal-fetch-dir"), ap.add_argument("--cal-write-dir")
    ap.add_argument("--kernel", default="batch_step<0>")
    ap.add_argument("--bench-json", help="the bench line of the profiled command (its stderr log or JSON)")
    ap.add_argument("--command", action="append", default=[], help="a command that made the profile (repeatable)")
    ap.add_argument("--out", help="summary file to write")
    args = ap.parse_args()
    if args.summarize_profile:
        text = profile_summary(args)
        if args.out:
            with open(args.out, "w") as f:
                f.write(text)
        print(text)
        return
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        bb = torch.empty_like(a)
        for _ in range(3):
            bb.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4, "copies": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; a multi-GPU run (sources "
                                   "sharded across GPUs, one reduction of the BC vectors) is not implemented"}))
        sys.exit(2)

    import torch
    from paper_2008_05718_amd import binding as b
    from paper_2008_05718_amd import workloads as W

    b.lib()  # fails loudly when libbc.so is missing
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    t0 = time.time()
    g, srcs = W.workload(args.workload)
    if args.sources > 0:
        srcs = srcs[:args.sources]
    log(f"[bench] generated {args.workload}: n={g.n} m={g.m} sources={len(srcs)} in {time.time() - t0:.1f}s")

    pol = {"auto": b.BC_POLICY_AUTO, "heuristic": b.BC_POLICY_HEURISTIC, "mlp": b.BC_POLICY_MLP,
           "tpv": b.BC_POLICY_FORCE_PUSH_TPV, "wpv": b.BC_POLICY_FORCE_PUSH_WPV,
           "pull": b.BC_POLICY_FORCE_PULL}[args.policy]
    torch.cuda.synchronize()
    t = time.perf_counter()
    G = b.Graph(g)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t
    log(f"[bench] bc_graph_create (host CSR in, validation, hub-first renumbering, upload): {create_s:.2f}s")
    weights_loaded = False
    if os.path.exists(args.weights):
        G.load_policy(np.load(args.weights))
        weights_loaded = True
    if pol == b.BC_POLICY_AUTO:  # the learned policy when trained weights exist (fixed, not tuned)
        pol = b.BC_POLICY_MLP if weights_loaded else b.BC_POLICY_HEURISTIC

    def timed(sources, nsteps, nwarm, H=None, **opts):
        H = H or G
        for _ in range(nwarm):
            H.run(sources, stream=stream, **opts)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        t = time.perf_counter()
        stats = []
        for _ in range(nsteps):
            H.run(sources, stream=stream, **opts)
            stats.append(H.stats())
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        gpu_ms = ev0.elapsed_time(ev1)
        return wall, gpu_ms, stats

    # graphs with arc weights run on the weighted engine (a persistent launch,
    # 16 sources per workgroup; no level policy or launch shape to tune, and
    # no per-source or heuristic leg)
    weighted = getattr(g, "weights", None) is not None
    wextra = {}
    if weighted:
        args.no_tune, args.no_plain, args.heuristic_steps = True, True, 0
        wextra = {"weighted_lanes": args.weighted_lanes}
    wlanes = 1 if args.weighted_lanes == 1 else 16

    # ---- batched (headline); launch configuration tuned on a sample first (untimed)
    gflags = (b.BC_RUN_NO_GRAPHS if args.no_graphs else 0) | (b.BC_RUN_NO_BLOCKS if args.no_blocks else 0)
    tuned = None
    tune_cached = False
    if not args.no_tune:
        if args.tune_cache and os.path.exists(args.tune_cache):
            b.bc_tune_cache_load(args.tune_cache)
        t = time.time()
        n0 = b.bc_tune_cache_size()
        tuned = G.autotune(srcs[:TUNE_SOURCES], batch=64, policy=pol, grid_blocks=args.grid,
                           flags=gflags | (b.BC_TUNE_FRESH if args.retune else 0),
                           lanes_per_entry=args.lanes_per_entry, policy_margin=args.policy_margin)
        tune_cached = b.bc_tune_cache_size() == n0 and not args.retune  # a miss adds an entry
        gflags |= b.BC_RUN_TUNED
        log(f"[bench] autotuned on {min(TUNE_SOURCES, len(srcs))} sources in {time.time() - t:.1f}s"
            f"{' (tune cache hit)' if tune_cached else ''}: {tuned}")
        if args.tune_cache_out:
            b.bc_tune_cache_save(args.tune_cache_out)
    wall, gpu_ms, stats = timed(srcs, args.steps, args.warmup, batch=64, policy=pol, flags=gflags,
                                grid_blocks=args.grid, lanes_per_entry=args.lanes_per_entry,
                                policy_margin=args.policy_margin, **wextra)
    st = stats[-1]
    headline_bits = G.scores().copy()
    ms_step = wall * 1e3 / args.steps
    work = traversed_edges(g, srcs)
    gteps = work * args.steps / wall / 1e9
    launches = sum(s["launches"] for s in stats)
    # dominant kernel: the 64-bit (batch_step<0>) or FP64 (batch_step<1>)
    # path-count pass with more device time.  The library times each pass
    # with HIP events on the stream it launches on; on a single graph the
    # batches run on concurrent replicas (own streams), so per-stream times
    # overlap: the device time of the timed region (events on the caller's
    # stream, which waits for every replica) is shared out by pass.
    mode_ms = [sum(s["mode_ms"][i] for s in stats) for i in (0, 1)]
    k = 0 if mode_ms[0] >= mode_ms[1] else 1
    k_launches = sum(s["mode_launches"][k] for s in stats)
    k_algo = sum(s["mode_algo_bytes"][k] for s in stats)
    share = mode_ms[k] / max(sum(mode_ms), 1e-12)
    dev_ms = gpu_ms * share
    avg_launch_us = dev_ms * 1e3 / max(k_launches, 1)
    trace_launch_us = mode_ms[k] * 1e3 / max(k_launches, 1)
    achieved_gbs = k_algo / max(dev_ms * 1e-3, 1e-12) / 1e9
    # the same bytes without the per-(vertex, source) slab term
    arcs_frac = sum(s["algo_bytes_arcs"] for s in stats) / max(sum(s["algo_bytes"] for s in stats), 1e-12)
    if weighted:
        kernel = f"weighted_run<{k}>" if wlanes == 1 else f"wbatch_run<{k}>"
    elif k == 0 and st.get("block_workgroups", 0) > 0:
        kernel = "block_run<0>"
    else:
        kernel = f"batch_step<{k}>"
    log(f"[bench] batched: {ms_step:.1f} ms/step, {gteps:.2f} GTEPS, launches/step={launches // args.steps}, "
        f"{kernel}: {k_launches} launches, {avg_launch_us:.2f} us each of device time ({trace_launch_us:.2f} us "
        f"on its stream), algo {achieved_gbs:.1f} GB/s, device ms per mode {[round(x, 1) for x in mode_ms]} "
        f"(host wall {wall * 1e3:.1f}, events {gpu_ms:.1f}), policy={st['policy']} "
        f"variants={st['variant_levels']} f64={st['f64_sources']} reached pairs={st['reached_pairs']} "
        f"block engine workgroups={st['block_workgroups']} chunks={st['block_chunks']}")
    if weighted:
        nu = max(-(-st["n_sources"] // wlanes), 1)  # sources (one per workgroup) or lane batches
        unit = "source" if wlanes == 1 else f"batch of {wlanes}"
        log(f"[bench] weighted: per {unit} {st['forward_levels'] / nu:.1f} relaxation rounds, "
            f"{st['arcs_scanned'] / nu / max(g.nnz, 1):.2f} x nnz arcs relaxed, "
            f"{st['steps'] / nu:.1f} DAG rounds, {st['lane_arcs'] / nu / max(g.nnz, 1):.2f} x nnz DAG-pass arcs"
            + ("" if wlanes == 1 else
               f"; (arc, source) pairs per source: relaxation {st['phase_lane_arcs'][1] / st['n_sources'] / g.nnz:.2f}"
               f" x nnz, DAG passes {st['phase_lane_arcs'][2] / st['n_sources'] / g.nnz:.2f} x nnz; device ms "
               f"summed over batches (relaxation, DAG rounds, dependencies) "
               f"{[round(x, 1) for x in st['phase_ms'][1:4]]}, longest batch {st['phase_ms'][4]:.1f} ms"))
    log("[bench] batched phase ms (fwd, sig, bwd, fin, bc):",
        [round(x, 1) for x in st["phase_ms"][1:6]], "variant ms:", [round(x, 1) for x in st["variant_ms"]])
    log("[bench] batched per phase: arcs", st["phase_arcs"][1:4], "lane arcs", st["phase_lane_arcs"][1:4],
        "pairs", st["phase_pairs"][1:4], "queue entries", st["queue_entries"], "batches", st["n_batches"])

    # ---- the same engine with the direction-optimising heuristic (learned vs Beamer)
    heur = None
    if args.heuristic_steps > 0 and pol == b.BC_POLICY_MLP:
        hw, _, hst = timed(srcs, args.heuristic_steps, 1, batch=64, policy=b.BC_POLICY_HEURISTIC, flags=gflags,
                           grid_blocks=args.grid, lanes_per_entry=args.lanes_per_entry,
                           policy_margin=args.policy_margin)
        same = bool(np.array_equal(G.scores().view(np.uint64), headline_bits.view(np.uint64)))
        hg = work * args.heuristic_steps / hw / 1e9
        heur = {"value": round(hg, 4), "unit": "GTEPS", "steps": args.heuristic_steps,
                "ms_per_step": round(hw * 1e3 / args.heuristic_steps, 3), "same_score_bits": same,
                "learned_over_heuristic": round(gteps / hg, 4), "variants": hst[-1]["variant_levels"]}
        log(f"[bench] heuristic policy: {hg:.2f} GTEPS, learned/heuristic = {gteps / hg:.4f}, same bits: {same}")
        if not same:
            raise SystemExit("the learned and the heuristic policy gave different score bits")

    # ---- plain per-source engine on a prefix of the same source list
    plain = None
    if not args.no_plain:
        ps = srcs if args.plain_sources <= 0 else srcs[:args.plain_sources]
        # the caller's vertex order and the library's default launch shape
        # (the tuned shape and the hub-first renumbering belong to the
        # batched path)
        with b.Graph(g, flags=b.BC_KEEP_ORDER) as P:
            if weights_loaded:
                P.load_policy(np.load(args.weights))
            pw, pg, pst = timed(ps, 1, 1, H=P, batch=1, policy=pol,
                                flags=b.BC_RUN_NO_GRAPHS if args.no_graphs else 0)
        pg_teps = traversed_edges(g, ps) / pw / 1e9
        plain = {"value": round(pg_teps, 4), "unit": "GTEPS", "ms_per_step": round(pw * 1e3, 2),
                 "sources": int(len(ps)), "variants": pst[-1]["variant_levels"],
                 "batched_over_plain": round(gteps / pg_teps, 2)}
        log(f"[bench] plain: {pw * 1e3:.1f} ms for {len(ps)} sources, {plain['value']} GTEPS; phase ms",
            [round(x, 1) for x in pst[-1]["phase_ms"][1:6]], "variant ms", [round(x, 1) for x in pst[-1]["variant_ms"]])

    # ---- oracle on the host, bounded sample of the same workload
    cpu = None if args.no_cpu else cpu_baseline(g, srcs, args.workload, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(gteps, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 path counts, f64 dependencies",
        "data": "synthetic (seeded generator, no dataset)",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "sources": int(len(srcs)),
                   "directed": bool(getattr(g, "directed", False)),
                   "arc_weights": (f"integers in [{int(g.weights.min())}, {int(g.weights.max())}]"
                                   if weighted else None),
                   "batch": wlanes if weighted else 64,
                   # the weighted engine has no level policy, captured chunks or launch shape
                   "policy": None if weighted else
                   {1: "heuristic", 2: "mlp", 3: "tpv", 4: "wpv", 5: "pull"}.get(st["policy"]),
                   "mlp_weights_loaded": None if weighted else weights_loaded,
                   "graph_chunk_steps": None if weighted else st["chunk_steps"],
                   "grid_blocks": None if weighted else st["grid_blocks"], "tuned": tuned,
                   "tune_cache_hit": tune_cached, "policy_margin": None if weighted else args.policy_margin},
        "create_s": round(create_s, 3),
        "heuristic": heur,
        "plain": plain,
        "roofline": {"bound": "hbm", "achieved": round(achieved_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(kernel, args.workload),
                     "kernel": kernel, "avg_launch_us": round(avg_launch_us, 3),
                     "avg_launch_us_on_stream": round(trace_launch_us, 3), "launches": int(k_launches),
                     "algo_bytes_per_launch": round(k_algo / max(k_launches, 1), 1),
                     "frac_without_slab_bytes": round(achieved_gbs * arcs_frac / HBM_PEAK_GBS, 4),
                     "target_frac": 0.40},
        "cpu_baseline": cpu,
    }
    G.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
