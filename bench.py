"""Benchmark: exact Brandes BC throughput (GTEPS = m x sources / s) on one MI355X.

One step = one complete BC run (forward + backward for every source, all
levels, scores summed) over the workload's source list, through libbc's C ABI.
Inputs are resident in HBM before the timed region (bc_graph_create is
outside it).  The batched engine (64 sources per traversal, level policy as
selected) is the headline value; the plain per-source engine is timed on the
same workload beside it.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload rmat18] [--gpus 1]
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


TUNE_SOURCES = 512  # autotuner sample: the first sources of the list (untimed)
KERNEL_SOURCES = ["paper_2008_05718_amd/csrc/bc_batched.hip", "paper_2008_05718_amd/csrc/bc_common.h",
                  "paper_2008_05718_amd/csrc/bc_api.hip",
                  "paper_2008_05718_amd/csrc/bc_dev.h", "paper_2008_05718_amd/build.py"]


def _code_only(text: str) -> str:
    """C/C++ source without comments and with whitespace collapsed."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_sources_sha256() -> str:
    """Hash of the sources the step kernel is built from; comments and
    whitespace of the HIP sources are ignored, so an edit of comments only
    keeps the recorded counters valid."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
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
    tag = {"batch_step<0>": "batch_step_u64", "batch_step<1>": "batch_step_f64"}.get(kernel)
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
        if vals.get("kernel_sources_sha256") != kernel_sources_sha256():
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat18")
    ap.add_argument("--policy", default="auto", choices=["auto", "heuristic", "mlp", "tpv", "wpv", "pull"])
    ap.add_argument("--plain-sources", type=int, default=0,
                    help="sources for the plain-engine leg (0 = the full list)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2008_05718_amd", "policy_weights.npy"))
    ap.add_argument("--sources", type=int, default=0, help="use only the first N sources (profiling runs)")
    ap.add_argument("--no-graphs", action="store_true", help="launch level steps one by one")
    ap.add_argument("--grid", type=int, default=0, help="workgroups per step launch (0 = library default)")
    ap.add_argument("--no-tune", action="store_true", help="skip bc_autotune (default: tune on the first 512 sources)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes 3 times (counter calibration)")
    args = ap.parse_args()
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

    if not os.path.exists(b.LIB_PATH):
        from paper_2008_05718_amd import build as hb
        hb.build()
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
    G = b.Graph(g)
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

    # ---- batched (headline); launch configuration tuned on a sample first (untimed)
    gflags = b.BC_RUN_NO_GRAPHS if args.no_graphs else 0
    tuned = None
    if not args.no_tune:
        t = time.time()
        tuned = G.autotune(srcs[:TUNE_SOURCES], batch=64, policy=pol, grid_blocks=args.grid, flags=gflags)
        gflags |= b.BC_RUN_TUNED
        log(f"[bench] autotuned on {min(TUNE_SOURCES, len(srcs))} sources in {time.time() - t:.1f}s: {tuned}")
    wall, gpu_ms, stats = timed(srcs, args.steps, args.warmup, batch=64, policy=pol, flags=gflags,
                                grid_blocks=args.grid)
    st = stats[-1]
    ms_step = wall * 1e3 / args.steps
    gteps = g.m * len(srcs) * args.steps / wall / 1e9
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
    kernel = f"batch_step<{k}>"
    log(f"[bench] batched: {ms_step:.1f} ms/step, {gteps:.2f} GTEPS, launches/step={launches // args.steps}, "
        f"{kernel}: {k_launches} launches, {avg_launch_us:.2f} us each of device time ({trace_launch_us:.2f} us "
        f"on its stream), algo {achieved_gbs:.1f} GB/s, device ms per mode {[round(x, 1) for x in mode_ms]} "
        f"(host wall {wall * 1e3:.1f}, events {gpu_ms:.1f}), policy={st['policy']} "
        f"variants={st['variant_levels']} f64={st['f64_sources']}")
    log("[bench] batched phase ms (fwd, sig, bwd, fin, bc):",
        [round(x, 1) for x in st["phase_ms"][1:6]], "variant ms:", [round(x, 1) for x in st["variant_ms"]])
    log("[bench] batched per phase: arcs", st["phase_arcs"][1:4], "lane arcs", st["phase_lane_arcs"][1:4],
        "pairs", st["phase_pairs"][1:4], "queue entries", st["queue_entries"], "batches", st["n_batches"])

    # ---- plain per-source engine on the same workload
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
        plain = {"value": round(g.m * len(ps) / pw / 1e9, 4), "unit": "GTEPS", "ms_per_step": round(pw * 1e3, 2),
                 "sources": int(len(ps)), "variants": pst[-1]["variant_levels"]}
        log(f"[bench] plain: {pw * 1e3:.1f} ms for {len(ps)} sources, {plain['value']} GTEPS; phase ms",
            [round(x, 1) for x in pst[-1]["phase_ms"][1:6]], "variant ms", [round(x, 1) for x in pst[-1]["variant_ms"]])

    # ---- oracle on the host, bounded sample of the same workload
    cpu = None
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        k = 0
        t = time.perf_counter()
        per = []
        while time.perf_counter() - t < args.cpu_seconds and k < len(srcs):
            t1 = time.perf_counter()
            oracle.bc(g, srcs[k:k + 1])
            per.append(time.perf_counter() - t1)
            k += 1
        el = time.perf_counter() - t
        cpu = {"value": round(g.m * k / el / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"first {k} of {len(srcs)} sources of {args.workload}, single-threaded C oracle"}
        log(f"[bench] oracle: {k} sources in {el:.1f}s -> {cpu['value']} GTEPS")

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
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "sources": int(len(srcs)), "batch": 64,
                   "policy": {1: "heuristic", 2: "mlp", 3: "tpv", 4: "wpv", 5: "pull"}.get(st["policy"]),
                   "mlp_weights_loaded": weights_loaded, "graph_chunk_steps": st["chunk_steps"],
                   "grid_blocks": st["grid_blocks"], "tuned": tuned},
        "plain": plain,
        "roofline": {"bound": "hbm", "achieved": round(achieved_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(kernel, args.workload),
                     "kernel": kernel, "avg_launch_us": round(avg_launch_us, 3),
                     "avg_launch_us_on_stream": round(trace_launch_us, 3), "launches": int(k_launches),
                     "algo_bytes_per_launch": round(k_algo / max(k_launches, 1), 1)},
        "cpu_baseline": cpu,
    }
    G.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
