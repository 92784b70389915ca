"""Parity at the full workload sizes, in the benchmark's launch configuration
(64-source batches, default policy with the trained weights loaded, captured
level chunks, concurrent replicas or sub-unions).

A whole run at these sizes is beyond the oracle, so each test checks
  * sampled sources one by one: d and integer sigma bit-exact, FP64 sigma and
    delta within 1e-10 relative, dumped from the full run itself;
  * the sum of the scores against the path-length excess of every source
    (sum_v delta_s(v) = sum_t (d(s, t) - 1), from a BFS-only checker);
  * every vertex's score on a prefix of the source list against the oracle;
  * that a detail run leaves the same score bits as the plain run.
"""
from __future__ import annotations

import os
import time

import numpy as np
import pytest

import oracle
from gpu_util import REL, assert_bc_close, check_detail, say
from paper_2008_05718_amd import binding as b
from paper_2008_05718_amd import workloads as W

pytestmark = pytest.mark.gpu
WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2008_05718_amd",
                       "policy_weights.npy")


def _graph(g):
    G = b.Graph(g)
    if os.path.exists(WEIGHTS):
        G.load_policy(np.load(WEIGHTS))
    return G


def _sum_check(bc, g, srcs):
    t = time.time()
    want = float(oracle.path_excess(g, srcs).sum())
    got = float(np.sum(bc, dtype=np.float64))
    say(f"  sum of scores {got:.6e} vs path-length excess {want:.6e} ({time.time() - t:.1f}s on the host)")
    assert abs(got - want) <= REL * want


def _full_case(name, dump_at, prefix, run_full_plain=True):
    t = time.time()
    g, srcs = W.workload(name)
    say(f"[fullsize {name}] n={g.n} m={g.m} sources={len(srcs)} (generated in {time.time() - t:.1f}s)")
    with _graph(g) as G:
        ref_bits = None
        if run_full_plain:
            t = time.time()
            G.run(srcs, batch=64)
            ref_bits = G.scores().copy()
            st = G.stats()
            say(f"  full run {time.time() - t:.2f}s, f64 sources {st['f64_sources']}, policy {st['policy']}")
            _sum_check(ref_bits, g, srcs)
        for k in dump_at:
            t = time.time()
            det = G.detail(srcs, dump_index=k, batch=64)
            say(f"  detail of source #{k} ({srcs[k]}): mode {det['mode']}, {det['n_levels']} levels, "
                f"{time.time() - t:.2f}s")
            check_detail(g, det, srcs[k])
            bits = G.scores()
            if ref_bits is None:
                ref_bits = bits.copy()
            assert np.array_equal(bits.view(np.uint64), ref_bits.view(np.uint64))
        t = time.time()
        G.run(srcs[:prefix], batch=64)
        got = G.scores()
    ref, modes = oracle.bc(g, srcs[:prefix])
    say(f"  prefix of {prefix} sources vs oracle ({time.time() - t:.1f}s), f64 sources {int(modes.sum())}")
    assert_bc_close(got, ref)
    return g, srcs


def test_rmat18_8192_sources():
    _full_case("rmat18", dump_at=[0, 4097, 8191], prefix=96)


def test_grid1024_4096_sources():
    # every source overflows 64-bit path counts: the whole run is the FP64 path
    _full_case("grid1024", dump_at=[0, 4095], prefix=24)


def test_rmat22_16384_sources():
    # the full list is dumped once (that run is also the score check); the
    # score sum is checked on a 256-source prefix, the oracle on 4 sources
    t = time.time()
    g, srcs = W.workload("rmat22")
    say(f"[fullsize rmat22] n={g.n} m={g.m} sources={len(srcs)} (generated in {time.time() - t:.1f}s)")
    with _graph(g) as G:
        t = time.time()
        det = G.detail(srcs, dump_index=9000, batch=64)
        say(f"  full run with detail of source #9000: mode {det['mode']}, {time.time() - t:.2f}s")
        check_detail(g, det, srcs[9000])
        full = G.scores().copy()
        assert np.isfinite(full).all() and (full >= 0).all()
        G.run(srcs[:256], batch=64)
        _sum_check(G.scores(), g, srcs[:256])
        G.run(srcs[:4], batch=64)
        got = G.scores()
    ref, _ = oracle.bc(g, srcs[:4])
    assert_bc_close(got, ref)


def _block(g, lo, hi):
    """Graph block [lo, hi) of a block-diagonal union as a CSR of its own."""
    rp = g.row_ptr[lo:hi + 1].astype(np.int64)
    col = g.col_idx[rp[0]:rp[-1]].astype(np.int64) - lo
    rr = np.repeat(np.arange(hi - lo), np.diff(rp))
    return W.csr_from_edges(hi - lo, rr, col)


def test_ba512_sampled_sources():
    # the full union (512 graphs, 12.3 M vertices) in the default launch
    # configuration (concurrent sub-unions), 8 sources from every graph:
    # details of three sources, the score sum against the path-length excess,
    # and three whole graphs' scores against the oracle
    t = time.time()
    g, _ = W.workload("ba512")
    off = g.vtx_offsets.astype(np.int64)
    rng = np.random.default_rng(77)
    srcs = np.concatenate([off[i] + rng.choice(off[i + 1] - off[i], 8, replace=False)
                           for i in range(len(off) - 1)]).astype(np.int32)
    say(f"[fullsize ba512] n={g.n} m={g.m} graphs={len(off) - 1} sources={len(srcs)} "
        f"(generated in {time.time() - t:.1f}s)")
    with _graph(g) as G:
        t = time.time()
        G.run(srcs, batch=64)
        got = G.scores().copy()
        say(f"  run {time.time() - t:.2f}s")
        _sum_check(got, g, srcs)
        for k in (0, 8 * 255 + 3, len(srcs) - 1):
            det = G.detail(srcs, dump_index=k, batch=64)
            check_detail(g, det, srcs[k])
    for i in (0, 255, 511):
        lo, hi = int(off[i]), int(off[i + 1])
        ref, _ = oracle.bc(_block(g, lo, hi), srcs[8 * i:8 * i + 8] - lo)
        assert_bc_close(got[lo:hi], ref)
