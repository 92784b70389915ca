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
    # the full list runs four times with a detail dump each (sources spread
    # over the list, so over batches held by different concurrent replicas);
    # every run leaves the same score bits; the score sum is checked on a
    # 256-source prefix and every vertex's score on a 64-source prefix
    t = time.time()
    g, srcs = W.workload("rmat22")
    say(f"[fullsize rmat22] n={g.n} m={g.m} sources={len(srcs)} (generated in {time.time() - t:.1f}s)")
    with _graph(g) as G:
        full = None
        for k in (0, 5003, 9000, 16383):
            t = time.time()
            det = G.detail(srcs, dump_index=k, batch=64)
            say(f"  full run with detail of source #{k}: mode {det['mode']}, {det['n_levels']} levels, "
                f"{time.time() - t:.2f}s")
            check_detail(g, det, srcs[k])
            bits = G.scores().copy()
            if full is None:
                full = bits
                assert np.isfinite(full).all() and (full >= 0).all()
            assert np.array_equal(bits.view(np.uint64), full.view(np.uint64))
        G.run(srcs[:256], batch=64)
        _sum_check(G.scores(), g, srcs[:256])
        G.run(srcs[:64], batch=64)
        got = G.scores()
    t = time.time()
    ref, _ = oracle.bc_sliced(g, srcs[:64], threads=16)
    say(f"  oracle on 64 sources: {time.time() - t:.1f}s on the host")
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
    g = _ba_all_graph()
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


# The whole BA workload, every vertex of every graph a source, in steps that
# each finish within a couple of minutes: the union is generated once, one
# run in the default launch configuration computes every score, and the
# host checks follow in parts.
_BA_ALL = {}


def _ba_all_graph():
    if "g" not in _BA_ALL:
        t = time.time()
        g, _ = W.workload("ba512")
        _BA_ALL["g"] = g
        say(f"[fullsize ba512 all sources] n={g.n} m={g.m} (generated in {time.time() - t:.1f}s)")
    return _BA_ALL["g"]


def test_ba512_all_sources_run():
    g = _ba_all_graph()
    with _graph(g) as G:
        t = time.time()
        G.run(None, batch=64)
        got = G.scores().copy()
        st = G.stats()
    say(f"  all {g.n} sources: {time.time() - t:.1f}s, batches {st['n_batches']}")
    assert np.isfinite(got).all() and (got >= 0).all()
    _BA_ALL["bc"] = got


def _ba_all_pick():
    g = _ba_all_graph()
    off = g.vtx_offsets.astype(np.int64)
    sizes = np.diff(off)
    order = np.argsort(sizes, kind="stable")
    whole = [int(order[0]), int(order[-1])] + [int(order[k]) for k in np.linspace(1, len(order) - 2, 14).astype(int)]
    chosen = set(whole)
    rest = [i for i in range(len(sizes)) if i not in chosen and sizes[i] <= 20000]
    excess = [int(i) for i in np.random.default_rng(2024).choice(rest, 48, replace=False)]
    return g, off, whole, excess


@pytest.mark.parametrize("part", [0, 1, 2, 3])
def test_ba512_all_sources_whole_graphs(part):
    # 16 whole graphs (the smallest, the largest, 14 spread over the size
    # range; every source of each) against the oracle, four per test
    if "bc" not in _BA_ALL:
        pytest.skip("needs test_ba512_all_sources_run in the same session")
    g, off, whole, _ = _ba_all_pick()
    got = _BA_ALL["bc"]
    t = time.time()
    for i in whole[part::4]:
        lo, hi = int(off[i]), int(off[i + 1])
        ref, _ = oracle.bc_sliced(_block(g, lo, hi), np.arange(hi - lo, dtype=np.int32), threads=16)
        assert_bc_close(got[lo:hi], ref, what=f"graph {i} (n={hi - lo})")
    say(f"  whole graphs {whole[part::4]} against the oracle: {time.time() - t:.1f}s on the host")


def test_ba512_all_sources_score_sums():
    # the score sum of 48 more graphs against their path-length excess
    if "bc" not in _BA_ALL:
        pytest.skip("needs test_ba512_all_sources_run in the same session")
    g, off, _, excess = _ba_all_pick()
    got = _BA_ALL["bc"]
    t = time.time()
    for i in excess:
        lo, hi = int(off[i]), int(off[i + 1])
        want = float(oracle.path_excess(_block(g, lo, hi), np.arange(hi - lo, dtype=np.int32)).sum())
        have = float(np.sum(got[lo:hi], dtype=np.float64))
        assert abs(have - want) <= REL * want, (i, have, want)
    say(f"  score sums of 48 more graphs: {time.time() - t:.1f}s on the host")


def test_rmat18_directed_8192_sources():
    # the directed benchmark workload at full size: dumps, the score sum
    # (hop-count excess over out-arcs) and an oracle prefix
    _full_case("rmat18_directed", dump_at=[0, 4097, 8191], prefix=96)


def test_rmat18_weighted_4096_sources():
    # the weighted benchmark workload at full size: repeatable bits, dumps
    # from the full run (int64 distances and uint64 counts bit-exact), and a
    # 48-source prefix against the oracle on 16 host threads
    t = time.time()
    g, srcs = W.workload("rmat18_weighted")
    say(f"[fullsize rmat18_weighted] n={g.n} m={g.m} sources={len(srcs)} (generated in {time.time() - t:.1f}s)")
    with _graph(g) as G:
        t = time.time()
        G.run(srcs)
        full = G.scores().copy()
        st = G.stats()
        say(f"  full run {time.time() - t:.2f}s, f64 sources {st['f64_sources']}, relaxation rounds "
            f"{st['forward_levels']}")
        for k in (0, 2049, 4095):
            det = G.detail(srcs, dump_index=k)
            check_detail(g, det, srcs[k])
            assert np.array_equal(G.scores().view(np.uint64), full.view(np.uint64))
        G.run(srcs[:48])
        got = G.scores()
    t = time.time()
    ref, _ = oracle.bc_sliced(g, srcs[:48], threads=16)
    say(f"  oracle on 48 sources: {time.time() - t:.1f}s on the host")
    assert_bc_close(got, ref)
