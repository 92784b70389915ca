"""The block engine: one persistent launch in which every workgroup runs the
batched level state machine alone over chunks of consecutive batches of one
small graph.  Checked against the oracle (d and uint64 path counts exact,
scores within 1e-10 relative), run to run for identical bits, against the
general engine to rounding, and through its fallbacks: sources whose path
counts overflow 64 bits run again in FP64 on the general engine, and runs
that exceed a workgroup's capacities run on the general engine instead."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import assert_bc_close, check_detail, say
from paper_2008_05718_amd import binding as b
from paper_2008_05718_amd import workloads as W

pytestmark = pytest.mark.gpu


def _g(n, edges):
    e = np.array(edges, dtype=np.int64).reshape(-1, 2)
    return W.csr_from_edges(n, e[:, 0], e[:, 1])


def _union():
    sizes = [50, 700, 120, 3000, 90, 400, 1500, 60, 250, 800, 30, 2200]
    gs = [W.barabasi_albert(n, 4, seed=500 + i) for i, n in enumerate(sizes)]
    gs[5] = W.grid(20, 0.1, 0.0, seed=3)
    # a heavy vertex (degree 2499 > one 1024-arc segment)
    gs.insert(3, _g(2500, [(0, i) for i in range(1, 2500)] + [(i, i + 1) for i in range(1, 2499, 2)]))
    return W.union(gs), gs


@pytest.mark.parametrize("K", [16, 64])
def test_union_all_sources_against_oracle(K):
    u, gs = _union()
    say(f"[block] union of {len(gs)} graphs, n={u.n}, K={K}")
    with b.Graph(u) as G:
        G.run(None, batch=K, flags=b.BC_RUN_BLOCKS)
        got = G.scores().copy()
        st = G.stats()
        say(f"  workgroups {st['block_workgroups']} chunks {st['block_chunks']} batches {st['n_batches']}")
        assert st["block_workgroups"] > 0 and st["block_chunks"] > 0
        assert st["n_batches"] == sum(-(-x.n // K) for x in gs)
        G.run(None, batch=K, flags=b.BC_RUN_BLOCKS)  # run to run: same bits
        assert np.array_equal(G.scores().view(np.uint64), got.view(np.uint64))
        G.run(None, batch=K, flags=b.BC_RUN_NO_BLOCKS)
        general = G.scores().copy()
        assert G.stats()["block_workgroups"] == 0
    for i, gg in enumerate(gs):
        lo, hi = u.vtx_offsets[i], u.vtx_offsets[i + 1]
        ref, _ = oracle.bc(gg)
        assert_bc_close(got[lo:hi], ref, what=f"graph {i}")
    assert np.max(np.abs(got - general) / np.maximum(np.abs(general), 1e-300)) <= 1e-12


def test_single_graph_default_and_accumulate():
    # ER(2000): the default path takes the block engine for the whole list;
    # two runs with BC_RUN_ACCUMULATE add up to the whole list
    g, srcs = W.workload("er2000")
    ref, _ = oracle.bc(g, srcs)
    with b.Graph(g) as G:
        G.run(srcs, batch=64)
        st = G.stats()
        say(f"[block er2000] workgroups {st['block_workgroups']} chunks {st['block_chunks']} ms {st['ms']:.2f}")
        assert st["block_workgroups"] > 0
        assert_bc_close(G.scores(), ref)
        G.run(srcs[:900], batch=64, flags=b.BC_RUN_BLOCKS)
        G.run(srcs[900:], batch=64, flags=b.BC_RUN_BLOCKS | b.BC_RUN_ACCUMULATE)
        assert_bc_close(G.scores(), ref)
        det = G.detail(srcs, dump_index=1234, batch=64)  # detail runs use the general engine
        check_detail(g, det, int(srcs[1234]))


def test_overflowed_sources_rerun_in_fp64():
    # a 60 x 60 grid (every corner-ish source overflows 64-bit counts) in a
    # union with BA graphs: the block pass hands the overflowed sources to
    # an FP64 pass of the general engine
    grid = W.grid(60, 0.05, 0.0, seed=21)
    gs = [W.barabasi_albert(900, 4, seed=31), grid, W.barabasi_albert(1500, 4, seed=32)]
    u = W.union(gs)
    srcs = np.arange(0, u.n, 3, dtype=np.int32)
    ref, modes = oracle.bc_sliced(u, srcs, threads=8)
    say(f"[block overflow] n={u.n} sources={len(srcs)} f64 (oracle) {int(modes.sum())}")
    assert modes.any()
    with b.Graph(u) as G:
        G.run(srcs, batch=64, flags=b.BC_RUN_BLOCKS)
        st = G.stats()
        assert st["block_workgroups"] > 0
        assert st["f64_sources"] == int(modes.sum())
        assert_bc_close(G.scores(), ref)


@pytest.mark.parametrize("L", [3000, 6000])
def test_paths_and_capacity_fallback(L):
    # paths: 64 sources spread along a path put a vertex on up to 64 levels
    # of a batch (the block engine holds that many queue entries per vertex
    # for graphs this small); a 3000-vertex path fits its 4,096 levels, a
    # 6000-vertex path does not and the run finishes on the general engine;
    # both give the oracle's scores
    g = _g(L, [(i, i + 1) for i in range(L - 1)])
    srcs = np.linspace(0, L - 1, 640).astype(np.int32)
    ref, _ = oracle.bc(g, srcs)
    with b.Graph(g) as G:
        G.run(srcs, batch=64, flags=b.BC_RUN_BLOCKS)
        st = G.stats()
        say(f"[block paths] path {L}: workgroups {st['block_workgroups']} max levels {st['max_levels']}")
        assert (st["block_workgroups"] > 0) == (L < 4096)
        assert_bc_close(G.scores(), ref)


def test_directed_graph_on_block_engine():
    g = W.rmat_directed(11, 8, seed=51)
    srcs = W.choose_sources(g, 600, seed=5)
    ref, _ = oracle.bc(g, srcs)
    with b.Graph(g) as G:
        G.run(srcs, batch=64, flags=b.BC_RUN_BLOCKS)
        assert G.stats()["block_workgroups"] > 0
        assert_bc_close(G.scores(), ref)
