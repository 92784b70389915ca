"""GPU parity on directed graphs (BC_DIRECTED): paths follow arcs, so the
forward phase pushes over out-arcs and pulls over in-arcs, and the backward
phase pulls from successors over out-arcs.  Checked against the oracle (its
directed form is pinned in tests/test_oracle_directed.py): d and uint64 path
counts bit for bit, scores and dependencies within 1e-10 relative; every
level variant and both summation forms give the same bits."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import assert_bc_close, check_detail, say
from paper_2008_05718_amd import binding as b
from paper_2008_05718_amd import workloads as W

pytestmark = pytest.mark.gpu

POLICIES = (b.BC_POLICY_HEURISTIC, b.BC_POLICY_FORCE_PUSH_TPV, b.BC_POLICY_FORCE_PUSH_WPV, b.BC_POLICY_FORCE_PULL)


def _dg(n, arcs):
    a = np.array(arcs, dtype=np.int64).reshape(-1, 2)
    return W.digraph_from_arcs(n, a[:, 0], a[:, 1])


def _run(g, srcs, **opts):
    with b.Graph(g) as G:
        G.run(srcs, **opts)
        return G.scores()


def test_directed_closed_forms():
    # directed path 0 -> 1 -> ... -> n-1: vertex i lies on i * (n - 1 - i) pairs;
    # directed cycle: every vertex carries (n - 1)(n - 2) / 2; out-star: 0
    n = 40
    path = _dg(n, [(i, i + 1) for i in range(n - 1)])
    cyc = _dg(n, [(i, (i + 1) % n) for i in range(n)])
    star = _dg(n, [(0, i) for i in range(1, n)])
    for batch in (1, 64):
        np.testing.assert_array_equal(_run(path, None, batch=batch), [i * (n - 1 - i) for i in range(n)])
        assert_bc_close(_run(cyc, None, batch=batch), np.full(n, (n - 1) * (n - 2) / 2))
        np.testing.assert_array_equal(_run(star, None, batch=batch), np.zeros(n))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_digraphs_against_oracle(seed):
    rng = np.random.default_rng(seed)
    n = 300
    m = 1500
    g = W.digraph_from_arcs(n, rng.integers(0, n, m), rng.integers(0, n, m))
    ref, _ = oracle.bc(g)
    outs = []
    with b.Graph(g) as G:
        for batch in (1, 64):
            for pol in POLICIES:
                for lpe in (-1.0, 64.0):
                    G.run(None, batch=batch, policy=pol, lanes_per_entry=lpe, flags=b.BC_RUN_ONE_QUEUE)
                    outs.append(((batch, pol, lpe), G.scores().copy()))
        det = G.detail(None, dump_index=17, batch=64)
        check_detail(g, det, 17)
    assert_bc_close(outs[0][1], ref)
    for key, v in outs:
        if key[0] == 64:
            assert np.array_equal(v.view(np.uint64), outs[8][1].view(np.uint64)), key
        assert_bc_close(v, ref)


def test_directed_heavy_vertices_split_by_larger_degree():
    # vertex 0 has out-degree 3000 and in-degree 1; vertex 4000 has in-degree
    # 3000 and out-degree 2: segments follow the larger degree in every phase
    n = 5000
    arcs = [(0, i) for i in range(1, 3001)] + [(i, 4000) for i in range(1, 3001)]
    arcs += [(4000, 4001), (4000, 4002), (4001, 0)]
    rng = np.random.default_rng(5)
    arcs += [tuple(x) for x in rng.integers(3001, 5000, size=(6000, 2))]
    g = _dg(n, arcs)
    srcs = np.array([0, 4001, 4000, 17, 3500, 4999], np.int32)
    ref, _ = oracle.bc(g, srcs)
    base = None
    with b.Graph(g) as G:
        for pol in POLICIES:
            G.run(srcs, batch=64, policy=pol)
            got = G.scores().copy()
            assert_bc_close(got, ref)
            if base is None:
                base = got
            assert np.array_equal(got.view(np.uint64), base.view(np.uint64)), pol
        for k in range(len(srcs)):
            det = G.detail(srcs, dump_index=k, batch=64)
            check_detail(g, det, int(srcs[k]))


def test_both_arcs_equal_the_undirected_engine():
    # a digraph holding both arcs of every edge is the undirected graph: same
    # adjacency, same order of every sum, so the same bits as an undirected
    # handle, both keeping the caller's numbering and source order
    und = W.rmat(11, 8, seed=31)
    rr = np.repeat(np.arange(und.n), np.diff(und.row_ptr.astype(np.int64)))
    dg = W.digraph_from_arcs(und.n, rr, und.col_idx.astype(np.int64))
    srcs = W.choose_sources(und, 150, seed=4)
    with b.Graph(und, flags=b.BC_KEEP_ORDER) as U:
        U.run(srcs, batch=64, flags=b.BC_RUN_ONE_QUEUE)
        u_bits = U.scores().copy()
    with b.Graph(dg, flags=b.BC_KEEP_ORDER) as D:
        D.run(srcs, batch=64, flags=b.BC_RUN_ONE_QUEUE)
        d_bits = D.scores().copy()
    assert np.array_equal(u_bits.view(np.uint64), d_bits.view(np.uint64))
    # without BC_KEEP_ORDER the digraph's sources are ranked: same scores to
    # rounding
    with b.Graph(dg) as D:
        D.run(srcs, batch=64, flags=b.BC_RUN_ONE_QUEUE)
        assert_bc_close(D.scores(), u_bits)


def test_directed_grid_overflows_to_fp64():
    # arcs right and down on a 40 x 40 grid: from the corner, sigma(i, j) =
    # C(i + j, i) passes 2^64 - 1, so the source runs again in FP64 mode
    L = 40
    arcs = [(i * L + j, i * L + j + 1) for i in range(L) for j in range(L - 1)]
    arcs += [(i * L + j, (i + 1) * L + j) for i in range(L - 1) for j in range(L)]
    g = _dg(L * L, arcs)
    srcs = np.array([0, 1, L, 5 * L + 7], np.int32)
    ref, modes = oracle.bc(g, srcs)
    assert modes[0] == 1
    for batch in (1, 64):
        with b.Graph(g) as G:
            det = G.detail(srcs, dump_index=0, batch=batch)
            check_detail(g, det, 0)
            assert G.stats()["f64_sources"] >= 1
            assert_bc_close(G.scores(), ref)


def test_directed_rmat_sources_against_oracle():
    g = W.rmat_directed(14, 16, seed=41)
    srcs = W.choose_sources(g, 256, seed=9)
    say(f"[directed rmat14] n={g.n} arcs={g.nnz}")
    with b.Graph(g) as G:
        G.run(srcs, batch=64)
        got = G.scores().copy()
        st = G.stats()
        say(f"  variants {st['variant_levels']} levels {st['max_levels']}")
        det = G.detail(srcs, dump_index=100, batch=64)
        check_detail(g, det, int(srcs[100]))
        assert np.array_equal(G.scores().view(np.uint64), got.view(np.uint64))
    ref, _ = oracle.bc_sliced(g, srcs, threads=8)
    assert_bc_close(got, ref)


def test_directed_multi_graph_refused():
    g = _dg(4, [(0, 1), (2, 3)])
    with pytest.raises(b.BCError) as ei:
        b.bc_graph_create_multi(np.array([0, 2, 4], np.int32), g.row_ptr, g.col_idx, flags=b.BC_DIRECTED)
    assert ei.value.status == 6


def test_directed_degenerate_inputs_and_accumulate():
    # no arcs at all, sinks and sources, an empty list, duplicates, accumulation
    empty = _dg(5, [])
    for K in (1, 64):
        assert (_run(empty, None, batch=K) == 0).all()
    g = _dg(6, [(0, 1), (1, 2), (3, 1)])  # 2 is a sink, 4 and 5 isolated
    ref, _ = oracle.bc(g)
    for K in (1, 8, 64):
        assert_bc_close(_run(g, None, batch=K), ref)
    with b.Graph(g) as G:
        G.run([2, 2, 4], batch=64)
        assert (G.scores() == 0).all()
        G.run([], batch=64)
        assert (G.scores() == 0).all()
    dg = W.rmat_directed(11, 6, seed=72)
    s1 = W.choose_sources(dg, 90, seed=1)
    s2 = W.choose_sources(dg, 40, seed=2)
    with b.Graph(dg) as G:
        for K in (1, 64):
            G.run(s1, batch=K)
            G.run(s2, batch=K, flags=b.BC_RUN_ACCUMULATE)
            ref, _ = oracle.bc(dg, np.concatenate([s1, s2]))
            assert_bc_close(G.scores(), ref)
            G.run(np.concatenate([s1[:5], s1[:5]]), batch=K)
            r1, _ = oracle.bc(dg, s1[:5])
            assert_bc_close(G.scores(), 2 * r1)
