"""GPU parity on graphs with positive integer arc weights (the forward phase
as a shortest-path computation; the weighted engines: 16 sources per
workgroup in lane batches, the default, and one source per workgroup).  Against the oracle,
whose weighted form is pinned in tests/test_oracle_weighted.py: int64
distances and uint64 path counts bit for bit, FP64 counts, dependencies
and scores within 1e-10 relative; runs repeat bit for bit; unit weights
agree with the unweighted engines."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import assert_bc_close, check_detail, say
from paper_2008_05718_amd import binding as b
from paper_2008_05718_amd import workloads as W

pytestmark = pytest.mark.gpu


LANES = [16, 1]


@pytest.mark.parametrize("lanes", LANES)
@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("wmax", [1, 3, 100])
def test_weighted_rmat_against_oracle(directed, wmax, lanes):
    base = W.rmat_directed(11, 8, seed=61) if directed else W.rmat(11, 8, seed=61)
    g = W.with_weights(base, 1, wmax, seed=7)
    srcs = W.choose_sources(base, 200, seed=3)
    ref, modes = oracle.bc(g, srcs)
    say(f"[weighted] directed={directed} wmax={wmax} lanes={lanes} n={g.n} f64 {int(modes.sum())}")
    with b.Graph(g) as G:
        G.run(srcs, weighted_lanes=lanes)
        got = G.scores().copy()
        G.run(srcs, weighted_lanes=lanes)
        assert np.array_equal(G.scores().view(np.uint64), got.view(np.uint64))
        for k in (0, 77, 199):
            det = G.detail(srcs, dump_index=k, weighted_lanes=lanes)
            check_detail(g, det, int(srcs[k]))
        st = G.stats()
        say(f"  relaxation rounds {st['forward_levels']}, DAG rounds {st['steps']}, arcs {st['arcs_scanned']}")
    assert_bc_close(got, ref)


def test_unit_weights_equal_unweighted_engine():
    base = W.rmat(12, 16, seed=62)
    g = W.with_weights(base, 1, 1, seed=1)
    srcs = W.choose_sources(base, 300, seed=4)
    with b.Graph(g) as G:
        G.run(srcs)
        wgot = G.scores().copy()
    with b.Graph(base, flags=b.BC_KEEP_ORDER) as U:
        U.run(srcs, batch=64, flags=b.BC_RUN_ONE_QUEUE)
        ugot = U.scores().copy()
    assert np.max(np.abs(wgot - ugot) / np.maximum(np.abs(ugot), 1e-300)) <= 1e-12


@pytest.mark.parametrize("lanes", LANES)
def test_weighted_grid_overflow_to_fp64(lanes):
    # unit weights on a 45 x 45 grid: counts from a corner pass 2^64, so the
    # sources run again with FP64 counts
    base = W.grid(45)
    g = W.with_weights(base, 1, 1, seed=2)
    srcs = np.array([0, 44, 22 * 45 + 22, 45 * 45 - 1, 100], np.int32)
    ref, modes = oracle.bc(g, srcs)
    assert modes[0] == 1
    with b.Graph(g) as G:
        G.run(srcs, weighted_lanes=lanes)
        assert G.stats()["f64_sources"] == int(modes.sum())
        assert_bc_close(G.scores(), ref)
        det = G.detail(srcs, dump_index=0, weighted_lanes=lanes)
        check_detail(g, det, 0)


def test_weighted_lane_batches_path_count_limit():
    # a path-count limit hands the sources whose counts pass it to the FP64
    # pass; within a lane batch the other sources keep their uint64 results.
    # Both engines, and both against the oracle.
    base = W.rmat(11, 8, seed=64)
    g = W.with_weights(base, 1, 2, seed=8)
    srcs = W.choose_sources(base, 120, seed=9)
    ref, _ = oracle.bc(g, srcs)
    lim = 119  # about half of the sources have a count above it
    over = []
    for s in srcs:  # sources with a path count above the limit
        o = oracle.source(g, int(s))
        over.append(o.mode == 1 or bool((o.sigma_u64[o.d >= 0] > lim).any()))
    want = sum(over)
    assert 0 < want < len(srcs)
    k_under, k_over = over.index(False), over.index(True)
    got = {}
    for lanes in LANES:
        with b.Graph(g) as G:
            G.run(srcs, weighted_lanes=lanes, sigma_limit=lim)
            assert G.stats()["f64_sources"] == want
            got[lanes] = G.scores().copy()
            det = G.detail(srcs, dump_index=k_under, weighted_lanes=lanes, sigma_limit=lim)
            check_detail(g, det, int(srcs[k_under]))
            # a source over the limit is dumped from the FP64 pass
            det = G.detail(srcs, dump_index=k_over, weighted_lanes=lanes, sigma_limit=lim)
            o = oracle.source(g, int(srcs[k_over]))
            assert det["mode"] == 1
            np.testing.assert_array_equal(det["d64"], o.d)
            r = o.d >= 0
            sig = np.ldexp(det["sigma_mant"][r].astype(np.longdouble), det["sigma_exp"][r].astype(np.int64))
            np.testing.assert_array_equal(sig, o.sigma_u64[r].astype(np.longdouble))
            inner = o.d >= 1
            assert_bc_close(det["delta"][inner], o.delta[inner])
        assert_bc_close(got[lanes], ref)
    assert_bc_close(got[16], got[1])


def test_weighted_closed_forms_and_errors():
    # a weighted path keeps the unweighted scores; weights < 1 and
    # asymmetric undirected weights are refused
    n = 30
    u = np.arange(n - 1)
    base = W.csr_from_edges(n, u, u + 1)
    g = W.with_weights(base, 1, 9, seed=5)
    with b.Graph(g) as G:
        G.run(None)
        np.testing.assert_array_equal(G.scores(), [2.0 * i * (n - 1 - i) for i in range(n)])
    bad = g.weights.copy()
    bad[3] = 0
    with pytest.raises(b.BCError) as e:
        b.bc_graph_create_weighted(g.row_ptr, g.col_idx, bad)
    assert e.value.status == 2
    asym = g.weights.copy()
    asym[0] += 1
    with pytest.raises(b.BCError) as e:
        b.bc_graph_create_weighted(g.row_ptr, g.col_idx, asym)
    assert e.value.status == 2


@pytest.mark.parametrize("lanes", LANES)
def test_weighted_heavy_vertices(lanes):
    # hubs above the lane-batched engine's light-entry degree (256): their
    # arcs are walked by a whole wavefront (sums as partials added in a
    # fixed order)
    base = W.rmat(13, 16, seed=63)
    g = W.with_weights(base, 1, 4, seed=6)
    deg = base.degrees()
    assert (deg > 256).sum() >= 4
    srcs = np.concatenate([np.argsort(-deg)[:4], W.choose_sources(base, 60, seed=5)]).astype(np.int32)
    ref, _ = oracle.bc(g, srcs)
    with b.Graph(g) as G:
        G.run(srcs, weighted_lanes=lanes)
        got = G.scores().copy()
        assert_bc_close(got, ref)
        det = G.detail(srcs, dump_index=1, weighted_lanes=lanes)
        check_detail(g, det, int(srcs[1]))
        assert np.array_equal(G.scores().view(np.uint64), got.view(np.uint64))


def test_weighted_degenerate_inputs_accumulate_and_duplicates():
    # one vertex, isolated vertices, a source that reaches nothing, an empty
    # source list, duplicates counted twice, accumulation across runs
    one = W.with_weights(W.CSR(np.array([0, 0], np.int32), np.zeros(0, np.int32)), 1, 5, seed=1)
    with b.Graph(one) as G:
        G.run([0, 0])
        assert G.scores().tolist() == [0.0]
    u = np.array([0, 1, 4])
    base = W.csr_from_edges(7, u, u + 1)  # 3 and 6 isolated
    g = W.with_weights(base, 1, 7, seed=3)
    ref, _ = oracle.bc(g)
    with b.Graph(g) as G:
        G.run(None)
        assert_bc_close(G.scores(), ref)
        G.run([])
        assert (G.scores() == 0).all()
        G.run([3, 3, 6])
        assert (G.scores() == 0).all()
        det = G.detail([3], dump_index=0)
        assert det["d64"].tolist() == [-1, -1, -1, 0, -1, -1, -1]
    dg = W.with_weights(W.rmat_directed(10, 6, seed=71), 1, 20, seed=4)
    s1 = W.choose_sources(dg, 50, seed=1)
    s2 = W.choose_sources(dg, 30, seed=2)
    with b.Graph(dg) as G:
        G.run(s1)
        G.run(s2, flags=b.BC_RUN_ACCUMULATE)
        ref, _ = oracle.bc(dg, np.concatenate([s1, s2]))
        assert_bc_close(G.scores(), ref)
        G.run(np.concatenate([s1[:5], s1[:5]]))
        r1, _ = oracle.bc(dg, s1[:5])
        assert_bc_close(G.scores(), 2 * r1)
        # a source listed 16 times fills one lane batch with the same vertex
        G.run(np.repeat(s1[:1], 16))
        r0, _ = oracle.bc(dg, s1[:1])
        assert_bc_close(G.scores(), 16 * r0)
        with pytest.raises(b.BCError) as e:
            G.run(s1, weighted_lanes=8)
        assert e.value.status == 1


@pytest.mark.parametrize("lanes", LANES)
def test_weighted_few_workgroups_many_batches(lanes):
    # a device-memory cap just above the graph leaves room for the state of
    # one or two workgroups, so each works through several chunks of several
    # batches: the reset between batches and chunks is exercised
    base = W.rmat(11, 8, seed=65)
    g = W.with_weights(base, 1, 50, seed=9)
    srcs = W.choose_sources(base, 300, seed=10)  # 19 lane batches, the last partial
    ref, _ = oracle.bc(g, srcs)
    with b.Graph(g) as G:
        floor = G.info()["device_bytes"]
        ran = False
        for extra_mib in range(1, 41):
            G.set_device_limit(floor + (extra_mib << 20))
            try:
                G.run(srcs, weighted_lanes=lanes)
            except b.BCError as e:
                assert e.status == 3, e  # refused before allocating
                assert G.info()["device_bytes"] <= floor + (extra_mib << 20)
                continue
            ran = True
            break
        assert ran
        say(f"[weighted few workgroups] lanes={lanes}: cap {extra_mib} MiB above the graph")
        got = G.scores().copy()
        assert_bc_close(got, ref)
        det = G.detail(srcs, dump_index=290, weighted_lanes=lanes)
        check_detail(g, det, int(srcs[290]))
        G.run(srcs, weighted_lanes=lanes)
        assert np.array_equal(G.scores().view(np.uint64), got.view(np.uint64))
