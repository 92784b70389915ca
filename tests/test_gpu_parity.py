"""GPU parity: libbc (through its C ABI) against the CPU oracle.

d and uint64 sigma must match bit for bit; BC, delta and FP64 sigma within
1e-10 relative per vertex (exact zeros must stay zero).  Both engines (plain
K=1 and batched K<=64), every level variant, graph capture on/off and several
batch widths must give bitwise-identical BC within one engine.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest

import oracle
from gpu_util import assert_bc_close, check_detail, run_bc, say
from paper_2008_05718_amd import binding as b
from paper_2008_05718_amd import workloads as W

pytestmark = pytest.mark.gpu
ENGINES = [1, 64]


def _g(n, edges):
    e = np.array(edges, dtype=np.int64).reshape(-1, 2)
    return W.csr_from_edges(n, e[:, 0], e[:, 1])


CLOSED = {
    "path50": (_g(50, [(i, i + 1) for i in range(49)]), lambda n: np.array([i * (n - 1 - i) for i in range(n)], float)),
    "star40": (_g(40, [(0, i) for i in range(1, 40)]), lambda n: np.array([(n - 1) * (n - 2) / 2] + [0] * (n - 1), float)),
    "cycle21": (_g(21, [(i, (i + 1) % 21) for i in range(21)]), lambda n: np.full(n, (n - 1) * (n - 3) / 8)),
    "cycle30": (_g(30, [(i, (i + 1) % 30) for i in range(30)]), lambda n: np.full(n, (n - 2) ** 2 / 8)),
    "complete17": (_g(17, list(itertools.combinations(range(17), 2))), lambda n: np.zeros(n)),
    "hypercube6": (_g(64, [(v, v ^ (1 << i)) for v in range(64) for i in range(6) if v < v ^ (1 << i)]),
                   lambda n: np.full(n, (6 * 2 ** 5 - 2 ** 6 + 1) / 2)),
    "k35": (_g(8, [(i, 3 + j) for i in range(3) for j in range(5)]),
            lambda n: np.array([math.comb(5, 2) / 3] * 3 + [math.comb(3, 2) / 5] * 5)),
}


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("name", sorted(CLOSED))
def test_closed_forms(name, engine):
    g, f = CLOSED[name]
    say(f"[closed] {name} engine={engine}")
    bc, st = run_bc(g, None, batch=engine)
    want = f(g.n)
    assert_bc_close(bc / 2.0, want, 1e-12)
    ref, _ = oracle.bc(g)
    assert_bc_close(bc, ref)


@pytest.mark.parametrize("engine", ENGINES)
def test_er2000_all_sources(engine):
    g, srcs = W.workload("er2000")
    say(f"[er2000] engine={engine}")
    ref, modes = oracle.bc(g, srcs)
    bc, st = run_bc(g, srcs, batch=engine)
    say("  stats", st)
    assert_bc_close(bc, ref)
    with b.Graph(g) as G:
        for idx in (0, 77, 1999):
            det = G.detail(srcs, dump_index=idx, batch=engine)
            check_detail(g, det, srcs[idx])


@pytest.mark.parametrize("engine", ENGINES)
def test_policies_and_capture_bit_identical(engine):
    g = W.rmat(12, 16, seed=21)
    srcs = W.choose_sources(g, 200, seed=5)
    say(f"[policies] rmat12 engine={engine}")
    ref, _ = oracle.bc(g, srcs)
    outs = {}
    with b.Graph(g) as G:
        for pol in (b.BC_POLICY_HEURISTIC, b.BC_POLICY_FORCE_PUSH_TPV, b.BC_POLICY_FORCE_PUSH_WPV,
                    b.BC_POLICY_FORCE_PULL):
            for flags in (0, b.BC_RUN_NO_GRAPHS):
                G.run(srcs, batch=engine, policy=pol, flags=flags)
                outs[(pol, flags)] = G.scores().copy()
                st = G.stats()
                if pol == b.BC_POLICY_FORCE_PULL:
                    assert st["variant_levels"][0] == st["variant_levels"][1] == 0
    base = outs[(b.BC_POLICY_HEURISTIC, 0)]
    assert_bc_close(base, ref)
    for k, v in outs.items():
        assert np.array_equal(v.view(np.uint64), base.view(np.uint64)), f"bits differ for {k}"


def test_batch_widths_bit_identical():
    # one state machine: every width adds the same terms in the same order;
    # the default (batches dealt to concurrent replicas, whose score vectors
    # are added at the end) groups the additions per replica instead
    g = W.rmat(12, 16, seed=22)
    srcs = W.choose_sources(g, 150, seed=6)
    say("[widths] rmat12")
    outs = []
    with b.Graph(g) as G:
        for K in (8, 16, 32, 64):
            G.run(srcs, batch=K, flags=b.BC_RUN_ONE_QUEUE)
            outs.append(G.scores().copy())
            assert G.stats()["n_batches"] == -(-150 // K)
        reps = {}
        for K in (16, 64):
            G.run(srcs, batch=K)
            reps[K] = G.scores().copy()
            assert G.stats()["n_batches"] == -(-150 // K)
            G.run(srcs, batch=K)  # run to run: same bits
            assert np.array_equal(G.scores().view(np.uint64), reps[K].view(np.uint64))
    for o in outs[1:]:
        assert np.array_equal(o.view(np.uint64), outs[0].view(np.uint64))
    ref, _ = oracle.bc(g, srcs)
    assert_bc_close(outs[0], ref)
    for r in reps.values():
        assert_bc_close(r, ref)
        assert_bc_close(r, outs[0], 1e-13)


@pytest.mark.parametrize("engine", ENGINES)
def test_rmat_details(engine):
    g = W.rmat(13, 16, seed=23)
    srcs = W.choose_sources(g, 130, seed=7)
    say(f"[rmat13 detail] engine={engine}")
    with b.Graph(g) as G:
        for idx in (0, 63, 64, 129):
            det = G.detail(srcs, dump_index=idx, batch=engine)
            check_detail(g, det, srcs[idx])
        ref, _ = oracle.bc(g, srcs)
        assert_bc_close(G.scores(), ref)


@pytest.mark.parametrize("engine", ENGINES)
def test_hub_first_relabelling_keeps_caller_ids(engine):
    # hubs placed last in the caller's numbering, so the internal renumbering
    # moves them; every output must still be in the caller's ids
    base = W.rmat(12, 16, seed=31)
    deg = np.diff(base.row_ptr)
    order = np.argsort(deg, kind="stable")  # caller id i -> vertex order[i]: hubs get the largest ids
    inv = np.empty_like(order)
    inv[order] = np.arange(base.n)
    src_v = np.repeat(np.arange(base.n), deg)
    g = W.csr_from_edges(base.n, inv[src_v], inv[base.col_idx.astype(np.int64)])
    srcs = W.choose_sources(g, 100, seed=5)
    srcs[3] = base.n - 1  # the largest hub as a source
    say(f"[relabel] engine={engine} n={g.n} max degree {deg.max()}")
    with b.Graph(g) as G, b.Graph(g, flags=b.BC_KEEP_ORDER) as H:
        G.run(srcs, batch=engine)
        got = G.scores()
        H.run(srcs, batch=engine)
        kept = H.scores()
        for idx in (0, 3, 99):
            det = G.detail(srcs, dump_index=idx, batch=engine)
            check_detail(g, det, srcs[idx])
            det_k = H.detail(srcs, dump_index=idx, batch=engine)
            assert np.array_equal(det["d"], det_k["d"])
        G.run(None, batch=engine)
        all_src = G.scores()
    ref, _ = oracle.bc(g, srcs)
    assert_bc_close(got, ref)
    assert_bc_close(kept, ref)
    assert np.max(np.abs(got - kept) / np.maximum(np.abs(kept), 1e-300)) <= 1e-13
    ref_all, _ = oracle.bc(g)
    assert_bc_close(all_src, ref_all)


def test_ranked_sources_make_list_order_irrelevant():
    # a handle with hubs takes the sources in its own rank order, so any
    # permutation of the same list gives the same bits; a caller-order handle
    # (BC_KEEP_ORDER) agrees to rounding
    g = W.rmat(12, 16, seed=43)
    srcs = W.choose_sources(g, 300, seed=9)
    rng = np.random.default_rng(4)
    say(f"[ranked] rmat12 sources={len(srcs)}")
    ref, _ = oracle.bc(g, srcs)
    with b.Graph(g) as G, b.Graph(g, flags=b.BC_KEEP_ORDER) as H:
        G.run(srcs, batch=64, flags=b.BC_RUN_ONE_QUEUE)
        first = G.scores().copy()
        for _ in range(2):
            G.run(rng.permutation(srcs), batch=64, flags=b.BC_RUN_ONE_QUEUE)
            assert np.array_equal(G.scores().view(np.uint64), first.view(np.uint64))
        G.run(rng.permutation(srcs), batch=64)  # concurrent replicas: same K, same bits
        again = G.scores().copy()
        G.run(rng.permutation(srcs), batch=64)
        assert np.array_equal(G.scores().view(np.uint64), again.view(np.uint64))
        H.run(srcs, batch=64)
        kept = H.scores()
        det = G.detail(srcs, dump_index=123, batch=64)  # position in the caller's list
        check_detail(g, det, srcs[123])
    assert_bc_close(first, ref)
    assert np.max(np.abs(first - kept) / np.maximum(np.abs(kept), 1e-300)) <= 1e-13


@pytest.mark.parametrize("engine", ENGINES)
def test_source_transitions_repeatable(engine):
    # every source (plain) or batch (batched) ends with a launch whose last
    # workgroup sets up the next one over words the other workgroups have
    # just reset; repeated runs over many such transitions must agree bit
    # for bit and with the oracle
    g = W.rmat(11, 16, seed=41)
    say(f"[transitions] rmat11 engine={engine} sources={g.n}")
    ref, _ = oracle.bc(g)
    with b.Graph(g) as G:
        first = None
        for rep in range(3):
            G.run(None, batch=engine, flags=b.BC_RUN_ONE_QUEUE)
            x = G.scores().copy()
            assert_bc_close(x, ref)
            if first is None:
                first = x
            assert np.array_equal(x.view(np.uint64), first.view(np.uint64)), f"run {rep} differs"


@pytest.mark.parametrize("engine", ENGINES)
def test_grid_uint64_overflow_fallback(engine):
    L = 40
    g = W.grid(L)
    # corner sources overflow uint64 (C(78, 39) > 2^64); central ones do not
    srcs = np.array([0, L - 1, L * L - 1, 20 * L + 20, 5 * L + 7, 0], dtype=np.int32)
    say(f"[grid40 overflow] engine={engine}")
    ref, modes = oracle.bc(g, srcs)
    assert modes.tolist() == [1, 1, 1, 0, 0, 1]
    with b.Graph(g) as G:
        G.run(srcs, batch=engine)
        assert G.stats()["f64_sources"] == 4
        assert_bc_close(G.scores(), ref)
        for idx in range(len(srcs)):
            det = G.detail(srcs, dump_index=idx, batch=engine)
            check_detail(g, det, srcs[idx])


@pytest.mark.parametrize("engine", ENGINES)
def test_sigma_limit_and_forced_f64(engine):
    g, _ = W.workload("er2000")
    srcs = np.arange(0, 2000, 13, dtype=np.int32)
    ref, _ = oracle.bc(g, srcs)
    say(f"[sigma limit / force f64] engine={engine}")
    with b.Graph(g) as G:
        G.run(srcs, batch=engine, sigma_limit=3)
        st = G.stats()
        assert 0 < st["f64_sources"] <= len(srcs)
        assert_bc_close(G.scores(), ref)
        G.run(srcs, batch=engine, flags=b.BC_RUN_FORCE_F64)
        assert G.stats()["f64_sources"] == len(srcs)
        assert_bc_close(G.scores(), ref)
        det = G.detail(srcs, dump_index=5, batch=engine, flags=b.BC_RUN_FORCE_F64)
        assert det["mode"] == 1
        o = oracle.source(g, int(srcs[5]))
        np.testing.assert_array_equal(det["d"], o.d)
        r = o.d >= 0
        got = np.ldexp(det["sigma_mant"][r], det["sigma_exp"][r])
        np.testing.assert_array_equal(got, o.sigma_u64[r].astype(np.float64))


@pytest.mark.parametrize("engine", ENGINES)
def test_heavy_vertices_segments(engine):
    # RMAT scale 14: vertices above one 1024-arc segment (max degree 3665);
    # every policy must split them the same way and give identical bits
    g = W.rmat(14, 16, seed=1)
    deg = g.degrees()
    hubs = np.argsort(-deg)[:3].astype(np.int32)
    srcs = np.concatenate([hubs, W.choose_sources(g, 90, seed=8)]).astype(np.int32)
    say(f"[heavy] rmat14 max degree {deg.max()} engine={engine}")
    ref, _ = oracle.bc(g, srcs)
    outs = []
    with b.Graph(g) as G:
        for pol in (b.BC_POLICY_HEURISTIC, b.BC_POLICY_FORCE_PUSH_TPV, b.BC_POLICY_FORCE_PUSH_WPV,
                    b.BC_POLICY_FORCE_PULL):
            G.run(srcs, batch=engine, policy=pol)
            outs.append(G.scores().copy())
        assert_bc_close(outs[0], ref)
        for o in outs[1:]:
            assert np.array_equal(o.view(np.uint64), outs[0].view(np.uint64))
        for idx in (0, 1, 50):
            det = G.detail(srcs, dump_index=idx, batch=engine, policy=b.BC_POLICY_FORCE_PULL)
            check_detail(g, det, srcs[idx])
        G.run(srcs[:20], batch=engine, flags=b.BC_RUN_FORCE_F64)
        r20, _ = oracle.bc(g, srcs[:20])
        assert_bc_close(G.scores(), r20)


def test_multi_graph_union_equals_per_graph():
    gs = [W.barabasi_albert(n, 4, seed=30 + i) for i, n in enumerate([60, 300, 150, 1000, 90])]
    gs.append(W.grid(12, 0.1, 0.0, seed=1))
    star = _g(2500, [(0, i) for i in range(1, 2500)] + [(i, i + 1) for i in range(1, 2499, 2)])
    gs.insert(2, star)  # a heavy vertex (degree 2499) inside the union
    u = W.union(gs)
    say("[multi] union of", [x.n for x in gs])
    with b.Graph(u) as G:
        for K in (16, 64):
            G.run(None, batch=K)
            got = G.scores()
            for i, gg in enumerate(gs):
                lo, hi = u.vtx_offsets[i], u.vtx_offsets[i + 1]
                ref, _ = oracle.bc(gg)
                assert_bc_close(got[lo:hi], ref)
        G.run(None, batch=1)
        ref_u, _ = oracle.bc(u)
        assert_bc_close(G.scores(), ref_u)


def test_fp64_first_pass_hands_back_small_counts():
    # a union of an 80 x 80 grid (every source overflows 64 bits) and an R-MAT
    # graph (no source does): the first batch is all grid sources, so the
    # rest runs in FP64 first; R-MAT sources must come back to the 64-bit
    # pass (their mode and integer counts exact), grid sources stay FP64
    grid = W.grid(80, 0.05, 0.0, seed=11)
    rm = W.rmat(10, 8, seed=12)
    u = W.union([grid, rm])
    gsrc = W.choose_sources(grid, 100, seed=1)
    rsrc = W.choose_sources(rm, 40, seed=2) + grid.n
    srcs = np.concatenate([gsrc[:64], rsrc[:20], gsrc[64:], rsrc[20:]]).astype(np.int32)
    say("[fp64 first] grid80 + rmat10, sources", len(srcs))
    ref, modes = oracle.bc(u, srcs)
    assert modes[:64].all() and not modes[64:84].any()
    with b.Graph(u) as G:
        G.run(srcs, batch=64, flags=b.BC_RUN_ONE_QUEUE)  # one list, so the FP64-first pass runs
        st = G.stats()
        assert st["f64_sources"] == int(modes.sum())
        assert_bc_close(G.scores(), ref)
        for idx in (70, 90, 130):  # R-MAT in the FP64-first part, grid, R-MAT at the end
            det = G.detail(srcs, dump_index=idx, batch=64, flags=b.BC_RUN_ONE_QUEUE)
            check_detail(u, det, srcs[idx])
        G.run(srcs, batch=64)  # default path (replicas)
        assert_bc_close(G.scores(), ref)


def test_many_graph_union_parts_bit_identical():
    # 12 graphs of uneven size: the handle runs them as concurrent parts; the
    # scores must equal one state machine's bit for bit and each graph's oracle
    sizes = [50, 700, 120, 3000, 90, 400, 1500, 60, 250, 800, 30, 2200]
    gs = [W.barabasi_albert(n, 4, seed=200 + i) for i, n in enumerate(sizes)]
    gs[5] = W.grid(20, 0.1, 0.0, seed=3)
    u = W.union(gs)
    srcs = np.concatenate([W.choose_sources(u, 600, seed=9), np.arange(0, u.n, 7)]).astype(np.int32)
    say("[parts] union of", len(gs), "graphs, sources", len(srcs))
    with b.Graph(u) as G:
        G.run(srcs, batch=64, flags=b.BC_RUN_ONE_QUEUE)
        one = G.scores().copy()
        G.run(srcs, batch=64, flags=b.BC_RUN_NO_BLOCKS)  # concurrent parts of the general engine
        parts = G.scores().copy()
        assert np.array_equal(one.view(np.uint64), parts.view(np.uint64))
        G.run(srcs[:300], batch=64, flags=b.BC_RUN_NO_BLOCKS)
        G.run(srcs[300:], batch=64, flags=b.BC_RUN_ACCUMULATE | b.BC_RUN_NO_BLOCKS)
        acc = G.scores().copy()
        for idx in (0, 333, len(srcs) - 1):
            det = G.detail(srcs, dump_index=idx, batch=64)
            check_detail(u, det, srcs[idx])
        assert np.array_equal(G.scores().view(np.uint64), parts.view(np.uint64))
    ref, _ = oracle.bc(u, srcs)
    assert_bc_close(parts, ref)
    assert_bc_close(acc, ref)


def test_invalid_inputs_and_handle_survives():
    good = W.grid(4)
    bad_cases = {
        "self_loop": W.CSR(np.array([0, 2, 3], np.int32), np.array([0, 1, 0], np.int32)),
        "asym": W.CSR(np.array([0, 1, 1], np.int32), np.array([1], np.int32)),
        "unsorted": W.CSR(np.array([0, 2, 3, 4], np.int32), np.array([2, 1, 0, 0], np.int32)),
        "dup": W.CSR(np.array([0, 2, 4], np.int32), np.array([1, 1, 0, 0], np.int32)),
        "range": W.CSR(np.array([0, 1, 2], np.int32), np.array([1, 5], np.int32)),
        "nonmono": W.CSR(np.array([0, 2, 1, 2], np.int32), np.array([1, 0], np.int32)),
    }
    for name, g in bad_cases.items():
        say(f"[invalid] {name}")
        with pytest.raises(b.BCError) as ei:
            b.Graph(g)
        assert ei.value.status == 2, name
    with pytest.raises(b.BCError) as ei:
        b.Graph(W.union([W.grid(3), W.grid(3)]), vtx_offsets=[0, 4, 18])
    assert ei.value.status == 2
    with b.Graph(good) as G:
        for bad in ([-1], [16], [3, 99]):
            with pytest.raises(b.BCError) as ei:
                G.run(bad)
            assert ei.value.status == 1
        with pytest.raises(b.BCError):
            G.run([0], batch=3)
        with pytest.raises(b.BCError):
            G.run([0], policy=b.BC_POLICY_MLP)  # no weights loaded
        G.run(None)
        ref, _ = oracle.bc(good)
        assert_bc_close(G.scores(), ref)


def test_degenerate_inputs():
    say("[degenerate]")
    one = W.CSR(np.array([0, 0], np.int32), np.zeros(0, np.int32))
    with b.Graph(one) as G:
        for K in (1, 64):
            G.run([0, 0], batch=K)
            assert G.scores().tolist() == [0.0]
    iso = _g(7, [(0, 1), (1, 2), (4, 5)])  # 3 and 6 isolated
    ref, _ = oracle.bc(iso)
    for K in (1, 8, 64):
        bc, _ = run_bc(iso, None, batch=K)
        assert_bc_close(bc, ref)
    with b.Graph(iso) as G:
        G.run([], batch=64)
        assert (G.scores() == 0).all()
        G.run([3, 3, 6], batch=64)
        assert (G.scores() == 0).all()
    # a handle with hubs ranks its sources: an empty list is still no source
    hub = W.rmat(10, 8, seed=5)
    with b.Graph(hub) as G:
        G.run(W.choose_sources(hub, 10, seed=1), batch=64)
        assert (G.scores() > 0).any()
        for K in (1, 64):
            G.run([], batch=K)
            assert (G.scores() == 0).all()


def test_accumulate_and_duplicates():
    g = W.rmat(11, 8, seed=24)
    s1 = W.choose_sources(g, 70, seed=1)
    s2 = W.choose_sources(g, 40, seed=2)
    say("[accumulate]")
    with b.Graph(g) as G:
        for K in (1, 64):
            G.run(s1, batch=K)
            G.run(s2, batch=K, flags=b.BC_RUN_ACCUMULATE)
            ref, _ = oracle.bc(g, np.concatenate([s1, s2]))
            assert_bc_close(G.scores(), ref)
            dup = np.concatenate([s1[:5], s1[:5]])
            G.run(dup, batch=K)
            r1, _ = oracle.bc(g, s1[:5])
            assert_bc_close(G.scores(), 2 * r1)


def test_torch_device_interop():
    import torch
    g = W.rmat(11, 8, seed=25)
    srcs = W.choose_sources(g, 100, seed=3)
    say("[torch interop]")
    stream = torch.cuda.Stream()
    rp = torch.from_numpy(g.row_ptr.astype(np.int32)).cuda()
    ci = torch.from_numpy(g.col_idx.astype(np.int32)).cuda()
    ref, _ = oracle.bc(g, srcs)
    with torch.cuda.stream(stream):
        with b.Graph(row_ptr=rp, col_idx=ci) as G:
            G.run(srcs, stream=stream, batch=64)
            out = torch.empty(g.n, dtype=torch.float64, device="cuda")
            G.scores(out, stream=stream)
    stream.synchronize()
    assert_bc_close(out.cpu().numpy(), ref)


def test_level_records_add_up_to_run_stats():
    g = W.rmat(12, 16, seed=44)
    srcs = W.choose_sources(g, 300, seed=12)
    say("[level stats] rmat12")
    with b.Graph(g) as G:
        for opts in ({"batch": 64}, {"batch": 64, "flags": b.BC_RUN_ONE_QUEUE}, {"batch": 1}):
            G.run(srcs, **opts)
            st = G.stats()
            lv = G.level_stats()
            L = len(lv["visits"])
            say(f"  {opts}: {L} levels, entries {lv['entries'][:8].tolist()}")
            assert L == st["max_levels"]
            assert int(lv["visits"].sum()) == st["forward_levels"]
            assert int(lv["entries"][1:].sum()) == st["queue_entries"]
            assert lv["variant"].sum(axis=0).tolist() == st["variant_levels"]
            assert int(lv["arcs"].sum()) == st["arcs_scanned"]
            # one forward step per batch (or source) at level 0; K = 1 has one entry per source
            assert int(lv["visits"][0]) == (st["n_batches"] if opts["batch"] > 1 else len(srcs))
            if opts["batch"] == 1:
                assert int(lv["entries"][0]) == len(srcs)
            assert (np.diff(lv["visits"]) <= 0).all()  # every batch that reaches l + 1 reached l
            assert (lv["ms"] >= 0).all() and lv["ms"].sum() > 0


def test_device_limit_refuses_before_allocating_and_falls_back():
    g = W.rmat(12, 16, seed=45)
    srcs = W.choose_sources(g, 400, seed=13)
    say("[device limit] rmat12")
    ref, _ = oracle.bc(g, srcs)
    with b.Graph(g) as G:
        G.run(srcs, batch=64, flags=b.BC_RUN_ONE_QUEUE)
        one = G.scores().copy()
        need = G.info()["device_bytes"]  # graph + one batched engine
    with b.Graph(g) as H:
        base = H.info()["device_bytes"]
        H.set_device_limit(base + (1 << 20))  # far too small for the batched engine
        with pytest.raises(b.BCError) as e:
            H.run(srcs, batch=64)
        assert e.value.status == 3 and "max_device_bytes" in e.value.message
        assert H.info()["device_bytes"] == base  # nothing was allocated
        H.set_device_limit(need + (4 << 20))  # one engine fits, concurrent replicas do not
        H.run(srcs, batch=64)
        assert H.info()["device_bytes"] <= need + (4 << 20)
        assert np.array_equal(H.scores().view(np.uint64), one.view(np.uint64))  # one state machine
        H.set_device_limit(0)
        H.run(srcs, batch=64)  # replicas now
        many = H.scores().copy()
        assert H.info()["device_bytes"] > need + (4 << 20)
        H.set_device_limit(need + (4 << 20))  # the replicas no longer fit: released
        assert H.info()["device_bytes"] <= need + (4 << 20)
        H.run(srcs, batch=64)
        assert np.array_equal(H.scores().view(np.uint64), one.view(np.uint64))
    assert_bc_close(one, ref)
    assert_bc_close(many, ref)


@pytest.mark.parametrize("case", ["grid", "rmat", "grid_f64"])
def test_entry_source_items_same_bits(case):
    # path-count and backward groups summed one thread per (entry, source)
    # pair or one wavefront lane per source: same sums in the same CSR order,
    # so the same bits; details of one source against the oracle
    if case == "rmat":
        g = W.rmat(12, 16, seed=23)
        srcs = W.choose_sources(g, 130, seed=8)
    else:
        g = W.grid(64, 0.1, 0.0 if case == "grid_f64" else 0.002, seed=9)
        srcs = W.choose_sources(g, 130, seed=8)
    flags = b.BC_RUN_ONE_QUEUE | (b.BC_RUN_FORCE_F64 if case == "grid_f64" else 0)
    say(f"[items] {case} n={g.n}")
    outs = {}
    with b.Graph(g) as G:
        for lpe in (-1.0, 0.0, 64.0):
            G.run(srcs, batch=64, flags=flags, lanes_per_entry=lpe)
            outs[lpe] = G.scores().copy()
        if case != "grid_f64":  # forced FP64 mode has no oracle counterpart for small counts
            det = G.detail(srcs, dump_index=77, batch=64, flags=flags, lanes_per_entry=64.0)
            check_detail(g, det, int(srcs[77]))
    for k, v in outs.items():
        assert np.array_equal(v.view(np.uint64), outs[-1.0].view(np.uint64)), f"bits differ for lanes_per_entry={k}"
    ref, _ = oracle.bc(g, srcs)
    assert_bc_close(outs[64.0], ref)
