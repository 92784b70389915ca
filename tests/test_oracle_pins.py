"""Pins for the CPU oracle: it is checked against things other than itself.

* brute force: every labelled graph on n <= 5 vertices by simple-path
  enumeration (Eq. 1 literally), random graphs up to n = 14 by exact walk
  counting;
* closed forms for path, star, complete, cycle, complete bipartite,
  hypercube and grid graphs;
* the uint64 overflow threshold of the corner-sourced grid;
* the per-source invariant sum_v delta_s(v) = sum_t (d(s, t) - 1);
* library routines: scipy's unweighted shortest paths (d) and networkx's
  betweenness (which halves undirected sums);
* planted mistakes: mutated copies of the oracle source must fail the pins.
"""
from __future__ import annotations

import itertools
import math
import os
import random
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from brute import bc_by_paths, bc_by_walks
from paper_2008_05718_amd import workloads as W

REL = 1e-12


def _g(n, edges):
    e = np.array(edges, dtype=np.int64).reshape(-1, 2)
    return W.csr_from_edges(n, e[:, 0], e[:, 1])


def _close(a, b, rel=REL):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300) or a == b


def _check_against_exact(n, edges, bc_exact, dist, cnt):
    g = _g(n, edges)
    bc, modes = oracle.bc(g)
    assert not modes.any()
    for v in range(n):
        ex = float(bc_exact[v])
        assert _close(bc[v], ex), (n, edges, v, bc[v], ex)
        if bc_exact[v] == 0:
            assert bc[v] == 0.0
    for s in range(n):
        det = oracle.source(g, s)
        assert det.d.tolist() == dist[s]
        assert det.sigma_u64.astype(object).tolist() == cnt[s]


def test_all_graphs_up_to_5_by_path_enumeration():
    for n in range(1, 6):
        pairs = list(itertools.combinations(range(n), 2))
        for mask in range(1 << len(pairs)):
            edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
            bcx, dist, cnt = bc_by_paths(n, edges)
            _check_against_exact(n, edges, bcx, dist, cnt)


def test_random_graphs_by_walk_counting():
    rng = random.Random(12345)
    for trial in range(120):
        n = rng.randint(6, 14)
        p = rng.choice([0.15, 0.3, 0.5, 0.8])
        edges = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < p]
        bcx, dist, cnt = bc_by_walks(n, edges)
        _check_against_exact(n, edges, bcx, dist, cnt)


def test_path_enumeration_agrees_with_walks():
    # the two definition-level checkers pin each other on n = 6
    rng = random.Random(7)
    for _ in range(40):
        edges = [(a, b) for a, b in itertools.combinations(range(6), 2) if rng.random() < 0.5]
        a = bc_by_paths(6, edges)
        b = bc_by_walks(6, edges)
        assert a[0] == b[0] and a[1] == b[1] and a[2] == b[2]


# ------------------------------------------------------------- closed forms
def _raw_half(bc):
    return bc / 2.0  # ordered-pair sums -> unordered-pair values


@pytest.mark.parametrize("n", [2, 3, 7, 50])
def test_path_graph(n):
    g = _g(n, [(i, i + 1) for i in range(n - 1)])
    bc, _ = oracle.bc(g)
    for i in range(n):
        assert _raw_half(bc)[i] == i * (n - 1 - i)


@pytest.mark.parametrize("n", [3, 4, 11, 40])
def test_star(n):
    g = _g(n, [(0, i) for i in range(1, n)])
    bc, _ = oracle.bc(g)
    assert _raw_half(bc)[0] == (n - 1) * (n - 2) / 2
    assert (bc[1:] == 0).all()


@pytest.mark.parametrize("n", [2, 5, 17])
def test_complete(n):
    g = _g(n, list(itertools.combinations(range(n), 2)))
    bc, _ = oracle.bc(g)
    assert (bc == 0).all()
    for s in (0, n - 1):
        det = oracle.source(g, s)
        assert (det.sigma_u64 == 1).all()


@pytest.mark.parametrize("n", [5, 9, 21, 4, 10, 30])
def test_cycle(n):
    g = _g(n, [(i, (i + 1) % n) for i in range(n)])
    bc, _ = oracle.bc(g)
    want = (n - 1) * (n - 3) / 8 if n % 2 else (n - 2) ** 2 / 8
    assert np.allclose(_raw_half(bc), want, rtol=REL, atol=0)
    if n % 2 == 0:
        det = oracle.source(g, 0)
        assert det.sigma_u64[n // 2] == 2  # antipode has two shortest paths


@pytest.mark.parametrize("a,b", [(1, 4), (2, 3), (3, 5), (6, 2)])
def test_complete_bipartite(a, b):
    edges = [(i, a + j) for i in range(a) for j in range(b)]
    g = _g(a + b, edges)
    bc, _ = oracle.bc(g)
    half = _raw_half(bc)
    # side-A vertex: C(b,2)/a ; side-B vertex: C(a,2)/b
    assert np.allclose(half[:a], math.comb(b, 2) / a, rtol=REL, atol=0)
    assert np.allclose(half[a:], math.comb(a, 2) / b, rtol=REL, atol=0)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
def test_hypercube(k):
    n = 1 << k
    edges = [(v, v ^ (1 << i)) for v in range(n) for i in range(k) if v < v ^ (1 << i)]
    g = _g(n, edges)
    bc, _ = oracle.bc(g)
    want = (k * 2 ** (k - 1) - 2 ** k + 1) / 2
    assert np.allclose(_raw_half(bc), want, rtol=REL, atol=0)
    det = oracle.source(g, 0)
    for v in range(n):
        h = bin(v).count("1")
        assert det.d[v] == h and det.sigma_u64[v] == math.factorial(h)


@pytest.mark.parametrize("L", [2, 5, 16])
def test_intact_grid_from_corner(L):
    g = W.grid(L)
    det = oracle.source(g, 0)
    for i in range(L):
        for j in range(L):
            v = i * L + j
            assert det.d[v] == i + j
            assert int(det.sigma_u64[v]) == math.comb(i + j, i)


def test_uint64_overflow_threshold():
    # corner-sourced L x L grid: sigma(i, j) = C(i + j, i).  C(67,33) < 2^64 - 1
    # < C(68,34), so L = 34 (max i + j = 66) stays in uint64 and L = 35 does not.
    assert math.comb(67, 33) < 2**64 - 1 < math.comb(68, 34)
    g34 = W.grid(34)
    d34 = oracle.source(g34, 0)
    assert d34.mode == 0
    assert int(d34.sigma_u64[33 * 34 + 33]) == math.comb(66, 33)
    g35 = W.grid(35)
    d35 = oracle.source(g35, 0)
    assert d35.mode == 1
    for (i, j) in [(34, 34), (34, 33), (20, 30), (0, 34)]:
        exact = np.longdouble(str(math.comb(i + j, i)))
        got = d35.sigma_ld[i * 35 + j]
        assert abs(got - exact) <= exact * np.longdouble(2.0) ** -60


def _invariant_check(g, sources):
    for s in sources:
        det = oracle.source(g, int(s))
        reach = det.d > 0
        want = float(np.sum(det.d[reach] - 1, dtype=np.float64))
        mask = det.d > 0
        got = float(np.sum(det.delta[mask], dtype=np.float64))
        assert _close(got, want, 1e-11), (s, got, want)


def test_dependency_sum_invariant_rmat_er():
    g = W.rmat(12, 16, seed=77)
    _invariant_check(g, W.choose_sources(g, 12, seed=9))
    g = W.erdos_renyi(500, 6.0, seed=3)
    _invariant_check(g, range(0, 500, 50))


def test_dependency_sum_invariant_f64_mode():
    g = W.grid(40)  # corner sources overflow uint64
    det = oracle.source(g, 0)
    assert det.mode == 1
    _invariant_check(g, [0, 40 * 40 - 1, 20 * 40 + 20])


def test_distances_match_scipy():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    g = W.rmat(11, 8, seed=5)
    A = csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    srcs = W.choose_sources(g, 6, seed=1)
    D = shortest_path(A, unweighted=True, indices=srcs)
    for k, s in enumerate(srcs):
        det = oracle.source(g, int(s))
        want = np.where(np.isinf(D[k]), -1, D[k]).astype(np.int64)
        assert (det.d == want).all()


def test_er2000_matches_networkx():
    import networkx as nx
    g = W.erdos_renyi(2000, 8.0, seed=1)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for v in range(g.n):
        for w in g.neighbors(v):
            if v < w:
                G.add_edge(v, int(w))
    ref = nx.betweenness_centrality(G, normalized=False)
    bc, modes = oracle.bc(g)
    assert not modes.any()
    for v in range(g.n):
        assert _close(bc[v] / 2.0, ref[v], 1e-11), (v, bc[v] / 2, ref[v])


def test_small_ba_matches_networkx_with_subset_sources():
    import networkx as nx
    g = W.barabasi_albert(300, 4, seed=11)
    G = nx.Graph()
    for v in range(g.n):
        for w in g.neighbors(v):
            if v < w:
                G.add_edge(v, int(w))
    ref = nx.betweenness_centrality(G, normalized=False)
    bc, _ = oracle.bc(g)
    for v in range(g.n):
        assert _close(bc[v] / 2.0, ref[v], 1e-11)


def test_f64_mode_grid_matches_networkx():
    # 36 x 36 grid: sources near a corner overflow uint64 (path counts up to
    # C(70, 35) ~ 1.1e20); networkx accumulates path counts in double.
    import networkx as nx
    L = 36
    g = W.grid(L)
    G = nx.grid_2d_graph(L, L)
    G = nx.relabel_nodes(G, {(i, j): i * L + j for i in range(L) for j in range(L)})
    srcs = [0, 1, L, L * L - 1, L * L - 2, 17 * L + 5, 3 * L + 30]
    ref = nx.betweenness_centrality_subset(G, sources=srcs, targets=list(G.nodes()), normalized=False)
    bc, modes = oracle.bc(g, srcs)
    assert modes.tolist() == [1, 1, 1, 1, 1, 0, 0]
    for v in range(g.n):
        assert _close(bc[v] / 2.0, ref[v], 1e-11), (v, bc[v] / 2, ref[v])


def test_sources_subset_and_duplicates_sum():
    g = W.erdos_renyi(120, 5.0, seed=2)
    a, _ = oracle.bc(g, [3, 7])
    b, _ = oracle.bc(g, [3])
    c, _ = oracle.bc(g, [7])
    assert np.allclose(a, b + c, rtol=1e-14, atol=0)
    d, _ = oracle.bc(g, [3, 3])
    assert np.allclose(d, 2 * b, rtol=1e-14, atol=0)


def test_disconnected_graph_unreachable_pairs_contribute_zero():
    # two disjoint paths: BC of each is its own path BC
    edges = [(0, 1), (1, 2), (3, 4), (4, 5), (5, 6)]
    g = _g(8, edges)  # vertex 7 isolated
    bc, _ = oracle.bc(g)
    assert list(bc / 2) == [0, 1, 0, 0, 2, 2, 0, 0]


# ---------------------------------------------------------- planted mistakes
MUTATIONS = {
    "drop_one_plus": ("(1.0 + w->dep_d[u])", "(w->dep_d[u])"),
    "inverted_ratio": ("((double)w->sig_u[v] / (double)w->sig_u[u])", "((double)w->sig_u[u] / (double)w->sig_u[v])"),
    "wrong_successor": ("if (w->dist[u] != w->dist[v] + 1) continue;",
                        "if (w->dist[u] != w->dist[v] + 1 && w->dist[u] != w->dist[v]) continue;"),
    "wrong_predecessor": ("if (w->dist[v] != w->dist[t] - 1) continue;", "if (w->dist[v] > w->dist[t]) continue;"),
    "count_source": ("for (int64_t i = 1; i < w.n_reached; ++i)", "for (int64_t i = 0; i < w.n_reached; ++i)"),
    "sigma_one_term": ("} else if (__builtin_add_overflow(su, w->sig_u[v], &su)) {",
                       "} else if ((su = w->sig_u[v]), 0) {"),
    "forward_order": ("for (int64_t k = w->n_reached - 1; k >= 0; --k) {", "for (int64_t k = 0; k < w->n_reached; ++k) {"),
    "sigma_over_out_arcs": ("for (int64_t e = w->in_row_ptr[t]; e < w->in_row_ptr[t + 1]; ++e) {\n            const int32_t v = w->in_col[e];",
                            "for (int64_t e = w->row_ptr[t]; e < w->row_ptr[t + 1]; ++e) {\n            const int32_t v = w->col[e];"),
    "distance_step": ("w->dist[x] = w->dist[v] + 1;\n                w->order", "w->dist[x] = w->dist[v] + 2;\n                w->order"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    old, new = MUTATIONS[name]
    src = open(os.path.join(os.path.dirname(oracle.__file__), "bc_oracle.c")).read()
    assert old in src, name
    with tempfile.TemporaryDirectory() as td:
        cpath = os.path.join(td, "m.c")
        so = os.path.join(td, "m.so")
        open(cpath, "w").write(src.replace(old, new))
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", cpath, "-o", so, "-lm"])
        monkeypatch.setattr(oracle, "_LIB", so)
        monkeypatch.setattr(oracle, "_lib", None)
        caught = False
        rng = random.Random(5)
        try:
            for trial in range(60):
                n = rng.randint(4, 8)
                edges = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < 0.45]
                bcx, dist, cnt = bc_by_walks(n, edges)
                _check_against_exact(n, edges, bcx, dist, cnt)
            # the directed pins (some mistakes only show when arcs are one-way)
            from test_oracle_directed import check_directed_against_exact, random_digraph_trials
            for n, arcs in random_digraph_trials(60, seed=7, nmax=8):
                bcx, dist, cnt = bc_by_walks(n, arcs, directed=True)
                check_directed_against_exact(n, arcs, bcx, dist, cnt)
        except AssertionError:
            caught = True
        monkeypatch.setattr(oracle, "_lib", None)
    assert caught, f"mutation {name} was not detected by the pins"


def test_path_excess_matches_scipy_and_closed_form():
    # the BFS-only checker used for full-size runs: scipy's unweighted
    # shortest paths (library routine) and the intact grid seen from a corner
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    g = W.union([W.rmat(10, 8, seed=8), W.erdos_renyi(300, 3.0, seed=2)])
    A = csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    srcs = W.choose_sources(g, 40, seed=3)
    D = shortest_path(A, unweighted=True, indices=srcs)
    want = [int(np.sum(row[np.isfinite(row) & (row > 0)] - 1)) for row in D]
    assert oracle.path_excess(g, srcs, threads=3).tolist() == want
    L = 30
    closed = sum(i + j - 1 for i in range(L) for j in range(L) if i + j > 0)
    assert oracle.path_excess(W.grid(L), [0]).tolist() == [closed]


def test_path_excess_equals_dependency_sums():
    g = W.rmat(11, 16, seed=21)
    srcs = W.choose_sources(g, 16, seed=5)
    ex = oracle.path_excess(g, srcs, threads=4)
    for s, e in zip(srcs, ex):
        det = oracle.source(g, int(s))
        assert _close(float(np.sum(det.delta[det.d > 0])), float(e), 1e-11)


def test_sliced_oracle_matches_single_thread():
    # the threaded helper used for large parity checks: same terms, grouped
    # per slice, so it agrees with the single-threaded oracle to rounding
    g = W.rmat(11, 16, seed=12)
    srcs = W.choose_sources(g, 37, seed=2)
    one, m1 = oracle.bc(g, srcs)
    many, m2 = oracle.bc_sliced(g, srcs, threads=5)
    assert np.array_equal(m1, m2)
    for v in range(g.n):
        assert _close(one[v], many[v], 1e-13)
        assert (one[v] == 0) == (many[v] == 0)
