"""Pins for the oracle on graphs with positive integer arc weights (the
forward phase as a single-source shortest-path computation), checked against
things other than itself:

* brute force: every graph on n <= 4 vertices with weights in {1, 2} and
  random graphs with n = 5, 6 by simple-path enumeration; random graphs up to
  n = 11 (undirected and directed) by counting walks of each total weight;
* unit weights reduce to the unweighted oracle, bit for bit (same
  adjacency, same order of every sum);
* scaling every weight by 3 scales distances by 3 and leaves path counts and
  scores unchanged, bit for bit;
* a weighted path and a weighted tree have the unweighted scores (one path
  per pair whatever the weights);
* library routines: scipy's Dijkstra distances and networkx's weighted
  betweenness (which halves undirected sums);
* planted mistakes in the weighted code must fail these pins.
"""
from __future__ import annotations

import itertools
import os
import random
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from brute import bc_by_weighted_paths, bc_by_weighted_walks
from paper_2008_05718_amd import workloads as W

REL = 1e-12


def _close(a, b, rel=REL):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300) or a == b


def _weighted(n, edges, weights, directed):
    """CSR with the given edge weights (undirected: both arcs)."""
    e = np.array(edges, dtype=np.int64).reshape(-1, 2)
    g = W.digraph_from_arcs(n, e[:, 0], e[:, 1]) if directed else W.csr_from_edges(n, e[:, 0], e[:, 1])
    wmap = {}
    for (a, b), w in zip(edges, weights):
        wmap[(a, b)] = w
        if not directed:
            wmap[(b, a)] = w
    rp = g.row_ptr.astype(np.int64)
    src = np.repeat(np.arange(n), np.diff(rp))
    g.weights = np.array([wmap[(int(a), int(b))] for a, b in zip(src, g.col_idx)], np.int32)
    if directed:
        irp = g.in_row_ptr.astype(np.int64)
        head = np.repeat(np.arange(n), np.diff(irp))
        g.in_weights = np.array([wmap[(int(t), int(h))] for t, h in zip(g.in_col_idx, head)], np.int32)
    return g


def check_weighted(n, edges, weights, directed, exact):
    bcx, dist, cnt = exact
    g = _weighted(n, edges, weights, directed)
    bc, modes = oracle.bc(g)
    assert not modes.any()
    for v in range(n):
        ex = float(bcx[v])
        assert _close(bc[v], ex), (n, edges, weights, v, bc[v], ex)
        if bcx[v] == 0:
            assert bc[v] == 0.0
    for s in range(n):
        det = oracle.source(g, s)
        assert det.d.tolist() == dist[s], (s, det.d.tolist(), dist[s])
        assert det.sigma_u64.astype(object).tolist() == cnt[s]


def _simple_edges(n, edges):
    return [(a, b) for a, b in edges if a != b]


def test_small_weighted_graphs_by_path_enumeration():
    for n in range(2, 5):
        pairs = list(itertools.combinations(range(n), 2))
        for mask in range(1 << len(pairs)):
            edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
            for wmask in range(1 << len(edges)):
                ws = [1 + (wmask >> i & 1) for i in range(len(edges))]
                check_weighted(n, edges, ws, False, bc_by_weighted_paths(n, edges, ws))
    rng = random.Random(3)
    for _ in range(150):
        n = rng.randint(5, 6)
        directed = rng.random() < 0.5
        cand = [(a, b) for a in range(n) for b in range(n) if a != b] if directed else \
            list(itertools.combinations(range(n), 2))
        edges = [e for e in cand if rng.random() < 0.45]
        ws = [rng.randint(1, 3) for _ in edges]
        check_weighted(n, edges, ws, directed, bc_by_weighted_paths(n, edges, ws, directed))


def random_weighted_trials(count, seed, nmax=11):
    rng = random.Random(seed)
    for _ in range(count):
        n = rng.randint(4, nmax)
        directed = rng.random() < 0.5
        p = rng.uniform(0.2, 0.6)
        cand = [(a, b) for a in range(n) for b in range(n) if a != b] if directed else \
            list(itertools.combinations(range(n), 2))
        edges = [e for e in cand if rng.random() < p]
        ws = [rng.randint(1, 4) for _ in edges]
        yield n, edges, ws, directed


def test_random_weighted_graphs_by_walk_counting():
    for n, edges, ws, directed in random_weighted_trials(120, seed=11):
        check_weighted(n, edges, ws, directed, bc_by_weighted_walks(n, edges, ws, directed))


@pytest.mark.parametrize("directed", [False, True])
def test_unit_weights_equal_the_unweighted_oracle(directed):
    g = W.rmat_directed(9, 8, seed=4) if directed else W.rmat(9, 8, seed=4)
    gw = W.with_weights(g, 1, 1, seed=1)
    srcs = W.choose_sources(g, 60, seed=2)
    a, ma = oracle.bc(g, srcs)
    b, mb = oracle.bc(gw, srcs)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64)) and np.array_equal(ma, mb)
    for s in srcs[:5]:
        x, y = oracle.source(g, int(s)), oracle.source(gw, int(s))
        assert np.array_equal(x.d.astype(np.int64), y.d) and np.array_equal(x.sigma_u64, y.sigma_u64)
        assert np.array_equal(x.delta.view(np.uint64), y.delta.view(np.uint64))


@pytest.mark.parametrize("directed", [False, True])
def test_scaled_weights_keep_counts_and_scores(directed):
    g = W.rmat_directed(9, 8, seed=5) if directed else W.rmat(9, 8, seed=5)
    gw = W.with_weights(g, 1, 5, seed=3)
    g3 = W.with_weights(g, 1, 5, seed=3)
    g3.weights = gw.weights * 3
    if directed:
        g3.in_weights = gw.in_weights * 3
    srcs = W.choose_sources(g, 50, seed=2)
    a, _ = oracle.bc(gw, srcs)
    b, _ = oracle.bc(g3, srcs)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    for s in srcs[:4]:
        x, y = oracle.source(gw, int(s)), oracle.source(g3, int(s))
        r = x.d >= 0
        assert np.array_equal(x.d[r] * 3, y.d[r]) and np.array_equal(x.sigma_u64, y.sigma_u64)


def test_weighted_path_and_tree_keep_unweighted_scores():
    rng = np.random.default_rng(7)
    n = 40
    path = [(i, i + 1) for i in range(n - 1)]
    g = _weighted(n, path, [int(x) for x in rng.integers(1, 9, n - 1)], False)
    bc, _ = oracle.bc(g)
    np.testing.assert_array_equal(bc, [2.0 * i * (n - 1 - i) for i in range(n)])
    parent = [int(rng.integers(0, i)) for i in range(1, 60)]
    tree = [(p, i + 1) for i, p in enumerate(parent)]
    t_unw = W.csr_from_edges(60, np.array([e[0] for e in tree]), np.array([e[1] for e in tree]))
    t_w = _weighted(60, tree, [int(x) for x in rng.integers(1, 20, len(tree))], False)
    a, _ = oracle.bc(t_unw)
    b, _ = oracle.bc(t_w)
    assert np.array_equal(a, b)


def test_distances_match_scipy_dijkstra():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    for directed in (False, True):
        g = W.rmat_directed(10, 8, seed=6) if directed else W.rmat(10, 8, seed=6)
        gw = W.with_weights(g, 1, 50, seed=4)
        A = csr_matrix((gw.weights.astype(np.float64), gw.col_idx, gw.row_ptr), shape=(g.n, g.n))
        srcs = W.choose_sources(g, 12, seed=1)
        D = dijkstra(A, directed=True, indices=srcs)
        for k, s in enumerate(srcs):
            det = oracle.source(gw, int(s))
            want = np.where(np.isfinite(D[k]), D[k], -1).astype(np.int64)
            assert np.array_equal(det.d, want)


def test_networkx_weighted_betweenness():
    import networkx as nx
    for directed in (False, True):
        g = W.rmat_directed(8, 6, seed=8) if directed else W.rmat(8, 6, seed=8)
        gw = W.with_weights(g, 1, 4, seed=5)
        G = nx.DiGraph() if directed else nx.Graph()
        G.add_nodes_from(range(g.n))
        rp = gw.row_ptr.astype(np.int64)
        for v in range(g.n):
            for e in range(rp[v], rp[v + 1]):
                G.add_edge(v, int(gw.col_idx[e]), weight=int(gw.weights[e]))
        ref = nx.betweenness_centrality(G, weight="weight", normalized=False)
        bc, _ = oracle.bc(gw)
        scale = 1.0 if directed else 2.0  # networkx halves undirected sums
        for v in range(g.n):
            assert _close(bc[v], scale * ref[v], 1e-9), (directed, v, bc[v], ref[v])


WMUTATIONS = {
    "hop_distance": ("const int64_t nd = d + (int64_t)w->wt[e];", "const int64_t nd = d + 1;"),
    "pred_ignores_weight": ("if (w->dist[v] < 0 || w->dist[v] + (int64_t)w->in_wt[e] != w->dist[t]) continue;",
                            "if (w->dist[v] < 0 || w->dist[v] >= w->dist[t]) continue;"),
    "succ_ignores_weight": ("if (w->dist[u] != w->dist[v] + (int64_t)w->wt[e]) continue; /* not a successor */",
                            "if (w->dist[u] <= w->dist[v]) continue; /* not a successor */"),
    "settle_first_copy": ("if (w->done[v] || d != w->dist[v]) continue; /* a stale copy */",
                          "if (0) continue; /* a stale copy */"),
}


@pytest.mark.parametrize("name", sorted(WMUTATIONS))
def test_planted_weighted_mistake_is_caught(name, monkeypatch):
    old, new = WMUTATIONS[name]
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
        try:
            for n, edges, ws, directed in random_weighted_trials(60, seed=13, nmax=8):
                check_weighted(n, edges, ws, directed, bc_by_weighted_walks(n, edges, ws, directed))
        except AssertionError:
            caught = True
        monkeypatch.setattr(oracle, "_lib", None)
    assert caught, f"mutation {name} was not detected by the pins"
