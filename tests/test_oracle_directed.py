"""Pins for the oracle on directed graphs (paths follow arcs; Eq. 1 over
ordered pairs), checked against things other than itself:

* every digraph on n <= 4 vertices by simple-path enumeration, random
  digraphs up to n = 11 by exact walk counting (tests/brute.py);
* closed forms: the directed path, the directed cycle, out- and in-stars;
* the graph with both arcs of every edge equals the undirected oracle bit
  for bit (same adjacency, same order of every sum);
* networkx's betweenness on directed graphs (ordered pairs, no halving);
* the per-source invariant sum_v delta_s(v) = sum_t (d(s, t) - 1).
"""
from __future__ import annotations

import itertools
import random

import numpy as np
import pytest

import oracle
from brute import bc_by_paths, bc_by_walks
from paper_2008_05718_amd import workloads as W


def _dg(n, arcs):
    a = np.array(arcs, dtype=np.int64).reshape(-1, 2)
    return W.digraph_from_arcs(n, a[:, 0], a[:, 1])


def _close(a, b, rel=1e-12):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300) or a == b


def check_directed_against_exact(n, arcs, bc_exact, dist, cnt):
    g = _dg(n, arcs)
    bc, modes = oracle.bc(g)
    assert not modes.any()
    for v in range(n):
        ex = float(bc_exact[v])
        assert _close(bc[v], ex), (n, arcs, v, bc[v], ex)
        if bc_exact[v] == 0:
            assert bc[v] == 0.0
    for s in range(n):
        det = oracle.source(g, s)
        assert det.d.tolist() == dist[s]
        assert det.sigma_u64.astype(object).tolist() == cnt[s]


def test_all_digraphs_up_to_4_by_path_enumeration():
    for n in range(1, 5):
        pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
        for mask in range(1 << len(pairs)):
            arcs = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
            bcx, dist, cnt = bc_by_paths(n, arcs, directed=True)
            check_directed_against_exact(n, arcs, bcx, dist, cnt)


def random_digraph_trials(count, seed, nmax=11):
    rng = random.Random(seed)
    for _ in range(count):
        n = rng.randint(3, nmax)
        p = rng.uniform(0.15, 0.5)
        arcs = [(a, b) for a in range(n) for b in range(n) if a != b and rng.random() < p]
        yield n, arcs


def test_random_digraphs_by_walk_counting():
    for n, arcs in random_digraph_trials(150, seed=11):
        bcx, dist, cnt = bc_by_walks(n, arcs, directed=True)
        check_directed_against_exact(n, arcs, bcx, dist, cnt)


def test_walks_agree_with_paths_on_digraphs():
    for n, arcs in random_digraph_trials(40, seed=12, nmax=6):
        a = bc_by_paths(n, arcs, directed=True)
        b = bc_by_walks(n, arcs, directed=True)
        assert a[0] == b[0] and a[1] == b[1] and a[2] == b[2]


@pytest.mark.parametrize("n", [2, 7, 40])
def test_directed_path(n):
    bc, _ = oracle.bc(_dg(n, [(i, i + 1) for i in range(n - 1)]))
    assert bc.tolist() == [float(i * (n - 1 - i)) for i in range(n)]


@pytest.mark.parametrize("n", [3, 8, 31])
def test_directed_cycle(n):
    # every ordered pair has one path; each vertex is interior to (n-1)(n-2)/2 of them
    bc, _ = oracle.bc(_dg(n, [(i, (i + 1) % n) for i in range(n)]))
    assert np.all(bc == (n - 1) * (n - 2) / 2)


@pytest.mark.parametrize("n", [5, 20])
def test_stars(n):
    out_star = _dg(n, [(0, i) for i in range(1, n)])
    in_star = _dg(n, [(i, 0) for i in range(1, n)])
    both = _dg(n, [(0, i) for i in range(1, n)] + [(i, 0) for i in range(1, n)])
    assert not oracle.bc(out_star)[0].any() and not oracle.bc(in_star)[0].any()
    bc, _ = oracle.bc(both)
    assert bc[0] == (n - 1) * (n - 2) and not bc[1:].any()


def test_both_arcs_equal_the_undirected_oracle_bitwise():
    u = W.rmat(10, 8, seed=14)
    src_v = np.repeat(np.arange(u.n), np.diff(u.row_ptr))
    d = W.digraph_from_arcs(u.n, src_v, u.col_idx)
    assert np.array_equal(d.row_ptr, u.row_ptr) and np.array_equal(d.in_col_idx, u.col_idx)
    srcs = W.choose_sources(u, 30, seed=1)
    a, _ = oracle.bc(u, srcs)
    b, _ = oracle.bc(d, srcs)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_directed_matches_networkx():
    nx = pytest.importorskip("networkx")
    g = W.rmat_directed(9, 6, seed=15)
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    for v in range(g.n):
        for w in g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]:
            G.add_edge(v, int(w))
    ref = nx.betweenness_centrality(G, normalized=False)
    bc, _ = oracle.bc(g)
    for v in range(g.n):
        assert _close(bc[v], ref[v], 1e-10), (v, bc[v], ref[v])


def test_directed_invariant_and_asymmetry():
    g = W.rmat_directed(11, 8, seed=16)
    assert not np.array_equal(g.row_ptr, g.in_row_ptr)  # genuinely directed
    srcs = W.choose_sources(g, 20, seed=2)
    ex = oracle.path_excess(g, srcs)
    for s, e in zip(srcs, ex):
        det = oracle.source(g, int(s))
        assert _close(float(np.sum(det.delta[det.d > 0])), float(e), 1e-11)
