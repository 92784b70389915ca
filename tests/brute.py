"""Definition-level checkers that pin the CPU oracle (pure Python, exact).

Neither function uses the Brandes recursion; both evaluate Eq. 1 of the paper
(Section "Background") directly:

    BC[v] = sum over ordered pairs s != v != t with sigma_st > 0 of
            sigma_st(v) / sigma_st

* ``bc_by_paths`` enumerates every simple path of the graph (depth-first),
  keeps the shortest ones per ordered pair, and counts them, and the ones
  through v, literally.  Exponential: only for n <= 6.
* ``bc_by_walks`` uses the textbook fact that every walk of length d(s, t)
  between s and t is a shortest path, so sigma_st = (A^d)[s, t] with
  d = min{k : (A^k)[s, t] > 0}, and a shortest s-t path passes through v iff
  d(s, v) + d(v, t) = d(s, t), in which case sigma_st(v) = sigma_sv * sigma_vt.
  Python integers keep every count exact.

Both return exact Fractions (ordered-pair convention), the distance matrix
(-1 = unreachable) and the path-count matrix.  With directed=True an edge
(a, b) is the arc a -> b only, and paths follow arcs.
"""
from __future__ import annotations

from fractions import Fraction


def _adj_lists(n, edges, directed=False):
    adj = [set() for _ in range(n)]
    for a, b in edges:
        if a != b:
            adj[a].add(b)
            if not directed:
                adj[b].add(a)
    return [sorted(x) for x in adj]


def bc_by_paths(n, edges, directed=False):
    adj = _adj_lists(n, edges, directed)
    # best[s][t] = (length, count, through-count list)
    dist = [[-1] * n for _ in range(n)]
    cnt = [[0] * n for _ in range(n)]
    through = [[[0] * n for _ in range(n)] for _ in range(n)]
    for s in range(n):
        dist[s][s] = 0
        cnt[s][s] = 1
        stack = [(s, [s])]
        while stack:
            v, path = stack.pop()
            for w in adj[v]:
                if w in path:
                    continue
                p2 = path + [w]
                L = len(p2) - 1
                if dist[s][w] == -1 or L < dist[s][w]:
                    dist[s][w] = L
                    cnt[s][w] = 0
                    through[s][w] = [0] * n
                if L == dist[s][w]:
                    cnt[s][w] += 1
                    for x in p2[1:-1]:
                        through[s][w][x] += 1
                stack.append((w, p2))
    bc = [Fraction(0)] * n
    for s in range(n):
        for t in range(n):
            if s == t or cnt[s][t] == 0:
                continue
            for v in range(n):
                if v != s and v != t and through[s][t][v]:
                    bc[v] += Fraction(through[s][t][v], cnt[s][t])
    return bc, dist, cnt


def bc_by_walks(n, edges, directed=False):
    A = [[0] * n for _ in range(n)]
    for a, b in edges:
        if a != b:
            A[a][b] = 1
            if not directed:
                A[b][a] = 1
    dist = [[-1] * n for _ in range(n)]
    cnt = [[0] * n for _ in range(n)]
    P = [[1 if i == j else 0 for j in range(n)] for i in range(n)]  # A^0
    for k in range(n):
        for s in range(n):
            for t in range(n):
                if dist[s][t] == -1 and P[s][t] > 0:
                    dist[s][t] = k
                    cnt[s][t] = P[s][t]
        # P <- P * A
        P = [[sum(P[i][l] * A[l][j] for l in range(n) if P[i][l]) for j in range(n)]
             for i in range(n)]
    bc = [Fraction(0)] * n
    for s in range(n):
        for t in range(n):
            if s == t or dist[s][t] < 0:
                continue
            for v in range(n):
                if v in (s, t) or dist[s][v] < 0 or dist[v][t] < 0:
                    continue
                if dist[s][v] + dist[v][t] == dist[s][t]:
                    bc[v] += Fraction(cnt[s][v] * cnt[v][t], cnt[s][t])
    return bc, dist, cnt


def _weighted_arcs(n, edges, weights, directed):
    arcs = {}
    for (a, b), w in zip(edges, weights):
        if a == b:
            continue
        arcs[(a, b)] = w
        if not directed:
            arcs[(b, a)] = w
    out = [[] for _ in range(n)]
    for (a, b), w in sorted(arcs.items()):
        out[a].append((b, w))
    return out


def bc_by_weighted_paths(n, edges, weights, directed=False):
    """Eq. 1 on a graph with positive integer arc weights by enumerating
    every simple path: per ordered pair the minimum total weight, the number
    of simple paths of that weight, and how many of them pass through each
    vertex.  Exponential: only for n <= 6."""
    adj = _weighted_arcs(n, edges, weights, directed)
    dist = [[-1] * n for _ in range(n)]
    cnt = [[0] * n for _ in range(n)]
    through = [[[0] * n for _ in range(n)] for _ in range(n)]
    for s in range(n):
        dist[s][s] = 0
        cnt[s][s] = 1
        stack = [(s, [s], 0)]
        while stack:
            v, path, L0 = stack.pop()
            for w, wt in adj[v]:
                if w in path:
                    continue
                p2 = path + [w]
                L = L0 + wt
                if dist[s][w] == -1 or L < dist[s][w]:
                    dist[s][w] = L
                    cnt[s][w] = 0
                    through[s][w] = [0] * n
                if L == dist[s][w]:
                    cnt[s][w] += 1
                    for x in p2[1:-1]:
                        through[s][w][x] += 1
                stack.append((w, p2, L))
    bc = [Fraction(0)] * n
    for s in range(n):
        for t in range(n):
            if s == t or cnt[s][t] == 0:
                continue
            for v in range(n):
                if v != s and v != t and through[s][t][v]:
                    bc[v] += Fraction(through[s][t][v], cnt[s][t])
    return bc, dist, cnt


def bc_by_weighted_walks(n, edges, weights, directed=False):
    """Eq. 1 by counting walks of each total weight: with positive weights a
    walk of the least total weight between s and t repeats no vertex, so the
    shortest s-t paths are exactly the s-t walks of total weight d(s, t).
    W[k][t] (walks from s of weight k ending at t) follows
    W[k][t] = sum over arcs v -> t of weight w <= k of W[k - w][v].  A
    shortest path passes through v iff d(s, v) + d(v, t) = d(s, t), then
    sigma_st(v) = sigma_sv * sigma_vt.  Python integers keep counts exact."""
    adj = _weighted_arcs(n, edges, weights, directed)
    into = [[] for _ in range(n)]
    for v in range(n):
        for t, w in adj[v]:
            into[t].append((v, w))
    maxw = max([w for lst in adj for _, w in lst], default=1)
    kmax = maxw * max(n - 1, 1)
    dist = [[-1] * n for _ in range(n)]
    cnt = [[0] * n for _ in range(n)]
    for s in range(n):
        W = [[0] * n for _ in range(kmax + 1)]
        W[0][s] = 1
        for k in range(1, kmax + 1):
            for t in range(n):
                W[k][t] = sum(W[k - w][v] for v, w in into[t] if w <= k)
        for t in range(n):
            for k in range(kmax + 1):
                if W[k][t] > 0:
                    dist[s][t] = k
                    cnt[s][t] = W[k][t]
                    break
    bc = [Fraction(0)] * n
    for s in range(n):
        for t in range(n):
            if s == t or dist[s][t] < 0:
                continue
            for v in range(n):
                if v in (s, t) or dist[s][v] < 0 or dist[v][t] < 0:
                    continue
                if dist[s][v] + dist[v][t] == dist[s][t]:
                    bc[v] += Fraction(cnt[s][v] * cnt[v][t], cnt[s][t])
    return bc, dist, cnt
