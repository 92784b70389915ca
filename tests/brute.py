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
