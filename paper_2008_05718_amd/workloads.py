"""Seeded synthetic graph generators (inputs only).

This module builds the undirected, unweighted inputs the betweenness-centrality
path is measured and tested on.  It holds none of the method's arithmetic: no
distances, path counts or dependencies are computed here.  Both the GPU path
and the CPU oracle consume its output, and nothing else is shared between them.

Every generator returns a :class:`CSR` with
  * ``row_ptr``  int32[n+1] (int64 when nnz >= 2**31),
  * ``col_idx``  int32[nnz],
symmetric (both arc directions stored), rows strictly ascending, no self-loops,
no duplicate arcs.  ``m = nnz // 2`` undirected edges.

The graph families stand in for the paper's datasets (Table 1: road networks,
Delaunay meshes, social/web graphs, random geometric graphs), which are not
available here:
  * R-MAT           -> power-law, small-diameter social/web graphs,
  * damaged grid    -> low-degree, high-diameter road/mesh graphs,
  * Erdos-Renyi     -> uniform-degree graphs,
  * Barabasi-Albert -> many small scale-free graphs of uneven size.
"""
from __future__ import annotations

import math
import random
from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSR:
    row_ptr: np.ndarray
    col_idx: np.ndarray
    name: str = ""
    # Block-diagonal unions of several graphs carry their vertex offsets
    # (int32[n_graphs+1]); a single graph has [0, n].
    vtx_offsets: np.ndarray | None = None
    meta: dict = field(default_factory=dict)
    # Directed graphs: row_ptr / col_idx hold the out-arcs and these the
    # in-arcs (the transpose, rows ascending).  None for undirected graphs,
    # whose symmetric adjacency is both.
    in_row_ptr: np.ndarray | None = None
    in_col_idx: np.ndarray | None = None
    # Weighted graphs: positive int32 arc weights aligned with col_idx (and
    # with in_col_idx for directed graphs); symmetric for undirected graphs.
    weights: np.ndarray | None = None
    in_weights: np.ndarray | None = None

    @property
    def directed(self) -> bool:
        return self.in_row_ptr is not None

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        """Edge count: undirected edges (each stored as two arcs), or arcs of
        a directed graph."""
        return self.nnz if self.directed else self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def neighbors(self, v: int) -> np.ndarray:
        return self.col_idx[self.row_ptr[v]:self.row_ptr[v + 1]]


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray, name: str = "") -> CSR:
    """Symmetrise an edge list, drop self-loops and duplicates, sort rows."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    if u.size:
        if u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n:
            raise ValueError("edge endpoint out of range")
    keys = np.concatenate([u * n + v, v * n + u])
    keys.sort()
    if keys.size:
        keep = np.empty(keys.size, dtype=bool)
        keep[0] = True
        np.not_equal(keys[1:], keys[:-1], out=keep[1:])
        keys = keys[keep]
    rows = keys // n
    cols = (keys - rows * n).astype(np.int32)
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] < 2**31:
        row_ptr = row_ptr.astype(np.int32)
    g = CSR(row_ptr, cols, name=name)
    g.vtx_offsets = np.array([0, n], dtype=np.int32)
    return g


def _rows(n: int, keys: np.ndarray):
    rows = keys // n
    cols = (keys - rows * n).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    if row_ptr[-1] < 2**31:
        row_ptr = row_ptr.astype(np.int32)
    return row_ptr, cols


def digraph_from_arcs(n: int, u: np.ndarray, v: np.ndarray, name: str = "") -> CSR:
    """Directed graph from arcs u -> v: self-loops and duplicate arcs
    dropped, out-rows and in-rows sorted ascending."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    if u.size and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("arc endpoint out of range")
    out_keys = np.unique(u * n + v)
    uu, vv = out_keys // n, out_keys % n
    in_keys = np.sort(vv * n + uu)
    rp, ci = _rows(n, out_keys)
    irp, ici = _rows(n, in_keys)
    g = CSR(rp, ci, name=name, in_row_ptr=irp, in_col_idx=ici)
    g.vtx_offsets = np.array([0, n], dtype=np.int32)
    return g


def rmat_directed(scale: int, edgefactor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
                  seed: int = 1) -> CSR:
    """R-MAT arcs (the sampled edges kept as directed arcs, not symmetrised),
    seeded random relabelling, duplicates and self-loops dropped."""
    und = rmat(scale, edgefactor, a, b, c, seed=seed, relabel=True, keep_arcs=True)
    u, v = und.meta.pop("arcs")
    g = digraph_from_arcs(1 << scale, u, v, name=f"rmatdir{scale}_ef{edgefactor}_s{seed}")
    g.meta.update(family="rmat_directed", scale=scale, edgefactor=edgefactor, seed=seed)
    return g


def with_weights(g: CSR, lo: int = 1, hi: int = 16, seed: int = 1) -> CSR:
    """The same graph with integer arc weights drawn uniformly from [lo, hi]:
    one weight per undirected edge (both arcs carry it), or one per arc of a
    directed graph (the in-arcs carry the weight of the same arc)."""
    rng = np.random.default_rng(seed)
    n = g.n
    rp = g.row_ptr.astype(np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    dst = g.col_idx.astype(np.int64)
    if g.directed:
        w = rng.integers(lo, hi + 1, size=g.nnz).astype(np.int32)
        key = src * n + dst  # ascending: out-rows are sorted
        irp = g.in_row_ptr.astype(np.int64)
        isrc = np.repeat(np.arange(n, dtype=np.int64), np.diff(irp))  # head of the in-arc
        ikey = g.in_col_idx.astype(np.int64) * n + isrc  # the same arc, tail * n + head
        iw = w[np.searchsorted(key, ikey)]
    else:
        a, b = np.minimum(src, dst), np.maximum(src, dst)
        ekey = a * n + b
        uniq, inv = np.unique(ekey, return_inverse=True)
        wu = rng.integers(lo, hi + 1, size=uniq.size).astype(np.int32)
        w = wu[inv]
        iw = None
    h = CSR(g.row_ptr, g.col_idx, name=g.name + f"_w{lo}-{hi}", vtx_offsets=g.vtx_offsets, meta=dict(g.meta),
            in_row_ptr=g.in_row_ptr, in_col_idx=g.in_col_idx, weights=w, in_weights=iw)
    h.meta.update(weights=(lo, hi, seed))
    return h


def csr_from_networkx(G) -> CSR:
    """Small helper for tests: relabel a networkx graph 0..n-1 in sorted order."""
    nodes = sorted(G.nodes())
    idx = {x: i for i, x in enumerate(nodes)}
    e = np.array([(idx[a], idx[b]) for a, b in G.edges()], dtype=np.int64).reshape(-1, 2)
    return csr_from_edges(len(nodes), e[:, 0], e[:, 1], name="nx")


# ---------------------------------------------------------------- Erdos-Renyi
def erdos_renyi(n: int, avg_degree: float, seed: int) -> CSR:
    """G(n, p) with p = avg_degree / (n - 1); every unordered pair drawn once."""
    rng = np.random.default_rng(seed)
    p = avg_degree / (n - 1)
    us, vs = [], []
    # Row by row keeps memory at O(n) per step for larger n.
    for i in range(n - 1):
        hit = np.nonzero(rng.random(n - 1 - i) < p)[0]
        if hit.size:
            us.append(np.full(hit.size, i, dtype=np.int64))
            vs.append(hit.astype(np.int64) + i + 1)
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    g = csr_from_edges(n, u, v, name=f"er_n{n}_d{avg_degree:g}_s{seed}")
    g.meta.update(family="er", n=n, avg_degree=avg_degree, seed=seed)
    return g


# ---------------------------------------------------------------------- R-MAT
def rmat(scale: int, edgefactor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 1, relabel: bool = True, keep_arcs: bool = False) -> CSR:
    """R-MAT (Chakrabarti et al.) with a seeded random vertex relabelling.

    edgefactor * 2**scale edges are sampled bit by bit from the quadrant
    probabilities (a, b, c, d = 1-a-b-c), then symmetrised and deduplicated.
    """
    n = 1 << scale
    E = edgefactor * n
    rng = np.random.default_rng(seed)
    src = np.zeros(E, dtype=np.int32)
    dst = np.zeros(E, dtype=np.int32)
    ab, abc = a + b, a + b + c
    chunk = 1 << 24
    for lo in range(0, E, chunk):
        hi = min(E, lo + chunk)
        s = np.zeros(hi - lo, dtype=np.int32)
        t = np.zeros(hi - lo, dtype=np.int32)
        for bit in range(scale):
            r = rng.random(hi - lo, dtype=np.float64)
            sb = r >= ab
            tb = ((r >= a) & (r < ab)) | (r >= abc)
            s |= sb.astype(np.int32) << bit
            t |= tb.astype(np.int32) << bit
        src[lo:hi] = s
        dst[lo:hi] = t
    if relabel:
        perm = rng.permutation(n).astype(np.int32)
        src = perm[src]
        dst = perm[dst]
    g = csr_from_edges(n, src, dst, name=f"rmat{scale}_ef{edgefactor}_s{seed}")
    g.meta.update(family="rmat", scale=scale, edgefactor=edgefactor,
                  abcd=(a, b, c, 1 - a - b - c), seed=seed)
    if keep_arcs:
        g.meta["arcs"] = (src, dst)
    return g


# ----------------------------------------------------------------------- grid
def grid(L: int, delete_frac: float = 0.0, shortcut_frac: float = 0.0,
         seed: int = 3, keep_lcc: bool = True) -> CSR:
    """L x L 4-neighbour grid, a fraction of edges deleted uniformly at random
    (without replacement), the largest connected component kept and relabelled
    compactly in row-major order, then round(shortcut_frac * m) uniform random
    long-range edges added (no duplicates, no self-loops).

    With delete_frac = shortcut_frac = 0 this is the intact grid whose vertex
    (i, j) has id i * L + j.
    """
    rng = np.random.default_rng(seed)
    ids = np.arange(L * L, dtype=np.int64).reshape(L, L)
    hu, hv = ids[:, :-1].ravel(), ids[:, 1:].ravel()
    vu, vv = ids[:-1, :].ravel(), ids[1:, :].ravel()
    u = np.concatenate([hu, vu])
    v = np.concatenate([hv, vv])
    E = u.size
    ndel = int(round(delete_frac * E))
    if ndel:
        drop = rng.choice(E, size=ndel, replace=False)
        keep = np.ones(E, dtype=bool)
        keep[drop] = False
        u, v = u[keep], v[keep]
    n = L * L
    if keep_lcc and ndel:
        from scipy.sparse import coo_matrix
        from scipy.sparse.csgraph import connected_components
        A = coo_matrix((np.ones(u.size, np.int8), (u, v)), shape=(n, n))
        ncomp, lab = connected_components(A, directed=False)
        big = np.argmax(np.bincount(lab))
        inside = lab == big
        newid = np.full(n, -1, dtype=np.int64)
        newid[inside] = np.arange(int(inside.sum()))
        sel = inside[u] & inside[v]
        u, v = newid[u[sel]], newid[v[sel]]
        n = int(inside.sum())
    m = u.size
    nsc = int(round(shortcut_frac * m))
    if nsc:
        existing = set((np.minimum(u, v) * n + np.maximum(u, v)).tolist())
        su, sv = [], []
        while len(su) < nsc:
            a_, b_ = rng.integers(0, n, size=2)
            if a_ == b_:
                continue
            key = min(a_, b_) * n + max(a_, b_)
            if key in existing:
                continue
            existing.add(key)
            su.append(a_)
            sv.append(b_)
        u = np.concatenate([u, np.array(su, np.int64)])
        v = np.concatenate([v, np.array(sv, np.int64)])
    g = csr_from_edges(n, u, v, name=f"grid{L}_del{delete_frac:g}_sc{shortcut_frac:g}_s{seed}")
    g.meta.update(family="grid", L=L, delete_frac=delete_frac,
                  shortcut_frac=shortcut_frac, seed=seed)
    return g


# ------------------------------------------------------------ Barabasi-Albert
def barabasi_albert(n: int, m0: int = 4, seed: int = 4) -> CSR:
    """Preferential attachment: start from the complete graph K_{m0}; every new
    vertex links to m0 distinct existing vertices chosen with probability
    proportional to their degree."""
    if n <= m0:
        raise ValueError("n must exceed m0")
    r = random.Random(seed)
    ends = np.empty(2 * (m0 * (m0 - 1) // 2 + (n - m0) * m0), dtype=np.int64)
    us = np.empty(m0 * (m0 - 1) // 2 + (n - m0) * m0, dtype=np.int64)
    vs = np.empty_like(us)
    k = 0
    e = 0
    for i in range(m0):
        for j in range(i + 1, m0):
            us[e], vs[e] = i, j
            ends[k], ends[k + 1] = i, j
            k += 2
            e += 1
    endsl = ends.tolist()  # Python list indexing is faster than numpy scalars
    rnd = r.random
    for w in range(m0, n):
        chosen = []
        while len(chosen) < m0:
            t = endsl[int(rnd() * k)]
            if t not in chosen:
                chosen.append(t)
        for t in chosen:
            us[e], vs[e] = w, t
            e += 1
            endsl[k] = w
            endsl[k + 1] = t
            k += 2
    g = csr_from_edges(n, us[:e], vs[:e], name=f"ba_n{n}_m{m0}_s{seed}")
    g.meta.update(family="ba", n=n, m0=m0, seed=seed)
    return g


def union(graphs: list[CSR], name: str = "union") -> CSR:
    """Block-diagonal union; graph g owns vertices [vtx_offsets[g], vtx_offsets[g+1])."""
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        offs[i + 1] = offs[i] + g.n
    rp_parts, ci_parts = [np.zeros(1, np.int64)], []
    base_arc = 0
    for i, g in enumerate(graphs):
        rp_parts.append(g.row_ptr[1:].astype(np.int64) + base_arc)
        ci_parts.append(g.col_idx.astype(np.int64) + offs[i])
        base_arc += g.nnz
    row_ptr = np.concatenate(rp_parts)
    col_idx = np.concatenate(ci_parts).astype(np.int32) if ci_parts else np.zeros(0, np.int32)
    if row_ptr[-1] < 2**31:
        row_ptr = row_ptr.astype(np.int32)
    u = CSR(row_ptr, col_idx, name=name)
    u.vtx_offsets = offs.astype(np.int32)
    u.meta.update(family="union", n_graphs=len(graphs))
    return u


def ba_collection(n_graphs: int, n_lo: int, n_hi: int, m0: int = 4, seed: int = 4) -> list[CSR]:
    """n_graphs BA graphs with n drawn log-uniform in [n_lo, n_hi]."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=n_graphs))).astype(int)
    return [barabasi_albert(int(s), m0, seed=seed * 100003 + i) for i, s in enumerate(sizes)]


# -------------------------------------------------------------------- sources
def choose_sources(g: CSR, k: int, seed: int, nonisolated: bool = True) -> np.ndarray:
    """k distinct sources drawn uniformly (without replacement) from the
    vertices of degree >= 1 (or all vertices), in the drawn order."""
    rng = np.random.default_rng(seed)
    pool = np.nonzero(g.degrees() > 0)[0] if nonisolated else np.arange(g.n)
    if k > pool.size:
        raise ValueError(f"asked for {k} sources, only {pool.size} eligible")
    return rng.choice(pool, size=k, replace=False).astype(np.int32)


# ------------------------------------------------------ the five workloads
def workload(name: str, small: bool = False):
    """Return (graph, sources) for a named workload.

    er2000     : G(2000, p = 8/1999), all sources                 (gen seed 1)
    rmat18     : R-MAT scale 18, ef 16, 8192 sources               (seed 2, src 1001)
    grid1024   : 1024^2 grid, -10% edges, LCC, +0.1% shortcuts, 4096 sources (seed 3, src 1002)
    ba512      : 512 BA graphs, n log-uniform [1e3, 1e5], all sources (seed 4)
    ba512_frac64 : the same union, every 64th vertex of every graph as a source
    rmat22     : R-MAT scale 22, ef 16, 16384 sources              (seed 5, src 1004)
    rmat18_directed : R-MAT scale 18 arcs kept directed, 8192 sources of out-degree >= 1
                      (seed 2, src 1001)
    rmat18_weighted : rmat18 with edge weights uniform in [1, 100], 4096 sources
                      (weight seed 6, src 1001)
    """
    if name == "er2000":
        g = erdos_renyi(2000, 8.0, seed=1)
        return g, np.arange(g.n, dtype=np.int32)
    if name == "rmat18":
        g = rmat(18, 16, seed=2)
        return g, choose_sources(g, 8192, seed=1001)
    if name == "grid1024":
        g = grid(1024, 0.10, 0.001, seed=3)
        return g, choose_sources(g, 4096, seed=1002)
    if name == "grid1024_noshortcut":
        g = grid(1024, 0.10, 0.0, seed=3)
        return g, choose_sources(g, 256, seed=1002)
    if name == "ba512":
        gs = ba_collection(512, 1000, 100000, 4, seed=4)
        u = union(gs, name="ba512")
        return u, np.arange(u.n, dtype=np.int32)
    if name == "ba512_frac64":
        # 1/64 of the all-sources work with the same mix of graph sizes:
        # every 64th vertex of every graph
        gs = ba_collection(512, 1000, 100000, 4, seed=4)
        u = union(gs, name="ba512")
        off = u.vtx_offsets.astype(np.int64)
        srcs = np.concatenate([np.arange(off[i], off[i + 1], 64) for i in range(len(off) - 1)])
        return u, srcs.astype(np.int32)
    if name == "rmat22":
        g = rmat(22, 16, seed=5)
        return g, choose_sources(g, 16384, seed=1004)
    if name == "rmat18_directed":
        g = rmat_directed(18, 16, seed=2)
        return g, choose_sources(g, 8192, seed=1001)
    if name == "rmat18_weighted":
        g = rmat(18, 16, seed=2)
        srcs = choose_sources(g, 4096, seed=1001)
        return with_weights(g, 1, 100, seed=6), srcs
    raise KeyError(name)
