"""CPU oracle for Brandes betweenness centrality -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The GPU library never loads it
and shares no code with it.

``bc_oracle.c`` is a plain single-threaded C implementation of Eq. 1-2 of
the paper's Section "Background", written out from their definitions:
breadth-first distances (Dijkstra's method for graphs with positive integer
arc weights, ``g.weights``), the path-count recurrence over predecessors, and
Eq. 2 as a sum over each vertex's successors.  This module compiles it with
gcc and wraps it with ctypes.  ``tests/brute.py`` holds definition-level
checkers (path enumeration, walk counting) used to pin the oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_bc.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (gcc -O2, no fast-math: evaluation order is kept)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    lib.oracle_bc_dir.restype = ctypes.c_int
    lib.oracle_bc_dir.argtypes = [ctypes.c_int32, P, P, P, P, P, P, P, ctypes.c_int64, P, P]
    lib.oracle_source_dir.restype = ctypes.c_int
    lib.oracle_source_dir.argtypes = [ctypes.c_int32, P, P, P, P, P, P, ctypes.c_int32, P, P, P, P, P]
    lib.oracle_path_excess.restype = ctypes.c_int
    lib.oracle_path_excess.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int64, P]
    lib.oracle_bc_w.restype = ctypes.c_int
    lib.oracle_bc_w.argtypes = [ctypes.c_int32, P, P, P, P, P, P, P, P, P, ctypes.c_int64, P, P]
    lib.oracle_source_w.restype = ctypes.c_int
    lib.oracle_source_w.argtypes = [ctypes.c_int32, P, P, P, P, P, P, P, P, ctypes.c_int32, P, P, P, P]
    lib.oracle_sizeof_long_double.restype = ctypes.c_int
    if lib.oracle_sizeof_long_double() != np.dtype(np.longdouble).itemsize:
        raise RuntimeError("long double size mismatch between gcc and numpy")
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _rp_arr(rp):
    rp = np.ascontiguousarray(rp)
    if rp.dtype == np.int64:
        return None, rp
    return np.ascontiguousarray(rp, dtype=np.int32), None


def _rp(g):
    return _rp_arr(g.row_ptr)


def _in_arcs(g):
    """(in_rp32, in_rp64, in_col) pointers' arrays of a directed graph, or
    Nones for an undirected one (its adjacency serves as both)."""
    if getattr(g, "in_row_ptr", None) is None:
        return None, None, None
    irp32, irp64 = _rp_arr(g.in_row_ptr)
    return irp32, irp64, np.ascontiguousarray(g.in_col_idx, dtype=np.int32)


def _weights(g):
    """(wt, in_wt) int32 arrays of a weighted graph (in_wt None when
    undirected), or (None, None)."""
    w = getattr(g, "weights", None)
    if w is None:
        return None, None
    iw = getattr(g, "in_weights", None)
    return (np.ascontiguousarray(w, dtype=np.int32),
            None if iw is None else np.ascontiguousarray(iw, dtype=np.int32))


def _bc_call(lib, g, rp32, rp64, col, irp32, irp64, icol, src, ns, out, modes):
    wt, iwt = _weights(g)
    if wt is None:
        return lib.oracle_bc_dir(g.n, _ptr(rp32), _ptr(rp64), _ptr(col), _ptr(irp32), _ptr(irp64), _ptr(icol),
                                 _ptr(src), ns, _ptr(out), _ptr(modes))
    return lib.oracle_bc_w(g.n, _ptr(rp32), _ptr(rp64), _ptr(col), _ptr(wt), _ptr(irp32), _ptr(irp64), _ptr(icol),
                           _ptr(iwt), _ptr(src), ns, _ptr(out), _ptr(modes))


def bc(g, sources=None):
    """Raw ordered-pair BC sums over ``sources`` (None = all vertices).  A
    graph with ``in_row_ptr`` / ``in_col_idx`` is directed (paths follow
    arcs); otherwise its symmetric adjacency is used both ways.

    Returns (bc float64[n], modes int32[len(sources)]) where mode 1 marks a
    source whose path counts exceed uint64 and were evaluated in long double.
    """
    lib = _load()
    rp32, rp64 = _rp(g)
    col = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    out = np.zeros(g.n, dtype=np.float64)
    if sources is None:
        src = None
        ns = g.n
    else:
        src = np.ascontiguousarray(sources, dtype=np.int32)
        ns = src.size
    modes = np.zeros(ns, dtype=np.int32)
    irp32, irp64, icol = _in_arcs(g)
    rc = _bc_call(lib, g, rp32, rp64, col, irp32, irp64, icol, src, ns, out, modes)
    if rc != 0:
        raise ValueError(f"oracle_bc failed with code {rc}")
    return out, modes


def bc_sliced(g, sources, threads: int = 0):
    """``bc(g, sources)`` with the source list cut into ``threads`` contiguous
    slices (0 = all cores, at most 16), each run by the single-threaded oracle
    on its own host thread with its own buffers; the partial score vectors
    are added in slice order.  Same terms as ``bc``, grouped per slice, so
    the result agrees with ``bc`` to rounding.  Returns (bc, modes)."""
    from concurrent.futures import ThreadPoolExecutor
    lib = _load()
    rp32, rp64 = _rp(g)
    col = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    modes = np.zeros(src.size, dtype=np.int32)
    nt = threads or min(16, os.cpu_count() or 1)
    nt = max(1, min(nt, src.size))
    bounds = np.linspace(0, src.size, nt + 1).astype(np.int64)
    parts = [np.zeros(g.n, dtype=np.float64) for _ in range(nt)]
    irp32, irp64, icol = _in_arcs(g)

    def work(i):
        lo, hi = int(bounds[i]), int(bounds[i + 1])
        if hi <= lo:
            return 0
        s = src[lo:hi]
        m = modes[lo:hi]
        return _bc_call(lib, g, rp32, rp64, col, irp32, irp64, icol, s, hi - lo, parts[i], m)

    with ThreadPoolExecutor(nt) as ex:
        rcs = list(ex.map(work, range(nt)))
    if any(rcs):
        raise ValueError(f"oracle_bc failed with codes {rcs}")
    out = np.zeros(g.n, dtype=np.float64)
    for p in parts:
        out += p
    return out, modes


class SourceDetail:
    __slots__ = ("d", "sigma_u64", "sigma_ld", "delta", "mode", "n_levels")


def source(g, s: int) -> SourceDetail:
    """Distances, path counts and dependencies for one source."""
    lib = _load()
    rp32, rp64 = _rp(g)
    col = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    n = g.n
    r = SourceDetail()
    r.d = np.empty(n, np.int32)
    r.sigma_u64 = np.empty(n, np.uint64)
    r.sigma_ld = np.empty(n, np.longdouble)
    r.delta = np.empty(n, np.float64)
    nl = np.zeros(1, np.int32)
    irp32, irp64, icol = _in_arcs(g)
    wt, iwt = _weights(g)
    if wt is None:
        mode = lib.oracle_source_dir(n, _ptr(rp32), _ptr(rp64), _ptr(col), _ptr(irp32), _ptr(irp64), _ptr(icol),
                                     int(s), _ptr(r.d), _ptr(r.sigma_u64), _ptr(r.sigma_ld), _ptr(r.delta), _ptr(nl))
    else:  # weighted: int64 distances; n_levels = number of distinct distances
        r.d = np.empty(n, np.int64)
        mode = lib.oracle_source_w(n, _ptr(rp32), _ptr(rp64), _ptr(col), _ptr(wt), _ptr(irp32), _ptr(irp64),
                                   _ptr(icol), _ptr(iwt), int(s), _ptr(r.d), _ptr(r.sigma_u64), _ptr(r.sigma_ld),
                                   _ptr(r.delta))
        nl[0] = len(np.unique(r.d[r.d >= 0])) if mode >= 0 else 0
    if mode < 0:
        raise ValueError(f"oracle_source failed with code {mode}")
    r.mode = int(mode)
    r.n_levels = int(nl[0])
    return r


def path_excess(g, sources, threads: int = 0) -> np.ndarray:
    """Per source, the sum over reached t != s of (d(s, t) - 1), as int64.

    This equals sum_v delta_s(v), so a BC vector over ``sources`` must sum to
    ``path_excess(g, sources).sum()``.  Only distances are computed (plain
    BFS); slices of the source list run on ``threads`` host threads (0 = all
    cores, at most 16), each call owning its buffers.
    """
    from concurrent.futures import ThreadPoolExecutor
    if getattr(g, "weights", None) is not None:
        raise ValueError("path_excess counts hops: it does not apply to weighted graphs")
    lib = _load()
    rp32, rp64 = _rp(g)
    col = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    out = np.zeros(src.size, dtype=np.int64)
    if src.size == 0:
        return out
    nt = threads or min(16, os.cpu_count() or 1)
    nt = max(1, min(nt, src.size))
    bounds = np.linspace(0, src.size, nt + 1).astype(np.int64)

    def work(i):
        lo, hi = int(bounds[i]), int(bounds[i + 1])
        if hi <= lo:
            return 0
        s = src[lo:hi]
        o = out[lo:hi]
        return lib.oracle_path_excess(g.n, _ptr(rp32), _ptr(rp64), _ptr(col), _ptr(s), hi - lo, _ptr(o))

    with ThreadPoolExecutor(nt) as ex:
        rcs = list(ex.map(work, range(nt)))
    if any(rcs):
        raise ValueError(f"oracle_path_excess failed with codes {rcs}")
    return out
