"""ctypes binding of libbc (include/bc.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libbc.so.  PyTorch, when used, only supplies device buffers
(``torch.Tensor`` on ``cuda``) and the current HIP stream.

The functions keep the C names (``bc_graph_create``, ``bc_run``,
``bc_scores``, ``bc_destroy``, ...).  ``Graph`` is a small owning wrapper.
If libbc.so has not been built the first call raises ``LibraryMissing``;
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbc.so")  # the in-tree build; no override

BC_OK = 0
STATUS = {0: "BC_OK", 1: "BC_ERR_INVALID_ARG", 2: "BC_ERR_INVALID_GRAPH", 3: "BC_ERR_OUT_OF_MEMORY",
          4: "BC_ERR_DEVICE", 5: "BC_ERR_SIGMA_RANGE", 6: "BC_ERR_NOT_SUPPORTED"}

BC_INPUT_DEVICE = 0x1
BC_SKIP_SYMMETRY_CHECK = 0x2
BC_KEEP_ORDER = 0x4
BC_DIRECTED = 0x8
BC_RUN_ACCUMULATE = 0x1
BC_RUN_NO_GRAPHS = 0x2
BC_RUN_FORCE_F64 = 0x4
BC_RUN_TUNED = 0x8
BC_RUN_ONE_QUEUE = 0x10
BC_RUN_BLOCKS = 0x20
BC_RUN_NO_BLOCKS = 0x40
BC_TUNE_FRESH = 0x80
BC_OUT_DEVICE = 0x1

BC_VARIANT_PUSH_TPV, BC_VARIANT_PUSH_WPV, BC_VARIANT_PULL = 0, 1, 2
BC_POLICY_AUTO = 0
BC_POLICY_HEURISTIC = 1
BC_POLICY_MLP = 2
BC_POLICY_FORCE_PUSH_TPV = 3
BC_POLICY_FORCE_PUSH_WPV = 4
BC_POLICY_FORCE_PULL = 5
BC_MLP_IN = 5
BC_MLP_OUT = 9
BC_MLP_PARAMS = 32 * 5 + 32 + 32 * 32 + 32 + 9 * 32 + 9
BC_LB_PACKED, BC_LB_RULE, BC_LB_ITEMS = 0, 1, 2

EXPORTS = ["bc_status_string", "bc_last_error", "bc_graph_create", "bc_graph_create_multi",
           "bc_graph_create_weighted", "bc_destroy",
           "bc_graph_info", "bc_run_options_init", "bc_run", "bc_scores", "bc_run_detail", "bc_run_stats",
           "bc_load_policy", "bc_mlp_loss_grad", "bc_mlp_train", "bc_mlp_predict", "bc_collect_level_times",
           "bc_autotune", "bc_set_device_limit", "bc_run_level_stats", "bc_mlp_loss_grad_noalloc",
           "bc_tune_cache_save", "bc_tune_cache_load", "bc_tune_cache_clear", "bc_tune_cache_size"]


class LibraryMissing(RuntimeError):
    pass


class BCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class RunOptions(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("batch", ctypes.c_int32), ("policy", ctypes.c_int32),
                ("alpha", ctypes.c_float), ("beta", ctypes.c_float), ("wpv_degree", ctypes.c_float),
                ("grid_blocks", ctypes.c_int32), ("chunk_steps", ctypes.c_int32),
                ("sigma_limit", ctypes.c_int64), ("lanes_per_entry", ctypes.c_float),
                ("policy_margin", ctypes.c_float), ("replicas", ctypes.c_int32),
                ("weighted_lanes", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class Detail(ctypes.Structure):
    _fields_ = [("d", ctypes.c_void_p), ("sigma_u64", ctypes.c_void_p), ("sigma_mant", ctypes.c_void_p),
                ("sigma_exp", ctypes.c_void_p), ("delta", ctypes.c_void_p), ("mode", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("d64", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("n_sources", ctypes.c_int64), ("n_batches", ctypes.c_int64), ("batch", ctypes.c_int32),
                ("policy", ctypes.c_int32), ("grid_blocks", ctypes.c_int32), ("chunk_steps", ctypes.c_int32),
                ("steps", ctypes.c_int64), ("launches", ctypes.c_int64), ("forward_levels", ctypes.c_int64),
                ("max_levels", ctypes.c_int64), ("variant_levels", ctypes.c_int64 * 3),
                ("f64_sources", ctypes.c_int64), ("arcs_scanned", ctypes.c_int64), ("lane_arcs", ctypes.c_int64),
                ("queue_entries", ctypes.c_int64), ("algo_bytes", ctypes.c_double), ("ms", ctypes.c_double),
                ("phase_ms", ctypes.c_double * 10), ("variant_ms", ctypes.c_double * 3),
                ("phase_arcs", ctypes.c_int64 * 10), ("phase_lane_arcs", ctypes.c_int64 * 10),
                ("phase_pairs", ctypes.c_int64 * 10), ("mode_launches", ctypes.c_int64 * 2),
                ("mode_ms", ctypes.c_double * 2), ("mode_algo_bytes", ctypes.c_double * 2),
                ("reached_pairs", ctypes.c_int64), ("algo_bytes_arcs", ctypes.c_double),
                ("block_workgroups", ctypes.c_int64), ("block_chunks", ctypes.c_int64)]


class LevelStats(ctypes.Structure):
    _fields_ = [("visits", ctypes.c_int64), ("entries", ctypes.c_int64), ("arcs", ctypes.c_int64),
                ("variant", ctypes.c_int64 * 3), ("ms", ctypes.c_double)]


_lib = None


def lib():
    """Load libbc.so (raises LibraryMissing if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is not built; run `python -m paper_2008_05718_amd.build`")
    # One HIP runtime per process: PyTorch bundles its own libamdhip64.so.7.
    # Importing torch first makes libbc.so bind to that same runtime, so torch
    # device buffers and streams are valid inside libbc.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    L.bc_status_string.restype = ctypes.c_char_p
    L.bc_status_string.argtypes = [ctypes.c_int]
    L.bc_last_error.restype = ctypes.c_char_p
    L.bc_last_error.argtypes = []
    L.bc_graph_create.restype = ctypes.c_int
    L.bc_graph_create.argtypes = [I32, I64, P, P, U32, ctypes.POINTER(P)]
    L.bc_graph_create_weighted.restype = ctypes.c_int
    L.bc_graph_create_weighted.argtypes = [I32, I64, P, P, P, U32, ctypes.POINTER(P)]
    L.bc_graph_create_multi.restype = ctypes.c_int
    L.bc_graph_create_multi.argtypes = [I32, P, I32, I64, P, P, U32, ctypes.POINTER(P)]
    L.bc_destroy.restype = None
    L.bc_destroy.argtypes = [P]
    L.bc_graph_info.restype = ctypes.c_int
    L.bc_graph_info.argtypes = [P, P, P, P, P]
    L.bc_run_options_init.restype = None
    L.bc_run_options_init.argtypes = [ctypes.POINTER(RunOptions)]
    L.bc_run.restype = ctypes.c_int
    L.bc_run.argtypes = [P, P, I64, ctypes.POINTER(RunOptions), P]
    L.bc_scores.restype = ctypes.c_int
    L.bc_scores.argtypes = [P, P, I64, U32, P]
    L.bc_run_detail.restype = ctypes.c_int
    L.bc_run_detail.argtypes = [P, P, I64, ctypes.POINTER(RunOptions), I64, ctypes.POINTER(Detail), P]
    L.bc_run_stats.restype = ctypes.c_int
    L.bc_run_stats.argtypes = [P, ctypes.POINTER(Stats)]
    L.bc_autotune.restype = ctypes.c_int
    L.bc_autotune.argtypes = [P, P, I64, ctypes.POINTER(RunOptions), ctypes.POINTER(RunOptions), P]
    L.bc_tune_cache_save.restype = ctypes.c_int
    L.bc_tune_cache_save.argtypes = [ctypes.c_char_p]
    L.bc_tune_cache_load.restype = ctypes.c_int
    L.bc_tune_cache_load.argtypes = [ctypes.c_char_p]
    L.bc_tune_cache_clear.restype = None
    L.bc_tune_cache_clear.argtypes = []
    L.bc_tune_cache_size.restype = I64
    L.bc_tune_cache_size.argtypes = []
    L.bc_load_policy.restype = ctypes.c_int
    L.bc_load_policy.argtypes = [P, P, I64]
    L.bc_mlp_loss_grad.restype = ctypes.c_int
    L.bc_mlp_loss_grad.argtypes = [P, P, P, P, I64, P, P, P]
    L.bc_mlp_loss_grad_noalloc.restype = ctypes.c_int
    L.bc_mlp_loss_grad_noalloc.argtypes = [P, P, P, P, I64, P, P, P]
    L.bc_mlp_train.restype = ctypes.c_int
    L.bc_mlp_train.argtypes = [P, P, P, P, I64, I32, ctypes.c_float, P, P]
    L.bc_mlp_predict.restype = ctypes.c_int
    L.bc_mlp_predict.argtypes = [P, P, I64, P, P]
    L.bc_set_device_limit.restype = ctypes.c_int
    L.bc_set_device_limit.argtypes = [P, I64]
    L.bc_run_level_stats.restype = ctypes.c_int
    L.bc_run_level_stats.argtypes = [P, P, I64, P]
    L.bc_collect_level_times.restype = ctypes.c_int
    L.bc_collect_level_times.argtypes = [P, P, I64, ctypes.POINTER(RunOptions), P, P, I64, P, P]
    _lib = L
    return L


def _check(status: int):
    if status != BC_OK:
        msg = lib().bc_last_error().decode(errors="replace")
        raise BCError(status, msg)


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr_i32(x):
    """Host numpy (contiguous int32) or torch tensor -> (pointer, keepalive, on_device)."""
    if _is_torch(x):
        import torch
        if x.dtype != torch.int32 or not x.is_contiguous():
            raise TypeError("torch inputs must be contiguous int32")
        return ctypes.c_void_p(x.data_ptr()), x, x.is_cuda
    a = np.ascontiguousarray(x, dtype=np.int32)
    return a.ctypes.data_as(ctypes.c_void_p), a, False


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(int(stream.cuda_stream))  # torch.cuda.Stream


def make_options(batch=0, policy=BC_POLICY_AUTO, flags=0, alpha=0.0, beta=0.0, wpv_degree=0.0,
                 grid_blocks=0, chunk_steps=0, sigma_limit=0, lanes_per_entry=0.0,
                 policy_margin=0.0, replicas=0, weighted_lanes=0) -> RunOptions:
    o = RunOptions()
    lib().bc_run_options_init(ctypes.byref(o))
    o.flags, o.batch, o.policy = flags, batch, policy
    o.alpha, o.beta, o.wpv_degree = alpha, beta, wpv_degree
    o.grid_blocks, o.chunk_steps, o.sigma_limit = grid_blocks, chunk_steps, sigma_limit
    o.lanes_per_entry = lanes_per_entry
    o.policy_margin = policy_margin
    o.replicas = replicas
    o.weighted_lanes = weighted_lanes
    return o


# ------------------------------------------------------------ C-named calls
def bc_graph_create(row_ptr, col_idx, flags: int = 0):
    rp, keep1, dev1 = _ptr_i32(row_ptr)
    ci, keep2, dev2 = _ptr_i32(col_idx)
    if dev1 != dev2:
        raise TypeError("row_ptr and col_idx must both be host or both be device arrays")
    n = (keep1.shape[0] if not _is_torch(keep1) else keep1.numel()) - 1
    nnz = keep2.shape[0] if not _is_torch(keep2) else keep2.numel()
    h = ctypes.c_void_p()
    _check(lib().bc_graph_create(n, nnz, rp, ci, flags | (BC_INPUT_DEVICE if dev1 else 0), ctypes.byref(h)))
    return h


def bc_graph_create_weighted(row_ptr, col_idx, weights, flags: int = 0):
    rp, keep1, dev1 = _ptr_i32(row_ptr)
    ci, keep2, dev2 = _ptr_i32(col_idx)
    wt, keep3, dev3 = _ptr_i32(weights)
    if not (dev1 == dev2 == dev3):
        raise TypeError("row_ptr, col_idx and weights must all be host or all be device arrays")
    n = (keep1.shape[0] if not _is_torch(keep1) else keep1.numel()) - 1
    nnz = keep2.shape[0] if not _is_torch(keep2) else keep2.numel()
    h = ctypes.c_void_p()
    _check(lib().bc_graph_create_weighted(n, nnz, rp, ci, wt, flags | (BC_INPUT_DEVICE if dev1 else 0),
                                          ctypes.byref(h)))
    return h


def bc_graph_create_multi(vtx_offsets, row_ptr, col_idx, flags: int = 0):
    vo = np.ascontiguousarray(vtx_offsets, dtype=np.int32)
    rp, keep1, dev1 = _ptr_i32(row_ptr)
    ci, keep2, dev2 = _ptr_i32(col_idx)
    if dev1 != dev2:
        raise TypeError("row_ptr and col_idx must both be host or both be device arrays")
    n = (keep1.shape[0] if not _is_torch(keep1) else keep1.numel()) - 1
    nnz = keep2.shape[0] if not _is_torch(keep2) else keep2.numel()
    h = ctypes.c_void_p()
    _check(lib().bc_graph_create_multi(vo.size - 1, vo.ctypes.data_as(ctypes.c_void_p), n, nnz, rp, ci,
                                       flags | (BC_INPUT_DEVICE if dev1 else 0), ctypes.byref(h)))
    return h


def bc_destroy(h):
    if h:
        lib().bc_destroy(h)


def bc_graph_info(h):
    n, nnz, ng, b = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().bc_graph_info(h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(ng), ctypes.byref(b)))
    return {"n": n.value, "nnz": nnz.value, "n_graphs": ng.value, "device_bytes": b.value}


def _sources(sources):
    if sources is None:
        return None, 0, None
    s = np.ascontiguousarray(sources, dtype=np.int32)
    return s.ctypes.data_as(ctypes.c_void_p), s.size, s


def bc_run(h, sources=None, options: RunOptions | None = None, stream=None):
    p, ns, keep = _sources(sources)
    _check(lib().bc_run(h, p, ns, ctypes.byref(options) if options is not None else None, _stream(stream)))


def bc_scores(h, out=None, stream=None):
    """Scores into a new numpy array, or into ``out`` (numpy or torch cuda float64)."""
    info = bc_graph_info(h)
    n = info["n"]
    if out is None:
        out = np.zeros(n, dtype=np.float64)
    if _is_torch(out):
        import torch
        if out.dtype != torch.float64 or not out.is_contiguous():
            raise TypeError("out must be contiguous float64")
        flags = BC_OUT_DEVICE if out.is_cuda else 0
        _check(lib().bc_scores(h, ctypes.c_void_p(out.data_ptr()), out.numel(), flags, _stream(stream)))
        return out
    if out.dtype != np.float64 or not out.flags.c_contiguous:
        raise TypeError("out must be contiguous float64")
    _check(lib().bc_scores(h, out.ctypes.data_as(ctypes.c_void_p), out.size, 0, _stream(stream)))
    return out


def bc_run_detail(h, sources, dump_index: int, options: RunOptions | None = None, stream=None) -> dict:
    n = bc_graph_info(h)["n"]
    p, ns, keep = _sources(sources)
    r = {"d": np.zeros(n, np.int32), "sigma_u64": np.zeros(n, np.uint64), "sigma_mant": np.zeros(n, np.float64),
         "sigma_exp": np.zeros(n, np.int32), "delta": np.zeros(n, np.float64), "d64": np.full(n, -1, np.int64)}
    det = Detail()
    for k in ("d", "sigma_u64", "sigma_mant", "sigma_exp", "delta", "d64"):
        setattr(det, k, r[k].ctypes.data_as(ctypes.c_void_p))
    _check(lib().bc_run_detail(h, p, ns, ctypes.byref(options) if options is not None else None, int(dump_index),
                               ctypes.byref(det), _stream(stream)))
    r["mode"] = det.mode
    r["n_levels"] = det.n_levels
    return r


def bc_run_stats(h) -> dict:
    s = Stats()
    _check(lib().bc_run_stats(h, ctypes.byref(s)))
    out = {}
    for name, _ in Stats._fields_:
        v = getattr(s, name)
        out[name] = list(v) if hasattr(v, "__len__") else v
    return out


def bc_set_device_limit(h, max_device_bytes: int):
    _check(lib().bc_set_device_limit(h, int(max_device_bytes)))


def bc_run_level_stats(h) -> dict:
    """Per-level records of the last run as arrays indexed by level."""
    nl = ctypes.c_int64()
    _check(lib().bc_run_level_stats(h, None, 0, ctypes.byref(nl)))
    k = nl.value
    recs = (LevelStats * max(k, 1))()
    _check(lib().bc_run_level_stats(h, ctypes.cast(recs, ctypes.c_void_p), k, ctypes.byref(nl)))
    return {"visits": np.array([r.visits for r in recs[:k]], np.int64),
            "entries": np.array([r.entries for r in recs[:k]], np.int64),
            "arcs": np.array([r.arcs for r in recs[:k]], np.int64),
            "variant": np.array([list(r.variant) for r in recs[:k]], np.int64).reshape(k, 3),
            "ms": np.array([r.ms for r in recs[:k]], np.float64)}


def bc_autotune(h, sample, options: RunOptions | None = None, stream=None) -> dict:
    """Measure the candidate launch configurations on ``sample`` (host source
    ids); returns the fastest as a dict of run options and keeps it in the
    handle for runs with BC_RUN_TUNED."""
    s = np.ascontiguousarray(sample, dtype=np.int32)
    best = RunOptions()
    _check(lib().bc_autotune(h, _p(s), s.size, ctypes.byref(options) if options is not None else None,
                             ctypes.byref(best), _stream(stream)))
    return {"batch": best.batch, "policy": best.policy, "grid_blocks": best.grid_blocks,
            "chunk_steps": best.chunk_steps, "wpv_degree": best.wpv_degree,
            "lanes_per_entry": best.lanes_per_entry, "replicas": best.replicas}


def bc_tune_cache_save(path: str):
    _check(lib().bc_tune_cache_save(os.fsencode(path)))


def bc_tune_cache_load(path: str):
    _check(lib().bc_tune_cache_load(os.fsencode(path)))


def bc_tune_cache_clear():
    lib().bc_tune_cache_clear()


def bc_tune_cache_size() -> int:
    return int(lib().bc_tune_cache_size())


def bc_load_policy(h, weights):
    if weights is None:
        _check(lib().bc_load_policy(h, None, 0))
        return
    w = np.ascontiguousarray(weights, dtype=np.float32)
    _check(lib().bc_load_policy(h, w.ctypes.data_as(ctypes.c_void_p), w.size))


def _f32(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def bc_mlp_loss_grad(weights, X, Y, mask):
    """(loss, grad float32[BC_MLP_PARAMS]) of the policy-network loss."""
    n = int(np.asarray(X).shape[0])
    w = _f32(weights, (BC_MLP_PARAMS,))
    x = _f32(X, (n, BC_MLP_IN))
    y = _f32(Y, (n, BC_MLP_OUT))
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(n, BC_MLP_OUT)
    loss = ctypes.c_float()
    grad = np.zeros(BC_MLP_PARAMS, np.float32)
    _check(lib().bc_mlp_loss_grad(_p(w), _p(x), _p(y), _p(m), n, ctypes.byref(loss), _p(grad), None))
    return float(loss.value), grad


def bc_mlp_loss_grad_noalloc(weights, X, Y, mask, loss, grad, stream=None):
    """Allocation-free loss and gradient: every argument is a contiguous
    torch cuda tensor (weights float32[BC_MLP_PARAMS], X float32[n][BC_MLP_IN],
    Y float32[n][BC_MLP_OUT], mask uint8[n][BC_MLP_OUT], loss float32[1], grad
    float32[BC_MLP_PARAMS]).  Enqueued on ``stream``; the outputs are valid
    once that stream's work is done."""
    import torch
    n = int(X.shape[0])
    for name, t, dt in (("weights", weights, torch.float32), ("X", X, torch.float32), ("Y", Y, torch.float32),
                        ("mask", mask, torch.uint8), ("loss", loss, torch.float32), ("grad", grad, torch.float32)):
        if not (_is_torch(t) and t.is_cuda and t.is_contiguous() and t.dtype == dt):
            raise TypeError(f"{name} must be a contiguous cuda tensor of {dt}")
    P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    _check(lib().bc_mlp_loss_grad_noalloc(P(weights), P(X), P(Y), P(mask), n, P(loss), P(grad), _stream(stream)))


def bc_mlp_train(weights, X, Y, mask, steps: int, lr: float):
    """Adam training; returns (new weights, final loss)."""
    n = int(np.asarray(X).shape[0])
    w = _f32(weights, (BC_MLP_PARAMS,)).copy()
    x = _f32(X, (n, BC_MLP_IN))
    y = _f32(Y, (n, BC_MLP_OUT))
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(n, BC_MLP_OUT)
    loss = ctypes.c_float()
    _check(lib().bc_mlp_train(_p(w), _p(x), _p(y), _p(m), n, int(steps), float(lr), ctypes.byref(loss), None))
    return w, float(loss.value)


def bc_mlp_predict(weights, X):
    n = int(np.asarray(X).shape[0])
    w = _f32(weights, (BC_MLP_PARAMS,))
    x = _f32(X, (n, BC_MLP_IN))
    y = np.zeros((n, BC_MLP_OUT), np.float32)
    _check(lib().bc_mlp_predict(_p(w), _p(x), n, _p(y), None))
    return y


def bc_collect_level_times(h, sources, cap: int = 100000, options: RunOptions | None = None, stream=None):
    """Timed steps of a real run: (features, log2 microseconds of each
    choice; NaN where a sample's choice is another one)."""
    s = np.ascontiguousarray(sources, dtype=np.int32)
    X = np.zeros((cap, BC_MLP_IN), np.float32)
    Y = np.zeros((cap, BC_MLP_OUT), np.float32)
    cnt = ctypes.c_int64()
    _check(lib().bc_collect_level_times(h, _p(s), s.size, ctypes.byref(options) if options is not None else None,
                                        _p(X), _p(Y), cap, ctypes.byref(cnt), _stream(stream)))
    k = cnt.value
    return X[:k].copy(), Y[:k].copy()


class Graph:
    """Owning handle: ``with Graph(csr) as g: g.run(sources); g.scores()``."""

    def __init__(self, csr=None, row_ptr=None, col_idx=None, vtx_offsets=None, flags: int = 0):
        weights = None
        if csr is not None:
            row_ptr, col_idx = csr.row_ptr, csr.col_idx
            if getattr(csr, "directed", False):
                flags |= BC_DIRECTED
            weights = getattr(csr, "weights", None)
            if vtx_offsets is None and getattr(csr, "vtx_offsets", None) is not None and len(csr.vtx_offsets) > 2:
                vtx_offsets = csr.vtx_offsets
        if weights is not None:
            self.h = bc_graph_create_weighted(row_ptr, col_idx, weights, flags)
        elif vtx_offsets is not None:
            self.h = bc_graph_create_multi(vtx_offsets, row_ptr, col_idx, flags)
        else:
            self.h = bc_graph_create(row_ptr, col_idx, flags)
        self.n = bc_graph_info(self.h)["n"]

    def run(self, sources=None, stream=None, **opts):
        bc_run(self.h, sources, make_options(**opts), stream)
        return self

    def scores(self, out=None, stream=None):
        return bc_scores(self.h, out, stream)

    def detail(self, sources, dump_index=0, stream=None, **opts):
        return bc_run_detail(self.h, sources, dump_index, make_options(**opts), stream)

    def stats(self):
        return bc_run_stats(self.h)

    def level_stats(self):
        return bc_run_level_stats(self.h)

    def set_device_limit(self, max_device_bytes: int):
        bc_set_device_limit(self.h, max_device_bytes)

    def load_policy(self, weights):
        bc_load_policy(self.h, weights)

    def autotune(self, sample, stream=None, **opts):
        return bc_autotune(self.h, sample, make_options(**opts), stream)

    def collect_level_times(self, sources, cap=100000, stream=None, **opts):
        return bc_collect_level_times(self.h, sources, cap, make_options(**opts), stream)

    def info(self):
        return bc_graph_info(self.h)

    def close(self):
        if getattr(self, "h", None):
            bc_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
