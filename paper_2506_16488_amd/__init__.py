"""MI355X (gfx950) exact point-to-point shortest paths: Python binding.

A thin ctypes layer over ``libppsp.so`` (C interface in ``include/ppsp.h``).
Every step of the search runs in the library's HIP kernels; this module only
marshals arguments. There is no CPU fallback: if the library is not built,
importing the functions raises.

Module-level functions carry the C names without the ``ppsp_`` prefix
(``graph_create``, ``query``, ``batch_query``, ``last_stats``, ...); the
``Graph`` class wraps a handle for convenience. PyTorch is used only to
obtain the caller's current HIP stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libppsp.so")

INF = (1 << 64) - 1

OK, E_INVALID, E_RANGE, E_OOM, E_OVERFLOW, E_NOCOORD, E_NOTSYM, E_DEVICE, E_BUSY, E_PATHCAP, E_NOPATH, \
    E_TIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, -11

ALGO = {"sssp": 0, "et": 1, "astar": 2, "bids": 3, "bidastar": 4}
BATCH = {"plain": 0, "plainstar": 1, "multi": 2, "sssp": 3, "vc": 4, "auto": 5}
SCHED = {"fixed": 0, "autotuned": 1, "learned": 2, "rho": 3}
SYMMETRIC = 1
WANT_PATH = 1
MEMO_H = 2
PULL = 4
DEVICE_IO = 8


class PPSPError(RuntimeError):
    def __init__(self, code: int, where: str):
        detail = last_error()
        super().__init__("%s failed: %s (%d)%s" % (where, status_str(code), code,
                                                   (": " + detail) if detail else ""))
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("sched", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("delta", ctypes.c_uint64)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_uint64), ("entries", ctypes.c_uint64),
                ("scanned_vertices", ctypes.c_uint64), ("scanned_arcs", ctypes.c_uint64),
                ("relax_success", ctypes.c_uint64), ("searches", ctypes.c_uint64),
                ("waves", ctypes.c_uint64), ("wall_ms", ctypes.c_double),
                ("relax_kernel_ms", ctypes.c_double), ("relax_launches", ctypes.c_uint64),
                ("carried", ctypes.c_uint64), ("retries", ctypes.c_uint64), ("relax_timed", ctypes.c_uint64),
                ("heavy_kernel_ms", ctypes.c_double), ("heavy_arcs", ctypes.c_uint64), ("heavy_chunks", ctypes.c_uint64),
                ("heavy_success", ctypes.c_uint64), ("dense_searches", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_uint64), ("theta_mode", ctypes.c_uint32), ("grid_blocks", ctypes.c_uint32),
                ("ms", ctypes.c_double), ("default_ms", ctypes.c_double), ("trials", ctypes.c_uint32),
                ("from_cache", ctypes.c_uint32), ("heavy_window", ctypes.c_uint32), ("local_chunks", ctypes.c_uint32),
                ("dense_min", ctypes.c_uint64), ("dense_ring", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerCounters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("admitted", "completed", "chunks", "rounds", "running", "slots",
                                               "pending", "restarts", "renumbers")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class FitReport(ctypes.Structure):
    _fields_ = [("label_hist", ctypes.c_uint32 * 8), ("rows", ctypes.c_uint64), ("loss_first", ctypes.c_double),
                ("loss_last", ctypes.c_double), ("train_acc", ctypes.c_double), ("label_ms", ctypes.c_double),
                ("train_ms", ctypes.c_double), ("c_round_ms", ctypes.c_double), ("c_arc_ns", ctypes.c_double),
                ("best_fixed_bin", ctypes.c_uint32), ("fallback_bin", ctypes.c_uint32),
                ("learned_ms", ctypes.c_double), ("fixed_ms", ctypes.c_double), ("c_entry_ns", ctypes.c_double),
                ("variants", ctypes.c_uint32), ("heldout", ctypes.c_uint32), ("heldout_learned_ms", ctypes.c_double),
                ("heldout_fixed_ms", ctypes.c_double), ("heldout_learned_cost", ctypes.c_double),
                ("heldout_fixed_cost", ctypes.c_double), ("plain_fallback", ctypes.c_uint32),
                ("dense_labels", ctypes.c_uint32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["label_hist"] = list(self.label_hist)
        return d


class TraceSpec(ctypes.Structure):
    _fields_ = [("bins", ctypes.c_void_p), ("bins_after", ctypes.c_void_p), ("switch_round", ctypes.c_void_p),
                ("network", ctypes.c_uint32), ("distinct", ctypes.c_uint32), ("cap", ctypes.c_uint64),
                ("feat", ctypes.c_void_p), ("row_pair", ctypes.c_void_p), ("row_round", ctypes.c_void_p),
                ("row_side", ctypes.c_void_p), ("row_bin", ctypes.c_void_p), ("nrows", ctypes.c_uint64),
                ("pair_rounds", ctypes.c_void_p), ("pair_arcs", ctypes.c_void_p), ("pair_entries", ctypes.c_void_p),
                ("dist", ctypes.c_void_p)]


MLP_FEATURES, MLP_BINS, MLP_OUTPUTS, MLP_PARAMS = 12, 8, 9, 5577

EXPORTS = ["ppsp_graph_create", "ppsp_graph_destroy", "ppsp_query", "ppsp_batch_query", "ppsp_last_stats",
           "ppsp_set_option", "ppsp_get_option", "ppsp_heuristic_fx", "ppsp_status_str", "ppsp_version",
           "ppsp_last_error", "ppsp_tune", "ppsp_server_create", "ppsp_server_submit", "ppsp_server_poll",
           "ppsp_server_wait", "ppsp_server_stats", "ppsp_server_destroy", "ppsp_mlp_forward", "ppsp_mlp_grad",
           "ppsp_mlp_train", "ppsp_mlp_load", "ppsp_sched_trace", "ppsp_mlp_fit",
           "ppsp_query_cover", "ppsp_sssp", "ppsp_batch_query_noalloc", "ppsp_sched_trace_ex"]

_lib_handle = None


def lib():
    """The loaded libppsp.so; raises if it has not been built."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(SO_PATH):
            raise ImportError("libppsp.so is not built (run __graft_entry__.build() or "
                              "python paper_2506_16488_amd/build.py)")
        # torch ships its own HIP runtime under the same soname; loading torch
        # first makes the library bind to that one runtime, so torch's streams
        # and device memory are valid here (two runtimes in one process do not
        # share devices).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(SO_PATH)
        u32, u64, i32, i64, P = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        L.ppsp_graph_create.argtypes = [ctypes.c_int, u32, u64, P, P, P, P, u32, u32, u32, P, ctypes.POINTER(P)]
        L.ppsp_graph_create.restype = ctypes.c_int
        L.ppsp_graph_destroy.argtypes = [P]
        L.ppsp_graph_destroy.restype = ctypes.c_int
        L.ppsp_query.argtypes = [P, u32, u32, ctypes.POINTER(Opts), P, ctypes.POINTER(u64), P, u32,
                                 ctypes.POINTER(u32)]
        L.ppsp_query.restype = ctypes.c_int
        L.ppsp_batch_query.argtypes = [P, P, u32, ctypes.POINTER(Opts), P, P, P, P, u64]
        L.ppsp_batch_query.restype = ctypes.c_int
        L.ppsp_batch_query_noalloc.argtypes = [P, P, u32, ctypes.POINTER(Opts), P, P]
        L.ppsp_batch_query_noalloc.restype = ctypes.c_int
        L.ppsp_sched_trace_ex.argtypes = [P, P, u32, ctypes.POINTER(Opts), ctypes.POINTER(TraceSpec)]
        L.ppsp_sched_trace_ex.restype = ctypes.c_int
        L.ppsp_last_stats.argtypes = [P, ctypes.POINTER(Stats)]
        L.ppsp_last_stats.restype = ctypes.c_int
        L.ppsp_set_option.argtypes = [P, ctypes.c_char_p, i64]
        L.ppsp_set_option.restype = ctypes.c_int
        L.ppsp_get_option.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(i64)]
        L.ppsp_get_option.restype = ctypes.c_int
        L.ppsp_heuristic_fx.argtypes = [i32, i32, i32, i32, u32, u32]
        L.ppsp_heuristic_fx.restype = u64
        L.ppsp_status_str.argtypes = [ctypes.c_int]
        L.ppsp_status_str.restype = ctypes.c_char_p
        L.ppsp_tune.argtypes = [P, P, u32, ctypes.POINTER(Opts), ctypes.c_char_p, ctypes.POINTER(TuneResult)]
        L.ppsp_tune.restype = ctypes.c_int
        L.ppsp_last_error.argtypes = []
        L.ppsp_last_error.restype = ctypes.c_char_p
        L.ppsp_version.argtypes = []
        L.ppsp_version.restype = ctypes.c_char_p
        L.ppsp_server_create.argtypes = [P, u32, ctypes.POINTER(Opts), u64, ctypes.POINTER(P)]
        L.ppsp_server_submit.argtypes = [P, u32, P, u32, ctypes.POINTER(u64)]
        L.ppsp_server_poll.argtypes = [P, u64, P, ctypes.POINTER(ctypes.c_double)]
        L.ppsp_server_wait.argtypes = [P, u64, P, ctypes.POINTER(ctypes.c_double), u32]
        L.ppsp_server_stats.argtypes = [P, ctypes.POINTER(ServerCounters)]
        L.ppsp_server_destroy.argtypes = [P]
        for f in ("create", "submit", "poll", "wait", "stats", "destroy"):
            getattr(L, "ppsp_server_" + f).restype = ctypes.c_int
        L.ppsp_mlp_forward.argtypes = [ctypes.c_int, P, P, u32, P]
        L.ppsp_mlp_grad.argtypes = [ctypes.c_int, P, P, P, u32, P, ctypes.POINTER(ctypes.c_double)]
        L.ppsp_mlp_train.argtypes = [ctypes.c_int, P, P, P, u32, u32, u32, ctypes.c_float, u64,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.ppsp_mlp_load.argtypes = [P, P]
        L.ppsp_sched_trace.argtypes = [P, P, u32, ctypes.POINTER(Opts), P, P, P, u64, ctypes.POINTER(u64), P, P]
        L.ppsp_mlp_fit.argtypes = [P, P, u32, ctypes.POINTER(Opts), P, u32, u64, u32, P, ctypes.POINTER(FitReport)]
        for f in ("forward", "grad", "train", "load", "fit"):
            getattr(L, "ppsp_mlp_" + f).restype = ctypes.c_int
        L.ppsp_sched_trace.restype = ctypes.c_int
        L.ppsp_query_cover.argtypes = [P, u32, u32, P, P, ctypes.POINTER(u32)]
        L.ppsp_query_cover.restype = ctypes.c_int
        L.ppsp_sssp.argtypes = [P, u32, ctypes.POINTER(Opts), P, P]
        L.ppsp_sssp.restype = ctypes.c_int
        _lib_handle = L
    return _lib_handle


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def current_stream():
    """The caller's current HIP stream from torch (None = default stream)."""
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


def _check(rc: int, where: str):
    if rc != OK:
        raise PPSPError(rc, where)


def status_str(code: int) -> str:
    try:
        return lib().ppsp_status_str(code).decode()
    except ImportError:
        return "status %d" % code


def last_error() -> str:
    try:
        return lib().ppsp_last_error().decode()
    except ImportError:
        return ""


def version() -> str:
    return lib().ppsp_version().decode()


def heuristic_fx(x0: int, y0: int, x1: int, y1: int, w_scale: int, frac_bits: int) -> int:
    return int(lib().ppsp_heuristic_fx(x0, y0, x1, y1, w_scale, frac_bits))


def make_opts(algo="bids", batch="plainstar", sched="fixed", delta=0, want_path=False, memo=False,
              pull=False) -> Opts:
    return Opts(ALGO[algo] if isinstance(algo, str) else int(algo),
                BATCH[batch] if isinstance(batch, str) else int(batch),
                SCHED[sched] if isinstance(sched, str) else int(sched),
                (WANT_PATH if want_path else 0) | (MEMO_H if memo else 0) | (PULL if pull else 0), int(delta))


REORDER = 4


def graph_create(n, row_ptr, col, w, coords=None, frac_bits=8, w_scale=1000, symmetric=True, device=0,
                 stream=None, reorder=False):
    """ppsp_graph_create: returns an opaque handle (c_void_p)."""
    rp = np.ascontiguousarray(row_ptr, np.uint64)
    col = np.ascontiguousarray(col, np.uint32)
    w = np.ascontiguousarray(w, np.uint32)
    xy = None if coords is None else np.ascontiguousarray(coords, np.int32).reshape(-1)
    h = ctypes.c_void_p()
    rc = lib().ppsp_graph_create(device, int(n), int(col.shape[0]), _ptr(rp), _ptr(col), _ptr(w), _ptr(xy),
                                 frac_bits, w_scale, (SYMMETRIC if symmetric else 0) | (REORDER if reorder else 0),
                                 stream if stream is not None else current_stream(), ctypes.byref(h))
    _check(rc, "ppsp_graph_create")
    return h


def graph_destroy(h):
    _check(lib().ppsp_graph_destroy(h), "ppsp_graph_destroy")


def query(h, s, t, opts: Opts, stream=None, want_path=False, path_cap=1 << 20):
    """ppsp_query: (distance, path or None)."""
    d = ctypes.c_uint64(0)
    plen = ctypes.c_uint32(0)
    path = np.empty(path_cap, np.uint32) if want_path else None
    rc = lib().ppsp_query(h, int(s), int(t), ctypes.byref(opts), stream if stream is not None else current_stream(),
                          ctypes.byref(d), _ptr(path), path_cap if want_path else 0, ctypes.byref(plen))
    if rc == E_PATHCAP and want_path:
        return query(h, s, t, opts, stream, want_path, int(plen.value))
    _check(rc, "ppsp_query")
    return int(d.value), (path[:plen.value].copy() if want_path else None)


def batch_query(h, pairs, opts: Opts, stream=None, want_path=False, path_cap=None):
    """ppsp_batch_query: distances (uint64, input order) and, with paths, (offsets, vertices)."""
    pairs = np.ascontiguousarray(pairs, np.uint32).reshape(-1, 2)
    k = pairs.shape[0]
    dist = np.empty(k, np.uint64)
    off = np.empty(k + 1, np.uint64) if want_path else None
    if want_path and path_cap is None:
        path_cap = max(1, 64 * k)
    vtx = np.empty(path_cap, np.uint32) if want_path else None
    st = stream if stream is not None else current_stream()
    for _ in range(8):
        rc = lib().ppsp_batch_query(h, _ptr(pairs), k, ctypes.byref(opts), st, _ptr(dist), _ptr(off), _ptr(vtx),
                                    path_cap if want_path else 0)
        if rc == E_PATHCAP and want_path:
            path_cap *= 4
            vtx = np.empty(path_cap, np.uint32)
            continue
        break
    _check(rc, "ppsp_batch_query")
    if want_path:
        return dist, (off, vtx[:int(off[k])].copy())
    return dist


def tune(h, pairs, opts: Opts, cache_path=None) -> dict:
    """ppsp_tune: choose Delta, threshold rule and launch shape on a sample batch."""
    pairs = np.ascontiguousarray(pairs, np.uint32).reshape(-1, 2)
    r = TuneResult()
    _check(lib().ppsp_tune(h, _ptr(pairs), pairs.shape[0], ctypes.byref(opts),
                           cache_path.encode() if cache_path else None, ctypes.byref(r)), "ppsp_tune")
    return r.as_dict()


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


def mlp_forward(params, X, device=0) -> np.ndarray:
    """Outputs [n][9] of feature rows X [n][12] (ppsp_mlp_forward): 8 bin logits, then the dense-mode logit."""
    p = _f32(params, (MLP_PARAMS,))
    X = _f32(X, (-1, MLP_FEATURES))
    out = np.empty((X.shape[0], MLP_OUTPUTS), np.float32)
    _check(lib().ppsp_mlp_forward(device, _ptr(p), _ptr(X), X.shape[0], _ptr(out)), "ppsp_mlp_forward")
    return out


def mlp_grad(params, X, y, device=0):
    """(mean cross-entropy loss, gradient) (ppsp_mlp_grad)."""
    p = _f32(params, (MLP_PARAMS,))
    X = _f32(X, (-1, MLP_FEATURES))
    y = np.ascontiguousarray(y, np.uint32)
    g = np.empty(MLP_PARAMS, np.float32)
    L = ctypes.c_double(0)
    _check(lib().ppsp_mlp_grad(device, _ptr(p), _ptr(X), _ptr(y), X.shape[0], _ptr(g), ctypes.byref(L)),
           "ppsp_mlp_grad")
    return L.value, g


def mlp_train(params, X, y, epochs, batch=512, lr=2e-3, seed=0, device=0):
    """(trained parameters, loss before, loss after) (ppsp_mlp_train)."""
    p = _f32(params, (MLP_PARAMS,)).copy()
    X = _f32(X, (-1, MLP_FEATURES))
    y = np.ascontiguousarray(y, np.uint32)
    l0, l1 = ctypes.c_double(0), ctypes.c_double(0)
    _check(lib().ppsp_mlp_train(device, _ptr(p), _ptr(X), _ptr(y), X.shape[0], int(epochs), int(batch), float(lr),
                                int(seed), ctypes.byref(l0), ctypes.byref(l1)), "ppsp_mlp_train")
    return p, l0.value, l1.value


def query_cover(pairs, directed=False):
    """(root per pair, 1 where the root is the pair's target, searches) of the
    query-graph vertex cover PPSP_BATCH_VC uses (ppsp_query_cover; host only)."""
    pairs = np.ascontiguousarray(pairs, np.uint32).reshape(-1, 2)
    k = pairs.shape[0]
    root = np.empty(k, np.uint32)
    ft = np.empty(k, np.uint8)
    size = ctypes.c_uint32(0)
    _check(lib().ppsp_query_cover(_ptr(pairs), k, 1 if directed else 0, _ptr(root), _ptr(ft), ctypes.byref(size)),
           "ppsp_query_cover")
    return root, ft, int(size.value)


def last_stats(h) -> dict:
    s = Stats()
    _check(lib().ppsp_last_stats(h, ctypes.byref(s)), "ppsp_last_stats")
    return s.as_dict()


def set_option(h, name: str, value: int):
    _check(lib().ppsp_set_option(h, name.encode(), int(value)), "ppsp_set_option")


def get_option(h, name: str) -> int:
    v = ctypes.c_int64(0)
    _check(lib().ppsp_get_option(h, name.encode(), ctypes.byref(v)), "ppsp_get_option")
    return int(v.value)


class Graph:
    """A graph resident on one GPU (owns a ppsp_graph handle)."""

    def __init__(self, n, row_ptr, col, w, coords=None, frac_bits=8, w_scale=1000, symmetric=True, device=0,
                 reorder=False):
        self.n = int(n)
        self.h = graph_create(n, row_ptr, col, w, coords, frac_bits, w_scale, symmetric, device, reorder=reorder)

    @classmethod
    def from_host(cls, g, device=0, w_scale=1000, reorder=False):
        """From any object with n, row_ptr, col, w, coords, frac_bits, symmetric."""
        return cls(g.n, g.row_ptr, g.col, g.w, getattr(g, "coords", None), getattr(g, "frac_bits", 8),
                   w_scale, getattr(g, "symmetric", True), device, reorder=reorder)

    def query(self, s, t, algo="bids", delta=0, want_path=False, memo=False, sched="fixed", pull=False):
        d, p = query(self.h, s, t, make_opts(algo, "plain", sched, delta, want_path, memo, pull), want_path=want_path)
        return (d, p) if want_path else d

    def batch_query(self, pairs, algo="bids", batch="plainstar", delta=0, want_path=False, memo=False,
                    sched="fixed", pull=False):
        return batch_query(self.h, pairs, make_opts(algo, batch, sched, delta, want_path, memo, pull),
                           want_path=want_path)

    def batch_query_device(self, pairs, dist, algo="bids", batch="plainstar", delta=0, sched="fixed"):
        """ppsp_batch_query with PPSP_DEVICE_IO: `pairs` (k x 2 int32/uint32) and `dist`
        (k int64, receives the distances; PPSP_INF reads as -1) are torch tensors on the
        graph's device, used in order on torch's current stream."""
        import torch
        assert pairs.is_cuda and dist.is_cuda and pairs.is_contiguous() and dist.is_contiguous()
        assert pairs.dtype in (torch.int32,) and dist.dtype == torch.int64
        k = pairs.shape[0]
        assert pairs.shape == (k, 2) and dist.shape == (k,)
        o = make_opts(algo, batch, sched, delta)
        o.flags |= DEVICE_IO
        _check(lib().ppsp_batch_query(self.h, ctypes.c_void_p(pairs.data_ptr()), k, ctypes.byref(o),
                                      current_stream(), ctypes.c_void_p(dist.data_ptr()), None, None, 0),
               "ppsp_batch_query")
        return dist

    def batch_query_noalloc(self, pairs, algo="bids", batch="plainstar", delta=0, sched="fixed", pull=False):
        """ppsp_batch_query_noalloc: the same distances, with every workspace
        buffer carved from the library's fixed device scratch (no allocation)."""
        pairs = np.ascontiguousarray(pairs, np.uint32).reshape(-1, 2)
        k = pairs.shape[0]
        dist = np.empty(k, np.uint64)
        o = make_opts(algo, batch, sched, delta, pull=pull)
        _check(lib().ppsp_batch_query_noalloc(self.h, _ptr(pairs), k, ctypes.byref(o), current_stream(), _ptr(dist)),
               "ppsp_batch_query_noalloc")
        return dist

    def batch_query_noalloc_device(self, pairs, dist, algo="bids", batch="plainstar", delta=0):
        """ppsp_batch_query_noalloc with PPSP_DEVICE_IO (torch tensors as in batch_query_device)."""
        import torch
        assert pairs.is_cuda and dist.is_cuda and pairs.dtype == torch.int32 and dist.dtype == torch.int64
        k = pairs.shape[0]
        assert pairs.shape == (k, 2) and dist.shape == (k,) and pairs.is_contiguous() and dist.is_contiguous()
        o = make_opts(algo, batch, "fixed", delta)
        o.flags |= DEVICE_IO
        _check(lib().ppsp_batch_query_noalloc(self.h, ctypes.c_void_p(pairs.data_ptr()), k, ctypes.byref(o),
                                              current_stream(), ctypes.c_void_p(dist.data_ptr())),
               "ppsp_batch_query_noalloc")
        return dist

    def sssp(self, s, delta=0, sched="fixed"):
        """Distances from s to every vertex (ppsp_sssp; PPSP_INF where unreachable)."""
        dist = np.empty(self.n, np.uint64)
        o = make_opts("sssp", "plain", sched, delta)
        _check(lib().ppsp_sssp(self.h, int(s), ctypes.byref(o), current_stream(), _ptr(dist)), "ppsp_sssp")
        return dist

    def stats(self) -> dict:
        return last_stats(self.h)

    def tune(self, pairs, algo="bids", batch="plainstar", cache_path=None) -> dict:
        return tune(self.h, pairs, make_opts(algo, batch), cache_path)

    def mlp_load(self, params):
        p = _f32(params, (MLP_PARAMS,))
        _check(lib().ppsp_mlp_load(self.h, _ptr(p)), "ppsp_mlp_load")

    def sched_trace(self, pairs, algo="bids", batch="plainstar", bins=None, cap=0, delta=0):
        """Fixed per-pair multiplier bins; returns (features [rows][12],
        row_pair, rows produced, pair_rounds, pair_arcs)."""
        pairs = np.ascontiguousarray(pairs, np.uint32).reshape(-1, 2)
        k = pairs.shape[0]
        b = None if bins is None else np.ascontiguousarray(np.broadcast_to(bins, (k,)), np.uint8)
        feat = np.empty((cap, MLP_FEATURES), np.float32)
        rowp = np.empty(cap, np.uint32)
        nrows = ctypes.c_uint64(0)
        pr = np.empty(k, np.uint32)
        pa = np.empty(k, np.uint64)
        _check(lib().ppsp_sched_trace(self.h, _ptr(pairs), k, ctypes.byref(make_opts(algo, batch, delta=delta)),
                                      _ptr(b), _ptr(feat) if cap else None, _ptr(rowp) if cap else None, int(cap),
                                      ctypes.byref(nrows), _ptr(pr), _ptr(pa)), "ppsp_sched_trace")
        kept = min(int(nrows.value), cap)
        return feat[:kept], rowp[:kept], int(nrows.value), pr, pa

    def sched_trace_ex(self, pairs, algo="bids", batch="plainstar", delta=0, bins=None, bins_after=None,
                       switch_round=None, network=False, distinct=False, cap=0):
        """ppsp_sched_trace_ex; returns a dict with rows (feat, pair, round,
        side, bin), nrows, and per pair rounds, arcs, entries and dist."""
        pairs = np.ascontiguousarray(pairs, np.uint32).reshape(-1, 2)
        k = pairs.shape[0]

        def per_pair(x, dt):
            return None if x is None else np.ascontiguousarray(np.broadcast_to(x, (k,)), dt)
        b, ba, sw = per_pair(bins, np.uint8), per_pair(bins_after, np.uint8), per_pair(switch_round, np.uint32)
        out = {"feat": np.empty((cap, MLP_FEATURES), np.float32), "pair": np.empty(cap, np.uint32),
               "round": np.empty(cap, np.uint32), "side": np.empty(cap, np.uint8), "bin": np.empty(cap, np.uint8),
               "pair_rounds": np.empty(k, np.uint32), "pair_arcs": np.empty(k, np.uint64),
               "pair_entries": np.empty(k, np.uint64), "dist": np.empty(k, np.uint64)}
        spec = TraceSpec(_ptr(b), _ptr(ba), _ptr(sw), 1 if network else 0, 1 if distinct else 0, int(cap),
                         _ptr(out["feat"]) if cap else None, _ptr(out["pair"]) if cap else None,
                         _ptr(out["round"]) if cap else None, _ptr(out["side"]) if cap else None,
                         _ptr(out["bin"]) if cap else None, 0, _ptr(out["pair_rounds"]), _ptr(out["pair_arcs"]),
                         _ptr(out["pair_entries"]), _ptr(out["dist"]))
        _check(lib().ppsp_sched_trace_ex(self.h, _ptr(pairs), k, ctypes.byref(make_opts(algo, batch, delta=delta)),
                                         ctypes.byref(spec)), "ppsp_sched_trace_ex")
        kept = min(int(spec.nrows), cap)
        for key in ("feat", "pair", "round", "side", "bin"):
            out[key] = out[key][:kept]
        out["nrows"] = int(spec.nrows)
        return out

    def mlp_fit(self, pairs, init, algo="bids", batch="plainstar", epochs=20, seed=0, delta=0, labels="single"):
        """Labels ("single": each pair timed alone; "batch": batch-aware),
        traces, trains and loads the learned schedule; returns (parameters,
        report dict)."""
        pairs = np.ascontiguousarray(pairs, np.uint32).reshape(-1, 2)
        p0 = _f32(init, (MLP_PARAMS,))
        out = np.empty(MLP_PARAMS, np.float32)
        rep = FitReport()
        mode = {"single": 0, "batch": 1, "counterfactual": 2}[labels]
        _check(lib().ppsp_mlp_fit(self.h, _ptr(pairs), pairs.shape[0], ctypes.byref(make_opts(algo, batch, delta=delta)),
                                  _ptr(p0), int(epochs), int(seed), mode, _ptr(out), ctypes.byref(rep)), "ppsp_mlp_fit")
        return out, rep.as_dict()

    def set_option(self, name, value):
        set_option(self.h, name, value)

    def get_option(self, name):
        return get_option(self.h, name)

    def close(self):
        if getattr(self, "h", None):
            graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass




class Server:
    """Continuous-batching server over resident graphs (ppsp_server_*): queries
    submitted while others run are admitted between rounds into free slots."""

    def __init__(self, graphs, algo="bidastar", delta=0, state_budget_bytes=1 << 30, sched="fixed"):
        """algo, delta and sched: one value for every graph, or a list with one per graph."""
        self.graphs = list(graphs)
        k = len(self.graphs)
        algos = list(algo) if isinstance(algo, (list, tuple)) else [algo] * k
        deltas = list(delta) if isinstance(delta, (list, tuple)) else [delta] * k
        scheds = list(sched) if isinstance(sched, (list, tuple)) else [sched] * k
        hs = (ctypes.c_void_p * k)(*[g.h for g in self.graphs])
        opts = (Opts * k)(*[make_opts(a, "plainstar", sc, delta=d) for a, d, sc in zip(algos, deltas, scheds)])
        h = ctypes.c_void_p()
        _check(lib().ppsp_server_create(hs, k, opts, int(state_budget_bytes), ctypes.byref(h)), "ppsp_server_create")
        self.h = h
        self.k = {}

    def submit(self, graph_id, pairs) -> int:
        pairs = np.ascontiguousarray(pairs, np.uint32).reshape(-1, 2)
        rid = ctypes.c_uint64(0)
        _check(lib().ppsp_server_submit(self.h, int(graph_id), _ptr(pairs), pairs.shape[0], ctypes.byref(rid)),
               "ppsp_server_submit")
        self.k[rid.value] = pairs.shape[0]
        return int(rid.value)

    def poll(self, rid):
        """(distances, latency_ms) once the request finished, else None."""
        d = np.empty(self.k[rid], np.uint64)
        lat = ctypes.c_double(0)
        rc = lib().ppsp_server_poll(self.h, rid, _ptr(d), ctypes.byref(lat))
        if rc == E_BUSY:
            return None
        _check(rc, "ppsp_server_poll")
        del self.k[rid]
        return d, lat.value

    def wait(self, rid, timeout_ms=60000):
        d = np.empty(self.k[rid], np.uint64)
        lat = ctypes.c_double(0)
        _check(lib().ppsp_server_wait(self.h, rid, _ptr(d), ctypes.byref(lat), int(timeout_ms)), "ppsp_server_wait")
        del self.k[rid]
        return d, lat.value

    def stats(self) -> dict:
        c = ServerCounters()
        _check(lib().ppsp_server_stats(self.h, ctypes.byref(c)), "ppsp_server_stats")
        return c.as_dict()

    def close(self):
        if getattr(self, "h", None):
            lib().ppsp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
