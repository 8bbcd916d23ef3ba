"""CPU oracle for exact point-to-point shortest-path distances.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does. It shares no code with the GPU library (``paper_2506_16488_amd``) and
does not import it.

The result being checked is the plain definition of d(s,t) (Section 1
problem statement, Section 2 notation): the minimum total weight of an s->t
path, 0 for s = t, and "infinity" (``INF`` = 2**64 - 1) when t is
unreachable. All of the method's search modes are exact (Theorems
bids-correctness and bdastar-correctness, the soundness of the early
termination and A* pruning rules of Sections 3.2-3.3), so the oracle is that
definition computed by textbook Dijkstra (``oracle.c``), pinned by
Floyd-Warshall, Bellman-Ford, closed forms and an optimality certificate in
the CPU test suite.

Readings of the paper that affect the expected values (all exact integer):
  * s = t gives 0 (the paper's update rule alone would not produce it).
  * unreachable pairs give INF (the disconnected-query rule of Appendix B).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

INF = (1 << 64) - 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, pthreads)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        u64, u32, P = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        L.oracle_dijkstra.argtypes = [u64, P, P, P, u32, u32, P, P]
        L.oracle_dijkstra.restype = u64
        L.oracle_pp_batch.argtypes = [u64, P, P, P, u64, P, P, ctypes.c_int]
        L.oracle_pp_batch.restype = None
        L.oracle_floyd_warshall.argtypes = [u64, P, P, P, P]
        L.oracle_floyd_warshall.restype = None
        L.oracle_bellman_ford.argtypes = [u64, P, P, P, u32, P]
        L.oracle_bellman_ford.restype = u64
        L.oracle_check_sssp.argtypes = [u64, P, P, P, u32, P, ctypes.POINTER(u64)]
        L.oracle_check_sssp.restype = ctypes.c_int
        L.oracle_check_path.argtypes = [u64, P, P, P, P, u64, u32, u32, u64, ctypes.POINTER(u64)]
        L.oracle_check_path.restype = ctypes.c_int
        _lib_handle = L
    return _lib_handle


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _csr(row_ptr, col, w):
    return (np.ascontiguousarray(row_ptr, np.uint64), np.ascontiguousarray(col, np.uint32),
            np.ascontiguousarray(w, np.uint32))


def sssp(n, row_ptr, col, w, s, parents=False):
    """Exact distances from s to every vertex (uint64, INF if unreachable)."""
    rp, col, w = _csr(row_ptr, col, w)
    dist = np.empty(n, np.uint64)
    par = np.empty(n, np.uint32) if parents else None
    _lib().oracle_dijkstra(n, _p(rp), _p(col), _p(w), s, 0xFFFFFFFF, _p(dist), _p(par))
    return (dist, par) if parents else dist


def pp(n, row_ptr, col, w, s, t):
    """d(s, t) by Dijkstra stopped when t is popped."""
    rp, col, w = _csr(row_ptr, col, w)
    dist = np.empty(n, np.uint64)
    return int(_lib().oracle_dijkstra(n, _p(rp), _p(col), _p(w), s, t, _p(dist), None))


def pp_batch(n, row_ptr, col, w, pairs, nthreads=None):
    """d(s_q, t_q) for an array of pairs (k, 2); one Dijkstra per pair."""
    rp, col, w = _csr(row_ptr, col, w)
    pairs = np.ascontiguousarray(pairs, np.uint32).reshape(-1, 2)
    out = np.empty(pairs.shape[0], np.uint64)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    _lib().oracle_pp_batch(n, _p(rp), _p(col), _p(w), pairs.shape[0], _p(pairs), _p(out), int(nthreads))
    return out


def floyd_warshall(n, row_ptr, col, w):
    """All-pairs distance matrix (n x n, uint64)."""
    rp, col, w = _csr(row_ptr, col, w)
    D = np.empty((n, n), np.uint64)
    _lib().oracle_floyd_warshall(n, _p(rp), _p(col), _p(w), _p(D))
    return D


def bellman_ford(n, row_ptr, col, w, s):
    rp, col, w = _csr(row_ptr, col, w)
    dist = np.empty(n, np.uint64)
    _lib().oracle_bellman_ford(n, _p(rp), _p(col), _p(w), s, _p(dist))
    return dist


def check_sssp(n, row_ptr, col, w, s, dist):
    """(code, vertex): code 0 iff dist is the exact distance function from s (w >= 1)."""
    rp, col, w = _csr(row_ptr, col, w)
    dist = np.ascontiguousarray(dist, np.uint64)
    bad = ctypes.c_uint64(0)
    rc = _lib().oracle_check_sssp(n, _p(rp), _p(col), _p(w), s, _p(dist), ctypes.byref(bad))
    return rc, bad.value


def check_path(n, row_ptr, col, w, path, s, t, d):
    """(code, info): code 0 iff path is an s->t path of total weight d."""
    rp, col, w = _csr(row_ptr, col, w)
    path = np.ascontiguousarray(path, np.uint32)
    bad = ctypes.c_uint64(0)
    rc = _lib().oracle_check_path(n, _p(rp), _p(col), _p(w), _p(path), path.shape[0], s, t, d,
                                  ctypes.byref(bad))
    return rc, bad.value
