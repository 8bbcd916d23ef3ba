"""Seeded synthetic inputs: graphs in CSR form, coordinates and s-t pairs.

This package is the only code shared by the CPU oracle tests and the GPU
path. It holds input construction only (no relaxation, pruning or heuristic
arithmetic). The heavy generators are C (``gen.c``, OpenMP) loaded through
ctypes; tiny test graphs are built with numpy.

The workloads are synthetic stand-ins for the paper's datasets
(Section 6, Table 3): a uniform-weight grid, road-like jittered lattices
(weights = ceil(1000 * Euclidean length), coordinates in fixed point with 8
fractional bits) and a power-law R-MAT graph with integer weights.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libppspgen.so")
_SRC = os.path.join(_HERE, "gen.c")

FRAC_BITS = 8  # fixed-point fractional bits of lattice coordinates


def build(force: bool = True) -> str:
    """Compile gen.c into libppspgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        u64, u32, i32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_double
        P = ctypes.c_void_p
        L.gen_rand.argtypes = [u64, u64, u64]; L.gen_rand.restype = u64
        L.gen_isqrt_floor.argtypes = [u64]; L.gen_isqrt_floor.restype = u64
        L.gen_isqrt_ceil.argtypes = [u64]; L.gen_isqrt_ceil.restype = u64
        L.gen_lattice_weight.argtypes = [i32, i32, u32]; L.gen_lattice_weight.restype = u32
        L.gen_grid_arcs.argtypes = [u32, u32]; L.gen_grid_arcs.restype = u64
        L.gen_grid.argtypes = [u32, u32, u32, u32, u64, P, P, P]; L.gen_grid.restype = None
        L.gen_lattice_coords.argtypes = [u32, u32, u64, P]; L.gen_lattice_coords.restype = None
        L.gen_lattice_rowptr.argtypes = [u32, dbl, u64, P]; L.gen_lattice_rowptr.restype = u64
        L.gen_lattice_arcs.argtypes = [u32, dbl, u64, P, u32, P, P, P]; L.gen_lattice_arcs.restype = None
        L.gen_rmat_begin.argtypes = [u32, u32, dbl, dbl, dbl, u32, u32, u64, ctypes.POINTER(u64)]
        L.gen_rmat_begin.restype = P
        L.gen_rmat_finish.argtypes = [P, P, P, P]; L.gen_rmat_finish.restype = None
        L.gen_lcc.argtypes = [u64, P, P, P]; L.gen_lcc.restype = u64
        L.gen_pairs_uniform.argtypes = [u64, P, u64, ctypes.c_int, u64, u64, P]
        L.gen_pairs_uniform.restype = None
        L.gen_pairs_hub.argtypes = [u64, P, u64, u64, u64, u64, u64, P]
        L.gen_pairs_hub.restype = None
        _lib_handle = L
    return _lib_handle


def _p(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


@dataclass
class Graph:
    """Host CSR graph. Arcs of vertex v are col[row_ptr[v]:row_ptr[v+1]]."""
    n: int
    row_ptr: np.ndarray            # uint64, n+1
    col: np.ndarray                # uint32, m
    w: np.ndarray                  # uint32, m
    coords: Optional[np.ndarray] = None   # int32, (n, 2) fixed point, or None
    frac_bits: int = FRAC_BITS
    symmetric: bool = True
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0])


def rand_u64(seed: int, stream: int, idx: int) -> int:
    return int(_lib().gen_rand(seed, stream, idx))


def isqrt_floor(x: int) -> int:
    return int(_lib().gen_isqrt_floor(x))


def isqrt_ceil(x: int) -> int:
    return int(_lib().gen_isqrt_ceil(x))


def lattice_weight(dx: int, dy: int, frac_bits: int = FRAC_BITS) -> int:
    return int(_lib().gen_lattice_weight(dx, dy, frac_bits))


def grid(R: int, C: int, wlo: int = 1, whi: int = 1000, seed: int = 1) -> Graph:
    """R x C 4-neighbour grid, weights uniform in [wlo, whi] per undirected edge."""
    L = _lib()
    n = R * C
    m = int(L.gen_grid_arcs(R, C))
    rp = np.empty(n + 1, np.uint64)
    col = np.empty(m, np.uint32)
    w = np.empty(m, np.uint32)
    L.gen_grid(R, C, wlo, whi, seed, _p(rp), _p(col), _p(w))
    return Graph(n, rp, col, w, name="grid%dx%d" % (R, C))


def lattice(Lside: int, p_diag: float = 0.05, seed: int = 2, frac_bits: int = FRAC_BITS) -> Graph:
    """Jittered Lside x Lside lattice with random short diagonals (road-like)."""
    L = _lib()
    n = Lside * Lside
    xy = np.empty((n, 2), np.int32)
    L.gen_lattice_coords(Lside, frac_bits, seed, _p(xy))
    rp = np.empty(n + 1, np.uint64)
    m = int(L.gen_lattice_rowptr(Lside, p_diag, seed, _p(rp)))
    col = np.empty(m, np.uint32)
    w = np.empty(m, np.uint32)
    L.gen_lattice_arcs(Lside, p_diag, seed, _p(xy), frac_bits, _p(rp), _p(col), _p(w))
    return Graph(n, rp, col, w, coords=xy, frac_bits=frac_bits, name="lattice%d" % Lside)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         wlo: int = 1, whi: int = 65535, seed: int = 4) -> Graph:
    """Symmetrised, deduplicated R-MAT graph with per-pair hashed weights."""
    L = _lib()
    m = ctypes.c_uint64(0)
    h = L.gen_rmat_begin(scale, edge_factor, a, b, c, wlo, whi, seed, ctypes.byref(m))
    n = 1 << scale
    rp = np.empty(n + 1, np.uint64)
    col = np.empty(m.value, np.uint32)
    w = np.empty(m.value, np.uint32)
    L.gen_rmat_finish(h, _p(rp), _p(col), _p(w))
    return Graph(n, rp, col, w, name="rmat%d" % scale)


def lcc(g: Graph) -> np.ndarray:
    """Vertices of the largest connected component, ascending (uint32)."""
    out = np.empty(g.n, np.uint32)
    k = int(_lib().gen_lcc(g.n, _p(g.row_ptr), _p(g.col), _p(out)))
    return out[:k].copy()


def pairs_uniform(n_or_cand, k: int, seed: int, distinct: bool = False, stream: int = 0) -> np.ndarray:
    """k uniform (s,t) pairs, shape (k,2) uint32, over range(n) or a candidate list."""
    out = np.empty((k, 2), np.uint32)
    if isinstance(n_or_cand, np.ndarray):
        cand = np.ascontiguousarray(n_or_cand, np.uint32)
        _lib().gen_pairs_uniform(cand.shape[0], _p(cand), k, int(distinct), seed, stream, _p(out))
    else:
        _lib().gen_pairs_uniform(int(n_or_cand), None, k, int(distinct), seed, stream, _p(out))
    return out


def pairs_hub(n_or_cand, n_hubs: int, k_hub: int, k: int, seed: int, batch: int = 0) -> np.ndarray:
    """Batch of k pairs: the first k_hub share sources drawn from n_hubs hubs."""
    out = np.empty((k, 2), np.uint32)
    if isinstance(n_or_cand, np.ndarray):
        cand = np.ascontiguousarray(n_or_cand, np.uint32)
        _lib().gen_pairs_hub(cand.shape[0], _p(cand), n_hubs, k_hub, k, seed, batch, _p(out))
    else:
        _lib().gen_pairs_hub(int(n_or_cand), None, n_hubs, k_hub, k, seed, batch, _p(out))
    return out


# ---- tiny graphs for tests (numpy) -----------------------------------------

def csr_from_edges(n: int, src, dst, w, symmetric: bool = True, coords=None) -> Graph:
    """CSR from an edge list; symmetric=True adds the reverse of every edge.
    Multi-edges and self-loops are kept as given."""
    src = np.asarray(src, np.int64); dst = np.asarray(dst, np.int64); w = np.asarray(w, np.uint32)
    if symmetric:
        src, dst, w = np.concatenate([src, dst]), np.concatenate([dst, src]), np.concatenate([w, w])
    order = np.lexsort((dst, src))
    src, dst, w = src[order], dst[order], w[order]
    rp = np.zeros(n + 1, np.uint64)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp).astype(np.uint64)
    return Graph(n, rp, dst.astype(np.uint32), w.astype(np.uint32), coords=coords, symmetric=symmetric)


def random_graph(n: int, m_edges: int, wmax: int, seed: int, wmin: int = 1,
                 symmetric: bool = True, allow_loops: bool = False) -> Graph:
    """Uniform random (multi)graph with m_edges edges, weights in [wmin, wmax]."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m_edges)
    dst = rng.integers(0, n, m_edges)
    if not allow_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    w = rng.integers(wmin, wmax + 1, src.shape[0])
    return csr_from_edges(n, src, dst, w, symmetric=symmetric)


# ---- the benchmark workloads -----------------------------------------------------

# The benchmark workloads by name: graph seed and pair seed 100 + graph seed.
WORKLOAD_SEEDS = {"grid256": 1, "lattice2048": 2, "lattice4096": 3, "rmat24": 4}


def workload_graph(name: str) -> Graph:
    """grid256: 256 x 256 grid, weights U[1, 1000]; lattice2048 / lattice4096:
    jittered lattices with 5% diagonals; rmat24: R-MAT scale 24, edge factor 16,
    weights U[1, 65535]."""
    seed = WORKLOAD_SEEDS[name]
    if name == "grid256":
        return grid(256, 256, 1, 1000, seed=seed)
    if name == "lattice2048":
        return lattice(2048, 0.05, seed=seed)
    if name == "lattice4096":
        return lattice(4096, 0.05, seed=seed)
    return rmat(24, 16, 0.57, 0.19, 0.19, 1, 65535, seed=seed)


def workload_pairs(name: str, g: Graph, batch: int = 0, cand: Optional[np.ndarray] = None) -> np.ndarray:
    """grid256: 64 distinct uniform pairs; lattice2048: 1,000 uniform pairs;
    lattice4096: batches of 1,024 (512 from 32 hubs, 512 uniform); rmat24: 256
    uniform pairs from the largest component (or `cand`)."""
    seed = 100 + WORKLOAD_SEEDS[name]
    if name == "grid256":
        return pairs_uniform(g.n, 64, seed, distinct=True)
    if name == "lattice2048":
        return pairs_uniform(g.n, 1000, seed)
    if name == "lattice4096":
        return pairs_hub(g.n, 32, 512, 1024, seed, batch)
    if cand is None:
        cand = lcc(g)
    return pairs_uniform(cand, 256, seed, stream=batch * 16)


# ---- learned-schedule network: initial parameters and synthetic rows ----------

MLP_SHAPES = [(64, 12), (64,), (64, 64), (64,), (9, 64), (9,)]


def mlp_init(seed: int) -> np.ndarray:
    """Initial parameters of the 12-64-64-9 network (flat float32, W1 b1 W2 b2
    W3 b3): weights uniform in +-sqrt(6 / fan_in), biases 0."""
    rng = np.random.default_rng(seed)
    out = []
    for shp in MLP_SHAPES:
        if len(shp) == 2:
            lim = np.sqrt(6.0 / shp[1])
            out.append(rng.uniform(-lim, lim, shp).reshape(-1))
        else:
            out.append(np.zeros(shp))
    return np.concatenate(out).astype(np.float32)


def mlp_rows(n: int, seed: int, learnable: bool = True, modes: bool = False):
    """n synthetic feature rows in [-1, 1) and labels: a bin in 0..7, plus 8 x
    a mode label (1 sparse, 2 dense) when modes=True (else 0: none). With
    learnable=True the bin is a fixed function of the first two features and
    the mode of the third."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, (n, 12)).astype(np.float32)
    if learnable:
        y = np.clip(np.floor(4.0 + 2.0 * X[:, 0] + 1.5 * X[:, 1]), 0, 7).astype(np.uint32)
        m = np.where(X[:, 2] > 0.2, 2, 1)
    else:
        y = rng.integers(0, 8, n).astype(np.uint32)
        m = rng.integers(1, 3, n)
    if modes:
        y = (y + 8 * m).astype(np.uint32)
    return X, y


# ---- batch patterns (query graphs of Section 4.1 and the batch experiments) ----

PATTERNS = ["star", "fork", "chain", "cycle", "bipartite", "clique", "separate", "random"]


def pattern_edges(kind: str, m: int = 6, k: int = 0, seed: int = 0):
    """Query-graph edges over vertices 0..m-1: star (one hub), fork (two hubs
    joined, each with leaves), chain (multi-stop), cycle, bipartite (halves,
    pairwise), clique (subset APSP), separate (disjoint pairs), random (k
    distinct pairs, k = 8 by default)."""
    if kind == "star":
        return [(0, j) for j in range(1, m)]
    if kind == "fork":
        h = m // 2
        return [(0, 1)] + [(0, j) for j in range(2, h + 1)] + [(1, j) for j in range(h + 1, m)]
    if kind == "chain":
        return [(j, j + 1) for j in range(m - 1)]
    if kind == "cycle":
        return [(j, (j + 1) % m) for j in range(m)]
    if kind == "bipartite":
        h = m // 2
        return [(a, b) for a in range(h) for b in range(h, m)]
    if kind == "clique":
        return [(a, b) for a in range(m) for b in range(a + 1, m)]
    if kind == "separate":
        return [(2 * j, 2 * j + 1) for j in range(m // 2)]
    if kind == "random":
        rng = np.random.default_rng(seed)
        allp = [(a, b) for a in range(m) for b in range(a + 1, m)]
        k = k or min(8, len(allp))
        return [allp[i] for i in sorted(rng.choice(len(allp), min(k, len(allp)), replace=False))]
    raise ValueError(kind)


def batch_pattern(kind: str, n_or_cand, seed: int, m: int = 6, k: int = 0) -> np.ndarray:
    """s-t pairs whose query graph is the pattern `kind` on m distinct
    vertices drawn uniformly (from range(n) or from the candidate array)."""
    rng = np.random.default_rng(seed)
    if isinstance(n_or_cand, (int, np.integer)):
        verts = rng.choice(int(n_or_cand), m, replace=False)
    else:
        verts = np.asarray(n_or_cand)[rng.choice(len(n_or_cand), m, replace=False)]
    e = pattern_edges(kind, m, k, seed + 1)
    return np.array([[verts[a], verts[b]] for a, b in e], np.uint32).reshape(-1, 2)


# ---- distance-rank targets (the fine-grained percentile study of Section 6) ----
# Selection only: the distances from the source are an input (from the oracle
# in tests, from the library under test in the benchmark).

UNREACHABLE = (1 << 64) - 1


def rank_ladder(reachable: int, first: int = 10) -> list:
    """Distance ranks first, 2*first, 4*first, ... below `reachable`, then the
    farthest vertex (rank `reachable`)."""
    out = []
    r = first
    while r < reachable:
        out.append(r)
        r *= 2
    if reachable > 0:
        out.append(reachable)
    return out


def targets_by_rank(dist, s: int, ranks) -> np.ndarray:
    """The vertices at the given 1-based distance ranks from s: the vertices
    other than s that s reaches, ordered by distance, ties by vertex id."""
    dist = np.asarray(dist, np.uint64)
    cand = np.nonzero(dist != np.uint64(UNREACHABLE))[0]
    cand = cand[cand != s]
    order = cand[np.lexsort((cand, dist[cand]))]
    return np.array([order[r - 1] for r in ranks], np.uint32)


def percentile_rank(reachable: int, x: float) -> int:
    """Rank of the x-th distance percentile target: the x% farthest vertex."""
    return max(1, min(reachable, int(np.ceil(x / 100.0 * reachable))))
