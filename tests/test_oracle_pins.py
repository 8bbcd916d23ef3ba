"""Pins for the CPU oracle: it must agree with what mathematics fixes.

Each check here is independent of the oracle's Dijkstra: brute force
(Floyd-Warshall, Bellman-Ford), closed forms (grids, paths, stars), a
library routine (scipy's csgraph Dijkstra), hand-worked fixtures under
tests/golden/, and the SSSP optimality certificate. A plausible mistake in
the oracle (a dropped relaxation, a wrong comparison, an off-by-one in the
heap, early exit before t is final) fails at least one of them.
"""
import os

import numpy as np
import pytest

import gen
import oracle

INF = oracle.INF
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _min_weight_matrix(g):
    """Dense matrix of minimum arc weights (for scipy, which sums duplicates)."""
    import scipy.sparse as sp
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))
    best = {}
    for a, b, ww in zip(src.tolist(), g.col.tolist(), g.w.tolist()):
        if a == b:
            continue
        k = (a, b)
        if k not in best or ww < best[k]:
            best[k] = ww
    if not best:
        return sp.csr_matrix((g.n, g.n))
    keys = np.array(list(best.keys()))
    vals = np.array(list(best.values()), dtype=np.float64)
    return sp.csr_matrix((vals, (keys[:, 0], keys[:, 1])), shape=(g.n, g.n))


@pytest.mark.parametrize("seed", range(60))
def test_dijkstra_matches_floyd_warshall(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    m = int(rng.integers(0, 3 * n + 1))
    wmax = int(rng.choice([1, 3, 10, 1000]))
    wmin = 0 if seed % 3 == 0 else 1          # zero weights allowed for distances
    g = gen.random_graph(n, m, wmax, seed=seed, wmin=wmin, symmetric=bool(seed % 2),
                         allow_loops=True)
    D = oracle.floyd_warshall(g.n, g.row_ptr, g.col, g.w)
    for s in range(n):
        dist = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s)
        assert np.array_equal(dist, D[s]), (seed, s)
    for s in range(n):
        for t in range(n):
            assert oracle.pp(g.n, g.row_ptr, g.col, g.w, s, t) == int(D[s, t])


@pytest.mark.parametrize("nthreads", [1, 3, 7])
def test_pp_batch_matches_floyd_warshall_and_single_queries(nthreads):
    """The batch checker that most GPU tests use: every entry equals the
    single-pair Dijkstra and the Floyd-Warshall matrix, whatever the thread
    count (pairs in shuffled order, duplicates, s = t and unreachable pairs)."""
    for seed in range(16):
        rng = np.random.default_rng(300 + seed)
        n = int(rng.integers(2, 36))
        g = gen.random_graph(n, int(rng.integers(0, 3 * n + 1)), int(rng.choice([1, 7, 1000])), seed=300 + seed,
                             wmin=seed % 2, symmetric=bool(seed % 3), allow_loops=True)
        D = oracle.floyd_warshall(g.n, g.row_ptr, g.col, g.w)
        allp = np.array([(s, t) for s in range(n) for t in range(n)], np.uint32)
        pairs = np.concatenate([allp[rng.permutation(len(allp))], allp[rng.integers(0, len(allp), 7)]])
        got = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs, nthreads=nthreads)
        assert np.array_equal(got, D[pairs[:, 0], pairs[:, 1]]), (seed, nthreads)
        one = [oracle.pp(g.n, g.row_ptr, g.col, g.w, int(s), int(t)) for s, t in pairs[:40]]
        assert got[:40].tolist() == one


@pytest.mark.parametrize("seed", range(12))
def test_dijkstra_matches_bellman_ford(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(50, 2000))
    g = gen.random_graph(n, int(rng.integers(n, 4 * n)), int(rng.choice([5, 65535])), seed=seed,
                         wmin=seed % 2, symmetric=seed < 6)
    for s in rng.integers(0, n, 4).tolist():
        assert np.array_equal(oracle.sssp(g.n, g.row_ptr, g.col, g.w, s),
                              oracle.bellman_ford(g.n, g.row_ptr, g.col, g.w, s))


@pytest.mark.parametrize("R,C,c", [(1, 1, 7), (1, 9, 3), (7, 5, 1), (16, 16, 5), (40, 3, 1000)])
def test_uniform_grid_closed_form(R, C, c):
    g = gen.grid(R, C, c, c, seed=3)           # every weight equals c
    for s in [0, R * C - 1, (R // 2) * C + C // 2]:
        dist = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s)
        rs, cs = divmod(s, C)
        r, cc = np.divmod(np.arange(R * C), C)
        assert np.array_equal(dist, (c * (np.abs(r - rs) + np.abs(cc - cs))).astype(np.uint64))


def test_path_graph_prefix_sums():
    rng = np.random.default_rng(7)
    n = 500
    w = rng.integers(1, 10**6, n - 1)
    g = gen.csr_from_edges(n, np.arange(n - 1), np.arange(1, n), w)
    pre = np.concatenate([[0], np.cumsum(w)]).astype(np.uint64)
    for s in [0, 17, 250, n - 1]:
        dist = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s)
        assert np.array_equal(dist, np.abs(pre.astype(np.int64) - int(pre[s])).astype(np.uint64))


def test_star_leaf_to_leaf():
    rng = np.random.default_rng(8)
    k = 50
    w = rng.integers(1, 5000, k)
    g = gen.csr_from_edges(k + 1, np.zeros(k, np.int64), np.arange(1, k + 1), w)
    for i in range(1, k + 1, 7):
        for j in range(1, k + 1, 5):
            exp = 0 if i == j else int(w[i - 1] + w[j - 1])
            assert oracle.pp(g.n, g.row_ptr, g.col, g.w, i, j) == exp


def test_disconnected_and_isolated():
    # two triangles, one isolated vertex
    g = gen.csr_from_edges(7, [0, 1, 2, 3, 4, 5], [1, 2, 0, 4, 5, 3], [1, 2, 3, 4, 5, 6])
    assert oracle.pp(g.n, g.row_ptr, g.col, g.w, 0, 3) == INF
    assert oracle.pp(g.n, g.row_ptr, g.col, g.w, 6, 0) == INF
    assert oracle.pp(g.n, g.row_ptr, g.col, g.w, 6, 6) == 0
    assert oracle.pp(g.n, g.row_ptr, g.col, g.w, 0, 2) == 3
    assert oracle.pp(g.n, g.row_ptr, g.col, g.w, 3, 5) == 6


def test_scipy_crosscheck_grid256():
    import scipy.sparse.csgraph as csg
    g = gen.workload_graph("grid256")
    M = _min_weight_matrix(g)
    srcs = [0, 12345, 65535]
    ref = csg.dijkstra(M, directed=True, indices=srcs)
    for i, s in enumerate(srcs):
        assert np.array_equal(oracle.sssp(g.n, g.row_ptr, g.col, g.w, s).astype(np.float64), ref[i])


def test_scipy_crosscheck_random_multigraph():
    import scipy.sparse.csgraph as csg
    g = gen.random_graph(3000, 9000, 100, seed=5, wmin=1, symmetric=False)
    M = _min_weight_matrix(g)
    ref = csg.dijkstra(M, directed=True, indices=[0, 1, 2])
    for s in range(3):
        d = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s).astype(np.float64)
        d[d == float(INF)] = np.inf
        assert np.array_equal(d, ref[s])


def test_certificate_accepts_oracle_and_rejects_planted_mistakes():
    g = gen.workload_graph("grid256")
    rng = np.random.default_rng(11)
    for s in rng.integers(0, g.n, 3).tolist():
        dist = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s)
        assert oracle.check_sssp(g.n, g.row_ptr, g.col, g.w, s, dist) == (0, 0)
        bad = dist.copy()
        v = (s + 777) % g.n
        bad[v] += 1                                       # too large: a tight arc is lost or infeasible
        assert oracle.check_sssp(g.n, g.row_ptr, g.col, g.w, s, bad)[0] in (2, 3)
        bad = dist.copy()
        bad[v] -= 1                                       # too small: no tight in-arc
        assert oracle.check_sssp(g.n, g.row_ptr, g.col, g.w, s, bad)[0] in (2, 3)
        bad = dist.copy()
        bad[s] = 1
        assert oracle.check_sssp(g.n, g.row_ptr, g.col, g.w, s, bad)[0] == 1


def test_certificate_reachability():
    g = gen.csr_from_edges(5, [0, 1, 3], [1, 2, 4], [2, 2, 2])
    dist = oracle.sssp(g.n, g.row_ptr, g.col, g.w, 0)
    assert oracle.check_sssp(g.n, g.row_ptr, g.col, g.w, 0, dist)[0] == 0
    bad = dist.copy()
    bad[3] = 5                                            # claims an unreachable vertex is reachable
    assert oracle.check_sssp(g.n, g.row_ptr, g.col, g.w, 0, bad)[0] in (2, 3, 4)


@pytest.mark.slow
def test_certificate_lattice2048_sampled():
    g = gen.workload_graph("lattice2048")
    for s in [0, 2048 * 1024 + 1024]:
        dist = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s)
        assert oracle.check_sssp(g.n, g.row_ptr, g.col, g.w, s, dist) == (0, 0)


def _walk_parents(par, s, t):
    path = [t]
    while path[-1] != s:
        path.append(int(par[path[-1]]))
        assert len(path) <= par.shape[0]
    return path[::-1]


def test_invariants_symmetry_triangle_parents():
    g = gen.grid(32, 32, 1, 50, seed=9)
    rng = np.random.default_rng(3)
    pts = rng.integers(0, g.n, 12).tolist()
    full = {s: oracle.sssp(g.n, g.row_ptr, g.col, g.w, s, parents=True) for s in pts}
    for s in pts:
        dist, par = full[s]
        for t in pts:
            assert dist[t] == full[t][0][s]                          # symmetry
            assert oracle.pp(g.n, g.row_ptr, g.col, g.w, s, t) == dist[t]  # early exit exact
            for v in pts:
                assert dist[t] <= dist[v] + full[v][0][t]            # triangle inequality
            path = _walk_parents(par, s, t)
            assert oracle.check_path(g.n, g.row_ptr, g.col, g.w, path, s, t, int(dist[t])) == (0, 0)


def test_meeting_identity():
    """d(s,t) = min_v d(s,v) + d(v,t) (the bidirectional meeting identity)."""
    g = gen.grid(24, 24, 1, 100, seed=12)
    ds = oracle.sssp(g.n, g.row_ptr, g.col, g.w, 5)
    dt = oracle.sssp(g.n, g.row_ptr, g.col, g.w, 500)
    assert int((ds + dt).min()) == int(ds[500])


def test_check_path_rejects_bad_paths():
    g = gen.grid(4, 4, 1, 1, seed=1)
    assert oracle.check_path(g.n, g.row_ptr, g.col, g.w, [0, 1, 2, 3], 0, 3, 3)[0] == 0
    assert oracle.check_path(g.n, g.row_ptr, g.col, g.w, [0, 2, 3], 0, 3, 2)[0] == 2
    assert oracle.check_path(g.n, g.row_ptr, g.col, g.w, [0, 1, 2, 3], 0, 3, 4)[0] == 3
    assert oracle.check_path(g.n, g.row_ptr, g.col, g.w, [1, 2, 3], 0, 3, 2)[0] == 1


def _read_golden(name):
    """Golden graph fixture: 'n N', 'e u v w' lines, 'q s t d' expected distances."""
    n, edges, queries = None, [], []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "n":
                n = int(line[1])
            elif line[0] == "e":
                edges.append(tuple(int(x) for x in line[1:4]))
            elif line[0] == "q":
                d = line[3]
                queries.append((int(line[1]), int(line[2]), INF if d == "inf" else int(d)))
    e = np.array(edges, dtype=np.int64).reshape(-1, 3)
    return gen.csr_from_edges(n, e[:, 0], e[:, 1], e[:, 2]), queries


@pytest.mark.parametrize("name", sorted(f for f in os.listdir(GOLDEN) if f.endswith(".graph")))
def test_golden_fixtures(name):
    g, queries = _read_golden(name)
    assert queries
    for s, t, d in queries:
        assert oracle.pp(g.n, g.row_ptr, g.col, g.w, s, t) == d, (name, s, t)
