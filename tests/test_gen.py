"""Input generator checks: sizes, symmetry, weight rules, determinism, pairs."""
import math

import numpy as np

import gen


def _arcs(g):
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr.astype(np.int64)))
    return src, g.col.astype(np.int64), g.w.astype(np.int64)


def _is_symmetric(g):
    s, d, w = _arcs(g)
    a = np.stack([s, d, w], 1)
    b = np.stack([d, s, w], 1)
    a = a[np.lexsort(a.T[::-1])]
    b = b[np.lexsort(b.T[::-1])]
    return np.array_equal(a, b)


def test_grid_shape_weights_symmetry():
    g = gen.grid(7, 9, 1, 1000, seed=3)
    assert g.n == 63 and g.m == 2 * (7 * 8 + 6 * 9)
    assert g.w.min() >= 1 and g.w.max() <= 1000
    assert _is_symmetric(g)
    for v in range(g.n):
        nb = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
        assert np.all(np.diff(nb.astype(np.int64)) > 0)
        r, c = divmod(v, 9)
        exp = sorted(x for x in [v - 9 if r else None, v - 1 if c else None, v + 1 if c < 8 else None,
                                 v + 9 if r < 6 else None] if x is not None)
        assert nb.tolist() == exp


def test_grid256_counts():
    g = gen.workload_graph("grid256")
    assert g.n == 65536 and g.m == 261120


def test_generators_deterministic():
    a, b = gen.lattice(64, 0.05, seed=9), gen.lattice(64, 0.05, seed=9)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.w, b.w) and np.array_equal(a.coords, b.coords)
    c = gen.lattice(64, 0.05, seed=10)
    assert not np.array_equal(a.coords, c.coords)
    assert np.array_equal(gen.pairs_uniform(1000, 50, 7), gen.pairs_uniform(1000, 50, 7))


def test_lattice_weights_exact_ceil():
    g = gen.lattice(48, 0.3, seed=5)
    assert _is_symmetric(g)
    s, d, w = _arcs(g)
    xy = g.coords.astype(np.int64)
    dx, dy = xy[d, 0] - xy[s, 0], xy[d, 1] - xy[s, 1]
    for k in range(0, s.shape[0], 7):
        q = 10**6 * int(dx[k] ** 2 + dy[k] ** 2)
        r = math.isqrt(q)
        r = r if r * r == q else r + 1                     # ceil(sqrt(q))
        assert int(w[k]) == -(-r // 256)                   # ceil(1000 * len) with len = sqrt(d2)/256
        # w >= 1000 * len exactly (consistency precondition of the heuristic)
        assert (int(w[k]) * 256) ** 2 >= q


def test_lattice_weight_golden():
    # hand-worked: len = 1 cell -> 1000; diagonal of a unit cell -> ceil(1414.2...) = 1415;
    # 1/256 cell -> ceil(3.90625) = 4; 3-4-5 triangle in cells -> 5000
    assert gen.lattice_weight(256, 0) == 1000
    assert gen.lattice_weight(256, 256) == 1415
    assert gen.lattice_weight(1, 0) == 4
    assert gen.lattice_weight(3 * 256, 4 * 256) == 5000
    assert gen.lattice_weight(-768, 1024) == 5000


def test_lattice_structure_and_diagonals():
    L = 64
    g = gen.lattice(L, 0.05, seed=2)
    n4 = 2 * 2 * L * (L - 1)
    ndiag = (g.m - n4) // 2
    assert g.m - n4 == 2 * ndiag and 0 < ndiag < 0.2 * (L - 1) ** 2
    cell = g.coords // 256
    assert np.array_equal(cell[:, 0], np.arange(g.n) % L) and np.array_equal(cell[:, 1], np.arange(g.n) // L)
    s, d, _ = _arcs(g)
    assert np.all(np.abs(cell[s] - cell[d]).max(1) == 1)     # only unit steps and diagonals


def test_isqrt_exact():
    rng = np.random.default_rng(1)
    vals = [0, 1, 2, 3, 4, 15, 16, 17, 2**32 - 1, 2**32, 2**62, 2**63 - 1, 2**64 - 1]
    vals += [int(x) for x in rng.integers(0, 2**63, 2000, dtype=np.int64)]
    vals += [k * k + e for k in [3037000499, 4294967295, 123456789] for e in (-1, 0, 1) if k * k + e < 2**64]
    for x in vals:
        assert gen.isqrt_floor(x) == math.isqrt(x)
        r = math.isqrt(x)
        assert gen.isqrt_ceil(x) == (r if r * r == x else r + 1)


def test_rmat_small():
    g = gen.rmat(10, 8, seed=4)
    assert g.n == 1024 and g.m > 0 and g.m % 2 == 0
    assert _is_symmetric(g)
    s, d, w = _arcs(g)
    assert np.all(s != d)                                     # no self-loops
    key = s * g.n + d
    assert np.unique(key).shape[0] == key.shape[0]            # no duplicate arcs
    assert w.min() >= 1 and w.max() <= 65535
    deg = np.diff(g.row_ptr.astype(np.int64))
    assert deg.max() > 8 * deg.mean()                         # skewed degrees
    for v in range(0, g.n, 37):
        nb = g.col[g.row_ptr[v]:g.row_ptr[v + 1]].astype(np.int64)
        assert np.all(np.diff(nb) > 0)


def test_lcc_and_pairs():
    # two components: a 5-path and a triangle, plus an isolated vertex
    g = gen.csr_from_edges(9, [0, 1, 2, 3, 5, 6, 7], [1, 2, 3, 4, 6, 7, 5], [1] * 7)
    assert gen.lcc(g).tolist() == [0, 1, 2, 3, 4]
    p = gen.pairs_uniform(gen.lcc(g), 200, seed=3)
    assert set(p.reshape(-1).tolist()) <= {0, 1, 2, 3, 4}
    p = gen.pairs_uniform(10, 500, seed=3, distinct=True)
    assert np.all(p[:, 0] != p[:, 1]) and p.max() < 10


def test_hub_pairs():
    p = gen.pairs_hub(1 << 20, 32, 512, 1024, seed=103)
    assert p.shape == (1024, 2)
    assert np.unique(p[:512, 0]).shape[0] <= 32
    assert np.unique(p[512:, 0]).shape[0] > 400


def test_batch_patterns():
    import itertools
    for kind in gen.PATTERNS:
        e = gen.pattern_edges(kind)
        assert all(0 <= a < 6 and 0 <= b < 6 and a != b for a, b in e), kind
        assert len(set(tuple(sorted(x)) for x in e)) == len(e), kind
        p = gen.batch_pattern(kind, 10_000, seed=1)
        assert p.shape == (len(e), 2) and len(set(p.reshape(-1).tolist())) <= 6
    sizes = {k: len(gen.pattern_edges(k)) for k in gen.PATTERNS}
    assert sizes == {"star": 5, "fork": 5, "chain": 5, "cycle": 6, "bipartite": 9, "clique": 15, "separate": 3,
                     "random": 8}
    # brute-force minimum vertex covers of the fixed patterns
    def min_cover(e):
        for c in range(7):
            for s in itertools.combinations(range(6), c):
                if all(a in s or b in s for a, b in e):
                    return c
    assert {k: min_cover(gen.pattern_edges(k)) for k in gen.PATTERNS if k != "random"} == \
        {"star": 1, "fork": 2, "chain": 3, "cycle": 3, "bipartite": 3, "clique": 5, "separate": 3}
    big = gen.batch_pattern("random", 10_000, seed=2, m=30, k=200)
    assert big.shape == (200, 2) and len(set(big.reshape(-1).tolist())) <= 30
