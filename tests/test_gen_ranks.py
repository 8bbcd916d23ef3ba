"""Distance-rank target selection for the percentile workloads (host only):
checked on a path graph, where ranks are positions, and against the oracle's
distances on a random graph."""
import numpy as np

import gen
import oracle


def test_rank_ladder():
    assert gen.rank_ladder(100) == [10, 20, 40, 80, 100]
    assert gen.rank_ladder(80) == [10, 20, 40, 80]
    assert gen.rank_ladder(5) == [5]
    assert gen.rank_ladder(0) == []
    assert gen.percentile_rank(1000, 1) == 10 and gen.percentile_rank(1000, 50) == 500
    assert gen.percentile_rank(1000, 99) == 990 and gen.percentile_rank(3, 0.1) == 1


def test_targets_on_a_path():
    n = 50
    g = gen.csr_from_edges(n, np.arange(n - 1), np.arange(1, n), np.ones(n - 1))
    d = oracle.sssp(g.n, g.row_ptr, g.col, g.w, 20)
    # distances from 20: 19 and 21 tie at 1 (smaller id first), then 18, 22, ...
    t = gen.targets_by_rank(d, 20, [1, 2, 3, 4, 49])
    assert t.tolist() == [19, 21, 18, 22, 49]


def test_targets_against_distances():
    g = gen.random_graph(800, 1500, 100, seed=5)
    s = 3
    d = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s)
    reach = int(np.sum(d != oracle.INF)) - 1
    ranks = gen.rank_ladder(reach)
    t = gen.targets_by_rank(d, s, ranks)
    for r, v in zip(ranks, t.tolist()):
        assert v != s and d[v] != oracle.INF
        before = np.sum((d < d[v]) & (d != oracle.INF)) - 1            # strictly closer, s excluded
        ties = np.sum((d == d[v]) & (np.arange(g.n) < v))
        assert before + ties + 1 == r
