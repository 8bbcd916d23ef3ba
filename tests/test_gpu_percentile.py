"""Single-source distances (ppsp_sssp) and the distance-rank study of
Section 6: targets at ranks 10, 20, 40, ... up to the farthest vertex from a
source, answered by every mode, against the oracle."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2506_16488_amd as P
    P.lib()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return P


def _directed(g, seed):
    rng = np.random.default_rng(seed)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))
    w = g.w.astype(np.int64) + rng.integers(0, 800, g.w.shape[0])
    return gen.csr_from_edges(g.n, src, g.col.astype(np.int64), w, symmetric=False, coords=g.coords)


@pytest.mark.parametrize("kind", ["lattice", "rmat", "random", "directed", "reordered"])
def test_sssp_all_distances(P, kind):
    if kind in ("lattice", "reordered"):
        g = gen.lattice(150, 0.1, seed=501)
    elif kind == "rmat":
        g = gen.rmat(12, 16, seed=502)
    elif kind == "random":
        g = gen.random_graph(4000, 3500, 300, seed=503, wmin=0)
    else:
        g = _directed(gen.lattice(100, 0.1, seed=504), 505)
    G = P.Graph.from_host(g, reorder=kind == "reordered")
    G.set_option("timeout_ms", 60000)
    for s in (0, g.n // 3, g.n - 1):
        assert np.array_equal(G.sssp(s), oracle.sssp(g.n, g.row_ptr, g.col, g.w, s)), (kind, s)
    assert np.array_equal(G.sssp(5, sched="autotuned"), oracle.sssp(g.n, g.row_ptr, g.col, g.w, 5))
    with pytest.raises(P.PPSPError) as e:
        G.sssp(g.n)
    assert e.value.code == P.E_RANGE
    G.close()


@pytest.mark.parametrize("kind", ["lattice", "rmat", "directed"])
def test_rank_ladder_every_mode(P, kind):
    if kind == "lattice":
        g = gen.lattice(120, 0.05, seed=511)
    elif kind == "rmat":
        g = gen.rmat(11, 16, seed=512)
    else:
        g = _directed(gen.lattice(80, 0.1, seed=513), 514)
    cand = gen.lcc(g) if kind == "rmat" else np.arange(g.n)
    s = int(cand[len(cand) // 2])
    d = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s)
    reach = int(np.sum(d != oracle.INF)) - 1
    ranks = gen.rank_ladder(reach) + [gen.percentile_rank(reach, x) for x in (1, 50, 99)]
    targets = gen.targets_by_rank(d, s, ranks)
    pairs = np.stack([np.full(len(targets), s, np.uint32), targets], 1)
    exp = d[targets]
    G = P.Graph.from_host(g)
    G.set_option("timeout_ms", 60000)
    algos = ["et", "bids", "sssp"] + (["astar", "bidastar"] if g.coords is not None else [])
    for algo in algos:
        for (ss, t), e in zip(pairs.tolist(), exp.tolist()):
            assert G.query(ss, t, algo=algo) == e, (kind, algo, t)
        assert np.array_equal(G.batch_query(pairs, algo=algo), exp), (kind, algo)
    assert np.array_equal(G.sssp(s)[targets], exp)
    G.close()
