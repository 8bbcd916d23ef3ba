"""GPU parity of the batch strategies of Sections 4.2 and 4.3 on the query-graph
patterns of the batch experiments (star, fork, chain, cycle, bipartite,
clique, separate, random over six sources; and 30 sources with 200 random
pairs), against the oracle."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

# minimum vertex cover of each six-vertex pattern
MIN_COVER = {"star": 1, "fork": 2, "chain": 3, "cycle": 3, "bipartite": 3, "clique": 5, "separate": 3}
STRATS = [("bids", "plain"), ("bids", "plainstar"), ("bids", "multi"), ("sssp", "sssp"), ("sssp", "vc"),
          ("bids", "auto")]


@pytest.fixture(scope="module")
def P():
    import paper_2506_16488_amd as P
    P.lib()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return P


def _check_paths(g, pairs, dist, off, vtx):
    for q in range(pairs.shape[0]):
        s, t = int(pairs[q, 0]), int(pairs[q, 1])
        path = vtx[int(off[q]):int(off[q + 1])]
        if dist[q] == oracle.INF:
            assert path.shape[0] == 0
        else:
            assert oracle.check_path(g.n, g.row_ptr, g.col, g.w, path, s, t, int(dist[q])) == (0, 0), q


@pytest.mark.parametrize("graph", ["lattice", "sparse"])
def test_patterns_all_strategies(P, graph):
    g = gen.lattice(96, 0.1, seed=90) if graph == "lattice" else gen.random_graph(4000, 5200, 500, seed=91)
    G = P.Graph.from_host(g)
    for j, kind in enumerate(gen.PATTERNS):
        pairs = gen.batch_pattern(kind, g.n, seed=200 + j)
        exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
        for algo, batch in STRATS:
            got = G.batch_query(pairs, algo=algo, batch=batch)
            assert np.array_equal(got, exp), (kind, algo, batch)
        if kind in MIN_COVER:
            G.batch_query(pairs, algo="sssp", batch="vc")
            assert G.stats()["searches"] == MIN_COVER[kind], kind
            G.batch_query(pairs, algo="sssp", batch="sssp")
            assert G.stats()["searches"] == len(set(int(s) for s in pairs[:, 0])), kind
        for algo, batch in [("sssp", "vc"), ("sssp", "sssp")]:
            d, (off, vtx) = G.batch_query(pairs, algo=algo, batch=batch, want_path=True)
            assert np.array_equal(d, exp)
            _check_paths(g, pairs, d, off, vtx)
    G.close()


def test_large_batch_thirty_sources(P):
    g = gen.lattice(128, 0.05, seed=92)
    pairs = gen.batch_pattern("random", g.n, seed=300, m=30, k=200)
    assert pairs.shape == (200, 2)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    G = P.Graph.from_host(g)
    for algo, batch in STRATS:
        assert np.array_equal(G.batch_query(pairs, algo=algo, batch=batch), exp), batch
    G.batch_query(pairs, algo="sssp", batch="vc")
    assert G.stats()["searches"] < 30          # a 200-edge graph on 30 vertices has a smaller cover
    # a big star: the greedy cover is its hub
    star = gen.batch_pattern("star", g.n, seed=301, m=40)
    G.batch_query(star, algo="sssp", batch="vc")
    assert G.stats()["searches"] == 1
    assert np.array_equal(G.batch_query(star, algo="bids", batch="auto"),
                          oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, star))
    G.close()


def test_strategy_errors_and_directed(P):
    g = gen.lattice(40, 0.2, seed=93)
    G = P.Graph.from_host(g)
    pairs = gen.batch_pattern("chain", g.n, seed=5)
    for algo, batch in [("bids", "vc"), ("bids", "sssp"), ("sssp", "auto"), ("et", "multi")]:
        with pytest.raises(P.PPSPError) as e:
            G.batch_query(pairs, algo=algo, batch=batch)
        assert e.value.code == P.E_INVALID
    G.close()



def _directed_graph(kind):
    if kind == "lattice":
        g = gen.lattice(90, 0.1, seed=95)
        rng = np.random.default_rng(96)
        w = (g.w.astype(np.int64) + rng.integers(0, 800, g.w.shape[0])).astype(np.uint32)
        return gen.csr_from_edges(g.n, np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64))),
                                  g.col.astype(np.int64), w.astype(np.int64), symmetric=False)
    if kind == "random":
        return gen.random_graph(3000, 9000, 200, seed=97, symmetric=False)
    r = gen.rmat(12, 16, seed=98)            # hubs: half of an R-MAT graph's arcs
    src = np.repeat(np.arange(r.n, dtype=np.int64), np.diff(r.row_ptr.astype(np.int64)))
    keep = np.random.default_rng(99).random(src.shape[0]) < 0.5
    return gen.csr_from_edges(r.n, src[keep], r.col[keep].astype(np.int64), r.w[keep].astype(np.int64),
                              symmetric=False)


@pytest.mark.parametrize("kind", ["lattice", "random", "hubs"])
def test_directed_patterns_all_strategies(P, kind):
    """Directed graphs (the adaptation to directed graphs): Multi-BiDS starts
    a forward search from every source and a backward one (on the transpose)
    from every target; VC-SSSP covers the bipartite query graph exactly."""
    d = _directed_graph(kind)
    D = P.Graph.from_host(d)
    D.set_option("timeout_ms", 60000)
    for j, pat in enumerate(gen.PATTERNS):
        pairs = gen.batch_pattern(pat, d.n, seed=600 + j)
        exp = oracle.pp_batch(d.n, d.row_ptr, d.col, d.w, pairs)
        for algo, batch in STRATS:
            assert np.array_equal(D.batch_query(pairs, algo=algo, batch=batch), exp), (kind, pat, algo, batch)
        real = pairs[pairs[:, 0] != pairs[:, 1]]
        D.batch_query(pairs, algo="sssp", batch="vc")
        assert D.stats()["searches"] == P.query_cover(real, directed=True)[2], pat
        D.batch_query(pairs, algo="bids", batch="multi")
        assert D.stats()["searches"] == len(set(real[:, 0].tolist())) + len(set(real[:, 1].tolist())), pat
        if kind != "random" or pat in ("star", "chain"):
            for algo, batch in [("sssp", "vc"), ("bids", "multi")]:
                dist, (off, vtx) = D.batch_query(pairs, algo=algo, batch=batch, want_path=True)
                assert np.array_equal(dist, exp)
                _check_paths(d, pairs, dist, off, vtx)
    # a reversed star: one backward search from the common target covers it
    star = gen.batch_pattern("star", d.n, seed=650, m=20)[:, ::-1].copy()
    exp = oracle.pp_batch(d.n, d.row_ptr, d.col, d.w, star)
    assert np.array_equal(D.batch_query(star, algo="sssp", batch="vc"), exp)
    assert D.stats()["searches"] == 1
    assert np.array_equal(D.batch_query(star, algo="bids", batch="auto"), exp)
    D.close()
