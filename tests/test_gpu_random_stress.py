"""Randomised GPU parity: many seeded graphs of varied shape (size, density,
weight range with zeros, multi-edges, several components), symmetric and
directed, with and without the reordered device copy, every applicable mode
and batch strategy against the oracle; paths validated where weights are
positive."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

INF = oracle.INF


@pytest.fixture(scope="module")
def P():
    import paper_2506_16488_amd as P
    P.lib()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return P


def _case(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.choice([5, 40, 300, 2000, 6000]))
    m = int(n * rng.choice([0.5, 1.2, 3.0, 8.0]))
    wmax = int(rng.choice([1, 10, 1000, 60000]))
    wmin = 0 if rng.random() < 0.3 else 1
    symmetric = bool(rng.random() < 0.7)
    g = gen.random_graph(n, max(m, 1), wmax, seed=seed, wmin=wmin, symmetric=symmetric)
    pairs = gen.pairs_uniform(n, int(min(60, n * n)), seed=seed + 1)
    return g, pairs, wmin > 0


@pytest.mark.parametrize("seed", range(64))
def test_random_graphs_every_mode(P, seed):
    g, pairs, positive = _case(1000 + seed)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    for reorder in (False, True):
        G = P.Graph.from_host(g, reorder=reorder)
        G.set_option("timeout_ms", 60000)
        strategies = [("sssp", "plainstar"), ("et", "plainstar"), ("bids", "plainstar"), ("bids", "plain"),
                      ("sssp", "sssp")]
        strategies += [("bids", "multi"), ("sssp", "vc"), ("bids", "auto")]   # bipartite query graph if directed
        for algo, batch in strategies:
            got = G.batch_query(pairs, algo=algo, batch=batch)
            assert np.array_equal(got, exp), (seed, reorder, algo, batch)
        if positive:
            dist, (off, vtx) = G.batch_query(pairs, algo="bids", want_path=True)
            assert np.array_equal(dist, exp)
            for q in range(pairs.shape[0]):
                s, t = int(pairs[q, 0]), int(pairs[q, 1])
                path = vtx[int(off[q]):int(off[q + 1])]
                if dist[q] == INF:
                    assert path.shape[0] == 0
                else:
                    assert oracle.check_path(g.n, g.row_ptr, g.col, g.w, path, s, t, int(dist[q])) == (0, 0), q
        # local chunks (a wave extracts its own additions in the same round)
        G.set_option("local_chunks", 8)
        G.set_option("local_chunks_plain", 8)
        for algo, batch in strategies[:4]:
            assert np.array_equal(G.batch_query(pairs, algo=algo, batch=batch), exp), (seed, reorder, algo, batch, "local")
        G.close()
