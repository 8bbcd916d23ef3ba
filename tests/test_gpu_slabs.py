"""The search-state slab reused across calls: batches of growing and
shrinking size and mode on one graph, with paths, memory waves and a server
taking the graph afterwards, must all keep the oracle's results."""
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


def test_slab_reuse_across_sizes_and_modes(P):
    g = gen.lattice(150, 0.1, seed=401)
    G = P.Graph.from_host(g)
    G.set_option("timeout_ms", 60000)
    for k, (m, algo) in enumerate([(40, "bidastar"), (40, "bids"), (90, "bidastar"), (7, "et"), (120, "bids"),
                                   (3, "astar"), (60, "bidastar"), (60, "bidastar")]):
        pairs = gen.pairs_uniform(g.n, m, seed=410 + k)
        exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
        assert np.array_equal(G.batch_query(pairs, algo=algo), exp), (k, m, algo)
    pairs = gen.pairs_uniform(g.n, 30, seed=420)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    for _ in range(3):
        dist, (off, vtx) = G.batch_query(pairs, algo="bidastar", want_path=True)
        assert np.array_equal(dist, exp)
        for q in range(pairs.shape[0]):
            assert oracle.check_path(g.n, g.row_ptr, g.col, g.w, vtx[off[q]:off[q + 1]], int(pairs[q, 0]),
                                     int(pairs[q, 1]), int(dist[q])) == (0, 0)
    # memory waves (a small budget): one slab, cleared before each wave
    G.set_option("mem_budget_mb", 1)
    pairs = gen.pairs_uniform(g.n, 50, seed=421)
    assert np.array_equal(G.batch_query(pairs, algo="bids"), oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs))
    assert G.stats()["waves"] > 1
    G.set_option("mem_budget_mb", 0)
    assert np.array_equal(G.batch_query(pairs, algo="bids"), oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs))
    # a server takes the graph after batches
    S = P.Server([G], algo="bidastar", state_budget_bytes=24 * g.n * 3)
    r = S.submit(0, pairs[:10])
    d, _ = S.wait(r, timeout_ms=60000)
    assert np.array_equal(d, oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs[:10]))
    S.close()
    assert np.array_equal(G.batch_query(pairs, algo="bidastar"), oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs))
    G.close()
