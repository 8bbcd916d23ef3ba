"""Rounds replayed through a captured hipGraph ("use_graph"): the captured
chunk of rounds (round kernel, hub-list kernel, control kernel) gives the
same distances as the host-driven launches, with odd and even chunk lengths,
on a lattice (Plain*, Multi-BiDS, the learned schedule) and on an R-MAT
graph whose hubs go through the hub-list kernel."""
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


@pytest.mark.parametrize("rps", [3, 8])
def test_graph_replay_lattice(P, rps):
    g = gen.lattice(150, 0.05, seed=120)
    pairs = gen.pairs_uniform(g.n, 48, seed=121)
    pairs[5, 1] = pairs[5, 0]
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    G = P.Graph.from_host(g)
    G.set_option("rounds_per_sync", rps)
    p = gen.mlp_init(122)
    p[-9:-1] = np.linspace(-1, 1, 8)
    G.mlp_load(p)
    for use in (0, 1):
        G.set_option("use_graph", use)
        print("replay lattice rps=%d use_graph=%d" % (rps, use), flush=True)
        assert np.array_equal(G.batch_query(pairs, algo="bidastar", batch="plainstar"), exp)
        assert np.array_equal(G.batch_query(pairs, algo="bids", batch="multi"), exp)
        assert np.array_equal(G.batch_query(pairs, algo="bidastar", sched="learned"), exp)
        assert np.array_equal(G.batch_query(pairs[:6], algo="et", batch="plain"), exp[:6])
    G.close()


@pytest.mark.parametrize("rps", [5, 16])
def test_graph_replay_rmat_hubs(P, rps):
    g = gen.rmat(14, 16, seed=123)
    assert int(np.max(np.diff(g.row_ptr.astype(np.int64)))) > 512
    pairs = gen.pairs_uniform(gen.lcc(g), 40, seed=124)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    G = P.Graph.from_host(g, reorder=True)
    G.set_option("rounds_per_sync", rps)
    G.set_option("use_graph", 1)
    print("replay rmat rps=%d" % rps, flush=True)
    assert np.array_equal(G.batch_query(pairs, algo="bids"), exp)
    G.set_option("theta_mode", 1)
    assert np.array_equal(G.batch_query(pairs, algo="bids", delta=3000), exp)
    G.close()
