"""GPU parity of the grouped state layout of bidirectional Plain* batches
(option plain_group: the words of one vertex for G searches, G / 2 queries,
side by side): every group size on lattices with heuristics, R-MAT graphs
with hub vertices and unreachable pairs, directed graphs, with paths, the
heuristic memo, pulled relaxations, dense frontiers, the learned schedule,
and memory waves that hold whole groups or fall back to groups of one
query, against the oracle."""
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


def _exp(g, pairs):
    return oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)


@pytest.mark.parametrize("grp", [2, 4, 16, 64])
def test_groups_lattice(P, grp):
    g = gen.lattice(130, 0.1, seed=300)
    pairs = gen.pairs_uniform(g.n, 45, seed=301)          # 45 queries: the last group is partly empty
    pairs[4, 1] = pairs[4, 0]
    pairs[9] = pairs[8][::-1]
    exp = _exp(g, pairs)
    G = P.Graph.from_host(g, reorder=True)
    G.set_option("timeout_ms", 60000)
    G.set_option("plain_group", grp)
    assert G.get_option("plain_group") == grp
    print("groups lattice", grp, flush=True)
    for algo in ["bidastar", "bids"]:
        assert np.array_equal(G.batch_query(pairs, algo=algo), exp), algo
    assert np.array_equal(G.batch_query(pairs, algo="bidastar", memo=True), exp)
    assert np.array_equal(G.batch_query(pairs, algo="bids", pull=True), exp)
    d, (off, vtx) = G.batch_query(pairs[:12], algo="bidastar", want_path=True)
    for q in range(12):
        s, t = int(pairs[q, 0]), int(pairs[q, 1])
        assert oracle.check_path(g.n, g.row_ptr, g.col, g.w, vtx[off[q]:off[q + 1]], s, t, int(d[q])) == (0, 0)
    G.set_option("dense_force", 1)
    assert np.array_equal(G.batch_query(pairs, algo="bidastar"), exp)
    G.set_option("dense_force", 0)
    p = gen.mlp_init(302)
    p[-9:-1] = np.linspace(-1, 1, 8)
    G.mlp_load(p)
    assert np.array_equal(G.batch_query(pairs, algo="bidastar", sched="learned"), exp)
    G.close()


@pytest.mark.parametrize("grp", [8, 32])
def test_groups_rmat_hubs_and_directed(P, grp):
    g = gen.rmat(15, 16, seed=303)
    assert int(np.max(np.diff(g.row_ptr.astype(np.int64)))) > 512
    pairs = np.concatenate([gen.pairs_uniform(gen.lcc(g), 50, seed=304), gen.pairs_uniform(g.n, 14, seed=305)])
    exp = _exp(g, pairs)
    assert np.any(exp == oracle.INF)
    G = P.Graph.from_host(g, reorder=True)
    G.set_option("timeout_ms", 60000)
    G.set_option("plain_group", grp)
    G.set_option("theta_mode", 1)
    print("groups rmat", grp, flush=True)
    assert np.array_equal(G.batch_query(pairs, algo="bids", delta=3000), exp)
    G.set_option("dense_min", 256)
    assert np.array_equal(G.batch_query(pairs, algo="bids", delta=1500), exp)
    G.close()
    d = gen.random_graph(300, 1500, 50, seed=306, wmin=1, symmetric=False)
    dp = gen.pairs_uniform(d.n, 40, seed=307)
    G = P.Graph.from_host(d)
    G.set_option("plain_group", grp)
    assert np.array_equal(G.batch_query(dp, algo="bids"), _exp(d, dp))
    G.close()


def test_groups_in_memory_waves(P):
    """A state budget of about 15 searches per wave: groups of 4 queries
    fill waves of 4 or 8 queries; groups of 32 queries do not fit and the
    waves fall back to groups of one query."""
    g = gen.workload_graph("grid256")
    pairs = gen.workload_pairs("grid256", g)
    exp = _exp(g, pairs)
    G = P.Graph.from_host(g)
    G.set_option("mem_budget_mb", 8)
    for grp in (8, 64):
        G.set_option("plain_group", grp)
        print("groups waves", grp, flush=True)
        assert np.array_equal(G.batch_query(pairs, algo="bids"), exp), grp
        assert G.stats()["waves"] > 1
    G.close()


def test_group_option_range(P):
    g = gen.grid(8, 8, 1, 5, seed=308)
    G = P.Graph.from_host(g)
    for bad in (0, 1, 3, 128):
        with pytest.raises(P.PPSPError):
            G.set_option("plain_group", bad)
    G.close()
