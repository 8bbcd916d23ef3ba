"""GPU parity of dense frontiers (the dense mode of Appendix B: a search's
frontier kept as bitmaps of n bits, one per step bucket, once it is large):
forced from the first round, switched on by frontier size, and off, on
lattices with heuristics, R-MAT graphs with hub vertices (the hub-list kernel
adds to the bitmaps), directed graphs and random multigraphs, in every mode
and batch strategy, against the oracle."""
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


def _modes(G, mode):
    G.set_option("timeout_ms", 60000)              # a round loop that never drained would return an error
    G.set_option("dense_force", 1 if mode == "forced" else 0)
    G.set_option("dense_min", 64 if mode == "auto" else 0)


@pytest.mark.parametrize("mode", ["off", "forced", "auto"])
def test_dense_lattice_all_modes(P, mode):
    g = gen.lattice(140, 0.1, seed=140)
    pairs = gen.pairs_uniform(g.n, 40, seed=141)
    pairs[3, 1] = pairs[3, 0]
    exp = _exp(g, pairs)
    G = P.Graph.from_host(g)
    _modes(G, mode)
    print("dense lattice", mode, flush=True)
    for algo in ["sssp", "et", "astar", "bids", "bidastar"]:
        for batch in ["plainstar", "plain"]:
            assert np.array_equal(G.batch_query(pairs[:12] if batch == "plain" else pairs, algo=algo, batch=batch),
                                  exp[:12] if batch == "plain" else exp), (algo, batch)
    assert np.array_equal(G.batch_query(pairs, algo="bids", batch="multi"), exp)
    assert np.array_equal(G.batch_query(pairs, algo="sssp", batch="vc"), exp)
    d, (off, vtx) = G.batch_query(pairs[:10], algo="bidastar", want_path=True)
    for q in range(10):
        s, t = int(pairs[q, 0]), int(pairs[q, 1])
        assert oracle.check_path(g.n, g.row_ptr, g.col, g.w, vtx[off[q]:off[q + 1]], s, t, int(d[q])) == (0, 0)
    assert np.array_equal(G.batch_query(pairs, algo="bidastar", memo=True), exp)
    G.close()


@pytest.mark.parametrize("delta", [1, 7, 300, 1 << 20])
def test_dense_bucket_widths(P, delta):
    """Bucket widths from 1 (most additions beyond the 8-bucket ring stay in
    the queue) to 2^20 (everything in one bucket, refilled every round), under
    each threshold rule."""
    g = gen.lattice(100, 0.05, seed=142)
    pairs = gen.pairs_uniform(g.n, 30, seed=143)
    exp = _exp(g, pairs)
    G = P.Graph.from_host(g)
    G.set_option("timeout_ms", 60000)
    G.set_option("dense_force", 1)
    for rule in (0, 1, 2, 3):
        G.set_option("theta_mode", rule)
        print("dense widths", delta, rule, flush=True)
        assert np.array_equal(G.batch_query(pairs, algo="bidastar", delta=delta), exp), rule
        assert np.array_equal(G.batch_query(pairs, algo="bids", delta=delta), exp), rule
    G.close()


@pytest.mark.parametrize("mode", ["forced", "auto"])
def test_dense_rmat_hubs_and_unreachable(P, mode):
    g = gen.rmat(15, 16, seed=144)
    assert int(np.max(np.diff(g.row_ptr.astype(np.int64)))) > 512
    pairs = np.concatenate([gen.pairs_uniform(gen.lcc(g), 40, seed=145), gen.pairs_uniform(g.n, 20, seed=146)])
    exp = _exp(g, pairs)
    assert np.any(exp == oracle.INF)
    G = P.Graph.from_host(g, reorder=True)
    _modes(G, mode)
    G.set_option("theta_mode", 1)
    print("dense rmat", mode, flush=True)
    for algo in ["bids", "et", "sssp"]:
        assert np.array_equal(G.batch_query(pairs, algo=algo, delta=3000), exp), algo
    assert np.array_equal(G.batch_query(pairs, algo="bids", batch="multi", delta=3000), exp)
    G.close()


def test_dense_directed_and_random(P):
    for seed in range(12):
        rng = np.random.default_rng(150 + seed)
        n = int(rng.integers(20, 400))
        g = gen.random_graph(n, int(rng.integers(n, 6 * n)), int(rng.choice([1, 9, 1000])), seed=150 + seed,
                             wmin=seed % 2, symmetric=bool(seed % 3))
        pairs = gen.pairs_uniform(n, 30, seed=170 + seed)
        exp = _exp(g, pairs)
        G = P.Graph.from_host(g)
        G.set_option("timeout_ms", 60000)
        G.set_option("dense_force", 1)
        print("dense random", seed, flush=True)
        for algo in ["bids", "et", "sssp"]:
            assert np.array_equal(G.batch_query(pairs, algo=algo), exp), (seed, algo)
        assert np.array_equal(G.batch_query(pairs, algo="bids", batch="multi"), exp), seed
        G.close()


def test_dense_with_learned_schedule(P):
    """A network picks each search's step; the switch to dense frontiers takes
    the step of that round as the bucket width."""
    g = gen.lattice(120, 0.05, seed=180)
    pairs = gen.pairs_uniform(g.n, 40, seed=181)
    exp = _exp(g, pairs)
    G = P.Graph.from_host(g)
    p = gen.mlp_init(182)
    p[-9:-1] = np.linspace(-1, 1, 8)
    G.mlp_load(p)
    G.set_option("timeout_ms", 60000)
    G.set_option("dense_min", 32)
    assert np.array_equal(G.batch_query(pairs, algo="bidastar", sched="learned"), exp)
    assert np.array_equal(G.batch_query(pairs, algo="bids", sched="learned"), exp)
    G.close()
