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
    switched = {}
    for algo in ["sssp", "et", "astar", "bids", "bidastar"]:
        for batch in ["plainstar", "plain"]:
            assert np.array_equal(G.batch_query(pairs[:12] if batch == "plain" else pairs, algo=algo, batch=batch),
                                  exp[:12] if batch == "plain" else exp), (algo, batch)
            switched[algo, batch] = G.stats()["dense_searches"]
    if mode == "off":
        assert not any(switched.values()), switched
    elif mode == "forced":
        assert all(switched.values()), switched
    else:
        assert switched["sssp", "plainstar"] > 0, switched
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


def _mode_net(dense):
    """Constant network: bin 4 (the base step) and a fixed frontier mode."""
    p = np.zeros(P_PARAMS, np.float32)
    p[-9 + 4] = 1.0
    p[-1] = 4.0 if dense else -4.0
    return p


P_PARAMS = 5577


@pytest.mark.parametrize("graph", ["lattice", "rmat"])
def test_dense_chosen_by_network(P, graph):
    """Option dense_learned: the network's mode output switches searches to
    dense frontiers (and a negative output never does); without the option
    the output is ignored. Distances are the oracle's in every case."""
    if graph == "lattice":
        g = gen.lattice(120, 0.05, seed=184)
        pairs = gen.pairs_uniform(g.n, 40, seed=185)
        algos = ["bidastar", "bids", "astar"]
    else:
        g = gen.rmat(14, 16, seed=186)
        pairs = np.concatenate([gen.pairs_uniform(gen.lcc(g), 30, seed=187), gen.pairs_uniform(g.n, 10, seed=188)])
        algos = ["bids", "et"]
    exp = _exp(g, pairs)
    G = P.Graph.from_host(g, reorder=graph == "rmat")
    G.set_option("timeout_ms", 60000)
    assert P.MLP_PARAMS == P_PARAMS
    for opt in (0, 1):
        G.set_option("dense_learned", opt)
        for dense in (False, True):
            G.mlp_load(_mode_net(dense))
            for algo in algos:
                print("dense by network", graph, opt, dense, algo, flush=True)
                assert np.array_equal(G.batch_query(pairs, algo=algo, sched="learned"), exp), (opt, dense, algo)
                n_dense = G.stats()["dense_searches"]
                if opt and dense:
                    assert n_dense > 0, algo
                else:
                    assert n_dense == 0, (opt, dense, algo, n_dense)
    G.close()


def test_dense_autotuned_setting_is_exact(P):
    """The autotuner's dense trials (switch size, ring, narrower steps) on an
    R-MAT graph with hubs: whatever it keeps, the autotuned batch is exact."""
    g = gen.rmat(14, 16, seed=189)
    lcc = gen.lcc(g)
    sample = gen.pairs_uniform(lcc, 24, seed=190)
    pairs = gen.pairs_uniform(lcc, 40, seed=191)
    exp = _exp(g, pairs)
    G = P.Graph.from_host(g, reorder=True)
    G.set_option("timeout_ms", 60000)
    tr = G.tune(sample, algo="bids", batch="plainstar")
    assert tr["dense_ring"] in (16, 32, 64) and tr["dense_min"] in (0, 1 << 16, 1 << 18), tr
    assert np.array_equal(G.batch_query(pairs, algo="bids", sched="autotuned"), exp)
    G.close()
