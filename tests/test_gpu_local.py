"""GPU parity with local chunks on (the "local_chunks" and
"local_chunks_plain" options): a wave extracts its own additions within the
round's threshold in the same launch.
Every mode, batch strategy, threshold rule and graph kind must still give the
oracle's distances bit for bit, and valid paths."""
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


def _graph(P, g, local, fill=0, **kw):
    G = P.Graph.from_host(g, **kw)
    G.set_option("timeout_ms", 60000)
    G.set_option("local_chunks", local)
    G.set_option("local_chunks_plain", local)
    G.set_option("local_chunks_small", local)
    G.set_option("local_fill", fill)
    return G


def _paths_ok(g, w, pairs, dist, off, vtx):
    for q in range(pairs.shape[0]):
        s, t = int(pairs[q, 0]), int(pairs[q, 1])
        path = vtx[int(off[q]):int(off[q + 1])]
        if dist[q] == INF:
            assert path.shape[0] == 0
        else:
            assert oracle.check_path(g.n, g.row_ptr, g.col, w, path, s, t, int(dist[q])) == (0, 0), q


@pytest.mark.parametrize("local", [0, 1, 4, 32])
def test_lattice_every_mode_and_strategy(P, local):
    g = gen.lattice(120, 0.1, seed=301)
    pairs = gen.pairs_uniform(g.n, 70, seed=302)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    G = _graph(P, g, local)
    for algo in ["sssp", "et", "astar", "bids", "bidastar"]:
        for batch in ["plainstar", "plain"]:
            assert np.array_equal(G.batch_query(pairs, algo=algo, batch=batch), exp), (algo, batch)
    for algo, batch in [("bids", "multi"), ("sssp", "sssp"), ("sssp", "vc"), ("bids", "auto")]:
        assert np.array_equal(G.batch_query(pairs, algo=algo, batch=batch), exp), (algo, batch)
    for algo in ["bids", "bidastar", "astar"]:
        dist, (off, vtx) = G.batch_query(pairs, algo=algo, want_path=True)
        assert np.array_equal(dist, exp)
        _paths_ok(g, g.w, pairs, dist, off, vtx)
    for q in range(8):
        s, t = int(pairs[q, 0]), int(pairs[q, 1])
        for algo in ["et", "astar", "bids", "bidastar"]:
            assert G.query(s, t, algo=algo) == exp[q], (q, algo)
    G.close()


@pytest.mark.parametrize("mode", [0, 1, 3])
def test_threshold_rules_and_partial_local(P, mode):
    """Other threshold rules; local chunks only in rounds with small frontiers."""
    g = gen.lattice(100, 0.05, seed=311)
    pairs = gen.pairs_uniform(g.n, 60, seed=312)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    G = _graph(P, g, 8, fill=3000)
    G.set_option("theta_mode", mode)
    for algo in ["bids", "bidastar", "et"]:
        assert np.array_equal(G.batch_query(pairs, algo=algo), exp), algo
    G.close()


def test_rmat_hubs_zero_weights_and_unreachable(P):
    r = gen.rmat(12, 16, seed=321)
    pairs = gen.pairs_uniform(r.n, 60, seed=322)
    exp = oracle.pp_batch(r.n, r.row_ptr, r.col, r.w, pairs)
    G = _graph(P, r, 8)
    for algo, batch in [("bids", "plainstar"), ("bids", "plain"), ("bids", "multi"), ("et", "plainstar"),
                        ("sssp", "vc")]:
        assert np.array_equal(G.batch_query(pairs, algo=algo, batch=batch), exp), (algo, batch)
    G.close()
    z = gen.random_graph(2500, 5000, 50, seed=323, wmin=0)
    pairs = gen.pairs_uniform(z.n, 80, seed=324)
    exp = oracle.pp_batch(z.n, z.row_ptr, z.col, z.w, pairs)
    assert np.any(exp == INF) and np.any(z.w == 0)
    G = _graph(P, z, 16)
    for algo, batch in [("bids", "plainstar"), ("bids", "plain"), ("bids", "multi"), ("et", "plainstar"),
                        ("sssp", "sssp")]:
        assert np.array_equal(G.batch_query(pairs, algo=algo, batch=batch), exp), (algo, batch)
    G.close()


def test_directed_memo_and_reordered(P):
    g = gen.lattice(80, 0.1, seed=331)
    rng = np.random.default_rng(332)
    w = (g.w.astype(np.int64) + rng.integers(0, 800, g.w.shape[0])).astype(np.uint32)
    pairs = gen.pairs_uniform(g.n, 50, seed=333)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, w, pairs)
    D = P.Graph(g.n, g.row_ptr, g.col, w, coords=g.coords, frac_bits=g.frac_bits, symmetric=False)
    D.set_option("timeout_ms", 60000)
    D.set_option("local_chunks", 8)
    D.set_option("local_chunks_plain", 8)
    for algo in ["bids", "bidastar", "et", "astar"]:
        for batch in ["plainstar", "plain"]:
            assert np.array_equal(D.batch_query(pairs, algo=algo, batch=batch), exp), (algo, batch)
    dist, (off, vtx) = D.batch_query(pairs, algo="bidastar", want_path=True)
    _paths_ok(g, w, pairs, dist, off, vtx)
    D.close()
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    G = _graph(P, g, 8, reorder=True)
    assert np.array_equal(G.batch_query(pairs, algo="bidastar", memo=True), exp)
    assert np.array_equal(G.batch_query(pairs, algo="bidastar"), exp)
    assert np.array_equal(G.batch_query(pairs, algo="bids", pull=True), exp)   # the pull pass runs without them
    G.close()


def test_options_checked(P):
    g = gen.lattice(20, 0.1, seed=341)
    G = P.Graph.from_host(g)
    assert G.get_option("local_chunks") == 16 and G.get_option("local_chunks_plain") == 0   # defaults
    assert G.get_option("local_chunks_small") == 4 and G.get_option("min_chunk") == 16
    assert G.get_option("local_time_pct") == 90 and G.get_option("defer_time_pct") == 105
    for name, bad in [("min_chunk", 0), ("min_chunk", 24), ("min_chunk", 128), ("local_chunks_small", -1),
                      ("local_time_pct", -1), ("defer_time_pct", -1), ("defer_time_pct", 50)]:
        with pytest.raises(P.PPSPError):
            G.set_option(name, bad)
    for name, bad in [("local_chunks", -1), ("local_chunks", 1025), ("local_chunks_plain", -1), ("local_fill", -1)]:
        with pytest.raises(P.PPSPError):
            G.set_option(name, bad)
    G.set_option("local_chunks", 12)
    assert G.get_option("local_chunks") == 12
    G.close()


@pytest.mark.parametrize("min_chunk", [1, 4, 64])
def test_chunk_sizes(P, min_chunk):
    """Small frontiers in chunks of min_chunk.. entries: same results for every
    mode (1 = one entry per wave, 64 = fixed chunks)."""
    g = gen.lattice(100, 0.1, seed=351)
    pairs = gen.pairs_uniform(g.n, 50, seed=352)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    G = _graph(P, g, 4)
    G.set_option("min_chunk", min_chunk)
    for algo, batch in [("bidastar", "plainstar"), ("bids", "plainstar"), ("bids", "multi"), ("et", "plain"),
                        ("sssp", "vc"), ("astar", "plainstar")]:
        assert np.array_equal(G.batch_query(pairs, algo=algo, batch=batch), exp), (algo, batch)
    for q in range(5):
        assert G.query(int(pairs[q, 0]), int(pairs[q, 1]), algo="bidastar") == exp[q]
    assert np.array_equal(G.sssp(int(pairs[0, 0])), oracle.sssp(g.n, g.row_ptr, g.col, g.w, int(pairs[0, 0])))
    G.close()


@pytest.mark.parametrize("pct,defer", [(0, 0), (1, 0), (30, 0), (80, 100), (0, 100), (1, 100), (80, 105)])
def test_local_time_limit(P, pct, defer):
    """The time limits on local chunks (1%: listed entries are handed to the
    next round almost at once; 0: no limit) and on queue chunks (100%: every
    wave slower than the mean hands on its remaining chunks): same results in
    every mode, on a batch large enough for full chunks."""
    g = gen.lattice(300, 0.05, seed=361)
    pairs = gen.pairs_uniform(g.n, 400, seed=362)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    G = P.Graph.from_host(g)
    G.set_option("timeout_ms", 60000)
    G.set_option("grid_blocks", 64)              # few workgroups: full chunks at this size
    G.set_option("local_time_pct", pct)
    G.set_option("defer_time_pct", defer)
    G.set_option("local_chunks_plain", 8)
    for algo, batch in [("bidastar", "plainstar"), ("astar", "plainstar"), ("bids", "plainstar"),
                        ("bids", "multi"), ("et", "plain")]:
        assert np.array_equal(G.batch_query(pairs, algo=algo, batch=batch), exp), (pct, algo, batch)
    dist, (off, vtx) = G.batch_query(pairs[:60], algo="bidastar", want_path=True)
    _paths_ok(g, g.w, pairs[:60], dist, off, vtx)
    G.close()
