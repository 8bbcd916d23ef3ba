"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Distances are integers and must be bit-exact (uint64, INF for unreachable).
Paths are not unique, so they are validated instead: consecutive vertices
are arcs, the weights sum to the distance, the ends are s and t.
"""
import os

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

INF = oracle.INF
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALGOS_PLAIN = ["sssp", "et", "bids"]
ALGOS_GEO = ["sssp", "et", "astar", "bids", "bidastar"]


@pytest.fixture(scope="module")
def P():
    import paper_2506_16488_amd as P
    P.lib()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return P


def _graph(P, g, **kw):
    G = P.Graph.from_host(g, **kw)
    G.set_option("timeout_ms", 60000)
    return G


def _oracle(g, pairs):
    return oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)


def _check_paths(g, pairs, dist, off, vtx):
    for q in range(pairs.shape[0]):
        s, t = int(pairs[q, 0]), int(pairs[q, 1])
        path = vtx[int(off[q]):int(off[q + 1])]
        if dist[q] == INF:
            assert path.shape[0] == 0
            continue
        rc = oracle.check_path(g.n, g.row_ptr, g.col, g.w, path, s, t, int(dist[q]))
        assert rc == (0, 0), (q, s, t, rc)


def test_grid256_all_modes(P):
    g = gen.workload_graph("grid256")
    pairs = gen.workload_pairs("grid256", g)
    exp = _oracle(g, pairs)
    G = _graph(P, g)
    for algo in ALGOS_PLAIN:
        for batch in ["plainstar", "plain"]:
            got = G.batch_query(pairs, algo=algo, batch=batch)
            assert np.array_equal(got, exp), (algo, batch)
    got = G.batch_query(pairs, algo="bids", batch="multi")
    assert np.array_equal(got, exp)
    # single-query entry point and the s = t special case
    for q in range(0, 64, 9):
        assert G.query(int(pairs[q, 0]), int(pairs[q, 1]), algo="bids") == int(exp[q])
    assert G.query(77, 77, algo="bids") == 0
    assert G.query(77, 77, algo="et") == 0
    G.close()


def test_grid256_paths(P):
    g = gen.workload_graph("grid256")
    pairs = gen.workload_pairs("grid256", g)
    G = _graph(P, g)
    for algo in ["et", "bids"]:
        for batch in ["plainstar", "multi"] if algo == "bids" else ["plainstar"]:
            dist, (off, vtx) = G.batch_query(pairs, algo=algo, batch=batch, want_path=True)
            assert np.array_equal(dist, _oracle(g, pairs))
            _check_paths(g, pairs, dist, off, vtx)
    d, path = G.query(5, 60000, algo="bids", want_path=True)
    assert oracle.check_path(g.n, g.row_ptr, g.col, g.w, path, 5, 60000, d) == (0, 0)
    d, path = G.query(9, 9, algo="bids", want_path=True)
    assert d == 0 and path.tolist() == [9]
    G.close()


@pytest.mark.parametrize("seed", range(16))
def test_random_small_graphs_all_pairs(P, seed):
    """Random multigraphs with zero weights, isolated vertices and several
    components: every pair, every mode, against Floyd-Warshall."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 60))
    m = int(rng.integers(0, 2 * n + 2))
    g = gen.random_graph(n, m, int(rng.choice([1, 5, 1000])), seed=seed, wmin=seed % 2)
    D = oracle.floyd_warshall(g.n, g.row_ptr, g.col, g.w)
    s, t = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pairs = np.stack([s.ravel(), t.ravel()], 1).astype(np.uint32)
    exp = D[pairs[:, 0], pairs[:, 1]]
    G = _graph(P, g)
    for algo in ALGOS_PLAIN:
        assert np.array_equal(G.batch_query(pairs, algo=algo, batch="plainstar"), exp), algo
    assert np.array_equal(G.batch_query(pairs, algo="bids", batch="multi"), exp)
    G.close()


def test_golden_fixtures_gpu(P):
    from test_oracle_pins import _read_golden
    for name in sorted(f for f in os.listdir(GOLDEN) if f.endswith(".graph")):
        g, queries = _read_golden(name)
        G = _graph(P, g)
        pairs = np.array([[s, t] for s, t, _ in queries], np.uint32)
        exp = np.array([d for _, _, d in queries], np.uint64)
        for algo in ALGOS_PLAIN:
            for batch in ["plainstar", "plain"]:
                assert np.array_equal(G.batch_query(pairs, algo=algo, batch=batch), exp), (name, algo)
        assert np.array_equal(G.batch_query(pairs, algo="bids", batch="multi"), exp), name
        G.close()


@pytest.mark.parametrize("L,p", [(40, 0.3), (200, 0.05)])
def test_lattice_heuristic_modes(P, L, p):
    g = gen.lattice(L, p, seed=L)
    pairs = gen.pairs_uniform(g.n, 100, seed=L + 1)
    exp = _oracle(g, pairs)
    G = _graph(P, g)
    for algo in ALGOS_GEO:
        got = G.batch_query(pairs, algo=algo, batch="plainstar")
        assert np.array_equal(got, exp), algo
    dist, (off, vtx) = G.batch_query(pairs[:20], algo="bidastar", want_path=True)
    _check_paths(g, pairs[:20], dist, off, vtx)
    dist, (off, vtx) = G.batch_query(pairs[:20], algo="astar", want_path=True)
    _check_paths(g, pairs[:20], dist, off, vtx)
    G.close()


def test_schedule_invariance(P):
    """Any threshold sequence gives the same distances (Theorems
    bids-correctness and bdastar-correctness hold for every stepping rule)."""
    g = gen.lattice(96, 0.1, seed=3)
    pairs = gen.pairs_uniform(g.n, 60, seed=4)
    exp = _oracle(g, pairs)
    G = _graph(P, g)
    for delta in [1, int(g.w.min()), 1000, 5000, 1 << 30]:
        for algo in ["bids", "bidastar", "astar", "et"]:
            assert np.array_equal(G.batch_query(pairs, algo=algo, delta=delta), exp), (delta, algo)
    G.close()


def test_batch_equals_alone_and_repeatable(P):
    g = gen.workload_graph("grid256")
    pairs = gen.pairs_uniform(g.n, 40, seed=9)
    G = _graph(P, g)
    batch = G.batch_query(pairs, algo="bids", batch="multi")
    for q in range(0, 40, 5):
        assert G.query(int(pairs[q, 0]), int(pairs[q, 1]), algo="bids") == int(batch[q])
    for _ in range(5):
        assert np.array_equal(G.batch_query(pairs, algo="bids", batch="plainstar"), batch)
    G.close()


def test_hub_batch_multi(P):
    g = gen.lattice(128, 0.05, seed=6)
    pairs = gen.pairs_hub(g.n, 4, 40, 80, seed=7)
    pairs = np.concatenate([pairs, pairs[:5, ::-1], pairs[:3]])        # mirrored and repeated
    exp = _oracle(g, pairs)
    G = _graph(P, g)
    for batch in ["multi", "plainstar", "plain"]:
        assert np.array_equal(G.batch_query(pairs, algo="bids", batch=batch), exp), batch
    dist, (off, vtx) = G.batch_query(pairs, algo="bids", batch="multi", want_path=True)
    _check_paths(g, pairs, dist, off, vtx)
    G.close()


def test_memory_waves(P):
    """A state budget below the batch size forces several waves."""
    g = gen.workload_graph("grid256")
    pairs = gen.workload_pairs("grid256", g)
    exp = _oracle(g, pairs)
    G = _graph(P, g)
    G.set_option("mem_budget_mb", 8)          # ~15 searches of 65,536 vertices per wave
    for batch in ["plainstar", "multi"]:
        assert np.array_equal(G.batch_query(pairs, algo="bids", batch=batch), exp)
        assert G.stats()["waves"] > 1
    G.close()


def test_error_paths(P):
    g = gen.grid(8, 8, 1, 5, seed=1)
    G = _graph(P, g)
    with pytest.raises(P.PPSPError) as e:
        G.query(0, 64, algo="bids")
    assert e.value.code == P.E_RANGE
    with pytest.raises(P.PPSPError) as e:
        G.query(0, 5, algo="astar")
    assert e.value.code == P.E_NOCOORD
    with pytest.raises(P.PPSPError) as e:
        G.batch_query(np.array([[0, 5]]), algo="et", batch="multi")
    assert e.value.code == P.E_INVALID
    G.close()
    d = gen.csr_from_edges(3, [0, 1], [1, 2], [1, 1], symmetric=False)
    D = P.Graph(d.n, d.row_ptr, d.col, d.w, symmetric=False)
    # the query graph of a directed batch is bipartite: sources forward, targets backward
    assert D.batch_query(np.array([[0, 2], [2, 0]]), algo="bids", batch="multi").tolist() == [2, INF]
    assert D.batch_query(np.array([[0, 2], [2, 0]]), algo="sssp", batch="vc").tolist() == [2, INF]
    assert D.query(0, 2, algo="bids") == 2                  # the backward search walks the transpose
    assert D.query(2, 0, algo="bids") == INF
    assert D.query(0, 2, algo="et") == 2
    assert D.query(2, 0, algo="et") == INF                 # directed: unreachable backwards
    D.close()
    z = gen.csr_from_edges(3, [0, 1], [1, 2], [0, 4])
    Z = P.Graph(z.n, z.row_ptr, z.col, z.w)
    assert Z.query(0, 2, algo="bids") == 4
    with pytest.raises(P.PPSPError) as e:
        Z.query(0, 2, algo="bids", want_path=True)
    assert e.value.code == P.E_NOPATH
    Z.close()


@pytest.mark.slow
def test_lattice2048_full_size_sampled(P):
    """The 2048^2 road-like lattice with all 1,000 pairs in one Plain* batch
    (the benchmark's launch configuration); 48 sampled pairs vs the oracle."""
    g = gen.workload_graph("lattice2048")
    pairs = gen.workload_pairs("lattice2048", g)
    G = _graph(P, g)
    got = {a: G.batch_query(pairs, algo=a, batch="plainstar") for a in ["bidastar", "bids"]}
    idx = np.arange(0, 1000, 21)
    exp = _oracle(g, pairs[idx])
    for a in got:
        assert np.array_equal(got[a][idx], exp), a
    assert np.array_equal(got["bids"], got["bidastar"])
    G.close()


@pytest.mark.parametrize("scale", [12, 16])
def test_rmat_heavy_vertices(P, scale):
    """Power-law graphs: hub vertices (degree > 512) take the heavy-list path;
    pairs from the largest component plus a few from outside it."""
    g = gen.rmat(scale, 16, seed=40 + scale)
    lcc = gen.lcc(g)
    pairs = np.concatenate([gen.pairs_uniform(lcc, 120, seed=scale), gen.pairs_uniform(g.n, 20, seed=scale + 1)])
    exp = _oracle(g, pairs)
    G = _graph(P, g)
    for algo in ["bids", "et", "sssp"]:
        assert np.array_equal(G.batch_query(pairs, algo=algo, batch="plainstar"), exp), algo
    assert np.array_equal(G.batch_query(pairs, algo="bids", batch="multi"), exp)
    dist, (off, vtx) = G.batch_query(pairs[:30], algo="bids", batch="multi", want_path=True)
    _check_paths(g, pairs[:30], dist, off, vtx)
    G.close()


def test_overflow_retries_keep_results_exact(P):
    """Tiny frontier-queue and heavy-list capacities force overflow: the wave
    is rerun with larger buffers and the answers are unchanged."""
    g = gen.rmat(14, 16, seed=77)
    lcc = gen.lcc(g)
    pairs = gen.pairs_uniform(lcc, 200, seed=78)
    exp = _oracle(g, pairs)
    G = _graph(P, g)
    for batch in ["plainstar", "multi"]:
        G.set_option("queue_cap", 4096)
        G.set_option("heavy_cap", 4)
        assert np.array_equal(G.batch_query(pairs, algo="bids", batch=batch), exp), batch
        assert G.stats()["retries"] > 0
        assert G.get_option("queue_cap") > 4096 and G.get_option("heavy_cap") > 4
    G.close()


@pytest.mark.parametrize("list_deg", [16, 100, 512])
def test_hub_list_degree_threshold(P, list_deg):
    """Vertices above list_deg degree relax their arcs through the hub-list
    kernel (16: nearly all of them; 512: only the hubs): the oracle's
    distances in every strategy that uses the list, paths included."""
    g = gen.rmat(13, 16, seed=82)
    lcc = gen.lcc(g)
    pairs = np.concatenate([gen.pairs_uniform(lcc, 50, seed=83), gen.pairs_uniform(g.n, 8, seed=84)])
    exp = _oracle(g, pairs)
    G = _graph(P, g, reorder=True)
    G.set_option("list_deg", list_deg)
    assert G.get_option("list_deg") == list_deg
    print("list_deg", list_deg, flush=True)
    for algo in ["bids", "et", "sssp"]:
        assert np.array_equal(G.batch_query(pairs, algo=algo), exp), algo
    assert G.stats()["heavy_arcs"] > 0
    assert np.array_equal(G.batch_query(pairs, algo="bids", batch="multi"), exp)
    dist, (off, vtx) = G.batch_query(pairs[:20], algo="bids", want_path=True)
    _check_paths(g, pairs[:20], dist, off, vtx)
    for bad in (15, 513):
        with pytest.raises(P.PPSPError):
            G.set_option("list_deg", bad)
    G.close()


@pytest.mark.parametrize("claim", [1, 3, 64])
def test_heavy_claim_sizes(P, claim):
    """The hub-list kernel's records claimed 1, 3 or 64 at a time (option
    heavy_claim), with and without dense frontiers and with frontier queues
    too small for a round (overflow reruns): the oracle's distances."""
    g = gen.rmat(14, 16, seed=79)
    lcc = gen.lcc(g)
    pairs = np.concatenate([gen.pairs_uniform(lcc, 60, seed=80), gen.pairs_uniform(g.n, 10, seed=81)])
    exp = _oracle(g, pairs)
    G = _graph(P, g, reorder=True)
    G.set_option("heavy_claim", claim)
    assert G.get_option("heavy_claim") == claim
    print("heavy claim", claim, flush=True)
    assert np.array_equal(G.batch_query(pairs, algo="bids"), exp)
    G.set_option("dense_min", 64)
    G.set_option("theta_mode", 1)
    assert np.array_equal(G.batch_query(pairs, algo="bids", delta=1500), exp)
    G.set_option("queue_cap", 4096)
    assert np.array_equal(G.batch_query(pairs, algo="bids", delta=1500), exp)
    assert G.stats()["retries"] > 0
    for bad in (0, 65):
        with pytest.raises(P.PPSPError):
            G.set_option("heavy_claim", bad)
    G.close()


@pytest.mark.slow
def test_lattice4096_hub_batch_sampled(P):
    """The 4096^2 lattice with a 1,024-pair hub batch (512 pairs from 32 hub
    sources, 512 uniform) as one Multi-BiDS wave of ~1,568 searches, and as
    Plain* bidirectional A*; sampled pairs against the oracle."""
    g = gen.workload_graph("lattice4096")
    pairs = gen.workload_pairs("lattice4096", g)
    idx = np.arange(0, 1024, 64)
    exp = _oracle(g, pairs[idx])
    G = _graph(P, g)
    got = G.batch_query(pairs, algo="bids", batch="multi")
    assert np.array_equal(got[idx], exp)
    assert G.stats()["searches"] < 1700                 # shared sources: fewer searches than 2 x 1,024
    assert np.array_equal(G.batch_query(pairs, algo="bidastar", batch="plainstar"), got)
    G.close()


@pytest.mark.slow
def test_rmat24_sampled(P):
    """R-MAT scale 24 (power law, hubs of degree ~400K) with the benchmark's
    256 pairs from the largest component: Multi-BiDS, then Plain* BiDS in the
    benchmark's setting (bucketed threshold, Delta 1433, dense frontiers with
    a ring of 64) under the fixed and the learned schedule (a network that may
    switch searches to dense frontiers); sampled pairs against the oracle,
    all 256 against each other."""
    g = gen.workload_graph("rmat24")
    lcc = gen.lcc(g)
    pairs = gen.workload_pairs("rmat24", g, cand=lcc)
    idx = np.arange(0, 256, 32)
    exp = _oracle(g, pairs[idx])
    G = _graph(P, g, reorder=True)
    G.set_option("timeout_ms", 240000)
    got = G.batch_query(pairs, algo="bids", batch="multi")
    assert np.array_equal(got[idx], exp)
    G.set_option("theta_mode", 1)
    G.set_option("dense_min", 1 << 18)
    G.set_option("dense_ring", 64)
    print("rmat24 plain* tuned setting", flush=True)
    assert np.array_equal(G.batch_query(pairs, algo="bids", batch="plainstar", delta=1433), got)
    assert G.stats()["dense_searches"] > 0
    p = gen.mlp_init(5)
    p[-9:-1] = np.linspace(-0.5, 0.5, 8)
    G.mlp_load(p)
    G.set_option("dense_learned", 1)
    print("rmat24 learned", flush=True)
    assert np.array_equal(G.batch_query(pairs, algo="bids", batch="plainstar", delta=1433, sched="learned"), got)
    G.close()


def test_autotune_changes_speed_not_results(P, tmp_path):
    g = gen.lattice(160, 0.05, seed=21)
    pairs = gen.pairs_uniform(g.n, 64, seed=22)
    exp = _oracle(g, pairs)
    G = _graph(P, g)
    cache = str(tmp_path / "tune.txt")
    r = G.tune(pairs[:32], algo="bidastar", batch="plainstar", cache_path=cache)
    assert r["delta"] > 0 and r["trials"] >= 6 and r["from_cache"] == 0
    got = G.batch_query(pairs, algo="bidastar", batch="plainstar", sched="autotuned")
    assert np.array_equal(got, exp)
    G.close()
    # a new handle on the same graph reads the choice back from the cache
    G2 = _graph(P, g)
    r2 = G2.tune(pairs[:32], algo="bidastar", batch="plainstar", cache_path=cache)
    assert r["local_chunks"] in (8, 16, 32)
    assert r2["from_cache"] == 1 and r2["delta"] == r["delta"] and r2["theta_mode"] == r["theta_mode"]
    assert r2["local_chunks"] == r["local_chunks"] and r2["heavy_window"] == r["heavy_window"]
    assert np.array_equal(G2.batch_query(pairs, algo="bidastar", sched="autotuned"), exp)
    G2.close()


def test_memoised_heuristic_same_results(P):
    """PPSP_MEMO_H (Section 5): the per-query memo of the heuristic changes
    nothing in the results, across waves (the epoch tag) and batch modes."""
    g = gen.lattice(150, 0.05, seed=61)
    pairs = gen.pairs_uniform(g.n, 80, seed=62)
    exp = _oracle(g, pairs)
    G = _graph(P, g)
    for algo in ["astar", "bidastar"]:
        for batch in ["plainstar", "plain"]:
            for _ in range(2):
                got = G.batch_query(pairs, algo=algo, batch=batch, memo=True)
                assert np.array_equal(got, exp), (algo, batch)
        dist, (off, vtx) = G.batch_query(pairs[:20], algo=algo, memo=True, want_path=True)
        _check_paths(g, pairs[:20], dist, off, vtx)
    # several memory waves share the memo through the epoch tag
    G.set_option("mem_budget_mb", 1)
    assert np.array_equal(G.batch_query(pairs, algo="bidastar", memo=True), exp)
    assert G.stats()["waves"] > 1
    assert G.query(int(pairs[3, 0]), int(pairs[3, 1]), algo="bidastar", memo=True) == int(exp[3])
    G.close()


@pytest.mark.parametrize("graph", ["lattice", "rmat", "random"])
def test_pull_relaxation_same_results(P, graph):
    """PPSP_PULL (Appendix B): pulling before pushing changes nothing in the
    results, in every mode and batch strategy, with hubs and unreachable pairs."""
    if graph == "lattice":
        g = gen.lattice(120, 0.1, seed=71)
    elif graph == "rmat":
        g = gen.rmat(12, 16, seed=72)
    else:
        g = gen.random_graph(2000, 3000, 300, seed=73)
    pairs = gen.pairs_uniform(g.n, 60, seed=74)
    exp = _oracle(g, pairs)
    G = _graph(P, g)
    algos = ALGOS_GEO if graph == "lattice" else ALGOS_PLAIN
    for algo in algos:
        assert np.array_equal(G.batch_query(pairs, algo=algo, pull=True), exp), algo
    assert np.array_equal(G.batch_query(pairs, algo="bids", batch="multi", pull=True), exp)
    assert np.array_equal(G.batch_query(pairs, algo="sssp", batch="vc", pull=True), exp)
    dist, (off, vtx) = G.batch_query(pairs[:20], algo="bids", pull=True, want_path=True)
    _check_paths(g, pairs[:20], dist, off, vtx)
    G.close()


@pytest.mark.parametrize("graph", ["lattice", "rmat"])
def test_bellman_ford_and_rho_schedules(P, graph):
    """The Bellman-Ford threshold (theta = infinity) and the rho-stepping-style
    schedule are stepping rules too: identical distances (Section 2)."""
    g = gen.lattice(100, 0.1, seed=81) if graph == "lattice" else gen.rmat(12, 16, seed=82)
    pairs = gen.pairs_uniform(g.n, 50, seed=83)
    exp = _oracle(g, pairs)
    G = _graph(P, g)
    algos = ["bids", "et", "sssp", "bidastar", "astar"] if graph == "lattice" else ["bids", "et", "sssp"]
    G.set_option("theta_mode", 3)
    for algo in algos:
        assert np.array_equal(G.batch_query(pairs, algo=algo), exp), ("bf", algo)
    bf_rounds = G.stats()["rounds"]
    G.set_option("theta_mode", 2)
    for rho in (16, 4096):
        G.set_option("rho", rho)
        for algo in algos:
            assert np.array_equal(G.batch_query(pairs, algo=algo, sched="rho"), exp), ("rho", rho, algo)
    assert np.array_equal(G.batch_query(pairs, algo="bids", batch="multi", sched="rho"), exp)
    assert bf_rounds > 0
    G.close()


def _directed_lattice(L, seed):
    """A lattice whose two directions of every edge carry independent extra
    weight (w >= 1000 * length still holds, so the heuristic stays consistent)."""
    g = gen.lattice(L, 0.1, seed=seed)
    rng = np.random.default_rng(seed + 1)
    w = g.w.astype(np.int64) + rng.integers(0, 800, g.w.shape[0])
    return g, w.astype(np.uint32)


def test_directed_bidirectional_searches(P):
    """Bidirectional search on directed graphs: the backward search runs on
    the transpose; distances and paths against the oracle on the same arcs."""
    g, w = _directed_lattice(90, 91)
    pairs = gen.pairs_uniform(g.n, 60, seed=92)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, w, pairs)
    rev = oracle.pp_batch(g.n, g.row_ptr, g.col, w, pairs[:, ::-1].copy())
    assert not np.array_equal(exp, rev)                   # the graph really is directed
    G = P.Graph(g.n, g.row_ptr, g.col, w, coords=g.coords, frac_bits=g.frac_bits, symmetric=False)
    G.set_option("timeout_ms", 60000)
    for algo in ["bids", "bidastar", "et", "astar", "sssp"]:
        for batch in ["plainstar", "plain"]:
            assert np.array_equal(G.batch_query(pairs, algo=algo, batch=batch), exp), (algo, batch)
    assert np.array_equal(G.batch_query(pairs[:, ::-1].copy(), algo="bidastar"), rev)
    for algo in ["bids", "bidastar"]:
        dist, (off, vtx) = G.batch_query(pairs[:25], algo=algo, want_path=True)
        for q in range(25):
            s0, t0 = int(pairs[q, 0]), int(pairs[q, 1])
            assert oracle.check_path(g.n, g.row_ptr, g.col, w, vtx[off[q]:off[q + 1]], s0, t0, int(dist[q])) == (0, 0)
    G.close()
    # random directed graph with unreachable pairs and (at this size) no hubs
    d = gen.random_graph(3000, 9000, 200, seed=93, symmetric=False)
    pairs = gen.pairs_uniform(d.n, 80, seed=94)
    exp = oracle.pp_batch(d.n, d.row_ptr, d.col, d.w, pairs)
    assert np.any(exp == INF)
    D = P.Graph(d.n, d.row_ptr, d.col, d.w, symmetric=False)
    for algo in ["bids", "et"]:
        assert np.array_equal(D.batch_query(pairs, algo=algo), exp), algo
    D.close()


def test_directed_hubs_heavy_path(P):
    """Directed graph with hubs (a random half of an R-MAT graph's arcs): the
    heavy list of a backward search indexes the transpose."""
    r = gen.rmat(12, 16, seed=95)
    src = np.repeat(np.arange(r.n, dtype=np.int64), np.diff(r.row_ptr.astype(np.int64)))
    keep = np.random.default_rng(96).random(src.shape[0]) < 0.5
    d = gen.csr_from_edges(r.n, src[keep], r.col[keep].astype(np.int64), r.w[keep].astype(np.int64), symmetric=False)
    assert np.max(np.diff(d.row_ptr.astype(np.int64))) > 512
    pairs = gen.pairs_uniform(d.n, 60, seed=97)
    exp = oracle.pp_batch(d.n, d.row_ptr, d.col, d.w, pairs)
    D = P.Graph(d.n, d.row_ptr, d.col, d.w, symmetric=False)
    D.set_option("timeout_ms", 60000)
    for algo in ["bids", "et", "sssp"]:
        assert np.array_equal(D.batch_query(pairs, algo=algo), exp), algo
    dist, (off, vtx) = D.batch_query(pairs[:20], algo="bids", want_path=True)
    assert np.array_equal(dist, exp[:20])
    _check_paths(d, pairs[:20], dist, off, vtx)
    D.close()


def test_edge_cases(P):
    """Empty and degenerate inputs, duplicates, distance overflow, a path
    buffer that is too small, and the host-side time limit."""
    g = gen.lattice(60, 0.1, seed=101)
    G = _graph(P, g)
    # empty batch
    for batch in ["plainstar", "multi"]:
        assert G.batch_query(np.zeros((0, 2), np.uint32), algo="bids", batch=batch).shape == (0,)
    d, (off, vtx) = G.batch_query(np.zeros((0, 2), np.uint32), algo="bids", want_path=True)
    assert d.shape == (0,) and off.tolist() == [0] and vtx.shape == (0,)
    # duplicates, reversed duplicates and self pairs in one batch
    base = gen.pairs_uniform(g.n, 20, seed=102)
    pairs = np.concatenate([base, base[:7], base[3:12, ::-1], np.array([[5, 5], [5, 5]], np.uint32)])
    exp = _oracle(g, pairs)
    for algo, batch in [("bids", "plainstar"), ("bidastar", "plain"), ("bids", "multi"), ("sssp", "vc"),
                        ("et", "plainstar")]:
        assert np.array_equal(G.batch_query(pairs, algo=algo, batch=batch), exp), (algo, batch)
    dist, (off, vtx) = G.batch_query(pairs, algo="bids", batch="multi", want_path=True)
    _check_paths(g, pairs, dist, off, vtx)
    # a path buffer that is too small reports PPSP_E_PATHCAP through the C ABI
    import ctypes
    pp = np.ascontiguousarray(base[:4])
    dd = np.empty(4, np.uint64)
    oo = np.empty(5, np.uint64)
    vv = np.empty(1, np.uint32)
    rc = P.lib().ppsp_batch_query(G.h, pp.ctypes.data, 4, ctypes.byref(P.make_opts("bids", "plainstar", want_path=True)),
                                  None, dd.ctypes.data, oo.ctypes.data, vv.ctypes.data, 1)
    assert rc == P.E_PATHCAP
    # the host-side time limit ends a long wave with PPSP_E_TIMEOUT (or it finished in time)
    G.set_option("timeout_ms", 1)
    G.set_option("rounds_per_sync", 1)
    try:
        assert np.array_equal(G.batch_query(base, algo="bids", delta=1), _oracle(g, base))
    except P.PPSPError as e:
        assert e.code == P.E_TIMEOUT
    G.set_option("timeout_ms", 60000)
    assert np.array_equal(G.batch_query(base, algo="bids"), _oracle(g, base))   # usable again
    G.close()
    # one vertex, no arcs
    one = gen.csr_from_edges(1, [], [], [])
    O = P.Graph(one.n, one.row_ptr, one.col, one.w)
    assert O.query(0, 0, algo="bids") == 0
    assert O.batch_query(np.array([[0, 0]], np.uint32), algo="bids", batch="multi").tolist() == [0]
    O.close()
    # isolated vertices only: every pair unreachable
    iso = gen.csr_from_edges(10, [0], [1], [3])
    I = P.Graph(iso.n, iso.row_ptr, iso.col, iso.w)
    q = np.array([[2, 7], [0, 1], [1, 0], [3, 9]], np.uint32)
    for algo, batch in [("bids", "plainstar"), ("bids", "multi"), ("sssp", "vc"), ("et", "plain")]:
        assert I.batch_query(q, algo=algo, batch=batch).tolist() == [INF, 3, 3, INF], (algo, batch)
    I.close()
    # distances past 2^32 - 2 report PPSP_E_OVERFLOW instead of a wrong value
    big = gen.csr_from_edges(4, [0, 1, 2], [1, 2, 3], [2 ** 31, 2 ** 31 - 10, 2 ** 31])
    B = P.Graph(big.n, big.row_ptr, big.col, big.w)
    assert B.query(0, 1, algo="bids") == 2 ** 31
    with pytest.raises(P.PPSPError) as e:
        B.query(0, 3, algo="et")
    assert e.value.code == P.E_OVERFLOW
    B.close()


@pytest.mark.parametrize("graph", ["lattice", "rmat", "directed"])
def test_reordered_graph_same_results(P, graph):
    """PPSP_REORDER renumbers the device copy (Morton order of the
    coordinates, else breadth-first); ids at the interface, distances and
    paths are the caller's."""
    if graph == "lattice":
        g = gen.lattice(110, 0.1, seed=111)
        algos = ["bidastar", "astar", "bids", "et", "sssp"]
    elif graph == "rmat":
        g = gen.rmat(12, 16, seed=112)
        algos = ["bids", "et", "sssp"]
    else:
        g = gen.random_graph(3000, 9000, 200, seed=113, symmetric=False)
        algos = ["bids", "et"]
    pairs = np.concatenate([gen.pairs_uniform(g.n, 50, seed=114), np.array([[7, 7]], np.uint32)])
    exp = _oracle(g, pairs)
    G = P.Graph.from_host(g, reorder=True)
    G.set_option("timeout_ms", 60000)
    for algo in algos:
        assert np.array_equal(G.batch_query(pairs, algo=algo), exp), algo
        assert G.query(int(pairs[1, 0]), int(pairs[1, 1]), algo=algo) == int(exp[1])
    if g.symmetric:
        for algo, batch in [("bids", "multi"), ("sssp", "vc")]:
            assert np.array_equal(G.batch_query(pairs, algo=algo, batch=batch), exp), batch
    dist, (off, vtx) = G.batch_query(pairs[:20], algo=algos[0], want_path=True)
    _check_paths(g, pairs[:20], dist, off, vtx)
    d1, p1 = G.query(int(pairs[2, 0]), int(pairs[2, 1]), algo=algos[0], want_path=True)
    assert d1 == int(exp[2]) and (d1 == INF or (int(p1[0]), int(p1[-1])) == (int(pairs[2, 0]), int(pairs[2, 1])))
    if g.symmetric:
        S = P.Server([G], algo=algos[0], state_budget_bytes=24 * g.n * 4)
        r = S.submit(0, pairs)
        assert np.array_equal(S.wait(r, timeout_ms=60000)[0], exp)
        S.close()
    G.close()


def test_device_resident_pairs_and_distances(P):
    """PPSP_DEVICE_IO: pairs and distances in device memory (torch tensors on the
    current stream), with duplicates, a self pair and unreachable pairs."""
    import torch
    g = gen.random_graph(3000, 2600, 100, seed=63)
    pairs = gen.pairs_uniform(g.n, 90, seed=64)
    pairs[3] = pairs[2]
    pairs[4, 1] = pairs[4, 0]
    exp = _oracle(g, pairs)
    assert np.any(exp == INF)
    G = _graph(P, g)
    dp = torch.from_numpy(pairs.astype(np.int32)).cuda()
    dd = torch.full((pairs.shape[0],), 7, dtype=torch.int64, device="cuda")
    for algo, batch in [("bids", "plainstar"), ("bids", "multi"), ("et", "plain"), ("sssp", "vc")]:
        dd.fill_(7)
        G.batch_query_device(dp, dd, algo=algo, batch=batch)
        assert np.array_equal(dd.cpu().numpy().view(np.uint64), exp), (algo, batch)
    e = torch.empty((0, 2), dtype=torch.int32, device="cuda")
    G.batch_query_device(e, torch.empty(0, dtype=torch.int64, device="cuda"))
    bad = dp.clone()
    bad[5, 1] = g.n
    with pytest.raises(P.PPSPError) as err:
        G.batch_query_device(bad, dd)
    assert err.value.code == P.E_RANGE
    G.close()
