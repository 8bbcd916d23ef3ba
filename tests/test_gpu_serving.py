"""GPU tests of the continuous-batching server (ppsp_server_* through the C-ABI).

Every request's distances must equal the oracle's and the same library's
answer for that request run alone (ppsp_batch_query before the server took
the graph), whatever else shares the device with it: queries are admitted
into a running round loop between rounds, and slots are reused.
"""
import time

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


def _oracle(g, pairs):
    return oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)


def _requests(graphs, sizes, seed):
    """Request i goes to graph i % len(graphs); a few self pairs mixed in."""
    out = []
    for i, k in enumerate(sizes):
        gi = i % len(graphs)
        p = gen.pairs_uniform(graphs[gi].n, k, seed=seed + i)
        if k > 2:
            p[1, 1] = p[1, 0]
        out.append((gi, p))
    return out


def _serve(P, hosts, algo, reqs, slots, stagger_s):
    Gs = [P.Graph.from_host(g) for g in hosts]
    alone = [Gs[gi].batch_query(p, algo=algo, batch="plainstar") for gi, p in reqs]
    budget = 24 * sum(g.n for g in hosts) * slots        # `slots` query slots per graph (2/3 of it is state)
    S = P.Server(Gs, algo=algo, state_budget_bytes=budget)
    assert S.stats()["slots"] == slots * len(hosts)
    ids = []
    for gi, p in reqs:
        ids.append(S.submit(gi, p))
        time.sleep(stagger_s)
    res = [S.wait(r, timeout_ms=120000) for r in ids]
    st = S.stats()
    S.close()
    for G in Gs:
        G.close()
    return alone, res, st


def test_server_isolation_and_admission(P):
    """Two resident lattices, BiD-A*, 4 slots each, 14 requests of 1..37
    queries submitted while earlier ones run: each request equals the oracle
    and its own run alone."""
    hosts = [gen.lattice(200, 0.05, seed=5), gen.lattice(120, 0.1, seed=6)]
    sizes = [1, 9, 37, 3, 16, 2, 25, 5, 12, 1, 30, 7, 4, 20]
    reqs = _requests(hosts, sizes, seed=500)
    alone, res, st = _serve(P, hosts, "bidastar", reqs, slots=4, stagger_s=0.002)
    for (gi, p), a, (d, lat) in zip(reqs, alone, res):
        exp = _oracle(hosts[gi], p)
        assert np.array_equal(a, exp)
        assert np.array_equal(d, exp)
        assert lat > 0
    nself = sum(int(np.sum(p[:, 0] == p[:, 1])) for _, p in reqs)
    assert st["admitted"] == sum(sizes) - nself
    assert st["completed"] == len(reqs)
    assert st["running"] == 0 and st["pending"] == 0


def test_server_mixed_algorithms(P):
    """One server, BiD-A* on a lattice and BiDS on an R-MAT graph (one
    algorithm per graph)."""
    hosts = [gen.lattice(150, 0.05, seed=11), gen.rmat(11, 16, seed=12)]
    Gs = [P.Graph.from_host(g) for g in hosts]
    reqs = _requests(hosts, [6, 20, 9, 13, 2, 30], seed=800)
    S = P.Server(Gs, algo=["bidastar", "bids"], state_budget_bytes=16 * sum(g.n for g in hosts) * 5)
    ids = [S.submit(gi, p) for gi, p in reqs]
    for (gi, p), r in zip(reqs, ids):
        d, _ = S.wait(r, timeout_ms=120000)
        assert np.array_equal(d, _oracle(hosts[gi], p))
    S.close()
    with pytest.raises(P.PPSPError):
        P.Server(Gs, algo=["bids", "bidastar"])             # no coordinates on the R-MAT graph
    with pytest.raises(P.PPSPError):
        P.Server([Gs[0], Gs[0]], algo="bids")               # a graph twice
    for G in Gs:
        G.close()


def test_server_bids_unreachable_and_hubs(P):
    """BiDS over a disconnected random graph and an R-MAT graph with hub
    vertices (heavy-list path): unreachable pairs return INF in the mix."""
    hosts = [gen.random_graph(3000, 2400, 100, seed=21), gen.rmat(12, 16, seed=52)]
    sizes = [8, 40, 3, 17, 1, 29, 11, 6]
    reqs = _requests(hosts, sizes, seed=700)
    alone, res, st = _serve(P, hosts, "bids", reqs, slots=6, stagger_s=0.0)
    n_inf = 0
    for (gi, p), a, (d, _) in zip(reqs, alone, res):
        exp = _oracle(hosts[gi], p)
        assert np.array_equal(a, exp)
        assert np.array_equal(d, exp)
        n_inf += int(np.sum(exp == oracle.INF))
    assert n_inf > 0, "the random graph should leave some pairs unreachable"


def test_server_single_slot_reuse(P):
    """One slot: every query reuses the slot its predecessor just left."""
    hosts = [gen.lattice(64, 0.2, seed=8)]
    reqs = _requests(hosts, [5, 1, 7, 3], seed=900)
    alone, res, _ = _serve(P, hosts, "bidastar", reqs, slots=1, stagger_s=0.0)
    for (gi, p), a, (d, _) in zip(reqs, alone, res):
        assert np.array_equal(d, _oracle(hosts[gi], p))
        assert np.array_equal(d, a)


def test_server_overflow_restarts_keep_results(P):
    """A queue far too small for the frontier: the server grows it and
    restarts the queries on the device; every result still equals the oracle."""
    hosts = [gen.lattice(120, 0.1, seed=14)]
    G = P.Graph.from_host(hosts[0])
    G.set_option("queue_cap", 256)
    reqs = _requests(hosts, [12, 5, 30, 8], seed=950)
    S = P.Server([G], algo="bidastar", state_budget_bytes=16 * hosts[0].n * 3 * 8)
    ids = [S.submit(0, p) for _, p in reqs]
    for (_, p), r in zip(reqs, ids):
        d, _ = S.wait(r, timeout_ms=120000)
        assert np.array_equal(d, _oracle(hosts[0], p))
    st = S.stats()
    assert st["restarts"] > 0 and st["completed"] == len(reqs)
    S.close()
    G.close()


def test_server_errors_and_release(P):
    g = gen.lattice(40, 0.3, seed=9)
    G = P.Graph.from_host(g)
    with pytest.raises(P.PPSPError):
        P.Server([G], algo="et")                        # one-directional modes are not served
    S = P.Server([G], algo="bids", state_budget_bytes=1 << 24)
    with pytest.raises(P.PPSPError) as e:
        G.query(0, 1, algo="bids")                      # reserved while served
    assert e.value.code == P.E_BUSY
    with pytest.raises(P.PPSPError) as e:
        G.set_option("rounds_per_sync", 4)
    assert e.value.code == P.E_BUSY
    assert P.lib().ppsp_graph_destroy(G.h) == P.E_BUSY
    with pytest.raises(P.PPSPError) as e:
        S.submit(0, np.array([[0, g.n]], np.uint32))
    assert e.value.code == P.E_RANGE
    with pytest.raises(P.PPSPError):
        S.submit(1, np.array([[0, 1]], np.uint32))      # no graph 1
    r = S.submit(0, np.zeros((0, 2), np.uint32))        # empty request completes at once
    d, _ = S.wait(r)
    assert d.shape == (0,)
    r = S.submit(0, np.array([[3, 3]], np.uint32))
    assert S.wait(r)[0].tolist() == [0]
    S.close()
    p = gen.pairs_uniform(g.n, 10, seed=1)
    assert np.array_equal(G.batch_query(p, algo="bids"), _oracle(g, p))  # usable again
    G.close()


def test_server_directed_graph(P):
    """A directed graph served with BiDS: the backward half of every admitted
    query walks the transpose."""
    g = gen.lattice(100, 0.1, seed=31)
    rng = np.random.default_rng(32)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))
    w = g.w.astype(np.int64) + rng.integers(0, 800, g.w.shape[0])
    d = gen.csr_from_edges(g.n, src, g.col.astype(np.int64), w, symmetric=False)
    reqs = _requests([d], [5, 17, 3, 30, 9], seed=33)
    exp = [_oracle(d, p) for _, p in reqs]
    rev = oracle.pp_batch(d.n, d.row_ptr, d.col, d.w, reqs[3][1][:, ::-1].copy())
    assert not np.array_equal(rev, exp[3])                   # the graph really is directed
    D = P.Graph.from_host(d)
    S = P.Server([D], algo="bids", state_budget_bytes=24 * d.n * 4)
    ids = [S.submit(0, p) for _, p in reqs]
    for r, e in zip(ids, exp):
        got, _ = S.wait(r, timeout_ms=120000)
        assert np.array_equal(got, e)
    S.close()
    D.close()


def test_server_renumbers_rounds_before_stamp_limit(P):
    """The round loop starts 40 rounds below the renumbering point (option
    server_round_base): the server renumbers its rounds from 0 while
    requests are on the device, restarts them, and every request still equals
    the oracle."""
    g = gen.lattice(160, 0.05, seed=31)
    G = P.Graph.from_host(g)
    G.set_option("rounds_per_sync", 16)
    G.set_option("server_round_base", 0xFFFFFF00 - 40)
    assert G.get_option("server_round_base") == 0xFFFFFF00 - 40
    reqs = [gen.pairs_uniform(g.n, k, seed=700 + i) for i, k in enumerate([5, 12, 3, 20, 8, 1, 15])]
    S = P.Server([G], algo="bidastar", state_budget_bytes=24 * g.n * 6)
    ids = [S.submit(0, p) for p in reqs]
    res = [S.wait(r, timeout_ms=120000) for r in ids]
    st = S.stats()
    S.close()
    G.close()
    assert st["renumbers"] >= 1, st
    for p, (d, _) in zip(reqs, res):
        assert np.array_equal(d, _oracle(g, p))


def test_server_4096_pair_request_across_slot_refills(P):
    """One request of 4,096 pairs on a server with 16 query slots per graph:
    it is admitted across hundreds of slot refills while a second graph's
    requests run beside it, and equals the oracle and its own run alone."""
    hosts = [gen.lattice(90, 0.05, seed=210), gen.rmat(12, 16, seed=211)]
    big = gen.pairs_uniform(hosts[0].n, 4096, seed=212)
    side = [gen.pairs_uniform(gen.lcc(hosts[1]), k, seed=213 + k) for k in (3, 40, 17)]
    Gs = [P.Graph.from_host(h) for h in hosts]
    alone = Gs[0].batch_query(big, algo="bidastar")
    alone_side = [Gs[1].batch_query(p, algo="bids") for p in side]
    budget = 24 * sum(h.n for h in hosts) * 16
    S = P.Server(Gs, algo=["bidastar", "bids"], state_budget_bytes=budget)
    assert S.stats()["slots"] == 32
    ids = [S.submit(0, big)] + [S.submit(1, p) for p in side]
    res = [S.wait(r, timeout_ms=300000) for r in ids]
    st = S.stats()
    S.close()
    for G in Gs:
        G.close()
    assert np.array_equal(res[0][0], alone)
    assert np.array_equal(res[0][0], _oracle(hosts[0], big))
    for p, a, (d, _) in zip(side, alone_side, res[1:]):
        assert np.array_equal(d, a) and np.array_equal(d, _oracle(hosts[1], p))
    assert st["admitted"] >= 4096 - int(np.sum(big[:, 0] == big[:, 1]))


def test_server_runs_the_learned_schedule(P):
    """Served graphs under the learned schedule (a network loaded on each):
    every search picks its step each round inside the server's round loop;
    every request equals the oracle and its run alone (batch, learned)."""
    hosts = [gen.lattice(150, 0.05, seed=220), gen.rmat(13, 16, seed=221)]
    reqs = [(0, gen.pairs_uniform(hosts[0].n, k, seed=222 + k)) for k in (1, 30, 9, 64)] + \
           [(1, gen.pairs_uniform(gen.lcc(hosts[1]), k, seed=240 + k)) for k in (5, 25, 2)]
    Gs = [P.Graph.from_host(h) for h in hosts]
    for i, G in enumerate(Gs):
        p = gen.mlp_init(230 + i)
        p[-9:-1] = np.linspace(-1, 1, 8)
        G.mlp_load(p)
    algos = ["bidastar", "bids"]
    alone = [Gs[gi].batch_query(p, algo=algos[gi], sched="learned") for gi, p in reqs]
    S = P.Server(Gs, algo=algos, sched="learned", state_budget_bytes=24 * sum(h.n for h in hosts) * 6)
    ids = []
    for gi, p in reqs:
        ids.append(S.submit(gi, p))
        time.sleep(0.002)
    res = [S.wait(r, timeout_ms=120000) for r in ids]
    S.close()
    for G in Gs:
        G.close()
    for (gi, p), a, (d, _) in zip(reqs, alone, res):
        assert np.array_equal(d, a) and np.array_equal(d, _oracle(hosts[gi], p))
