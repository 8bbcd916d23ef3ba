"""GPU tests of the learned step schedule: inference and training kernels
against the FP64 reference (oracle.mlp), exactness of searches under any
network, tracing, and the fit recipe."""
import numpy as np
import pytest

import gen
import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2506_16488_amd as P
    P.lib()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return P


def _params(seed, noise=0.05):
    p = gen.mlp_init(seed).astype(np.float64)
    p += np.random.default_rng(seed + 1).normal(0, noise, p.shape)
    return p.astype(np.float32)


def test_forward_matches_fp64_reference(P):
    for seed in (1, 2):
        p = _params(seed)
        X, _ = gen.mlp_rows(3000, seed + 10, learnable=False)
        got = P.mlp_forward(p, X)
        exp = mlp.forward(p.astype(np.float64), X)
        assert np.max(np.abs(got - exp)) <= 1e-5 * (1 + np.max(np.abs(exp))), seed
    assert P.mlp_forward(_params(3), np.zeros((0, 12), np.float32)).shape == (0, 9)


@pytest.mark.parametrize("n", [1, 37, 5000])
def test_gradient_matches_fp64_reference(P, n):
    p = _params(4)
    X, y = gen.mlp_rows(n, 20 + n, learnable=False, modes=True)
    y[::3] %= 8                                              # some rows without a mode label
    L, g = P.mlp_grad(p, X, y)
    Le, ge = mlp.grad(p.astype(np.float64), X, y)
    assert abs(L - Le) <= 1e-5 * (1 + abs(Le))
    scale = np.max(np.abs(ge))
    assert np.max(np.abs(g - ge)) <= 1e-4 * scale + 1e-7, n


def test_adam_step_matches_reference(P):
    """One full-batch step (batch = n, one epoch: the shuffle cannot matter)."""
    p = _params(5)
    X, y = gen.mlp_rows(512, 30, learnable=False)
    lr = 1e-3
    got, l0, l1 = P.mlp_train(p, X, y, epochs=1, batch=512, lr=lr, seed=3)
    _, g = mlp.grad(p.astype(np.float64), X, y)
    exp, _, _ = mlp.adam_step(p.astype(np.float64), np.zeros_like(g), np.zeros_like(g), g, 1, lr)
    # parameters whose gradient is far from zero (where fp32 and fp64 agree on its sign)
    big = np.abs(g) > 1e-3 * np.max(np.abs(g))
    assert big.sum() > 1000
    assert np.max(np.abs(got[big] - exp[big])) <= 2e-6
    assert np.max(np.abs(got - p)) <= lr * 1.0001          # a first Adam step never exceeds lr
    assert abs(l0 - mlp.loss(p.astype(np.float64), X, y)) < 1e-5
    assert abs(l1 - mlp.loss(got.astype(np.float64), X, y)) < 1e-5


def test_training_learns_a_rule(P):
    X, y = gen.mlp_rows(20000, 40, learnable=True, modes=True)
    p, l0, l1 = P.mlp_train(gen.mlp_init(41), X, y, epochs=15, batch=256, lr=3e-3, seed=42)
    assert l1 < 0.5 * l0, (l0, l1)
    z = P.mlp_forward(p, X)
    acc = np.mean(np.argmax(z[:, :8], axis=1) == y % 8)
    assert acc > 0.85, acc
    assert np.mean((z[:, 8] > 0) == (y // 8 == 2)) > 0.9                  # the mode output learned too
    Xt, yt = gen.mlp_rows(4000, 43, learnable=True, modes=True)
    zt = mlp.forward(p.astype(np.float64), Xt)
    assert np.mean(np.argmax(zt[:, :8], axis=1) == yt % 8) > 0.8
    # same seed, same result
    p2, _, _ = P.mlp_train(gen.mlp_init(41), X, y, epochs=15, batch=256, lr=3e-3, seed=42)
    assert np.array_equal(p, p2)


def _bias_only(b, dense=False):
    """A network that always picks bin b (and a dense frontier if asked)."""
    p = np.zeros(P_PARAMS, np.float32)
    p[-9:-1] = -5.0
    p[-9 + b] = 5.0
    p[-1] = 5.0 if dense else -5.0
    return p


P_PARAMS = 5577


def test_learned_schedule_is_exact(P):
    g = gen.lattice(96, 0.1, seed=50)
    pairs = np.concatenate([gen.pairs_uniform(g.n, 60, seed=51), np.array([[5, 5], [7, 9000]], np.uint32)])
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    G = P.Graph.from_host(g)
    with pytest.raises(P.PPSPError) as e:
        G.batch_query(pairs, algo="bids", sched="learned")      # no network loaded
    assert e.value.code == P.E_INVALID
    for params in [_params(60), _params(61, noise=0.5), _bias_only(0), _bias_only(7)]:
        G.mlp_load(params)
        for algo in ["sssp", "et", "astar", "bids", "bidastar"]:
            for batch in ["plainstar", "plain"]:
                got = G.batch_query(pairs, algo=algo, batch=batch, sched="learned")
                assert np.array_equal(got, exp), (algo, batch)
        assert np.array_equal(G.batch_query(pairs, algo="bids", batch="multi", sched="learned"), exp)
        d, (off, vtx) = G.batch_query(pairs[:10], algo="bidastar", sched="learned", want_path=True)
        for q in range(10):
            s, t = int(pairs[q, 0]), int(pairs[q, 1])
            assert oracle.check_path(g.n, g.row_ptr, g.col, g.w, vtx[off[q]:off[q + 1]], s, t, int(d[q])) == (0, 0)
    bad = _params(62)
    bad[100] = np.nan
    with pytest.raises(P.PPSPError):
        G.mlp_load(bad)
    G.close()


def test_learned_schedule_unreachable_and_hubs(P):
    g = gen.rmat(12, 16, seed=52)
    pairs = gen.pairs_uniform(g.n, 80, seed=53)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    assert np.any(exp == oracle.INF)
    G = P.Graph.from_host(g)
    G.mlp_load(_params(63, noise=0.3))
    for algo in ["bids", "et"]:
        assert np.array_equal(G.batch_query(pairs, algo=algo, sched="learned"), exp), algo
    G.close()


def test_trace_rows_and_costs(P):
    g = gen.lattice(128, 0.05, seed=70)
    pairs = gen.pairs_uniform(g.n, 40, seed=71)
    G = P.Graph.from_host(g)
    tot = {}
    for b in (0, 4, 7):
        feat, rowp, nrows, pr, pa = G.sched_trace(pairs, algo="bidastar", bins=b, cap=200000)
        assert nrows == feat.shape[0] > 0
        assert np.all(np.isfinite(feat)) and np.max(np.abs(feat)) < 4
        assert np.all(rowp < pairs.shape[0])
        assert np.all(pr > 0) and np.all(pa > 0)
        # each pair's rows: about one per search and round
        cnt = np.bincount(rowp, minlength=pairs.shape[0])
        assert np.all(cnt <= 2 * pr)
        tot[b] = (int(pr.sum()), int(pa.sum()))
    # A larger step needs fewer rounds until Delta covers a hop (one hop per
    # round bounds them from below; a stale entry checked every other round
    # can add a last round to a search), and scans more arcs.
    assert tot[0][0] > tot[4][0], tot
    assert tot[7][0] <= tot[4][0] + len(pairs), tot
    assert tot[0][1] < tot[4][1] < tot[7][1], tot
    # the fixed-bin run computes the same distances
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    assert np.array_equal(G.batch_query(pairs, algo="bidastar"), exp)
    G.close()


def test_fit_recipe(P):
    g = gen.lattice(128, 0.05, seed=80)
    train = gen.pairs_uniform(g.n, 24, seed=81)
    G = P.Graph.from_host(g)
    params, rep = G.mlp_fit(train, gen.mlp_init(82), algo="bidastar", epochs=5, seed=83)
    assert sum(rep["label_hist"]) == 24
    assert rep["rows"] > 0 and rep["loss_last"] <= rep["loss_first"]
    assert 0.0 <= rep["train_acc"] <= 1.0
    _check_referee(rep, params)
    test = gen.pairs_uniform(g.n, 50, seed=84)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, test)
    assert np.array_equal(G.batch_query(test, algo="bidastar", sched="learned"), exp)
    assert np.array_equal(G.batch_query(test, algo="bids", sched="learned"), exp)
    # batch-aware labels: fitted costs are non-negative, the best fixed bin is reported
    params, rep = G.mlp_fit(train, gen.mlp_init(85), algo="bidastar", epochs=5, seed=86, labels="batch")
    assert sum(rep["label_hist"]) == 24 and 0 <= rep["best_fixed_bin"] < 8
    assert rep["c_round_ms"] >= 0 and rep["c_arc_ns"] >= 0
    assert np.array_equal(G.batch_query(test, algo="bidastar", sched="learned"), exp)
    _check_referee(rep, params)
    G.close()


def _check_referee(rep, params):
    """The fixed-Delta referee: either the trained network won on the sample
    batch, or the installed (returned) network is the constant one for the
    faster fixed multiplier."""
    assert rep["learned_ms"] > 0 and rep["fixed_ms"] > 0
    fb = rep["fallback_bin"]
    assert 0 <= fb <= 8
    if fb == 8:
        assert rep["learned_ms"] <= rep["fixed_ms"]
    else:
        assert rep["fixed_ms"] < rep["learned_ms"]
        assert np.count_nonzero(params) == 1 and params[-9 + fb] == 1.0


def test_constant_network_is_exact(P):
    """The fallback network (zero weights, one output bias) is a valid learned
    schedule: every search keeps one multiplier and the distances are exact."""
    g = gen.lattice(96, 0.05, seed=87)
    test = gen.pairs_uniform(g.n, 40, seed=88)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, test)
    G = P.Graph.from_host(g)
    for b in (0, 4, 7):
        p = np.zeros(P.MLP_PARAMS, np.float32)
        p[-9 + b] = 1.0
        G.mlp_load(p)
        for algo in ("bidastar", "bids"):
            assert np.array_equal(G.batch_query(test, algo=algo, sched="learned"), exp), (b, algo)
    G.close()


def _bf16(p):
    """fp32 -> bf16 (round to nearest even) -> fp32, written out from the
    format's definition: keep the top 16 bits after adding half an ulp."""
    u = np.ascontiguousarray(p, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


def test_in_round_inference_matches_reference(P):
    """The network inside the control kernel (bf16 weights, fp32 arithmetic)
    picks, on every traced row, the argmax of the FP64 reference evaluated on
    the bf16-rounded parameters and the row's recorded features (rows whose
    two best logits are within 1e-3 of each other are skipped: fp32 and fp64
    may order them differently). The run is exact."""
    g = gen.lattice(128, 0.05, seed=90)
    pairs = gen.pairs_uniform(g.n, 40, seed=91)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    G = P.Graph.from_host(g)
    G.set_option("ml_every", 1)                 # the network decides after every round
    seen = set()
    for seed, noise in ((92, 0.3), (93, 1.0), (94, 2.0)):
        p = _params(seed, noise)
        G.mlp_load(p)
        tr = G.sched_trace_ex(pairs, algo="bidastar", network=True, cap=400000)
        assert np.array_equal(tr["dist"], exp)
        n = len(tr["bin"])
        assert tr["nrows"] == n > 100
        z = mlp.forward(_bf16(p).astype(np.float64), tr["feat"].astype(np.float64))[:, :8]
        top = np.sort(z, axis=1)
        clear = top[:, -1] - top[:, -2] > 1e-3 * (1 + np.abs(top[:, -1]))
        assert clear.mean() > 0.9, clear.mean()
        assert np.array_equal(tr["bin"][clear].astype(np.int64), np.argmax(z, axis=1)[clear])
        seen |= set(np.unique(tr["bin"]).tolist())
        assert np.all(tr["side"] <= 1) and np.all(tr["pair"] < len(pairs))
    assert len(seen) >= 2, seen                 # more than one output compared
    G.close()


def test_switched_schedule_rows_and_exactness(P):
    """Traced switches (the counterfactual replays of the labels): a pair runs
    bin 2 until the step for its switch round and bin 6 from then on; every
    row records the bin its step used, the distances are exact, and with
    distinct = 1 equal pairs with different schedules are traced apart."""
    g = gen.lattice(128, 0.05, seed=95)
    pairs = gen.pairs_uniform(g.n, 30, seed=96)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    G = P.Graph.from_host(g)
    sw = np.array([1 + 3 * (i % 5) for i in range(30)], np.uint32)
    tr = G.sched_trace_ex(pairs, algo="bidastar", bins=2, bins_after=6, switch_round=sw, cap=300000)
    assert np.array_equal(tr["dist"], exp)
    want = np.where(tr["round"] + 1 >= sw[tr["pair"]], 6, 2)
    assert np.array_equal(tr["bin"], want)
    assert np.all(tr["pair_rounds"] > 0) and np.all(tr["pair_arcs"] > 0) and np.all(tr["pair_entries"] > 0)
    # one pair three times: bins 0, 4 and 7 from round 1 on, kept apart
    rep = np.repeat(pairs[:1], 3, axis=0)
    tr = G.sched_trace_ex(rep, algo="bids", bins=4, bins_after=np.array([0, 4, 7], np.uint8),
                          switch_round=1, distinct=True)
    assert np.all(tr["dist"] == exp[0])
    # a smaller step needs more rounds and scans fewer arcs (a stale entry
    # checked every other round can add one round to a search)
    assert tr["pair_rounds"][0] > tr["pair_rounds"][1] and tr["pair_rounds"][2] <= tr["pair_rounds"][1] + 1
    assert tr["pair_arcs"][0] <= tr["pair_arcs"][2]
    G.close()


def test_counterfactual_fit_on_rmat_gains(P):
    """label_mode 2 on a mid-size R-MAT graph (scale 17) with the bucketed
    threshold rule: the labels come from replays that switch bins at decision
    rounds, the referee times 12 held-out pairs against the plain fixed path, and
    the trained schedule's fitted cost on those held-out pairs is below the
    base multiplier's. Distances stay exact."""
    g = gen.rmat(17, 16, seed=130)
    lcc = gen.lcc(g)
    sample = gen.pairs_uniform(lcc, 48, seed=131)
    test = gen.pairs_uniform(lcc, 40, seed=132)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, test)
    G = P.Graph.from_host(g, reorder=True)
    G.set_option("theta_mode", 1)
    delta = int(np.mean(g.w)) // 16
    print("counterfactual fit, rmat17", flush=True)
    params, rep = G.mlp_fit(sample, gen.mlp_init(133), algo="bids", epochs=30, seed=134, delta=delta,
                            labels="counterfactual")
    print({k: v for k, v in rep.items()}, flush=True)
    assert rep["heldout"] == 12 and rep["variants"] > 0 and rep["variants"] % 16 == 0
    assert sum(rep["label_hist"]) == rep["variants"] // 16
    assert 0 <= rep["dense_labels"] <= rep["variants"] // 16
    assert rep["rows"] > 0 and rep["loss_last"] <= rep["loss_first"]
    assert rep["c_round_ms"] >= 0 and rep["c_arc_ns"] >= 0 and rep["c_entry_ns"] >= 0
    assert rep["plain_fallback"] == (1 if rep["heldout_fixed_ms"] < rep["heldout_learned_ms"] else 0)
    assert np.array_equal(G.batch_query(test, algo="bids", sched="learned", delta=delta), exp)
    assert rep["heldout_learned_cost"] < rep["heldout_fixed_cost"], rep
    G.close()
