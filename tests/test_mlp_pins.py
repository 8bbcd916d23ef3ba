"""Pins of the FP64 network reference (oracle.mlp) on the CPU.

The learned schedule is not in the paper, so these pins come from the
network's own definition: finite differences of the loss check the
chain-rule gradient, closed forms check the loss, and Adam (Kingma and Ba,
Algorithm 1) is pinned by the closed forms of its moment recurrences under a
constant and a sign-alternating gradient over several steps.
"""
import numpy as np

import gen
from oracle import mlp


def _rows(n, seed):
    return gen.mlp_rows(n, seed, learnable=False)


def test_param_count_and_layout():
    assert mlp.NPARAM == 5577 == 64 * 12 + 64 + 64 * 64 + 64 + 9 * 64 + 9
    p = np.arange(mlp.NPARAM, dtype=np.float64)
    w = mlp.unpack(p)
    assert w["W1"][0, 1] == 1 and w["b1"][0] == 768 and w["W2"][0, 0] == 832
    assert w["b2"][0] == 4928 and w["W3"][0, 0] == 4992 and w["W3"][8, 63] == 5567
    assert w["b3"][0] == 5568 and w["b3"][8] == 5576
    assert np.array_equal(mlp.pack(w), p)


def test_zero_weights_give_bias_logits_and_closed_form_loss():
    p = np.zeros(mlp.NPARAM)
    w = mlp.unpack(p.copy())
    b3 = np.array([0.5, -1.0, 2.0, 0.0, 0.25, -0.5, 1.0, 3.0, -0.7])
    p[-9:] = b3
    X, y = _rows(50, 1)
    z = mlp.forward(p, X)
    assert z.shape == (50, 9) and np.allclose(z, b3[None, :])
    lse = np.log(np.exp(b3[:8]).sum())
    assert np.isclose(mlp.loss(p, X, y), np.mean(lse - b3[y]))          # no mode labels
    # with mode labels: + log(1 + e^z8) for sparse rows, + log(1 + e^z8) - z8 for dense ones
    Xm, ym = gen.mlp_rows(60, 2, learnable=False, modes=True)
    b, m = ym % 8, ym // 8
    assert set(m.tolist()) == {1, 2}
    expect = np.mean(lse - b3[b] + np.log1p(np.exp(-0.7)) - (m == 2) * (-0.7))
    assert np.isclose(mlp.loss(p, Xm, ym), expect)
    assert w["W1"].shape == (64, 12)


def test_uniform_logits_loss_is_log8():
    """All outputs 0: the bin term is log 8 and a labelled mode adds log 2."""
    p = np.zeros(mlp.NPARAM)
    X, y = _rows(30, 2)
    assert np.isclose(mlp.loss(p, X, y), np.log(8.0))
    Xm, ym = gen.mlp_rows(30, 3, learnable=False, modes=True)
    assert np.isclose(mlp.loss(p, Xm, ym), np.log(8.0) + np.log(2.0))


def test_single_path_network_closed_form():
    """Only hidden units 0 of both layers and output 3 connected: the logit
    is w3 * relu(w2 * relu(w1 . x + b1) + b2) + b3 by hand."""
    p = np.zeros(mlp.NPARAM)
    w = mlp.unpack(p)
    w["W1"][0, :] = np.linspace(-1, 1, 12)
    w["b1"][0] = 0.1
    w["W2"][0, 0] = 1.5
    w["b2"][0] = -0.2
    w["W3"][3, 0] = 2.0
    w["b3"][3] = 0.3
    w["W3"][8, 0] = -1.0                     # the mode output through the same path
    X, _ = _rows(20, 3)
    a = np.maximum(X.astype(np.float64) @ np.linspace(-1, 1, 12) + 0.1, 0)
    expect = 2.0 * np.maximum(1.5 * a - 0.2, 0) + 0.3
    z = mlp.forward(p, X)
    assert np.allclose(z[:, 3], expect)
    assert np.allclose(z[:, 8], -np.maximum(1.5 * a - 0.2, 0))
    assert np.allclose(np.delete(z, [3, 8], axis=1), 0)


def test_gradient_matches_finite_differences():
    p = gen.mlp_init(7).astype(np.float64)
    p += np.random.default_rng(8).normal(0, 0.05, p.shape)      # nonzero biases too
    X, y = gen.mlp_rows(40, 9, learnable=False, modes=True)
    y[::3] %= 8                                                  # a third of the rows without a mode label
    L, g = mlp.grad(p, X, y)
    assert np.isclose(L, mlp.loss(p, X, y))
    rng = np.random.default_rng(10)
    # every parameter block, a few coordinates each
    idx = np.concatenate([rng.choice(np.arange(a, b), min(12, b - a), replace=False)
                          for a, b in [(0, 768), (768, 832), (832, 4928), (4928, 4992), (4992, 5568), (5568, 5577)]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, y) - mlp.loss(p - e, X, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so the step is
    -lr * g / (|g| + eps)."""
    rng = np.random.default_rng(11)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    lr = 1e-3
    p1, m, v = mlp.adam_step(p, np.zeros(100), np.zeros(100), g, 1, lr)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_closed_form_t1_to_5():
    """A constant gradient g from zero moments: m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so the bias-corrected moments are exactly g and g^2
    at every t and each step moves p by -lr g / (|g| + eps). A dropped or
    mis-indexed bias correction changes the step size after t = 1."""
    rng = np.random.default_rng(21)
    p0 = rng.normal(size=64)
    g = rng.normal(size=64) * 10.0 ** rng.integers(-3, 3, 64)
    lr, b1, b2, eps = 2e-3, 0.9, 0.999, 1e-8
    p, m, v = p0.copy(), np.zeros(64), np.zeros(64)
    for t in range(1, 6):
        p, m, v = mlp.adam_step(p, m, v, g, t, lr)
        assert np.allclose(m, (1 - b1 ** t) * g, rtol=1e-12, atol=0)
        assert np.allclose(v, (1 - b2 ** t) * g * g, rtol=1e-12, atol=0)
        assert np.allclose(p, p0 - t * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_adam_alternating_gradient_closed_form_t1_to_5():
    """Gradients g, -g, g, -g, ...: m_t = (1 - b1) g (b1^t - (-1)^t) / (1 + b1)
    (the geometric sum of the recurrence) and v_t = (1 - b2^t) g^2; the update
    divides by the bias corrections 1 - b1^t and 1 - b2^t of step t."""
    rng = np.random.default_rng(22)
    p0 = rng.normal(size=32)
    g = rng.normal(size=32)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    p, m, v = p0.copy(), np.zeros(32), np.zeros(32)
    expect = p0.copy()
    for t in range(1, 6):
        gt = g if t % 2 == 1 else -g
        p, m, v = mlp.adam_step(p, m, v, gt, t, lr)
        mt = (1 - b1) * g * (b1 ** t - (-1.0) ** t) / (1 + b1)
        vt = (1 - b2 ** t) * g * g
        assert np.allclose(m, mt, rtol=1e-12, atol=1e-15)
        assert np.allclose(v, vt, rtol=1e-12, atol=0)
        expect = expect - lr * (mt / (1 - b1 ** t)) / (np.sqrt(vt / (1 - b2 ** t)) + eps)
        assert np.allclose(p, expect, rtol=1e-12, atol=1e-15)
    # the step sizes differ from a no-bias-correction update after t = 1
    assert not np.allclose(m / (1 - b1 ** 5), m)


def test_gradient_descent_lowers_loss():
    p = gen.mlp_init(12).astype(np.float64)
    X, y = gen.mlp_rows(200, 13, learnable=True)
    L0, g = mlp.grad(p, X, y)
    assert mlp.loss(p - 0.05 * g, X, y) < L0
