"""Pins of the FP64 network reference (oracle.mlp) on the CPU.

The learned schedule is not in the paper, so these pins come from the
network's own definition: finite differences of the loss check the
chain-rule gradient, closed forms check the loss, and Adam's first step
has a closed form.
"""
import numpy as np

import gen
from oracle import mlp


def _rows(n, seed):
    return gen.mlp_rows(n, seed, learnable=False)


def test_param_count_and_layout():
    assert mlp.NPARAM == 5512
    p = np.arange(mlp.NPARAM, dtype=np.float64)
    w = mlp.unpack(p)
    assert w["W1"][0, 1] == 1 and w["b1"][0] == 768 and w["W2"][0, 0] == 832
    assert w["b2"][0] == 4928 and w["W3"][0, 0] == 4992 and w["b3"][7] == 5511
    assert np.array_equal(mlp.pack(w), p)


def test_zero_weights_give_bias_logits_and_closed_form_loss():
    p = np.zeros(mlp.NPARAM)
    w = mlp.unpack(p.copy())
    b3 = np.array([0.5, -1.0, 2.0, 0.0, 0.25, -0.5, 1.0, 3.0])
    p[-8:] = b3
    X, y = _rows(50, 1)
    z = mlp.forward(p, X)
    assert np.allclose(z, b3[None, :])
    lse = np.log(np.exp(b3).sum())
    assert np.isclose(mlp.loss(p, X, y), np.mean(lse - b3[y]))
    assert w["W1"].shape == (64, 12)


def test_uniform_logits_loss_is_log8():
    p = np.zeros(mlp.NPARAM)
    X, y = _rows(30, 2)
    assert np.isclose(mlp.loss(p, X, y), np.log(8.0))


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
    X, _ = _rows(20, 3)
    a = np.maximum(X.astype(np.float64) @ np.linspace(-1, 1, 12) + 0.1, 0)
    expect = 2.0 * np.maximum(1.5 * a - 0.2, 0) + 0.3
    z = mlp.forward(p, X)
    assert np.allclose(z[:, 3], expect)
    assert np.allclose(np.delete(z, 3, axis=1), 0)


def test_gradient_matches_finite_differences():
    p = gen.mlp_init(7).astype(np.float64)
    p += np.random.default_rng(8).normal(0, 0.05, p.shape)      # nonzero biases too
    X, y = _rows(40, 9)
    L, g = mlp.grad(p, X, y)
    assert np.isclose(L, mlp.loss(p, X, y))
    rng = np.random.default_rng(10)
    # every parameter block, a few coordinates each
    idx = np.concatenate([rng.choice(np.arange(a, b), min(12, b - a), replace=False)
                          for a, b in [(0, 768), (768, 832), (832, 4928), (4928, 4992), (4992, 5504), (5504, 5512)]])
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


def test_gradient_descent_lowers_loss():
    p = gen.mlp_init(12).astype(np.float64)
    X, y = gen.mlp_rows(200, 13, learnable=True)
    L0, g = mlp.grad(p, X, y)
    assert mlp.loss(p - 0.05 * g, X, y) < L0
