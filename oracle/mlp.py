"""FP64 CPU reference of the learned step schedule's network.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``): the test suite uses
it to check the GPU inference and training kernels; the product path never
imports it, and it shares no code with the GPU library.

The paper does not learn its schedule. It motivates one: the best step
Delta of the stepping framework (Section 2) depends on the query, and every
threshold sequence keeps the distances exact (Theorems bids-correctness and
bdastar-correctness hold for any stepping rule); and its sparse/dense frontier
switch (Appendix B) only changes the container. The network is therefore
pinned not by the paper but by its own definition, written out here in
float64:

    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  z = W3 h2 + b3   (z: 9 outputs)
    a label y = bin + 8 m: bin in 0..7, m = 0 (no mode label), 1 (sparse), 2 (dense)
    loss = mean over rows of  [log(sum_{b<8} exp z_b) - z_bin]                  (softmax cross-entropy)
                            + [m > 0] (log(1 + exp z_8) - [m = 2] z_8)          (logistic loss)

with parameters in one flat vector, row-major, in the order W1 [64][12],
b1 [64], W2 [64][64], b2 [64], W3 [9][64], b3 [9]. Its gradient is written
out by the chain rule and pinned by finite differences of ``loss`` in the
CPU tests (the two share no arithmetic beyond the forward pass), and Adam
follows Kingma and Ba (2015), Algorithm 1.
"""
from __future__ import annotations

import numpy as np

F, H, K = 12, 64, 8
O = K + 1                                          # the bin logits and the dense-mode logit
SHAPES = [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (O, H)), ("b3", (O,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)   # 5577


def unpack(p):
    """Flat parameter vector -> dict of float64 arrays (views)."""
    p = np.asarray(p, np.float64)
    assert p.shape == (NPARAM,)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in SHAPES])


def forward(p, X):
    """Outputs [n][9] of rows X [n][12]: 8 bin logits, then the mode logit."""
    w = unpack(p)
    X = np.asarray(X, np.float64)
    h1 = np.maximum(X @ w["W1"].T + w["b1"], 0.0)
    h2 = np.maximum(h1 @ w["W2"].T + w["b2"], 0.0)
    return h2 @ w["W3"].T + w["b3"]


def _split(y):
    y = np.asarray(y)
    return y % K, y // K


def loss(p, X, y):
    """Mean over rows of the bin cross-entropy plus, where a mode label is
    given, the logistic loss of the mode logit."""
    z = forward(p, X)
    b, m = _split(y)
    zb = z[:, :K]
    zm = zb.max(axis=1, keepdims=True)
    lse = np.log(np.exp(zb - zm).sum(axis=1)) + zm[:, 0]
    ce = lse - zb[np.arange(z.shape[0]), b]
    z8 = z[:, K]
    logistic = np.logaddexp(0.0, z8) - (m == 2) * z8
    return float(np.mean(ce + (m > 0) * logistic))


def grad(p, X, y):
    """(loss, gradient as a flat vector) by the chain rule."""
    w = unpack(p)
    X = np.asarray(X, np.float64)
    y = np.asarray(y)
    n = X.shape[0]
    a1 = X @ w["W1"].T + w["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w["W3"].T + w["b3"]
    b, m = _split(y)
    zb = z[:, :K]
    zm = zb.max(axis=1, keepdims=True)
    e = np.exp(zb - zm)
    s = e.sum(axis=1, keepdims=True)
    z8 = z[:, K]
    L = float(np.mean(np.log(s[:, 0]) + zm[:, 0] - zb[np.arange(n), b]
                      + (m > 0) * (np.logaddexp(0.0, z8) - (m == 2) * z8)))
    dz = np.zeros_like(z)
    dz[:, :K] = e / s
    dz[np.arange(n), b] -= 1.0
    # d/dz of log(1 + e^z) - t z is sigmoid(z) - t
    dz[:, K] = (m > 0) * (1.0 / (1.0 + np.exp(-z8)) - (m == 2))
    dz /= n
    g = {"W3": dz.T @ h2, "b3": dz.sum(axis=0)}
    dh2 = dz @ w["W3"]
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ w["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return L, pack(g)


def adam_step(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1); returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
