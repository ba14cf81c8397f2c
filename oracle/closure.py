"""FP64 reference of the learned boundary closure's network (test
infrastructure): the forward map and the gradient of the mean squared error,
written out layer by layer.

Parameters, flat: in_scale, g_max, W1[64][10], b1[64], W2[64][64], b2[64],
W3[64][64], b3[64], W4[64], b4.  Network: x -> tanh(W1 s x + b1) ->
tanh(W2 . + b2) -> tanh(W3 . + b3) -> y = W4 . + b4, with s the input
scale and x the 10 raw inputs divided by their root mean square (plus
1e-30 under the root); the closure's r- is g_max tanh(y) r+.  A sample row
is X[11]: the 10 raw inputs (p and Z |u_t| now, then the square roots of
their running mean squares over 4 time scales), then r+, the outgoing
characteristic (p + Z n.u) / 2.  The network does not depend on what the
inputs mean.  The gradient is checked against central finite differences
in the tests, so the backward formulas below are pinned independently.
"""
from __future__ import annotations

import numpy as np

H, NIN = 64, 10
NPARAM = 2 + H * NIN + H + 2 * (H * H + H) + H + 1


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (NPARAM,)
    o = 2
    parts = {}
    for name, shape in (("W1", (H, NIN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
                        ("W3", (H, H)), ("b3", (H,)), ("W4", (H,)), ("b4", ())):
        size = int(np.prod(shape)) if shape else 1
        parts[name] = w[o:o + size].reshape(shape) if shape else w[o]
        o += size
    return w[0], w[1], parts


def forward(w, X):
    """r- for each sample row X[n][11]; also returns the hidden layers."""
    s_in, g_max, p = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    raw = X[:, :NIN]
    x = s_in * raw / np.sqrt(np.mean(raw * raw, axis=1, keepdims=True) + 1e-30)
    h1 = np.tanh(x @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    h3 = np.tanh(h2 @ p["W3"].T + p["b3"])
    th = np.tanh(h3 @ p["W4"] + p["b4"])
    rp = X[:, NIN]
    return g_max * th * rp, (x, h1, h2, h3, th, rp)


def loss_and_grad(w, X, T):
    """Mean squared error (1/n) sum (r- - T)^2 and its gradient with respect
    to the flat parameters (zero for the two scales)."""
    s_in, g_max, p = unpack(w)
    r, (x, h1, h2, h3, th, rp) = forward(w, X)
    e = r - np.asarray(T, dtype=np.float64)
    n = len(e)
    loss = float(np.mean(e * e))
    dy = 2.0 * e / n * g_max * rp * (1.0 - th * th)   # d loss / d (W4 h3 + b4)
    g = {"W4": dy @ h3, "b4": dy.sum()}
    d3 = np.outer(dy, p["W4"]) * (1.0 - h3 * h3)  # d loss / d pre-activation 3
    g["W3"], g["b3"] = d3.T @ h2, d3.sum(0)
    d2 = (d3 @ p["W3"]) * (1.0 - h2 * h2)
    g["W2"], g["b2"] = d2.T @ h1, d2.sum(0)
    d1 = (d2 @ p["W2"]) * (1.0 - h1 * h1)
    g["W1"], g["b1"] = d1.T @ x, d1.sum(0)
    flat = [np.zeros(2)] + [np.ravel(g[k]) for k in ("W1", "b1", "W2", "b2", "W3", "b3", "W4")]
    flat.append(np.array([g["b4"]]))
    return loss, np.concatenate(flat)


def init_params(seed, in_scale=1.0, g_max=1.0):
    """Glorot-uniform weights, zero biases (random networks for the tests)."""
    rng = np.random.default_rng(seed)
    w = np.zeros(NPARAM)
    w[0], w[1] = in_scale, g_max
    o = 2
    for fan_in, fan_out in ((NIN, H), (H, H), (H, H)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        w[o:o + fan_out * fan_in] = rng.uniform(-lim, lim, fan_out * fan_in)
        o += fan_out * fan_in + fan_out
    lim = np.sqrt(6.0 / (H + 1))
    w[o:o + H] = rng.uniform(-lim, lim, H)
    return w
