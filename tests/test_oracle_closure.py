"""Pins of the closure network's FP64 reference: the gradient against central
finite differences of the loss, and the forward map on special parameters."""
import numpy as np

from oracle.closure import NPARAM, forward, init_params, loss_and_grad


def test_parameter_count():
    assert NPARAM == 9091


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    w = init_params(7, in_scale=1.7, g_max=0.6)
    w[2:] += 0.05 * rng.standard_normal(NPARAM - 2)   # nonzero biases too
    X = rng.standard_normal((33, 11))
    T = rng.standard_normal(33)
    _, g = loss_and_grad(w, X, T)
    assert g[0] == 0.0 and g[1] == 0.0
    idx = np.concatenate([rng.choice(np.arange(2, NPARAM), 120, replace=False), [NPARAM - 1]])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (loss_and_grad(wp, X, T)[0] - loss_and_grad(wm, X, T)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_special_cases():
    X = np.random.default_rng(0).standard_normal((5, 11))
    rp = X[:, 10]
    # zero weights: r- = g_max tanh(b4) r+ for any input
    w = np.zeros(NPARAM)
    w[0], w[1], w[-1] = 2.0, 0.5, 0.25
    r, _ = forward(w, X)
    assert np.allclose(r, 0.5 * np.tanh(0.25) * rp, rtol=1e-15, atol=0)
    # a gain that saturates at +-g_max bounds |r-| by g_max |r+|
    w[-1] = 40.0
    r, _ = forward(w, X)
    assert np.all(np.abs(r) <= 0.5 * np.abs(rp) + 1e-15)
    assert np.allclose(r, 0.5 * rp, rtol=1e-15, atol=0)
    # one path: x0 -> unit 0 of each layer -> output, tanh composed four
    # times; the input reaches it divided by the rms of the 10 raw inputs
    w = np.zeros(NPARAM)
    w[0], w[1] = 0.5, 1.0
    o = 2
    w[o] = 1.0                                  # W1[0][0]
    o += 64 * 10 + 64
    w[o] = 1.0                                  # W2[0][0]
    o += 64 * 64 + 64
    w[o] = 1.0                                  # W3[0][0]
    o += 64 * 64 + 64
    w[o] = 2.0                                  # W4[0]
    x = np.zeros((1, 11))
    x[0, 0], x[0, 1], x[0, 10] = 0.8, 0.6, 0.3  # rms of the inputs: sqrt(1/10)
    r, _ = forward(w, x)
    a = 0.5 * 0.8 * np.sqrt(10.0)
    assert abs(r[0] - 0.3 * np.tanh(2.0 * np.tanh(np.tanh(np.tanh(a))))) < 1e-15
    # the map is invariant to the amplitude of the inputs
    r2, _ = forward(w, np.concatenate([1e-3 * x[:, :10], x[:, 10:]], axis=1))
    assert abs(r2[0] - r[0]) < 1e-12
