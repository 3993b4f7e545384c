"""Pins of the FP64 reference of the learned-guess network."""
import numpy as np

from oracle import mlp_ref as M


def test_parameter_count():
    assert M.NPARAM == 1377


def test_zero_network_outputs_bias():
    w = np.zeros(M.NPARAM)
    w[-1] = 0.37
    X = np.random.default_rng(0).normal(size=(5, 8))
    assert np.allclose(M.forward(w, X), 0.37)
    loss, g = M.loss_grad(w, X, np.zeros(5))
    assert abs(loss - 0.37 ** 2) < 1e-15
    assert abs(g[-1] - 2 * 0.37) < 1e-15          # dL/db3 = 2 mean(y - t)
    assert np.abs(g[:-1]).max() == 0.0             # nothing else moves through zero weights


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    w = rng.normal(scale=0.3, size=M.NPARAM)
    X = rng.normal(size=(7, 8))
    t = rng.normal(size=7)
    loss, g = M.loss_grad(w, X, t)
    h = 1e-6
    idx = rng.choice(M.NPARAM, 60, replace=False).tolist() + [0, 255, 256, 1376]
    for k in idx:
        e = np.zeros(M.NPARAM)
        e[k] = h
        fd = (M.loss_grad(w + e, X, t)[0] - M.loss_grad(w - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * (1 + abs(g[k])), k


def test_small_weights_linear_regime():
    """With tiny first-layer weights tanh is linear: y ~ W3 tanh(W2 (W1 x + b1) + b2) + b3."""
    rng = np.random.default_rng(2)
    p = {name: rng.normal(scale=1e-4, size=shape) for name, shape in M.SHAPES}
    X = rng.normal(size=(4, 8))
    w = M.pack(p)
    lin = (p["W3"] @ (p["W2"] @ (p["W1"] @ X.T + p["b1"][:, None]) + p["b2"][:, None]) + p["b3"][:, None])[0]
    assert np.allclose(M.forward(w, X), lin, rtol=1e-6, atol=1e-18)
