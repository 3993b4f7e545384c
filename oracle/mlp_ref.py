"""FP64 reference of the learned-guess network (test infrastructure only).

Network: 8 -> 32 -> 32 -> 1, tanh on both hidden layers, linear output:
  h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = W3 h2 + b3,
parameters packed as W1[32][8], b1[32], W2[32][32], b2[32], W3[1][32], b3[1]
(1377 values).  Loss: mean squared error L = (1/N) sum_n (y_n - t_n)^2.
Gradients by plain back-propagation (chain rule written out layer by layer).
Only the test suite uses this module.
"""
from __future__ import annotations

import numpy as np

SHAPES = [("W1", (32, 8)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)), ("W3", (1, 32)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = w[o:o + n].reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(w, X):
    """X: [N][8] -> y [N]."""
    p = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    return (h2 @ p["W3"].T + p["b3"])[:, 0]


def loss_grad(w, X, t):
    """Mean squared error and its gradient with respect to the packed parameters."""
    p = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    N = X.shape[0]
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.tanh(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.tanh(a2)
    y = (h2 @ p["W3"].T + p["b3"])[:, 0]
    r = y - t
    loss = float(np.mean(r * r))
    g3 = (2.0 / N) * r                      # dL/dy
    gW3 = g3[None, :] @ h2                   # [1][32]
    gb3 = np.array([g3.sum()])
    d2 = (g3[:, None] * p["W3"]) * (1.0 - h2 * h2)   # dL/da2 [N][32]
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (1.0 - h1 * h1)            # dL/da1 [N][32]
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    grad = pack(dict(W1=gW1, b1=gb1, W2=gW2, b2=gb2, W3=gW3, b3=gb3))
    return loss, grad
