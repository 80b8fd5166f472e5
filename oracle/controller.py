"""FP64 reference of the controller's MLP (the `rpca_mlp_*` entry points).

TEST INFRASTRUCTURE, like the rest of this directory: only the test suite may
use it. It restates the network that the library's header documents -- 10
inputs, two tanh layers of 64 units, two outputs y_k = lo_k + (hi_k - lo_k)
sigmoid(z_k) with (lo, hi) = (g_min, 1) and (w_min, w_max) -- and its loss
1/2 sum_k (y_k - t_k)^2, with the gradient written out by the chain rule. The
parameter vector follows the header's order: W1 (64 x 10, row-major), b1, W2
(64 x 64), b2, W3 (2 x 64), b3 (2).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 10, 64, 2
G_MIN, W_MIN, W_MAX = 0.5, 0.5, 2.0
LO = np.array([G_MIN, W_MIN])
SPAN = np.array([1.0 - G_MIN, W_MAX - W_MIN])
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p: np.ndarray) -> dict:
    out, at = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(p[at:at + k], dtype=np.float64).reshape(shape)
        at += k
    return out


def forward(p: np.ndarray, X: np.ndarray):
    """Y (n x 2) for the rows of X, with the intermediates the gradient needs."""
    q = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ q["W1"].T + q["b1"])
    h2 = np.tanh(h1 @ q["W2"].T + q["b2"])
    z = h2 @ q["W3"].T + q["b3"]
    sg = 1.0 / (1.0 + np.exp(-z))
    y = LO + SPAN * sg
    return y, (X, h1, h2, sg)


def loss(p: np.ndarray, X: np.ndarray, T: np.ndarray) -> float:
    y, _ = forward(p, X)
    return float(np.mean(0.5 * np.sum((y - np.asarray(T, dtype=np.float64)) ** 2, axis=1)))


def grad(p: np.ndarray, X: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Gradient of the mean loss over the rows of X (chain rule, layer by
    layer from the outputs back)."""
    q = unpack(p)
    y, (X, h1, h2, sg) = forward(p, X)
    n = X.shape[0]
    dz = (y - np.asarray(T, dtype=np.float64)) * SPAN * sg * (1.0 - sg) / n   # n x 2
    g_W3 = dz.T @ h2
    g_b3 = dz.sum(axis=0)
    dz2 = (dz @ q["W3"]) * (1.0 - h2 ** 2)
    g_W2 = dz2.T @ h1
    g_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ q["W2"]) * (1.0 - h1 ** 2)
    g_W1 = dz1.T @ X
    g_b1 = dz1.sum(axis=0)
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_W3.ravel(), g_b3])


def sgd_step(p: np.ndarray, X: np.ndarray, T: np.ndarray, lr: float) -> np.ndarray:
    return np.asarray(p, dtype=np.float64) - lr * grad(p, X, T)
