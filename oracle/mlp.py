"""FP64 reference of the far-field correction network (test infrastructure).

h = W3 relu(W2 relu(W1 f + b1) + b2) + b3, W1: 64x8, W2: 64x64, W3: 2x64,
parameters packed as W1, b1, W2, b2, W3, b3 (row-major, 4866 values).
Loss of a batch (f_b, y_b): L = 1/(2B) sum_b |h(f_b) - y_b|^2.
The gradient is the chain rule written out layer by layer.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 8, 64, 2
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(w):
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    assert w.size == N_PARAM
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = w[o:o + k].reshape(shp)
        o += k
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1)
                           for name, _ in SHAPES])


def init(seed: int, out_scale: float = 0.1) -> np.ndarray:
    """He-normal hidden layers, small output layer, zero biases."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.normal(0, np.sqrt(2.0 / N_IN), (N_H, N_IN)), "b1": np.zeros(N_H),
         "W2": rng.normal(0, np.sqrt(2.0 / N_H), (N_H, N_H)), "b2": np.zeros(N_H),
         "W3": rng.normal(0, out_scale / np.sqrt(N_H), (N_OUT, N_H)), "b3": np.zeros(N_OUT)}
    return pack(p)


def forward(w, X):
    p = unpack(w)
    X = np.asarray(X, dtype=np.float64).reshape(-1, N_IN)
    z1 = X @ p["W1"].T + p["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = np.maximum(z2, 0.0)
    h = a2 @ p["W3"].T + p["b3"]
    return h, (X, z1, a1, z2, a2)


def loss_grad(w, X, Y):
    """Returns (L, dL/dw packed)."""
    p = unpack(w)
    h, (X, z1, a1, z2, a2) = forward(w, X)
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, N_OUT)
    B = X.shape[0]
    r = h - Y
    L = 0.5 * float(np.sum(r * r)) / B
    dh = r / B
    g = {"W3": dh.T @ a2, "b3": dh.sum(0)}
    da2 = dh @ p["W3"]
    dz2 = da2 * (z2 > 0)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(0)
    da1 = dz2 @ p["W2"]
    dz1 = da1 * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return L, pack(g)
