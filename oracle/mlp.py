"""FP64 reference of the far-field correction network (test infrastructure).

h = W3 relu(W2 relu(W1 f + b1) + b2) + b3, W1: 64x8, W2: 64x64, W3: 2x64,
parameters packed as W1, b1, W2, b2, W3, b3 (row-major, 4866 values).
Loss of a batch (f_b, y_b): L = 1/(2B) sum_b |h(f_b) - y_b|^2.
The gradient is the chain rule written out layer by layer.

Training is Adam (Kingma and Ba, "Adam: A Method for Stochastic
Optimization", ICLR 2015, Algorithm 1) with its default moment decays
beta1 = 0.9, beta2 = 0.999 and epsilon = 1e-8, bias-corrected, on
minibatches drawn with replacement: row b of the minibatch of step t is
draw b of the SplitMix64 stream (seed, t, 64) modulo the sample count (the
stream state 0 is replaced by 1).  The network is not part of the paper; its
training is an extension of the method.
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


# ------------------------------------------------------------------ Adam

ADAM_BETA1, ADAM_BETA2, ADAM_EPS = 0.9, 0.999, 1e-8
MINIBATCH_TAG = 64


def adam_step(w, g, m, v, t, lr, beta1=ADAM_BETA1, beta2=ADAM_BETA2, eps=ADAM_EPS):
    """One Adam update at step number t >= 1 (Kingma and Ba 2015, Alg. 1):
    first and second raw moment estimates decayed by beta1 and beta2, each
    divided by (1 - beta^t) to remove the bias of their zero start, and the
    parameters moved by lr * m_hat / (sqrt(v_hat) + eps).
    Returns new (w, m, v); the inputs are not modified."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * (g * g)
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def minibatch_rows(n_samples: int, batch: int, seed: int, t: int) -> np.ndarray:
    """Rows of the minibatch of step t: SplitMix64 draws 0..batch-1 of the
    stream (seed, level t, tag 64), each modulo n_samples."""
    from . import draws, splitmix64_at

    state = (int(seed) ^ (int(t) << 48) ^ (MINIBATCH_TAG << 32)) & 0xFFFFFFFFFFFFFFFF
    if state == 0:
        r = np.array([splitmix64_at(1, b) for b in range(batch)], dtype=np.uint64)
    else:
        r = draws(seed, t, MINIBATCH_TAG, 0, batch)
    return (r % np.uint64(n_samples)).astype(np.int64)


def train(w, m, v, X, Y, steps: int, batch: int, lr: float, seed: int, step0: int = 0):
    """`steps` Adam steps on minibatches of the samples (X, Y), step numbers
    step0+1 ... step0+steps.  Returns (w, m, v, losses) with the minibatch
    loss before each step."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, N_IN)
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, N_OUT)
    w = np.array(w, dtype=np.float64)
    m = np.array(m, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    losses = []
    for it in range(steps):
        t = step0 + it + 1
        rows = minibatch_rows(X.shape[0], batch, seed, t)
        L, g = loss_grad(w, X[rows], Y[rows])
        losses.append(L)
        w, m, v = adam_step(w, g, m, v, t, lr)
    return w, m, v, np.array(losses)
