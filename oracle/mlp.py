"""16-64-64-1 tanh MLP in FP64: forward, analytic backward, Adam (oracle).

Not in the paper: this is the learned warm start of the entropy filter's per-element
search.  Inputs x (16 features) are standardised with a fixed mean/std,
    h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y^ = w3 . h2 + b3,
the loss is the mean squared error over a batch, the optimiser Adam.

Flat parameter layout (5,313 values):
    W1 [64][16] | b1 [64] | W2 [64][64] | b2 [64] | w3 [64] | b3 [1]
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 16, 64
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("w3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(w):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = w[o:o + n].reshape(shape)
        o += n
    return out


def glorot_init(seed=43):
    """Glorot-uniform weights, zero biases, from numpy PCG64(seed)."""
    rng = np.random.default_rng(seed)
    w = np.zeros(N_PARAMS)
    P = unpack(w)
    for name, fan_in, fan_out in (("W1", N_IN, N_H), ("W2", N_H, N_H)):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        P[name][...] = rng.uniform(-a, a, size=P[name].shape)
    a = np.sqrt(6.0 / (N_H + 1))
    P["w3"][...] = rng.uniform(-a, a, size=N_H)
    return w


def forward(w, X):
    P = unpack(np.asarray(w, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ P["W1"].T + P["b1"])
    h2 = np.tanh(h1 @ P["W2"].T + P["b2"])
    return h2 @ P["w3"] + P["b3"][0]


def loss_and_grad(w, X, y):
    """MSE loss mean((y^ - y)^2) and its gradient with respect to the flat parameters."""
    P = unpack(np.asarray(w, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    B = X.shape[0]
    h1 = np.tanh(X @ P["W1"].T + P["b1"])
    h2 = np.tanh(h1 @ P["W2"].T + P["b2"])
    yh = h2 @ P["w3"] + P["b3"][0]
    r = yh - y
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B                                  # dL/dy^
    g = np.zeros(N_PARAMS)
    G = unpack(g)
    G["w3"][...] = h2.T @ dy
    G["b3"][0] = dy.sum()
    d2 = np.outer(dy, P["w3"]) * (1.0 - h2 * h2)      # [B][64]
    G["W2"][...] = d2.T @ h1
    G["b2"][...] = d2.sum(axis=0)
    d1 = (d2 @ P["W2"]) * (1.0 - h1 * h1)
    G["W1"][...] = d1.T @ X
    G["b1"][...] = d1.sum(axis=0)
    return loss, g


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t = 1-based step count); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def batches(n, batch, steps, seed):
    """Deterministic minibatch index lists: epochs of PCG64(seed) permutations."""
    rng = np.random.default_rng(seed)
    out, perm, pos = [], rng.permutation(n), 0
    for _ in range(steps):
        if pos + batch > n:
            perm, pos = rng.permutation(n), 0
        out.append(perm[pos:pos + batch])
        pos += batch
    return out


def train(w, X, y, steps, batch=256, seed=44, lr=1e-3):
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    hist = []
    for t, idx in enumerate(batches(X.shape[0], batch, steps, seed), start=1):
        loss, g = loss_and_grad(w, X[idx], y[idx])
        w, m, v = adam_step(w, g, m, v, t, lr)
        hist.append(loss)
    return w, np.array(hist)
