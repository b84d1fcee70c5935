"""Rank-predictor network — test infrastructure, FP64 NumPy.

A small fully connected network maps 8 geometric features of an admissible
block to the natural logarithm of its adaptive ACA rank:

    h1 = relu(W1 x + b1)      (64)
    h2 = relu(W2 h1 + b2)     (64)
    y  = W3 . h2 + b3         (scalar)

trained by mean squared error on log-ranks with Adam (Kingma & Ba 2015:
m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2, p <- p - lr mhat /
(sqrt(vhat) + eps) with bias-corrected mhat, vhat).  Inputs are
standardized with a mean and a standard deviation per feature.

The parameter vector is a data format shared with the GPU kernels (not code):
W1 (64 x 8, row-major), b1 (64), W2 (64 x 64, row-major), b2 (64), W3 (64),
b3 (1); 4801 numbers.  The gradient here is written out by hand
(backpropagation) and pinned by finite differences in the tests.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 8, 64
N_PARAMS = N_H * N_IN + N_H + N_H * N_H + N_H + N_H + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + N_H * N_IN].reshape(N_H, N_IN); o += N_H * N_IN
    b1 = p[o:o + N_H]; o += N_H
    W2 = p[o:o + N_H * N_H].reshape(N_H, N_H); o += N_H * N_H
    b2 = p[o:o + N_H]; o += N_H
    W3 = p[o:o + N_H]; o += N_H
    b3 = p[o:o + 1]; o += 1
    assert o == N_PARAMS
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, np.ravel(W3), np.ravel(b3)]).astype(np.float64)


def init(seed: int = 0) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((N_H, N_IN)) * np.sqrt(2.0 / N_IN)
    W2 = rng.standard_normal((N_H, N_H)) * np.sqrt(2.0 / N_H)
    W3 = rng.standard_normal(N_H) * np.sqrt(2.0 / N_H)
    return pack(W1, np.zeros(N_H), W2, np.zeros(N_H), W3, np.zeros(1))


def standardize(X, mean, std):
    return (np.asarray(X, dtype=np.float64) - mean) / std


def forward(p, X):
    """X: (n, 8) standardized features -> (y (n,), cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3[0]
    return y, (X, z1, h1, z2, h2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - t) ** 2))


def grad(p, X, t):
    """Loss mean((y - t)^2) and its gradient with respect to p."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    y, (X, z1, h1, z2, h2) = forward(p, X)
    n = X.shape[0]
    dy = 2.0 * (y - t) / n                    # (n,)
    gW3 = h2.T @ dy
    gb3 = np.array([dy.sum()])
    d2 = np.outer(dy, W3) * (z2 > 0)          # (n, 64)
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (z1 > 0)                 # (n, 64)
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    return float(np.mean((y - t) ** 2)), pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def train(X, t, order, batch, lr=1e-3, p0=None, seed=0):
    """Minibatch Adam over the sample order given (one index array per
    epoch, concatenated): batches are consecutive runs of `batch` indices.
    Returns (p, per-step losses)."""
    p = init(seed) if p0 is None else np.array(p0, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    order = np.asarray(order)
    for s, a in enumerate(range(0, order.size - batch + 1, batch)):
        idx = order[a:a + batch]
        L, g = grad(p, X[idx], t[idx])
        losses.append(L)
        p, m, v = adam(p, g, m, v, s + 1, lr)
    return p, np.array(losses)


def predicted_rank(y, margin=0.25):
    """Allocation width from a predicted log-rank: ceil(exp(y) (1 + margin))."""
    return np.ceil(np.exp(y) * (1.0 + margin)).astype(np.int64)
