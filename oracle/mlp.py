"""CPU float64 reference of the learned cost model -- test infrastructure only.

Only ``tests/`` may import this module (it checks the GPU training kernels).
It shares no code with the GPU package.

The model is the 3-layer perceptron the tuner's cost model uses:
    z1 = x W1 + b1, a1 = relu(z1), z2 = a1 W2 + b2, a2 = relu(z2), y = a2 w3 + b3,
with loss L = (1/N) sum_s (y_s - t_s)^2, and the Adam update of Kingma & Ba
(2015, Algorithm 1).  Parameters are one flat vector in the order
W1 (IN x H, row-major), b1, W2 (H x H), b2, w3, b3.  Everything is float64 and
written out step by step (no batching tricks beyond numpy matrix products).
"""
from __future__ import annotations

import numpy as np

IN, H = 6, 64
NPARAM = IN * H + H + H * H + H + H + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == NPARAM
    o = 0
    W1 = p[o:o + IN * H].reshape(IN, H); o += IN * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def forward(p, X):
    """Model outputs y (N,) and the intermediate values (z1, a1, z2, a2)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1 + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2 + b2
    a2 = np.maximum(z2, 0.0)
    y = a2 @ w3 + b3
    return y, (z1, a1, z2, a2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def gradient(p, X, t):
    """d loss / d p by the chain rule, layer by layer (ReLU derivative 0 at 0)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = X.shape[0]
    y, (z1, a1, z2, a2) = forward(p, X)
    gy = 2.0 * (y - t) / n                 # dL/dy
    g_w3 = a2.T @ gy
    g_b3 = gy.sum()
    g_z2 = np.outer(gy, w3) * (z2 > 0)     # dL/dz2
    g_W2 = a1.T @ g_z2
    g_b2 = g_z2.sum(axis=0)
    g_z1 = (g_z2 @ W2.T) * (z1 > 0)        # dL/dz1
    g_W1 = X.T @ g_z1
    g_b1 = g_z1.sum(axis=0)
    return pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
