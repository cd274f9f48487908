"""Cost-model network oracle: a plain fp64 CPU implementation used to check
the GPU kernels of the schedule autotuner's cost model.

TEST INFRASTRUCTURE ONLY.  The product package never imports this module.

The paper has no learned component; this network only predicts how long a
decode schedule takes and never touches pixel or bin bits.  It is a
two-hidden-layer perceptron with ReLU units and one linear output:

    z1 = W1 x + b1,  h1 = max(z1, 0)
    z2 = W2 h1 + b2, h2 = max(z2, 0)
    y  = w3 . h2 + b3

trained on the mean squared error L = (1/N) sum_s (y_s - t_s)^2.  Gradients
are the chain rule written out layer by layer (backpropagation, Rumelhart,
Hinton and Williams, Nature 1986); the update is Adam (Kingma and Ba, ICLR
2015) with bias correction.  Parameters are packed in one vector in the order
W1 (H x D, row-major), b1 (H), W2 (H x H, row-major), b2 (H), w3 (H), b3 (1).
"""
from __future__ import annotations

import numpy as np


def nparams(d_in: int, hidden: int) -> int:
    return hidden * d_in + hidden + hidden * hidden + hidden + hidden + 1


def unpack(p: np.ndarray, d_in: int, hidden: int):
    p = np.asarray(p, dtype=np.float64)
    H, D = hidden, d_in
    o = 0
    W1 = p[o:o + H * D].reshape(H, D); o += H * D
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward(p, x, d_in: int, hidden: int) -> np.ndarray:
    """Predictions for the rows of x (N x D)."""
    W1, b1, W2, b2, w3, b3 = unpack(p, d_in, hidden)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.maximum(x @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ w3 + b3


def loss(p, x, t, d_in: int, hidden: int) -> float:
    y = forward(p, x, d_in, hidden)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(p, x, t, d_in: int, hidden: int):
    """(dL/dp packed like p, L) by backpropagation.  The derivative of ReLU
    at exactly zero is taken as 0."""
    W1, b1, W2, b2, w3, b3 = unpack(p, d_in, hidden)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    N = x.shape[0]
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    gy = 2.0 * (y - t) / N                     # dL/dy_s
    g_w3 = h2.T @ gy
    g_b3 = gy.sum()
    g_z2 = np.outer(gy, w3) * (z2 > 0)         # dL/dz2
    g_W2 = g_z2.T @ h1
    g_b2 = g_z2.sum(axis=0)
    g_z1 = (g_z2 @ W2) * (z1 > 0)              # dL/dz1
    g_W1 = g_z1.T @ x
    g_b1 = g_z1.sum(axis=0)
    g = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])
    return g, float(np.mean((y - t) ** 2))


def adam(p, g, m, v, step: int, lr: float, beta1: float, beta2: float, eps: float):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return np.asarray(p, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def init(d_in: int, hidden: int, seed: int) -> np.ndarray:
    """He-scaled normal weights, zero biases (He et al., ICCV 2015)."""
    rng = np.random.default_rng(seed)
    H, D = hidden, d_in
    parts = [rng.normal(0, np.sqrt(2.0 / D), H * D), np.zeros(H),
             rng.normal(0, np.sqrt(2.0 / H), H * H), np.zeros(H),
             rng.normal(0, np.sqrt(1.0 / H), H), np.zeros(1)]
    return np.concatenate(parts)
