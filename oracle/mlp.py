"""Learned split network: forward pass, mean-squared-error loss, back-propagation and Adam (oracle).

Test infrastructure (see the package docstring). Plain NumPy FP64, written from the definitions:

  network   3 -> 64 -> 64 -> 2:  h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = W3 h2 + b3
  loss      L = (1 / (2 n)) sum_s sum_o (y_so - t_so)^2      (mean over samples and the 2 outputs)
  gradients by the chain rule (d tanh(u) / du = 1 - tanh(u)^2), summed over samples
  Adam      m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
            p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)      (Kingma & Ba, 2015)

The parameter vector is laid out as W1 [64 x 3], b1 [64], W2 [64 x 64], b2 [64], W3 [2 x 64], b3 [2]
(row-major, 4546 values). The network and its training follow the learned-split description of the
method (an MLP mapping (log Nside, log FWHM, log target error) to (theta_cut, l_cut)); the paper
itself has no network, so no value here is printed in it.
"""
from __future__ import annotations

import numpy as np

SIZES = (3, 64, 64, 2)
N_PARAMS = 64 * 3 + 64 + 64 * 64 + 64 + 2 * 64 + 2


def unpack(p: np.ndarray):
    """Views (W1, b1, W2, b2, W3, b3) of the flat parameter vector."""
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (N_PARAMS,)
    o = 0
    out = []
    for shape in [(64, 3), (64,), (64, 64), (64,), (2, 64), (2,)]:
        k = int(np.prod(shape))
        out.append(p[o:o + k].reshape(shape))
        o += k
    return out


def forward(p, x):
    """Outputs y [n, 2] and the hidden activations (h1, h2) for inputs x [n, 3]."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.tanh(x @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ W3.T + b3, h1, h2


def loss(p, x, t) -> float:
    y, _, _ = forward(p, x)
    return float(np.sum((y - np.asarray(t, dtype=np.float64)) ** 2) / (2.0 * len(x)))


def gradient(p, x, t):
    """dL/dp as a flat vector (same layout as p), by back-propagation."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    y, h1, h2 = forward(p, x)
    n = len(x)
    dy = (y - np.asarray(t, dtype=np.float64)) / n          # dL/dy
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dh2 = (dy @ W3) * (1.0 - h2 * h2)                        # through tanh
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * (1.0 - h1 * h1)
    gW1 = dh1.T @ x
    gb1 = dh1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def finite_difference(p, x, t, idx, step: float = 1e-6):
    """Central differences of the loss for the parameters idx."""
    p = np.array(p, dtype=np.float64)
    out = np.empty(len(idx))
    for k, i in enumerate(idx):
        q = p.copy()
        q[i] += step
        lp = loss(q, x, t)
        q[i] -= 2 * step
        lm = loss(q, x, t)
        out[k] = (lp - lm) / (2 * step)
    return out


def adam(p, x, t, steps: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """Full-batch Adam from p; returns (p, loss history)."""
    p = np.array(p, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    hist = []
    for s in range(1, steps + 1):
        hist.append(loss(p, x, t))
        g = gradient(p, x, t)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        p = p - lr * (m / (1 - b1 ** s)) / (np.sqrt(v / (1 - b2 ** s)) + eps)
    return p, np.array(hist)
