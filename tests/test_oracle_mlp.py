"""Pins of the oracle's learned-split network (oracle/mlp.py): back-propagation against central
finite differences, the forward pass against scalar loops written from the layer definitions, the
first Adam step against its closed form (lr * g / (|g| + eps)), and descent on a fit problem."""
import math

import numpy as np
import pytest

from oracle import mlp


def _params(seed, scale=0.5):
    return np.random.default_rng(seed).normal(0.0, scale, mlp.N_PARAMS)


def _data(seed, n=37):
    g = np.random.default_rng(seed)
    x = g.uniform(-1, 1, (n, 3))
    t = np.stack([np.sin(2 * x[:, 0]) + x[:, 1] * x[:, 2], np.cos(x[:, 1]) - 0.5 * x[:, 0]], axis=1)
    return x, t


def test_layout_and_size():
    assert mlp.N_PARAMS == 4546
    parts = mlp.unpack(np.arange(mlp.N_PARAMS, dtype=float))
    assert [p.shape for p in parts] == [(64, 3), (64,), (64, 64), (64,), (2, 64), (2,)]
    assert parts[0][0, 1] == 1 and parts[1][0] == 192 and parts[5][1] == mlp.N_PARAMS - 1


def test_forward_matches_scalar_loops():
    p = _params(1)
    x, _ = _data(2, n=3)
    y, h1, h2 = mlp.forward(p, x)
    W1, b1, W2, b2, W3, b3 = [a.tolist() for a in mlp.unpack(p)]
    for s in range(3):
        a1 = [math.tanh(sum(W1[i][k] * x[s][k] for k in range(3)) + b1[i]) for i in range(64)]
        a2 = [math.tanh(sum(W2[i][k] * a1[k] for k in range(64)) + b2[i]) for i in range(64)]
        out = [sum(W3[o][k] * a2[k] for k in range(64)) + b3[o] for o in range(2)]
        assert np.allclose(h1[s], a1, rtol=0, atol=1e-14)
        assert np.allclose(h2[s], a2, rtol=0, atol=1e-14)
        assert np.allclose(y[s], out, rtol=0, atol=1e-13)


def test_backprop_matches_finite_differences():
    p = _params(3)
    x, t = _data(4)
    g = mlp.gradient(p, x, t)
    idx = np.random.default_rng(5).choice(mlp.N_PARAMS, 200, replace=False)
    idx = np.concatenate([idx, [0, 191, 192, 255, 256, 4351, 4352, 4479, 4480, 4543, 4544, 4545]])
    fd = mlp.finite_difference(p, x, t, idx)
    assert np.allclose(g[idx], fd, rtol=1e-6, atol=1e-9)


def test_first_adam_step_closed_form():
    p = _params(6)
    x, t = _data(7)
    g = mlp.gradient(p, x, t)
    lr, eps = 1e-3, 1e-8
    p1, hist = mlp.adam(p, x, t, steps=1, lr=lr, eps=eps)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
    assert hist[0] == pytest.approx(mlp.loss(p, x, t))


def test_adam_descends():
    p = _params(8, scale=0.2)
    x, t = _data(9, n=64)
    _, hist = mlp.adam(p, x, t, steps=300, lr=3e-3)
    assert hist[-1] < 0.2 * hist[0]
