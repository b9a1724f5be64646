"""Pins of the float64 MLP oracle (learned PP controller) against closed forms,
finite differences and the published Adam behaviour."""
import math

import numpy as np
import pytest

from oracle import mlp


def _params(d, H, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 0.7, mlp.n_params(d, H))


@pytest.mark.parametrize("d,H,B", [(5, 64, 17), (7, 64, 9), (3, 4, 1)])
def test_gradient_matches_central_differences(d, H, B):
    rng = np.random.default_rng(d * 100 + H)
    p = _params(d, H, 1)
    X = rng.normal(size=(B, d))
    t = rng.normal(size=B)
    _, g = mlp.loss_and_grad(p, X, t, d, H)
    h = 1e-6
    fd = np.empty_like(p)
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = h
        fd[k] = (mlp.loss(p + e, X, t, d, H) - mlp.loss(p - e, X, t, d, H)) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-7 * np.linalg.norm(fd)


def test_forward_special_case_constant_hidden_layer():
    # W1 = 0: every hidden unit is tanh(b1_j) whatever the input, so
    # y = sum_j W2_j tanh(b1_j) + b2 for every sample.
    d, H = 4, 3
    b1 = np.array([math.atanh(0.5), 0.0, math.atanh(-0.25)])
    W2 = np.array([2.0, 7.0, 4.0])
    p = mlp.pack(np.zeros((H, d)), b1, W2, 0.125)
    y, h = mlp.forward(p, np.random.default_rng(0).normal(size=(6, d)), d, H)
    assert np.allclose(h, [0.5, 0.0, -0.25], rtol=0, atol=1e-15)
    assert np.allclose(y, 2.0 * 0.5 + 4.0 * -0.25 + 0.125, rtol=0, atol=1e-15)


def test_forward_brute_force_single_sample():
    d, H = 3, 5
    p = _params(d, H, 3)
    x = np.array([0.3, -1.2, 0.7])
    W1, b1, W2, b2 = mlp.unpack(p, d, H)
    want = b2
    for j in range(H):
        z = b1[j]
        for i in range(d):
            z += W1[j, i] * x[i]
        want += W2[j] * math.tanh(z)
    y, _ = mlp.forward(p, x[None, :], d, H)
    assert abs(y[0] - want) <= 1e-14 * (1 + abs(want))


def test_adam_first_step_has_magnitude_lr():
    # With m = v = 0 the bias-corrected first step is lr * g / (|g| + eps).
    g = np.array([3.0, -0.01, 1e-3, -250.0])
    p0 = np.zeros_like(g)
    lr = 0.05
    p1, m, v = mlp.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    assert np.allclose(p1, -lr * np.sign(g), rtol=0, atol=lr * 1e-8 / 1e-3 * 1.01)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_converges_on_quadratic():
    p = np.array([0.0])
    m = np.zeros(1)
    v = np.zeros(1)
    for s in range(1, 3001):
        g = 2.0 * (p - 3.0)
        p, m, v = mlp.adam_step(p, g, m, v, s, 0.01)
    assert abs(p[0] - 3.0) < 1e-3


def test_training_reduces_loss_on_smooth_target():
    d, H, B = 2, 16, 64
    rng = np.random.default_rng(5)
    X = rng.uniform(-2, 2, size=(B, d))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1]
    p = rng.normal(0, 0.3, mlp.n_params(d, H))
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    L0 = mlp.loss(p, X, t, d, H)
    for s in range(1, 1501):
        _, g = mlp.loss_and_grad(p, X, t, d, H)
        p, m, v = mlp.adam_step(p, g, m, v, s, 0.01)
    assert mlp.loss(p, X, t, d, H) < 0.02 * L0


def test_features_and_label_known_values():
    f = mlp.features([0.1, 1.0, 0.01], 0, 0.99)
    assert np.allclose(f, [-1.0, 0.0, -2.0, 0.0, 2.0], atol=1e-10)
    M = [np.arange(1.0, 7.0).reshape(3, 2), np.ones((4, 2))]
    Mt = [M[0] * (1 + 1e-3), M[1] * (1 - 1e-2)]
    assert abs(mlp.label(Mt, M) - (-2.0)) < 1e-12
