"""Pins of the FP64 reference perceptron (oracle/mlp.py) that do not reuse
its own formulas: tabulated normal-CDF values for GELU, a weight choice that
turns the network into a closed-form linear map, central finite differences
for the hand-written gradient, and the bias-corrected first Adam step."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_tabulated_values():
    # GELU(x) = x Phi(x); Phi(1) = 0.8413447460685429, Phi(2) = 0.9772498680518208 (normal tables)
    assert mlp.gelu(np.array(0.0)) == 0.0
    assert abs(mlp.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(np.array(2.0)) - 2 * 0.9772498680518208) < 1e-15
    x = np.linspace(-5, 5, 41)
    # Phi(x) + Phi(-x) = 1  =>  GELU(x) - GELU(-x) = x
    assert np.allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-15)
    # derivative: central differences
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_prime(x), fd, atol=1e-8)
    assert mlp.gelu_prime(np.array(0.0)) == 0.5


def test_forward_linear_regime_closed_form():
    """With every pre-activation shifted by +40, GELU is the identity to
    within 40 * Phi(-40) ~ 1e-348, so the network is W3 W2 W1 x + const."""
    rng = np.random.default_rng(5)
    W1 = rng.uniform(-0.3, 0.3, (64, 5))
    W2 = rng.uniform(-0.1, 0.1, (64, 64))          # not symmetric: a transposed use would show
    W3 = rng.uniform(-0.2, 0.2, 64)
    shift = 40.0
    b1 = np.full(64, shift)
    b2 = shift - W2 @ np.full(64, shift)          # cancel the carried shift of layer 1
    b3 = 0.25
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, [b3]])
    X = rng.uniform(-1, 1, (17, 5))
    M = (W3[None, :] @ W2 @ W1).ravel()            # 5-vector
    expect = X @ M + shift * W3.sum() + b3
    assert np.allclose(mlp.forward(p, X), expect, rtol=0, atol=1e-12)


def test_forward_zero_weights():
    p = np.zeros(mlp.N_PARAMS)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    # biases only: output = W3 . GELU(b2) + b3 regardless of the input
    p[mlp.N_HID * 5 + mlp.N_HID + mlp.N_HID * mlp.N_HID:][:mlp.N_HID] = 1.0           # b2
    p[-1 - mlp.N_HID:-1] = np.arange(mlp.N_HID) / 64.0                                   # W3
    p[-1] = -0.5
    X = np.random.default_rng(0).standard_normal((4, 5))
    expect = (np.arange(64) / 64.0).sum() * 0.8413447460685429 - 0.5
    assert np.allclose(mlp.forward(p, X), expect, atol=1e-14)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(11)
    p = mlp.init_params(3) + rng.normal(0, 0.05, mlp.N_PARAMS)     # non-zero biases too
    X = rng.normal(0, 1, (23, 5))
    t = rng.normal(0, 1, 23)
    L, g = mlp.loss_and_grad(p, X, t)
    assert abs(L - np.mean((mlp.forward(p, X) - t) ** 2)) < 1e-14
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 200, replace=False), [0, 320, 384, 4480, 4544, 4608]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, X, t)[0] - mlp.loss_and_grad(p - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, np.abs(g).max()), (i, fd, g[i])


def test_adam_constant_gradient_moves_lr_per_step():
    """With bias correction, a constant gradient g gives m_hat = g and
    v_hat = g^2 exactly, so each step moves every parameter by lr g/(|g|+eps)."""
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    p = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-2, 1e-8
    for step in range(1, 6):
        p, m, v = mlp.adam_step(p, m, v, g, step, lr=lr, eps=eps)
        assert np.allclose(p, -step * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)


def test_init_is_glorot_uniform():
    p = mlp.init_params(0)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    assert np.abs(W1).max() <= math.sqrt(6.0 / 69) and np.abs(W2).max() <= math.sqrt(6.0 / 128)
    assert not b1.any() and not b2.any() and b3 == 0.0
    assert np.array_equal(p, mlp.init_params(0))


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (64, 5))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]
    p = mlp.init_params(1)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    L0 = mlp.loss_and_grad(p, X, t)[0]
    for step in range(1, 301):
        L, g = mlp.loss_and_grad(p, X, t)
        p, m, v = mlp.adam_step(p, m, v, g, step, lr=3e-3)
    assert mlp.loss_and_grad(p, X, t)[0] < 0.05 * L0
