"""Pins of the FP64 MLP oracle (oracle/mlp.py) against what mathematics fixes:
the GELU closed form at known points, finite differences of the loss, a
network whose hidden weights vanish, and Adam's first step."""
import math

import numpy as np
import pytest

import synth
from oracle import mlp


def test_parameter_count_and_layout():
    assert mlp.n_params() == 6 * 128 + 128 + 2 * (128 * 128 + 128) + 128 + 1 == 34049
    theta = np.arange(mlp.n_params(), dtype=np.float64)
    (W1, b1), (W2, b2), (W3, b3), (W4, b4) = mlp.unpack(theta)
    assert W1.shape == (128, 6) and W1[0, 1] == 1 and b1[0] == 768
    assert W2[0, 0] == 896 and W4.shape == (1, 128) and b4[0] == 34048


def test_gelu_closed_form():
    # GELU(z) = z Phi(z); Phi(1) = 0.8413447460685429, Phi(-1) = 1 - Phi(1)
    assert mlp.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-15)
    assert mlp.gelu(np.array([-1.0]))[0] == pytest.approx(-(1 - 0.8413447460685429), rel=1e-14)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu(np.array([9.0]))[0] == pytest.approx(9.0, rel=1e-15)
    assert abs(mlp.gelu(np.array([-9.0]))[0]) < 1e-17
    # derivative: Phi(0) + 0 = 1/2; at 1: Phi(1) + phi(1)
    assert mlp.gelu_grad(np.array([0.0]))[0] == 0.5
    assert mlp.gelu_grad(np.array([1.0]))[0] == pytest.approx(
        0.8413447460685429 + math.exp(-0.5) / math.sqrt(2 * math.pi), rel=1e-15)


def test_gradient_matches_central_differences():
    theta = synth.mlp_init(918).astype(np.float64)
    rng = np.random.default_rng(3)
    theta += 0.05 * rng.standard_normal(theta.size)   # nonzero biases too
    X, t = synth.mlp_batch(16, seed=5)
    L, g = mlp.backward(theta, X, t)
    assert L == pytest.approx(mlp.loss(theta, X, t), rel=1e-15)
    idx = np.concatenate([rng.choice(mlp.n_params(), 60, replace=False),
                          [0, 767, 768, 895, 34047, 34048]])
    h = 1e-5
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (mlp.loss(theta + e, X, t) - mlp.loss(theta - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])


def test_vanishing_hidden_weights_give_the_output_bias():
    theta = np.zeros(mlp.n_params())
    theta[-1] = 0.7                                   # b4
    X, t = synth.mlp_batch(10, seed=1)
    y, _ = mlp.forward(theta, X)
    assert np.all(y == 0.7)
    L, g = mlp.backward(theta, X, t)
    assert L == pytest.approx(np.mean((0.7 - t.astype(np.float64)) ** 2))
    assert g[-1] == pytest.approx(2 * np.mean(0.7 - t.astype(np.float64)))
    # GELU(0) = 0: every activation is zero, so every weight gradient but b4's
    # and W4's (times zero activations) vanishes, and W4 gets nothing either
    assert np.all(g[:-1] == 0.0)


def test_adam_first_step_moves_by_lr_sign():
    theta = np.array([1.0, -2.0, 3.0])
    g = np.array([0.3, -1e-3, 5.0])
    new, m, v = mlp.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    # bias-corrected moments equal g and g^2 at k = 1: the step is lr * sign(g)
    assert np.allclose(theta - new, 0.01 * np.sign(g), rtol=1e-9)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
