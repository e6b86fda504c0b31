"""Pins of the FP64 surrogate reference: the exact GELU at known points, the gradient
against central finite differences of the loss, and the closed-form first Adam step."""
import math

import numpy as np
import pytest

import workloads
from oracle import mlp


def test_gelu_values():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # GELU(1) = Phi(1) (standard normal CDF at 1)
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(np.array([-1.0]))[0] + (1 - 0.8413447460685429)) < 1e-15
    assert abs(mlp.gelu(np.array([10.0]))[0] - 10.0) < 1e-15
    assert abs(mlp.gelu(np.array([-10.0]))[0]) < 1e-20
    z = np.linspace(-4, 4, 41)
    fd = (mlp.gelu(z + 1e-6) - mlp.gelu(z - 1e-6)) / 2e-6
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-8)
    assert mlp.gelu_grad(np.array([0.0]))[0] == 0.5


def test_gradient_matches_finite_differences():
    p = workloads.mlp_params(seed=1)
    X, T = workloads.mlp_batch(16, seed=2)
    L, g = mlp.loss_grad(p, X, T)
    assert abs(L - mlp.loss(p, X, T)) < 1e-15
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(np.arange(0, 640), 8, replace=False),   # W1
                          rng.choice(np.arange(640, 768), 4, replace=False),  # b1
                          rng.choice(np.arange(768, 17152), 12, replace=False),  # W2
                          rng.choice(np.arange(17152, 17280), 4, replace=False),  # b2
                          rng.choice(np.arange(17280, 17664), 6, replace=False),  # W3
                          np.arange(17664, 17667)])  # b3
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, T) - mlp.loss(p - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(g[i])), i


def test_first_adam_step_moves_by_lr_times_sign():
    """With zero moments, bias correction makes the first Adam update -lr * g/(|g| + eps)."""
    rng = np.random.default_rng(4)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    q, m, v = mlp.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-2, eps=1e-12)
    assert np.allclose(q, p - 1e-2 * np.sign(g), atol=1e-12)
    assert mlp.NPARAMS == 17667
