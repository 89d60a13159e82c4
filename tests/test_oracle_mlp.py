"""Pins of the refinement-classifier oracle: GELU against its defining
integral, the gradient against central finite differences, the loss at
closed-form points and Adam's first step (whose size is lr in every
coordinate with a nonzero gradient)."""
import math

import numpy as np
from scipy import integrate

from oracle import mlp


def test_gelu_matches_the_normal_cdf_integral():
    for z in (-3.0, -0.7, 0.0, 0.4, 2.5):
        phi, _ = integrate.quad(lambda t: math.exp(-0.5 * t * t) / math.sqrt(2 * math.pi), -np.inf, z)
        assert abs(mlp.gelu(np.array([z]))[0] - z * phi) < 1e-14


def test_gelu_prime_by_differences():
    z = np.linspace(-4, 4, 17)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_prime(z)).max() < 1e-8


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init(1) + 0.05 * rng.standard_normal(mlp.N_PARAMS)
    X = rng.standard_normal((7, 64))
    y = (rng.random(7) < 0.5).astype(float)
    g = mlp.backward(theta, X, y)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [mlp.N_PARAMS - 1, 4096 + 3, 2 * 4096 + 64 + 5]])  # b3, b1, b2 entries
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (mlp.loss(theta + e, X, y) - mlp.loss(theta - e, X, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_loss_closed_forms():
    theta = np.zeros(mlp.N_PARAMS)
    X = np.ones((3, 64))
    # zero network: logit 0, loss log 2 for any labels
    assert abs(mlp.loss(theta, X, np.array([0.0, 1.0, 1.0])) - math.log(2)) < 1e-15
    theta[-1] = 2.0  # bias only: logit 2
    assert abs(mlp.loss(theta, X, np.array([1.0, 1.0, 1.0])) - math.log1p(math.exp(-2))) < 1e-15


def test_adam_first_step_has_size_lr():
    theta = np.zeros(5)
    grad = np.array([3.0, -0.2, 0.0, 1e-3, -7.0])
    new, m, v = mlp.adam_step(theta, grad, np.zeros(5), np.zeros(5), 1, lr=0.01, eps=1e-300)
    expect = -0.01 * np.sign(grad)
    assert np.allclose(new, expect, rtol=0, atol=1e-15)
