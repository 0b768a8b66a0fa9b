"""Pins for the FP64 reference MLP: central finite differences, Adam on a
quadratic, and a loss that falls on a learnable target."""
import numpy as np
import pytest

from oracle import mlp as M


@pytest.mark.parametrize("nout", [1, 2])
def test_backward_matches_finite_differences(nout):
    rng = np.random.default_rng(3)
    p = M.init_params(nout, seed=1) + 0.05 * rng.standard_normal(M.param_count(nout))
    x = rng.standard_normal((7, M.NIN))
    t = rng.standard_normal((7, nout))
    y, cache = M.forward(p, nout, x)
    _, dy = M.mse(y, t)
    g = M.backward(p, nout, x, cache, dy)
    idx = rng.choice(p.size, 120, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (M.loss(p + e, nout, x, t) - M.loss(p - e, nout, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_silu_derivative():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    assert np.allclose(fd, M.dsilu(z), atol=1e-8)


def test_adam_minimises_quadratic():
    p = np.array([3.0, -2.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for step in range(1, 2001):
        g = 2 * p
        p, m, v = M.adam(p, g, m, v, 0.05, 0.9, 0.999, 1e-8, step)
    assert np.abs(p).max() < 1e-2


def test_loss_decreases_on_learnable_target():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((256, M.NIN))
    t = np.tanh(x[:, :2] @ np.array([[1.0, -0.5], [0.3, 0.8]]))[:, :1]
    p = M.init_params(1, seed=2)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = M.loss(p, 1, x, t)
    for step in range(1, 301):
        y, c = M.forward(p, 1, x)
        _, dy = M.mse(y, t)
        p, m, v = M.adam(p, M.backward(p, 1, x, c, dy), m, v, 3e-3, 0.9, 0.999, 1e-8, step)
    assert M.loss(p, 1, x, t) < 0.1 * l0


# Kingma and Ba, Algorithm 1: with bias correction the first step moves every
# parameter by lr * g / (|g| + eps), whatever the scale of g, and a constant
# gradient keeps the corrected moments at g and g^2, so every step has that size.
def check_adam_first_step_and_constant_gradient(adam):
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    g = np.array([3.0, -0.02, 150.0, -7.5])
    p0 = np.array([0.5, -1.0, 2.0, 0.0])
    p1, m, v = adam(p0, g, np.zeros(4), np.zeros(4), lr, b1, b2, eps, 1)
    assert np.allclose(p1 - p0, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    p = p1
    for step in range(2, 6):
        q, m, v = adam(p, g, m, v, lr, b1, b2, eps, step)
        assert np.allclose(q - p, -lr * g / (np.abs(g) + eps), rtol=1e-9, atol=0)
        p = q


def test_adam_bias_corrected_steps():
    check_adam_first_step_and_constant_gradient(M.adam)


def test_planted_adam_without_bias_correction():
    def no_correction(p, g, m, v, lr, b1, b2, eps, step):
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        return p - lr * m / (np.sqrt(v) + eps), m, v

    def shifted_correction(p, g, m, v, lr, b1, b2, eps, step):
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        return p - lr * (m / (1 - b1 ** (step + 1))) / (np.sqrt(v / (1 - b2 ** (step + 1))) + eps), m, v

    for bad in (no_correction, shifted_correction):
        with pytest.raises(AssertionError):
            check_adam_first_step_and_constant_gradient(bad)
