"""Pins of the network oracle: finite differences, closed forms (no GPU)."""
import numpy as np
import pytest
from scipy.stats import norm

from oracle import mlp


def test_param_count():
    assert mlp.n_params() == 157460


def test_gelu_is_z_times_normal_cdf():
    z = np.linspace(-6, 6, 101)
    assert np.abs(mlp.gelu(z) - z * norm.cdf(z)).max() < 1e-15
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.abs(mlp.gelu_grad(z) - fd).max() < 1e-8


def test_gradient_vs_central_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(1) * 0.7
    x = rng.normal(size=(5, 80))
    t = rng.normal(size=(5, 20))
    _, g = mlp.loss_and_grad(p, x, t)
    idx = rng.choice(p.size, 60, replace=False)
    idx = np.concatenate([idx, [0, p.size - 1, 256 * 80 + 3, p.size - 25]])
    h = 1e-5
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, x, t)[0] - mlp.loss_and_grad(p - e, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_closed_form():
    # first step with bias correction: p - lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3])
    opt = mlp.Adam(3)
    p1 = opt.step(np.zeros(3), g, 0.01)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_later_steps_closed_form():
    # a constant gradient g: m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so with the bias
    # correction every step moves by lr g / (|g| + eps); a wrong correction exponent at t >= 2
    # (or none) changes steps 2 and 3
    g = np.array([0.3, -2.0, 1e-3, 7.5])
    opt = mlp.Adam(4)
    p = np.zeros(4)
    for t in range(1, 4):
        p = opt.step(p, g, 0.01)
        assert np.allclose(p, -0.01 * t * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0), t
    # a gradient that flips sign at t = 2: m_2 = (b1 (1 - b1) - (1 - b1)) g, v_2 = (1 - b2^2) g^2
    opt = mlp.Adam(4)
    p1 = opt.step(np.zeros(4), g, 0.01)
    p2 = opt.step(p1, -g, 0.01)
    mh = (0.9 * 0.1 - 0.1) / (1 - 0.9 ** 2)
    assert np.allclose(p2 - p1, -0.01 * mh * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0)


def test_adam_is_invariant_to_gradient_scale():
    rng = np.random.default_rng(4)
    gs = [rng.normal(size=50) for _ in range(4)]
    a, b = mlp.Adam(50, eps=0.0), mlp.Adam(50, eps=0.0)
    pa = pb = np.zeros(50)
    for g in gs:
        pa = a.step(pa, g, 1e-2)
        pb = b.step(pb, 1000.0 * g, 1e-2)
    assert np.allclose(pa, pb, rtol=1e-12, atol=1e-15)


def test_loss_decreases_on_a_linear_target():
    rng = np.random.default_rng(3)
    p = mlp.init_params(2)
    A = rng.normal(size=(80, 20)) * 0.1
    opt = mlp.Adam(p.size)
    losses = []
    for it in range(150):
        x = rng.normal(size=(64, 80))
        loss, g = mlp.loss_and_grad(p, x, x @ A)
        losses.append(loss)
        p = opt.step(p, g, 1e-3)
    assert np.mean(losses[-10:]) < 0.25 * np.mean(losses[:5])


def test_features_layout_and_sign():
    E, d, Np = 6, 2, 10
    w = np.arange(E * d * Np, dtype=float).reshape(E, d, Np)
    nbr = np.array([[1, 2, 3], [0, 4, 5], [3, 0, 1], [2, 5, 0], [5, 1, 2], [4, 3, 1]])
    sign = np.array([1, -1, 1, -1, 1, -1.0])
    x = mlp.features(w, nbr, sign, 2.0, np.array([1, 4]))
    assert x.shape == (2, 80)
    assert np.array_equal(x[0, :20], -w[1].ravel() / 2) and np.array_equal(x[0, 20:40], -w[0].ravel() / 2)
    assert np.array_equal(x[1, 60:], w[2].ravel() / 2)
