"""Pins of the float64 selector-network reference (oracle/mlp.py).

The chain-rule gradient is checked against central finite differences of the
loss, the GELU derivative against finite differences of GELU, Adam against a
hand-computed first step and against convergence on a quadratic, and the
features against their definitions on constructed particle sets.
"""
import math

import numpy as np
import pytest

from oracle import mlp as M


def test_parameter_count():
    assert M.N_PARAMS == 4929


def test_gelu_derivative_finite_difference():
    z = np.linspace(-6, 6, 97)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - M.gelu_grad(z))) < 1e-8
    # limits: gelu(z) ~ z for large z, ~ 0 for very negative z
    assert abs(M.gelu(10.0) - 10.0) < 1e-12 and abs(M.gelu(-10.0)) < 1e-12
    # exact at 0 and symmetric part: gelu(z) - gelu(-z) = z
    assert np.allclose(M.gelu(z) - M.gelu(-z), z, atol=1e-15)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    theta = M.init_params(3)
    X = rng.normal(size=(17, M.N_IN)); T = rng.normal(size=17)
    g = M.gradient(theta, X, T)
    idx = rng.choice(M.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [M.N_PARAMS - 1, 0, 640, 640 + 64, 640 + 64 + 4096]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta); e[i] = h
        fd = (M.loss(theta + e, X, T) - M.loss(theta - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_adam_first_step_and_convergence():
    th = np.array([1.0, -2.0]); m = np.zeros(2); v = np.zeros(2)
    grad = np.array([0.5, -4.0])
    th2, m2, v2 = M.adam_step(th, m, v, grad, 1, 0.1)
    # first step moves every coordinate by lr * sign(grad) (bias-corrected)
    assert np.allclose(th2, th - 0.1 * np.sign(grad), atol=1e-7)
    # minimise (theta - 3)^2
    th = np.array([0.0]); m = np.zeros(1); v = np.zeros(1)
    for k in range(1, 2001):
        th, m, v = M.adam_step(th, m, v, 2 * (th - 3.0), k, 0.05)
    assert abs(th[0] - 3.0) < 1e-3


def test_training_reduces_loss_on_smooth_target():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(256, M.N_IN)); T = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]
    th = M.init_params(0); m = np.zeros_like(th); v = np.zeros_like(th)
    l0 = M.loss(th, X, T)
    for k in range(1, 301):
        th, m, v = M.adam_step(th, m, v, M.gradient(th, X, T), k, 3e-3)
    assert M.loss(th, X, T) < 0.1 * l0


def test_features_definitions():
    # 4 x 4 lattice in [0, 4]^2 with alternating circulations
    c = np.arange(4) + 0.5
    yy, xx = np.meshgrid(c, c, indexing="ij")
    x = xx.ravel(); y = yy.ravel(); g = np.where((np.arange(16) % 2) == 0, 1.0, -3.0)
    f = M.features(x, y, g, sigma=0.25, p=7, levels=2, side=4.0)
    assert f[0] == 7 and f[1] == 2
    assert f[2] == pytest.approx(4.0) and f[3] == pytest.approx(0.0)
    assert f[4] == pytest.approx(math.log2((4.0 / 4) / 0.25))
    assert f[5] == pytest.approx(math.log2(0.25 / 1.0))
    assert f[6] == pytest.approx(-1.0 / math.sqrt(5.0))
    assert f[7] == pytest.approx(math.log10(32.0 / 3.0))
    assert f[8] == pytest.approx(math.sqrt(1.25) / 4.0) and f[9] == pytest.approx(math.sqrt(1.25) / 4.0)


def test_near_distance_feature():
    """f4 with the distance cut-off: the larger of the leaf side and the near
    radius clamped to four leaf sides (6 sigma for the automatic radius)."""
    c = np.arange(4) + 0.5
    yy, xx = np.meshgrid(c, c, indexing="ij")
    x = xx.ravel(); y = yy.ravel(); g = np.ones(16)
    # leaf side 1.0 (L = 2 of side 4), sigma 0.25
    f = lambda r: M.features(x, y, g, sigma=0.25, p=7, levels=2, side=4.0, radius=r)[4]
    assert f(0.0) == pytest.approx(math.log2(1.0 / 0.25))      # paper split: w_L
    assert f(0.5) == pytest.approx(math.log2(1.0 / 0.25))      # a < w_L
    assert f(2.5) == pytest.approx(math.log2(2.5 / 0.25))      # w_L < a < 4 w_L
    assert f(9.0) == pytest.approx(math.log2(4.0 / 0.25))      # clamped to 4 w_L
    assert f(-1.0) == pytest.approx(math.log2(1.5 / 0.25))     # automatic: 6 sigma
    # every other feature ignores the radius
    a = M.features(x, y, g, sigma=0.25, p=7, levels=2, side=4.0, radius=2.5)
    b = M.features(x, y, g, sigma=0.25, p=7, levels=2, side=4.0)
    assert np.array_equal(np.delete(a, 4), np.delete(b, 4))
