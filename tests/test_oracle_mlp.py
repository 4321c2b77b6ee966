"""Pins of the learned-proposer oracle: finite differences, closed forms."""
import math

import numpy as np
import pytest

from oracle import mlp


def _theta(D, seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(mlp.n_params(D)) * scale


def test_gelu_closed_forms():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5, abs=1e-15)
    # GELU(z) - GELU(-z) = z  (since Phi(z) + Phi(-z) = 1)
    z = np.linspace(-4, 4, 17)
    np.testing.assert_allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-14)
    # derivative matches central differences
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), rtol=1e-8, atol=1e-9)


def test_bce_closed_forms():
    assert mlp.bce_with_logits(np.array([0.0]), np.array([1.0])) == pytest.approx(math.log(2.0))
    z = np.array([3.0, -2.0])
    y = np.array([1.0, 0.0])
    want = np.mean([math.log1p(math.exp(-3.0)), math.log1p(math.exp(-2.0))])
    assert mlp.bce_with_logits(z, y) == pytest.approx(want, rel=1e-14)
    # large logits stay finite
    assert np.isfinite(mlp.bce_with_logits(np.array([800.0, -800.0]), np.array([0.0, 1.0])))


def test_backward_matches_finite_differences():
    D = 12
    theta = _theta(D, 1)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((7, D))
    y = rng.integers(0, 2, size=7).astype(np.float64)
    g = mlp.backward(theta, X, y, D)
    h = 1e-6
    idx = rng.choice(theta.size, size=60, replace=False)
    for i in np.concatenate([idx, [theta.size - 1, theta.size - 2, 0]]):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        num = (mlp.bce_with_logits(mlp.forward(tp, X, D)[0], y)
               - mlp.bce_with_logits(mlp.forward(tm, X, D)[0], y)) / (2 * h)
        # central-difference roundoff is about eps * |L| / h = 1.5e-10
        assert g[i] == pytest.approx(num, rel=1e-6, abs=5e-10), i


def test_output_gradient_is_sigmoid_minus_label():
    """dL/db3 = mean(sigma(z) - y)."""
    D = 11
    theta = _theta(D, 3)
    X = np.random.default_rng(4).standard_normal((9, D))
    y = (np.arange(9) % 2).astype(np.float64)
    z, _ = mlp.forward(theta, X, D)
    g = mlp.backward(theta, X, y, D)
    assert g[-1] == pytest.approx(np.mean(1 / (1 + np.exp(-z)) - y), rel=1e-12)


def test_adam_first_step_is_lr_times_sign():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = mlp.adam(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(t1, theta - 0.01 * np.sign(g), rtol=1e-6)


def test_features_closed_forms():
    front = np.array([[10, 0], [0, 10], [6, 6]], np.int64)   # normalised: (1,0), (0,1), (.6,.6)
    cands = np.array([[0.5, 0.5], [1.0, 0.0]])
    hits = np.array([[0.5, 0.5]])
    misses = np.zeros((0, 2))
    f = mlp.features(front, cands, hits, misses)
    # w = (.5,.5): v = (.5, .5, .6) -> max .6 at (.6,.6); 2nd .5; fewer than 8 points -> smallest .5
    np.testing.assert_allclose(f[0, :3], [0.6, 0.1, 0.1], atol=1e-12)
    assert f[0, 3] == pytest.approx(math.hypot(0.4, 0.6))      # nearest other point
    assert f[0, 4] == pytest.approx(1 / 3)
    assert f[0, 5] == pytest.approx(0.0, abs=1e-7)              # same direction as the hit
    assert f[0, 6] == pytest.approx(math.pi / 2)                # no misses
    assert f[0, 7] == pytest.approx(0.0)
    # w = (1,0): argmax is (1,0), angle to the hit is pi/4, |w - 1/2| = 1/2
    np.testing.assert_allclose(f[1, [0, 5, 7]], [1.0, math.pi / 4, 0.5], atol=1e-12)
    assert mlp.features(np.zeros((0, 2), np.int64), cands, hits, misses)[:, :5].sum() == 0.0
