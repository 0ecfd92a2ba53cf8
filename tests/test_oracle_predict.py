"""Pins for oracle.direct.predictive_mean (Sec. 4.1 predictive-mean cache)."""
import math

import numpy as np
import pytest

from oracle import direct, kernels


@pytest.mark.parametrize("kind", [kernels.RBF, kernels.MATERN52])
def test_single_training_point_closed_form(kind):
    x = np.array([[0.3, -1.0]])
    y = np.array([2.5])
    Xs = np.array([[0.0, 0.0], [0.3, -1.0], [2.0, 1.0]])
    a2, s2, ls = 1.7, 0.2, [0.8, 1.3]
    mu, v = direct.predictive_mean(x, y, Xs, kind, ls, a2, s2)
    assert v[0] == pytest.approx(y[0] / (a2 + s2), rel=1e-14)
    for i in range(3):
        r2 = sum(((Xs[i, m] - x[0, m]) / ls[m]) ** 2 for m in range(2))
        want = a2 * float(kernels.kfun(kind, r2)) * y[0] / (a2 + s2)
        assert mu[i] == pytest.approx(want, rel=1e-13)


def test_training_points_identity_and_far_field():
    g = np.random.default_rng(1)
    X = g.standard_normal((40, 3))
    y = np.sin(X).sum(1)
    a2, s2 = 1.3, 0.05
    mu, v = direct.predictive_mean(X, y, X, kernels.RBF, [0.9], a2, s2)
    np.testing.assert_allclose(mu, y - s2 * v, rtol=1e-10, atol=1e-10)   # a^2 K v = y - s^2 v
    far = X + 1e3
    mu_far, _ = direct.predictive_mean(X, y, far, kernels.RBF, [0.9], a2, s2)
    assert np.all(np.abs(mu_far) < 1e-300 + 1e-12)                       # prior mean 0


def test_interpolates_at_vanishing_noise():
    x = np.linspace(-3, 3, 15)[:, None]
    y = np.cos(x[:, 0])
    mu, _ = direct.predictive_mean(x, y, x, kernels.MATERN52, [0.5], 1.0, 1e-10)
    np.testing.assert_allclose(mu, y, atol=1e-6)
