"""Pins for oracle.kernels: closed forms against independent library definitions."""
import math

import numpy as np
import pytest
import scipy.special
import scipy.stats

from oracle import kernels


def matern_general(nu, r):
    """Textbook Matern via the modified Bessel function (Rasmussen & Williams eq. 4.14)."""
    r = np.asarray(r, dtype=np.float64)
    t = np.sqrt(2 * nu) * r
    out = np.ones_like(t)
    nz = t > 0
    out[nz] = (2 ** (1 - nu) / scipy.special.gamma(nu)) * t[nz] ** nu * scipy.special.kv(nu, t[nz])
    return out


R = np.array([0.0, 1e-3, 0.25, 0.5, 1.0, 1.7, 3.0, 6.5])


@pytest.mark.parametrize("kind,nu", [(kernels.MATERN12, 0.5), (kernels.MATERN32, 1.5), (kernels.MATERN52, 2.5)])
def test_matern_closed_forms_match_bessel_definition(kind, nu):
    np.testing.assert_allclose(kernels.kfun(kind, R ** 2), matern_general(nu, R), rtol=1e-12, atol=1e-15)


def test_rbf_matches_gaussian_density():
    # exp(-r^2/2) = sqrt(2 pi) * phi(r), phi the standard normal density
    np.testing.assert_allclose(kernels.kfun(kernels.RBF, R ** 2),
                               math.sqrt(2 * math.pi) * scipy.stats.norm.pdf(R), rtol=1e-13)


def test_unit_diagonal_and_symmetry():
    g = np.random.default_rng(0)
    X = g.standard_normal((30, 4))
    for kind in (kernels.RBF, kernels.MATERN52, kernels.MATERN12, kernels.MATERN32):
        K = kernels.kernel_matrix(X, X, kind, [0.7, 1.1, 2.0, 0.5], 1.0)
        np.testing.assert_allclose(np.diag(K), 1.0, rtol=0, atol=0)
        np.testing.assert_array_equal(K, K.T)


def test_ard_distance_against_loop():
    g = np.random.default_rng(1)
    X1, X2 = g.standard_normal((5, 3)), g.standard_normal((4, 3))
    ls = [0.5, 2.0, 1.3]
    D = kernels.scaled_sqdist(X1, X2, ls)
    for i in range(5):
        for j in range(4):
            want = math.fsum(((X1[i, m] - X2[j, m]) / ls[m]) ** 2 for m in range(3))
            assert abs(D[i, j] - want) <= 1e-14 * max(1.0, want)


def test_bad_lengthscales_rejected():
    with pytest.raises(ValueError):
        kernels.lengthscale_vector([1.0, -1.0], 2)
    with pytest.raises(ValueError):
        kernels.lengthscale_vector([1.0, 2.0, 3.0], 2)
