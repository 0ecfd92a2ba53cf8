"""Dense direct solve (oracle; test infrastructure only).

Sec. 2.2: the exact GP computations need v = K~^{-1} y with
K~ = a^2 K + s^2 I, classically by a Cholesky factorisation at O(N^3) cost.
This materialises K~ in float64 and solves by LAPACK Cholesky; it is the
reference the iterative solvers are compared with on small problems.
`predictive_mean` forms the cached mean of Sec. 4.1 from the same solve.
"""

import numpy as np
import scipy.linalg

from .kernels import kernel_matrix


def ktilde(X, kind, lengthscale, outputscale, noise):
    """K~ = a^2 K(X, X) + s^2 I, float64."""
    K = kernel_matrix(X, X, kind, lengthscale, outputscale)
    K[np.diag_indices_from(K)] += noise
    return K


def solve(X, B, kind, lengthscale, outputscale, noise):
    """U* = K~^{-1} B by Cholesky (float64)."""
    A = ktilde(X, kind, lengthscale, outputscale, noise)
    B = np.asarray(B, dtype=np.float64)
    c, low = scipy.linalg.cho_factor(A, lower=True)
    return scipy.linalg.cho_solve((c, low), B)


def predictive_mean(X, y, Xs, kind, lengthscale, outputscale, noise):
    """mu(x*) = a^2 K(x*, X) v with the cache v = K~^{-1} y (the predictive-mean
    cache of Sec. 4.1; Rasmussen & Williams Eq. 2.25 with K~ = a^2 K + s^2 I).
    Returns (mu, v), float64."""
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    v = solve(X, y[:, None], kind, lengthscale, outputscale, noise)[:, 0]
    Ks = kernel_matrix(Xs, X, kind, lengthscale, outputscale)
    return Ks @ v, v
