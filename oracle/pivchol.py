"""Pivoted Cholesky preconditioner (oracle; test infrastructure only).

Sec. 5.2, "Preconditioning": k steps of the pivoted Cholesky decomposition of
the kernel matrix need only single rows (columns) of K and its diagonal, which
is constant for a stationary kernel; they give K~ ~= L_k L_k^T + s^2 I, and the
Woodbury identity (Eq. woodbury) turns that into the preconditioner
    P^{-1} w = s^-2 w - s^-4 L_k (I + s^-2 L_k^T L_k)^{-1} L_k^T w,
whose inner k x k system is solved directly (Cholesky here, in float64).

Readings where the paper is silent: the factorised matrix is a^2 K (noise
enters only through the Woodbury form); each step pivots on the largest
remaining diagonal entry, the lowest index winning ties (the first step is
always a tie because the diagonal is constant); the factorisation stops early
when the largest remaining diagonal entry is <= stop_rel * a^2.
"""

import numpy as np
import scipy.linalg

from .kernels import kfun, scaled_sqdist


def pivoted_cholesky(X, kind, lengthscale, outputscale, rank, stop_rel=1e-12):
    """Greedy pivoted Cholesky of a^2 K(X, X).

    Returns (L, pivots, residual_diag) with L of shape n x m (m <= rank),
    pivots of length m, and the remaining diagonal of a^2 K - L L^T.
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if rank < 0 or rank > n:
        raise ValueError("rank must lie in [0, n]")
    diag = np.full(n, float(outputscale))
    L = np.zeros((n, rank))
    piv = []
    for m in range(rank):
        p = int(np.argmax(diag))                    # first maximum = lowest index
        if not diag[p] > stop_rel * outputscale:
            break
        col = outputscale * kfun(kind, scaled_sqdist(X, X[p:p + 1], lengthscale))[:, 0]
        lm = (col - L[:, :m] @ L[p, :m]) / np.sqrt(diag[p])
        L[:, m] = lm
        diag = diag - lm * lm
        piv.append(p)
    m = len(piv)
    return L[:, :m].copy(), np.array(piv, dtype=np.int64), diag


class WoodburyPreconditioner:
    """P^{-1} w = s^-2 w - s^-4 L (I + s^-2 L^T L)^{-1} L^T w  (Eq. woodbury)."""

    def __init__(self, L, noise):
        if not noise > 0:
            raise ValueError("the Woodbury form needs a positive noise")
        self.L = np.asarray(L, dtype=np.float64)
        self.noise = float(noise)
        k = self.L.shape[1]
        C = np.eye(k) + (self.L.T @ self.L) / self.noise
        self.cf = scipy.linalg.cho_factor(C, lower=True) if k else None

    def __call__(self, W):
        W = np.asarray(W, dtype=np.float64)
        out = W / self.noise
        if self.cf is None:
            return out
        T = self.L.T @ W
        return out - (self.L @ scipy.linalg.cho_solve(self.cf, T)) / self.noise ** 2


def build(X, kind, lengthscale, outputscale, noise, rank, stop_rel=1e-12):
    """Pivoted Cholesky of a^2 K followed by the Woodbury preconditioner."""
    L, piv, diag = pivoted_cholesky(X, kind, lengthscale, outputscale, rank, stop_rel)
    return WoodburyPreconditioner(L, noise), L, piv, diag
