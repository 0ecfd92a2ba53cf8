"""Covariance functions, float64 (oracle; test infrastructure only).

Paper: App. C (Experimental details) gives the RBF, Matern-1/2 and rational
quadratic forms with distance d and lengthscale l; Table 1's caption uses ARD,
i.e. one lengthscale per input dimension.  The paper names Matern-3/2 and
Matern-5/2 (Tables A.2-A.5) but prints no formula for them; the textbook
half-integer closed forms of Rasmussen & Williams (cited in Sec. 2.2) are used.

Scaled squared distance:  r^2(x, x') = sum_m ((x_m - x'_m) / l_m)^2.
"""

import numpy as np

RBF = 0
MATERN52 = 1
MATERN12 = 2
MATERN32 = 3

KIND_NAMES = {RBF: "rbf", MATERN52: "matern52", MATERN12: "matern12", MATERN32: "matern32"}


def lengthscale_vector(lengthscale, d):
    """Broadcast a scalar (isotropic) or length-d (ARD) lengthscale to d values."""
    ls = np.asarray(lengthscale, dtype=np.float64).reshape(-1)
    if ls.size == 1:
        ls = np.full(d, ls[0])
    if ls.size != d:
        raise ValueError("lengthscale must have 1 or d entries")
    if np.any(~np.isfinite(ls)) or np.any(ls <= 0):
        raise ValueError("lengthscales must be finite and positive")
    return ls


def scaled_sqdist(X1, X2, lengthscale):
    """r^2 between every row of X1 (n1 x d) and X2 (n2 x d), by direct differences."""
    X1 = np.asarray(X1, dtype=np.float64)
    X2 = np.asarray(X2, dtype=np.float64)
    ls = lengthscale_vector(lengthscale, X1.shape[1])
    A = X1 / ls
    B = X2 / ls
    diff = A[:, None, :] - B[None, :, :]
    return np.einsum("ijk,ijk->ij", diff, diff)


def kfun(kind, r2):
    """Unit-outputscale stationary kernel value as a function of r^2 (r^2 >= 0)."""
    r2 = np.maximum(np.asarray(r2, dtype=np.float64), 0.0)
    if kind == RBF:
        return np.exp(-0.5 * r2)
    r = np.sqrt(r2)
    if kind == MATERN12:
        return np.exp(-r)
    if kind == MATERN32:
        t = np.sqrt(3.0) * r
        return (1.0 + t) * np.exp(-t)
    if kind == MATERN52:
        t = np.sqrt(5.0) * r
        return (1.0 + t + t * t / 3.0) * np.exp(-t)
    raise ValueError(f"unknown kernel kind {kind}")


def kernel_matrix(X1, X2, kind, lengthscale, outputscale):
    """a^2 K(X1, X2) materialised (small inputs only)."""
    return outputscale * kfun(kind, scaled_sqdist(X1, X2, lengthscale))
