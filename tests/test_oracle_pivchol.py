"""Pins for oracle.pivchol (pivoted Cholesky + Woodbury preconditioner)."""
import numpy as np
import scipy.linalg.lapack

from oracle import kernels, pivchol


def points(n=40, d=2, seed=0):
    return np.random.default_rng(seed).uniform(-3, 3, size=(n, d))


def test_full_rank_reproduces_kernel_matrix():
    X = points()
    a2 = 1.7
    L, piv, diag = pivchol.pivoted_cholesky(X, kernels.RBF, 0.4, a2, rank=40, stop_rel=0.0)
    K = kernels.kernel_matrix(X, X, kernels.RBF, 0.4, a2)
    assert L.shape == (40, 40)
    np.testing.assert_allclose(L @ L.T, K, rtol=0, atol=1e-10 * a2)
    assert sorted(piv.tolist()) == list(range(40))


def test_pivots_match_lapack_dpstrf():
    X = points(n=30, seed=1)
    K = kernels.kernel_matrix(X, X, kernels.MATERN52, 0.7, 1.0)
    c, piv_lapack, rank, info = scipy.linalg.lapack.dpstrf(K, tol=-1.0, lower=1)
    k = 12
    L, piv, _ = pivchol.pivoted_cholesky(X, kernels.MATERN52, 0.7, 1.0, rank=k)
    assert piv.tolist() == (piv_lapack[:k] - 1).tolist()
    # LAPACK's factor, permuted back, has the same first k columns
    Lp = np.tril(c)[:, :k]
    Lfull = np.zeros_like(Lp)
    Lfull[piv_lapack - 1] = Lp
    np.testing.assert_allclose(L, Lfull, rtol=0, atol=1e-10)


def test_trace_residual_nonincreasing_and_consistent():
    X = points(n=60, seed=2)
    K = kernels.kernel_matrix(X, X, kernels.RBF, 1.0, 1.0)
    prev = np.inf
    for k in (0, 1, 3, 8, 20):
        L, piv, diag = pivchol.pivoted_cholesky(X, kernels.RBF, 1.0, 1.0, rank=k)
        tr = np.trace(K - L @ L.T)
        assert abs(tr - diag.sum()) <= 1e-9
        assert tr <= prev + 1e-12
        prev = tr


def test_early_stop_on_tiny_residual_diagonal():
    X = np.repeat(points(n=5, seed=3), 4, axis=0)   # 5 distinct points, each 4 times
    L, piv, diag = pivchol.pivoted_cholesky(X, kernels.RBF, 0.5, 1.0, rank=15)
    assert L.shape[1] == 5


def test_woodbury_equals_dense_inverse():
    X = points(n=50, seed=4)
    s2 = 0.03
    P, L, piv, _ = pivchol.build(X, kernels.RBF, 0.6, 1.0, s2, rank=10)
    W = np.random.default_rng(5).standard_normal((50, 3))
    want = np.linalg.solve(L @ L.T + s2 * np.eye(50), W)
    np.testing.assert_allclose(P(W), want, rtol=1e-9, atol=1e-9 * np.abs(want).max())
    P0 = pivchol.WoodburyPreconditioner(np.zeros((50, 0)), s2)
    np.testing.assert_allclose(P0(W), W / s2)
