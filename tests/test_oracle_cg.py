"""Pins for oracle.cg (Alg. 1 and Alg. 2, batched over columns) and oracle.direct."""
import math

import numpy as np
import pytest

from oracle import cg, direct, kernels, kmvm, pivchol


def small_problem(n=48, d=2, R=3, noise=0.05, ls=0.8, kind=kernels.RBF, seed=0):
    g = np.random.default_rng(seed)
    X = g.standard_normal((n, d))
    B = g.standard_normal((n, R))
    A = direct.ktilde(X, kind, ls, 1.0, noise)
    return X, B, A


def test_direct_solve_residual_and_lu():
    X, B, A = small_problem()
    U = direct.solve(X, B, kernels.RBF, 0.8, 1.0, 0.05)
    assert np.linalg.norm(A @ U - B) / np.linalg.norm(B) <= 1e-12
    np.testing.assert_allclose(U, np.linalg.solve(A, B), rtol=1e-9, atol=1e-9)


def test_lse_dot_equals_inner_product():
    g = np.random.default_rng(1)
    w, z = g.standard_normal(200), g.standard_normal(200)
    z = np.where(w * z < 0, -z, z)           # make the product positive
    z[::7] = 0.0                             # zero terms must contribute nothing
    val, ok = cg.lse_dot(w, z)
    want = math.fsum((w * z).tolist())
    assert ok and abs(math.exp(val) - want) <= 1e-14 * want
    # mixed signs with a positive total
    w2, z2 = g.standard_normal(300), g.standard_normal(300)
    tot = math.fsum((w2 * z2).tolist())
    if tot < 0:
        z2 = -z2
        tot = -tot
    val2, ok2 = cg.lse_dot(w2, z2)
    assert ok2 and abs(math.exp(val2) - tot) <= 1e-12 * abs(tot) * 300
    # very large and very small magnitudes beyond float64 products stay finite in log scale
    v3, ok3 = cg.lse_dot(np.full(4, 1e200), np.full(4, 1e200))
    assert ok3 and abs(v3 - (400 * math.log(10) + math.log(4))) < 1e-10
    assert cg.lse_dot(w2, -z2)[1] is False    # negative inner product: breakdown
    assert cg.lse_dot(np.zeros(5), np.ones(5))[1] is False


@pytest.mark.parametrize("algo", ["plain", "enhanced"])
@pytest.mark.parametrize("use_pc", [False, True])
def test_finite_termination_matches_direct(algo, use_pc):
    X, B, A = small_problem()
    n = A.shape[0]
    P = None
    if use_pc:
        P = pivchol.build(X, kernels.RBF, 0.8, 1.0, 0.05, rank=6)[0]
    U, st = cg.solve(lambda V: A @ V, B, tol=1e-10, max_iter=n, algo=algo, precond=P)
    U_ref = np.linalg.solve(A, B)
    assert np.all(st["converged"])
    assert np.all(st["iters"] <= n)
    np.testing.assert_allclose(U, U_ref, rtol=0, atol=1e-8 * np.abs(U_ref).max())


def test_reorthogonalisation_has_no_effect_in_double():
    # Sec. 7: apart from re-orthogonalisation the modifications have no effect
    # in single or double precision.  In float64, before orthogonality is lost,
    # all three variants produce the same iterates; later, re-orthogonalisation
    # can only help (the plain recurrences drift once Ritz values converge).
    X, B, A = small_problem(n=120, noise=0.5, seed=3)
    f = lambda V: A @ V
    U1, s1 = cg.solve(f, B, tol=1e-30, max_iter=10, algo="enhanced", reorth=True)
    U2, s2 = cg.solve(f, B, tol=1e-30, max_iter=10, algo="enhanced", reorth=False)
    U3, s3 = cg.solve(f, B, tol=1e-30, max_iter=10, algo="plain")
    assert np.all(s1["iters"] == 10)
    np.testing.assert_allclose(U1, U2, rtol=0, atol=1e-9 * np.abs(U2).max())
    np.testing.assert_allclose(U2, U3, rtol=0, atol=1e-10 * np.abs(U3).max())
    ref = np.linalg.solve(A, B)
    err = lambda U: np.linalg.norm(U - ref) / np.linalg.norm(ref)
    Ur, _ = cg.solve(f, B, tol=1e-30, max_iter=20, algo="enhanced", reorth=True)
    Up, _ = cg.solve(f, B, tol=1e-30, max_iter=20, algo="plain")
    assert err(Ur) <= err(Up)


def test_exact_preconditioner_one_iteration():
    X, B, A = small_problem()
    Ainv = np.linalg.inv(A)
    U, st = cg.solve(lambda V: A @ V, B, tol=1e-10, max_iter=10, precond=lambda W: Ainv @ W)
    assert np.all(st["iters"] == 1)
    np.testing.assert_allclose(U, np.linalg.solve(A, B), rtol=1e-8, atol=1e-10)


def test_residuals_orthogonal_in_preconditioner_inner_product():
    X, B, A = small_problem(n=80, noise=0.02, seed=5)
    P = pivchol.build(X, kernels.RBF, 0.8, 1.0, 0.02, rank=5)[0]
    res = []

    def mvm(V):
        return A @ V

    # record r_k through a wrapping preconditioner (it is applied once per residual)
    def rec(W):
        res.append(W[:, 0].copy())
        return P(W)

    cg.solve(mvm, B[:, :1], tol=1e-30, max_iter=12, precond=rec, algo="enhanced")
    Rm = np.array(res)
    Z = np.array([P(r[:, None])[:, 0] for r in Rm])
    G = Rm @ Z.T
    nrm = np.sqrt(np.abs(np.diag(G)))
    off = G / np.outer(nrm, nrm) - np.eye(len(Rm))
    assert np.abs(off).max() <= 1e-10


def test_euclidean_reorth_differs_under_preconditioning_only():
    X, B, A = small_problem(n=80, noise=0.02, seed=6)
    f = lambda V: A @ V
    U_p, _ = cg.solve(f, B, tol=1e-30, max_iter=15, reorth_inner="P")
    U_e, _ = cg.solve(f, B, tol=1e-30, max_iter=15, reorth_inner="euclid")
    np.testing.assert_allclose(U_p, U_e, rtol=0, atol=1e-9 * np.abs(U_p).max())
    P = pivchol.build(X, kernels.RBF, 0.8, 1.0, 0.02, rank=5)[0]
    U_p2, _ = cg.solve(f, B, tol=1e-30, max_iter=40, precond=P, reorth_inner="P")
    U_e2, _ = cg.solve(f, B, tol=1e-30, max_iter=40, precond=P, reorth_inner="euclid")
    ref = np.linalg.solve(A, B)
    err_p = np.linalg.norm(U_p2 - ref) / np.linalg.norm(ref)
    err_e = np.linalg.norm(U_e2 - ref) / np.linalg.norm(ref)
    # the literal Euclidean projection removes true residual components and stalls
    assert err_p < 1e-10 and err_e > 0.1


def test_zero_column_and_breakdown_and_freezing():
    X, B, A = small_problem()
    B = B.copy(); B[:, 1] = 0.0
    U, st = cg.solve(lambda V: A @ V, B, tol=1e-8, max_iter=100)
    assert np.all(U[:, 1] == 0) and st["converged"][1] and st["iters"][1] == 0
    # an indefinite operator breaks the logsumexp step size
    U, st = cg.solve(lambda V: -(A @ V), B[:, :1] + 1.0, tol=1e-8, max_iter=20)
    assert st["breakdown"][0] and not st["converged"][0]
    # per-column freezing: a loose and a tight column stop at different counts
    B2 = np.stack([B[:, 0], B[:, 0]], 1)
    U, st = cg.solve(lambda V: A @ V, B2, tol=1e-3, max_iter=200, min_iter=2)
    assert st["converged"].all() and st["iters"][0] == st["iters"][1]
    assert np.all(st["rel_res"] <= 1e-3)


def test_min_iter_and_loose_tolerance():
    X, B, A = small_problem()
    U, st = cg.solve(lambda V: A @ V, B, tol=1.0, max_iter=100, min_iter=10)
    assert np.all(st["iters"] == 10) and st["converged"].all()
    U, st = cg.solve(lambda V: A @ V, B, tol=1.0, max_iter=100, min_iter=0)
    assert np.all(st["iters"] == 0) and np.all(U == 0)


def test_warm_start_from_solution():
    X, B, A = small_problem()
    U_ref = np.linalg.solve(A, B)
    U, st = cg.solve(lambda V: A @ V, B, tol=1e-8, max_iter=50, x0=U_ref)
    assert np.all(st["iters"] == 0)
    np.testing.assert_allclose(U, U_ref)


def test_true_relative_residual_pins():
    """oracle.cg.true_relative_residual, pinned by closed forms.

    * the exact (LU) solution of a well-conditioned system: <= 1e-12;
    * u = 0: exactly 1 in every nonzero column, whatever its scale;
    * a zero right-hand side solved by 0: 0 (not a division by zero);
    * K~ = c I with u_c = t_c b_c: the residual is |1 - c t_c| column by
      column, independently of each column's norm (per-column normalisation,
      no transposed axis, no shared scale).
    """
    X, B, A = small_problem(n=40, R=3)
    mvm = lambda V: A @ V
    U = np.linalg.solve(A, B)
    assert np.all(cg.true_relative_residual(mvm, B, U) <= 1e-12)
    got = cg.true_relative_residual(mvm, B * np.array([1.0, 1e3, 1e-3]), np.zeros_like(B))
    np.testing.assert_array_equal(got, np.ones(3))
    B0 = B.copy()
    B0[:, 1] = 0.0
    U0 = np.linalg.solve(A, B0)
    got = cg.true_relative_residual(mvm, B0, U0)
    assert got[1] == 0.0 and np.all(got[[0, 2]] <= 1e-12)
    c = 2.5
    t = np.array([0.4, 0.3, 0.5])                    # c t = 1, 0.75, 1.25
    Bs = B * np.array([1.0, 1e4, 1e-4])
    got = cg.true_relative_residual(lambda V: c * V, Bs, Bs * t)
    np.testing.assert_allclose(got, np.abs(1.0 - c * t), rtol=1e-14, atol=1e-15)
    # a single column given as a vector
    got = cg.true_relative_residual(lambda V: c * V, Bs[:, 2], Bs[:, 2] * t[2])
    np.testing.assert_allclose(got, [0.25], rtol=1e-14)


@pytest.mark.parametrize("algo", ["plain", "enhanced"])
@pytest.mark.parametrize("use_pc", [False, True])
def test_per_column_iteration_caps_equal_separate_runs(algo, use_pc):
    """Per-column caps (matched-iteration runs) give each column exactly what a
    run of that column alone with that scalar cap gives."""
    X, B, A = small_problem(n=60, R=4, seed=3)
    P = pivchol.build(X, kernels.RBF, 0.8, 1.0, 0.05, rank=5)[0] if use_pc else None
    # the same matrix-vector call per column in both runs, so that the block
    # and the single-column runs differ only by the summation order of the
    # column-wise reductions (last-bit differences); an off-by-one cap or a
    # column that saw another column's step would differ at O(1)
    mvm = lambda V: np.column_stack([A @ V[:, j] for j in range(V.shape[1])])
    pre = None if P is None else (lambda W: np.column_stack([P(W[:, [j]])[:, 0]
                                                              for j in range(W.shape[1])]))
    caps = [3, 0, 7, 5]       # short of convergence: no rounding-noise trajectories
    U, st = cg.solve(mvm, B, tol=0.0, max_iter=caps, algo=algo, precond=pre)
    np.testing.assert_array_equal(st["iters"], caps)
    assert np.all(U[:, 1] == 0.0)                    # cap 0: the initial guess
    for c, m in enumerate(caps):
        Uc, sc = cg.solve(mvm, B[:, c:c + 1], tol=0.0, max_iter=m, algo=algo, precond=pre)
        assert sc["iters"][0] == m
        np.testing.assert_allclose(U[:, c], Uc[:, 0], rtol=0,
                                   atol=1e-9 * max(1.0, np.abs(Uc).max()))
    with pytest.raises(ValueError):
        cg.solve(lambda V: A @ V, B, tol=0.0, max_iter=[1, -1, 2, 3])
