"""Pins for oracle.train: Eq. (loss)/(gradient), Eq. (approx_loss)/(approx),
the App. C priors and Adam, and the SplitMix64 probe generator."""
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from oracle import kernels, train
from golden_values import paper_values

KINDS = [kernels.RBF, kernels.MATERN52, kernels.MATERN32, kernels.MATERN12]


def _problem(seed, n=12, d=3):
    g = np.random.default_rng(seed)
    X = g.standard_normal((n, d))
    y = np.sin(X).sum(1) + 0.1 * g.standard_normal(n)
    return X, y


def _theta(d, ard):
    ls = np.array([0.9, 1.4, 0.7][:d]) if ard else np.array([1.1])
    return ls, 1.3, 0.2


def _fd(f, x, h):
    return (f(x + h) - f(x - h)) / (2 * h)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("ard", [True, False])
def test_nll_gradient_matches_finite_differences(kind, ard):
    X, y = _problem(1)
    ls, a2, s2 = _theta(3, ard)
    g = train.nll_grad(X, y, kind, ls, a2, s2, ard)
    nl = len(ls)
    for p in range(nl + 2):
        def f(t):
            l2, o2, n2 = ls.copy(), a2, s2
            if p < nl:
                l2[p] = t
            elif p == nl:
                o2 = t
            else:
                n2 = t
            return train.nll(X, y, kind, l2, o2, n2)
        x0 = ls[p] if p < nl else (a2 if p == nl else s2)
        want = _fd(f, x0, 1e-5 * x0)
        assert abs(g[p] - want) <= 1e-6 * (1 + abs(want)), (p, g[p], want)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("ard", [True, False])
def test_pseudo_loss_gradient_is_derivative_of_pseudo_loss(kind, ard):
    """Eq. (approx) is the theta-derivative of Eq. (approx_loss) with U fixed;
    the finite differences perturb the closed-form kernel (kernels.kfun)."""
    X, y = _problem(2)
    n = len(y)
    g = np.random.default_rng(3)
    B = np.column_stack([y, g.choice([-1.0, 1.0], size=(n, 4))])
    U = g.standard_normal(B.shape)          # any fixed U: the identity is algebraic
    ls, a2, s2 = _theta(3, ard)
    grad = train.pseudo_loss_grad(X, U, B, kind, ls, a2, ard)
    nl = len(ls)
    for p in range(nl + 2):
        def f(t):
            l2, o2, n2 = ls.copy(), a2, s2
            if p < nl:
                l2[p] = t
            elif p == nl:
                o2 = t
            else:
                n2 = t
            return train.pseudo_loss(X, U, B, kind, l2, o2, n2)
        x0 = ls[p] if p < nl else (a2 if p == nl else s2)
        want = _fd(f, x0, 1e-5 * x0)
        assert abs(grad[p] - want) <= 1e-6 * (1 + abs(want)), (p, grad[p], want)


@pytest.mark.parametrize("kind", [kernels.RBF, kernels.MATERN52])
def test_hutchinson_mean_over_all_sign_vectors_is_exact(kind):
    """Averaged over all 2^n Rademacher vectors, (1/M) sum z z^T = I, so with
    exact solves Eq. (approx) equals Eq. (gradient), first line."""
    n, d = 8, 2
    X, y = _problem(4, n=n, d=d)
    Z = np.array([[1.0 if (k >> i) & 1 else -1.0 for i in range(n)] for k in range(2 ** n)]).T
    ls, a2, s2 = np.array([0.8, 1.3]), 0.9, 0.15
    A = train.ktilde(X, kind, ls, a2, s2)
    B = np.column_stack([y, Z])
    U = scipy.linalg.solve(A, B, assume_a="pos")
    est = train.pseudo_loss_grad(X, U, B, kind, ls, a2, True)
    exact = train.nll_grad(X, y, kind, ls, a2, s2, True)
    np.testing.assert_allclose(est, exact, rtol=1e-10, atol=1e-12)


def test_estimator_is_noisy_but_unbiased_on_few_probes():
    """With a handful of probes the estimate differs from the exact gradient,
    and its average over many independent probe draws approaches it."""
    n, d = 40, 2
    X, y = _problem(5, n=n, d=d)
    ls, a2, s2 = np.array([0.8, 1.3]), 0.9, 0.15
    A = train.ktilde(X, kernels.RBF, ls, a2, s2)
    exact = train.nll_grad(X, y, kernels.RBF, ls, a2, s2, True)
    g = np.random.default_rng(6)
    ests = []
    for _ in range(400):
        B = np.column_stack([y, g.choice([-1.0, 1.0], size=(n, 4))])
        U = scipy.linalg.solve(A, B, assume_a="pos")
        ests.append(train.pseudo_loss_grad(X, U, B, kernels.RBF, ls, a2, True))
    ests = np.array(ests)
    sem = ests.std(0) / np.sqrt(len(ests))
    assert np.all(ests.std(0) > 0)
    assert np.all(np.abs(ests.mean(0) - exact) < 5 * sem + 1e-12)


def test_row_partition_adds_up_and_scale_bounds():
    X, y = _problem(7, n=15)
    g = np.random.default_rng(8)
    B = np.column_stack([y, g.choice([-1.0, 1.0], size=(15, 3))])
    U = g.standard_normal(B.shape)
    ls, a2, _ = _theta(3, True)
    full = train.pseudo_loss_grad(X, U, B, kernels.MATERN52, ls, a2, True)
    parts = sum(train.pseudo_loss_grad(X, U, B, kernels.MATERN52, ls, a2, True, rows=r)
                for r in (range(0, 4), range(4, 11), range(11, 15)))
    np.testing.assert_allclose(parts, full, rtol=1e-12, atol=1e-12)
    scale = train.pseudo_loss_grad_scale(X, U, B, kernels.MATERN52, ls, a2, True)
    assert np.all(np.abs(full) <= scale * (1 + 1e-12))


def test_data_fit_is_half_y_v():
    X, y = _problem(9)
    A = train.ktilde(X, kernels.RBF, [1.0], 1.0, 0.1)
    B = np.column_stack([y, np.ones_like(y)])
    U = np.linalg.solve(A, B)
    assert train.data_fit(U, B) == pytest.approx(0.5 * y @ np.linalg.solve(A, y), rel=1e-12)


def test_priors_are_the_papers_and_match_scipy():
    pv = paper_values()
    assert train.PRIOR_LENGTHSCALE == (pv["prior_lengthscale_alpha"], pv["prior_lengthscale_beta"])
    assert train.PRIOR_OUTPUTSCALE == (pv["prior_outputscale_alpha"], pv["prior_outputscale_beta"])
    assert train.PRIOR_NOISE == (pv["prior_noise_alpha"], pv["prior_noise_beta"])
    assert train.NOISE_FLOOR == pv["noise_floor"]
    for (a, b) in (train.PRIOR_LENGTHSCALE, train.PRIOR_OUTPUTSCALE, train.PRIOR_NOISE):
        for x in (0.05, 0.7, 3.0, 12.0):
            want = scipy.stats.gamma.logpdf(x, a, scale=1.0 / b)
            assert train.gamma_logpdf(x, a, b) == pytest.approx(want, rel=1e-12, abs=1e-12)
            fd = _fd(lambda t: scipy.stats.gamma.logpdf(t, a, scale=1.0 / b), x, 1e-6 * x)
            assert train.gamma_logpdf_grad(x, a, b) == pytest.approx(fd, rel=1e-6, abs=1e-8)
    # the paper's noise start of 2 is the mode (alpha - 1) / beta of its prior
    a, b = train.PRIOR_NOISE
    assert (a - 1) / b == pytest.approx(pv["noise_init"])


def test_softplus_round_trip_and_constraint():
    th = np.array([0.3, 2.0, 7.5, 0.01])
    raw = train.raw_from(th, 2)
    np.testing.assert_allclose(train.constrained(raw, 2), th, rtol=1e-12)
    assert train.constrained(np.array([0.0, 0.0, -50.0, 0.0]), 2)[3] > train.NOISE_FLOOR
    np.testing.assert_allclose(train.softplus(np.array([0.0])), [np.log(2.0)], rtol=1e-15)
    for x in (-3.0, 0.0, 2.5):
        assert train.sigmoid(x) == pytest.approx(_fd(lambda t: float(train.softplus(t)), x, 1e-6), rel=1e-8)


@pytest.mark.parametrize("ard", [True, False])
def test_raw_gradient_matches_finite_differences_of_objective(ard):
    X, y = _problem(10, n=10, d=2)
    n = len(y)
    nl = 2 if ard else 1
    th0 = np.concatenate([[0.8, 1.2][:nl], [1.5, 0.3]])
    raw = train.raw_from(th0, nl)
    gth = train.nll_grad(X, y, kernels.RBF, th0[:nl], th0[nl], th0[nl + 1], ard)
    g = train.raw_gradient(raw, gth, n, nl)
    for p in range(nl + 2):
        def f(t):
            r2 = raw.copy()
            r2[p] = t
            return train.objective(r2, X, y, kernels.RBF, ard)
        assert g[p] == pytest.approx(_fd(f, raw[p], 1e-5), rel=1e-6, abs=1e-10)


def test_adam_first_step_closed_form_and_quadratic():
    g = np.array([0.5, -2.0, 1e-3])
    raw, m, v = train.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), 1, g, lr=0.1)
    np.testing.assert_allclose(raw, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)
    # minimises a quadratic
    x, m, v = np.array([3.0, -1.0]), np.zeros(2), np.zeros(2)
    for t in range(1, 2001):
        x, m, v = train.adam_step(x, m, v, t, 2 * x, lr=0.05)
    assert np.all(np.abs(x) < 1e-2)


def test_splitmix64_published_outputs():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "splitmix64.txt")
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(tuple(int(t) for t in line.split()))
    assert len(rows) == 6
    for seed, k, want in rows:
        assert train.splitmix64(seed, k) == want


def test_rademacher_probes_signs_and_balance():
    Z = train.rademacher_probes(11, 3, 400, 5)
    assert set(np.unique(Z)) == {-1.0, 1.0}
    assert abs(Z.mean()) < 4 / np.sqrt(Z.size)
    # steps draw different blocks from one stream
    assert not np.array_equal(Z, train.rademacher_probes(11, 4, 400, 5))
    # entry (i, c) of step t is counter (t n + i) M + c
    k = (3 * 400 + 17) * 5 + 2
    assert Z[17, 2] == (-1.0 if train.splitmix64(11, k) >> 63 else 1.0)


def test_training_lowers_objective_and_estimator_tracks_exact():
    """Adam with the exact gradient lowers the objective; steps taken with
    Eq. (approx) from exact solves and many probes stay close to it."""
    g = np.random.default_rng(12)
    n, d = 60, 2
    X = g.standard_normal((n, d))
    y = np.sin(2 * X[:, 0]) + 0.5 * X[:, 1] + 0.1 * g.standard_normal(n)
    th0 = np.array([0.693, 0.693, 0.693, 2.0])
    nl = 2
    raw0 = train.raw_from(th0, nl)
    th = train.train_exact(X, y, kernels.RBF, True, th0, 30)
    assert train.objective(train.raw_from(th, nl), X, y, kernels.RBF, True) < \
        train.objective(raw0, X, y, kernels.RBF, True) - 0.05
    raw, m, v = raw0.copy(), np.zeros(4), np.zeros(4)
    for t in range(1, 11):
        raw, m, v = train.estimator_step(X, y, kernels.RBF, True, raw, m, v, t, seed=5, M=64)
    th10 = train.train_exact(X, y, kernels.RBF, True, th0, 10)
    np.testing.assert_allclose(train.constrained(raw, nl), th10, rtol=0.15)
