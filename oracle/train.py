"""Hyperparameter training (oracle; test infrastructure only).

Sec. 2.2, Eq. (loss): the negative log marginal likelihood
    L(theta) = 1/2 log|K~| + 1/2 y^T K~^{-1} y + N/2 log(2 pi),
    K~ = a^2 K + s^2 I,  theta = (lengthscale(s) l, outputscale a^2, noise s^2).
Eq. (gradient), first line: dL/dtheta = 1/2 tr(K~^{-1} dK~) - 1/2 v^T dK~ v
with v = K~^{-1} y; the second line replaces the trace by Hutchinson's
estimate over probe vectors z_j.
Sec. 5.3 (loss function), Eq. (cg): U = K~^{-1} [y, z_1, ..., z_M] from one
multi-right-hand-side solve; Eq. (approx_loss) is the pseudo-loss
    Lt(theta) = 1/(2M) sum_j u_j^T (K~_theta z_j) - 1/2 u_0^T (K~_theta u_0)
with the solutions held fixed, and Eq. (approx) its gradient, the same
expression with K~_theta replaced by dK~/dtheta.  The probe law is not printed;
Rademacher (+-1) probes are used.
App. C (experimental setup): Gamma(3, 6) prior on each lengthscale,
Gamma(2, 0.15) on the outputscale, Gamma(1.1, 0.05) on the noise, noise
constrained above 1e-4 and started at 2, Adam for 50 or 100 steps.  Readings
where the paper is silent: Gamma(alpha, beta) has rate beta; the positive
parameters are softplus of unconstrained "raw" values (noise = 1e-4 +
softplus(raw)); the objective is (L - sum of log priors) / N; Adam uses
beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and step size 0.1.

Derivatives of the covariance functions are written out from their closed
forms (kernels.kfun) with r^2 = sum_m (x_m - x'_m)^2 / l_m^2:
    dk/dl_m = a^2 kappa'(r^2) * dr^2/dl_m,   dr^2/dl_m = -2 (x_m - x'_m)^2 / l_m^3,
    kappa'(r^2) = d kappa / d(r^2):
        RBF          -1/2 exp(-r^2/2)
        Matern-1/2   -exp(-r) / (2 r)            (0 where x = x')
        Matern-3/2   -3/2 exp(-sqrt3 r)
        Matern-5/2   -5/6 (1 + sqrt5 r) exp(-sqrt5 r)
    dk/da^2 = kappa(r^2),  dK~/ds^2 = I.
An isotropic lengthscale's derivative is the sum over m.

Probe generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used counter-style: value k of
stream `seed` is mix(seed + (k + 1) * 0x9E3779B97F4A7C15), and the Rademacher
entry is +1 when the top bit is 0, else -1.  Entry (i, c) of the probe block of
training step t (n rows, M probes) has k = (t * n + i) * M + c.

Parity status: pinned in tests/test_oracle_train.py by finite differences of
the exact likelihood and of the pseudo-loss, by the exact Hutchinson mean over
all 2^n sign vectors, by scipy's Gamma density, by Adam's closed-form first
step and by the published SplitMix64 output sequence.
"""

from math import lgamma

import numpy as np
import scipy.linalg

from .kernels import RBF, MATERN12, MATERN32, MATERN52, kfun, lengthscale_vector

NOISE_FLOOR = 1e-4
PRIOR_LENGTHSCALE = (3.0, 6.0)
PRIOR_OUTPUTSCALE = (2.0, 0.15)
PRIOR_NOISE = (1.1, 0.05)


# ---------------------------------------------------------------- kernel derivatives
def dkappa_dr2(kind, r2):
    """d kappa / d(r^2) of the unit-outputscale kernel, elementwise."""
    r2 = np.maximum(np.asarray(r2, dtype=np.float64), 0.0)
    if kind == RBF:
        return -0.5 * np.exp(-0.5 * r2)
    r = np.sqrt(r2)
    if kind == MATERN12:
        out = np.zeros_like(r)
        nz = r > 0
        out[nz] = -np.exp(-r[nz]) / (2.0 * r[nz])
        return out
    if kind == MATERN32:
        return -1.5 * np.exp(-np.sqrt(3.0) * r)
    if kind == MATERN52:
        t = np.sqrt(5.0) * r
        return -(5.0 / 6.0) * (1.0 + t) * np.exp(-t)
    raise ValueError(f"unknown kernel kind {kind}")


def n_lengthscales(d, ard):
    return d if ard else 1


def dktilde(X, kind, lengthscale, outputscale, ard, rows=None):
    """The matrices dK~/dtheta for theta = (l_1..l_L, a^2, s^2), L = d or 1.

    X is n x d; `lengthscale` has d entries if ard, else 1.  Returns a list of
    float64 arrays in that order, each holding the rows `rows` (an index
    array; all n rows when None) of the n x n derivative."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    sel = np.arange(n) if rows is None else np.asarray(rows)
    ls = lengthscale_vector(lengthscale, d)
    diff2 = [((X[sel, None, m] - X[None, :, m]) / ls[m]) ** 2 for m in range(d)]
    r2 = np.sum(diff2, axis=0)
    kp = dkappa_dr2(kind, r2)
    per_dim = [outputscale * kp * (-2.0 * diff2[m] / ls[m]) for m in range(d)]
    if ard:
        dls = per_dim
    else:
        dls = [np.sum(per_dim, axis=0)]
    eye_rows = np.zeros((sel.size, n))
    eye_rows[np.arange(sel.size), sel] = 1.0        # rows `sel` of the identity
    return dls + [kfun(kind, r2), eye_rows]


def ktilde(X, kind, lengthscale, outputscale, noise):
    X = np.asarray(X, dtype=np.float64)
    ls = lengthscale_vector(lengthscale, X.shape[1])
    A = X / ls
    r2 = np.sum((A[:, None, :] - A[None, :, :]) ** 2, axis=2)
    K = outputscale * kfun(kind, r2)
    return K + noise * np.eye(X.shape[0])


# ---------------------------------------------------------------- Eq. loss / gradient
def nll(X, y, kind, lengthscale, outputscale, noise):
    """Eq. (loss) by a dense Cholesky factorisation."""
    A = ktilde(X, kind, lengthscale, outputscale, noise)
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    c, low = scipy.linalg.cho_factor(A, lower=True)
    v = scipy.linalg.cho_solve((c, low), y)
    logdet = 2.0 * np.sum(np.log(np.diag(c)))
    return 0.5 * logdet + 0.5 * y @ v + 0.5 * len(y) * np.log(2.0 * np.pi)


def nll_grad(X, y, kind, lengthscale, outputscale, noise, ard):
    """Eq. (gradient), first line, with the trace formed exactly."""
    A = ktilde(X, kind, lengthscale, outputscale, noise)
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    Ainv = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A, lower=True), np.eye(len(y)))
    v = Ainv @ y
    out = []
    for D in dktilde(X, kind, lengthscale, outputscale, ard):
        out.append(0.5 * np.sum(Ainv * D) - 0.5 * v @ D @ v)   # tr(A^-1 D), A^-1 symmetric
    return np.array(out)


# ---------------------------------------------------------------- Eq. approx_loss / approx
def _split(U, B):
    U = np.asarray(U, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if U.shape != B.shape or U.ndim != 2 or U.shape[1] < 2:
        raise ValueError("U and B must both be n x (M + 1) with M >= 1")
    return U[:, 0], U[:, 1:], B[:, 1:]


def pseudo_loss(X, U, B, kind, lengthscale, outputscale, noise):
    """Eq. (approx_loss): B = [y, z_1..z_M], U the (detached) solutions."""
    u0, Up, Z = _split(U, B)
    A = ktilde(X, kind, lengthscale, outputscale, noise)
    M = Z.shape[1]
    return np.sum(Up * (A @ Z)) / (2.0 * M) - 0.5 * u0 @ (A @ u0)


def _w_rows(U, B, sel):
    """Rows sel of W = 1/(2M) sum_j u_j z_j^T - 1/2 u_0 u_0^T."""
    u0, Up, Z = _split(U, B)
    M = Z.shape[1]
    return Up[sel] @ Z.T / (2.0 * M) - 0.5 * np.outer(u0[sel], u0)


def pseudo_loss_grad(X, U, B, kind, lengthscale, outputscale, ard, rows=None):
    """Eq. (approx) for theta = (l.., a^2, s^2).

    rows (optional index array) keeps only the terms whose left index i is in
    rows: sum_{i in rows} sum_j dK~_ij W_ij with
    W = 1/(2M) sum_j u_j z_j^T - 1/2 u_0 u_0^T, so that a partition of the
    rows adds up to the whole gradient."""
    sel = np.arange(np.asarray(U).shape[0]) if rows is None else np.asarray(rows)
    W = _w_rows(U, B, sel)
    return np.array([np.sum(D * W) for D in dktilde(X, kind, lengthscale, outputscale, ard, sel)])


def pseudo_loss_grad_scale(X, U, B, kind, lengthscale, outputscale, ard, rows=None):
    """sum |dK~_ij| |W_ij| per component: the size of the terms Eq. (approx)
    adds, against which a rounding error is measured."""
    sel = np.arange(np.asarray(U).shape[0]) if rows is None else np.asarray(rows)
    W = np.abs(_w_rows(U, B, sel))
    return np.array([np.sum(np.abs(D) * W) for D in dktilde(X, kind, lengthscale, outputscale, ard, sel)])


def data_fit(U, B, rows=None):
    """1/2 y^T K~^{-1} y = 1/2 y^T u_0, the data-fit half of Eq. (loss)
    (the terms of the rows `rows` only, when given)."""
    y = np.asarray(B, dtype=np.float64)[:, 0]
    u0 = np.asarray(U, dtype=np.float64)[:, 0]
    sel = np.arange(len(y)) if rows is None else np.asarray(rows)
    return 0.5 * float(y[sel] @ u0[sel])


# ---------------------------------------------------------------- priors and parameters
def gamma_logpdf(x, alpha, beta):
    """log Gamma(x; shape alpha, rate beta)."""
    x = np.asarray(x, dtype=np.float64)
    return alpha * np.log(beta) - lgamma(alpha) + (alpha - 1.0) * np.log(x) - beta * x


def gamma_logpdf_grad(x, alpha, beta):
    x = np.asarray(x, dtype=np.float64)
    return (alpha - 1.0) / x - beta


def softplus(x):
    x = np.asarray(x, dtype=np.float64)
    return np.logaddexp(0.0, x)


def softplus_inv(y):
    y = np.asarray(y, dtype=np.float64)
    return y + np.log(-np.expm1(-y))


def sigmoid(x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def constrained(raw, nl):
    """theta from raw values: l and a^2 = softplus(raw), s^2 = 1e-4 + softplus(raw)."""
    raw = np.asarray(raw, dtype=np.float64)
    th = softplus(raw)
    th[nl + 1] += NOISE_FLOOR
    return th


def raw_from(theta, nl):
    theta = np.array(theta, dtype=np.float64)
    theta[nl + 1] -= NOISE_FLOOR
    return softplus_inv(theta)


def log_prior(theta, nl):
    th = np.asarray(theta, dtype=np.float64)
    return (np.sum(gamma_logpdf(th[:nl], *PRIOR_LENGTHSCALE))
            + gamma_logpdf(th[nl], *PRIOR_OUTPUTSCALE) + gamma_logpdf(th[nl + 1], *PRIOR_NOISE))


def log_prior_grad(theta, nl):
    th = np.asarray(theta, dtype=np.float64)
    g = np.empty_like(th)
    g[:nl] = gamma_logpdf_grad(th[:nl], *PRIOR_LENGTHSCALE)
    g[nl] = gamma_logpdf_grad(th[nl], *PRIOR_OUTPUTSCALE)
    g[nl + 1] = gamma_logpdf_grad(th[nl + 1], *PRIOR_NOISE)
    return g


def objective(raw, X, y, kind, ard, priors=True):
    """(L(theta) - sum log priors) / N at theta = constrained(raw)."""
    n, d = np.asarray(X).shape
    nl = n_lengthscales(d, ard)
    th = constrained(raw, nl)
    val = nll(X, y, kind, th[:nl], th[nl], th[nl + 1])
    if priors:
        val -= log_prior(th, nl)
    return val / n


def raw_gradient(raw, grad_theta, n, nl, priors=True):
    """Chain rule from dL/dtheta to d objective / d raw (softplus' = sigmoid)."""
    raw = np.asarray(raw, dtype=np.float64)
    th = constrained(raw, nl)
    g = np.asarray(grad_theta, dtype=np.float64).copy()
    if priors:
        g = g - log_prior_grad(th, nl)
    return g / n * sigmoid(raw)


def adam_step(raw, m, v, t, g, lr=0.1, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Alg. 1); t counts from 1."""
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return np.asarray(raw, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------- probes
_GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64(seed, k):
    """Value k (k >= 0) of the SplitMix64 stream seeded with `seed`, as Python ints."""
    z = (seed + (k + 1) * _GAMMA) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def rademacher_probes(seed, step, n, M):
    """n x M probe block of training step `step` (entries +-1, float64)."""
    out = np.empty((n, M))
    for i in range(n):
        for c in range(M):
            out[i, c] = -1.0 if splitmix64(seed, (step * n + i) * M + c) >> 63 else 1.0
    return out


# ---------------------------------------------------------------- training loops
def train_exact(X, y, kind, ard, theta0, steps, lr=0.1, priors=True):
    """Adam on the objective with the exact gradient (Eq. gradient, first line)."""
    n, d = np.asarray(X).shape
    nl = n_lengthscales(d, ard)
    raw = raw_from(theta0, nl)
    m = np.zeros_like(raw)
    v = np.zeros_like(raw)
    for t in range(1, steps + 1):
        th = constrained(raw, nl)
        g = nll_grad(X, y, kind, th[:nl], th[nl], th[nl + 1], ard)
        raw, m, v = adam_step(raw, m, v, t, raw_gradient(raw, g, n, nl, priors), lr=lr)
    return constrained(raw, nl)


def estimator_step(X, y, kind, ard, raw, m, v, t, seed, M, lr=0.1, priors=True):
    """One training step as the method takes it, with exact solves: probes of
    step t - 1, U = K~^{-1}[y, Z] (Cholesky), Eq. (approx), chain rule, Adam."""
    n, d = np.asarray(X).shape
    nl = n_lengthscales(d, ard)
    th = constrained(raw, nl)
    B = np.column_stack([np.asarray(y, dtype=np.float64).reshape(-1), rademacher_probes(seed, t - 1, n, M)])
    A = ktilde(X, kind, th[:nl], th[nl], th[nl + 1])
    U = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A, lower=True), B)
    g = pseudo_loss_grad(X, U, B, kind, th[:nl], th[nl], ard)
    return adam_step(raw, m, v, t, raw_gradient(raw, g, n, nl, priors), lr=lr)
