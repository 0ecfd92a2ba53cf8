"""Conjugate-gradient solvers for K~ U = B (oracle; test infrastructure only).

Two algorithms, both run on all right-hand-side columns at once with separate
step sizes per column (mBCG, App. A):

* ``algo="plain"``: standard preconditioned CG, App. A Alg. 2.
* ``algo="enhanced"``: the enhanced-stability CG of Sec. 5.2 / Alg. 1:
  step sizes kept in log scale through the logsumexp form of positive inner
  products (Sec. 5.2, "Rescaling Conjugate Gradients") and explicit
  Gram-Schmidt re-orthogonalisation of each new residual against the previous
  ones (Sec. 5.2, "Re-orthogonalization").

Sign convention as in both algorithms: r = K~ x - b, and the search direction
is minus the preconditioned residual plus beta times the previous direction.

Readings of the printed algorithms (each is also listed in the design notes):
  * the loop runs while a column is NOT converged (both listings print the
    comparison the other way round, which would never start);
  * with a preconditioner the directions are built from z = P(r), not r
    (d_0 = -z_0, d_{k+1} = -z_{k+1} + beta d_k); identical when P is identity;
  * re-orthogonalisation uses the inner product induced by the preconditioner:
    basis u_j = r_j / sqrt(gamma_j), w_j = z_j / sqrt(gamma_j) with
    gamma_j = r_j^T z_j, and r <- r - (w_j^T r) u_j for j = 0..k in order
    (modified Gram-Schmidt, the order of Alg. 1).  Without a preconditioner this
    is exactly the Euclidean projection against the normalised residuals that
    the paper describes; ``reorth_inner="euclid"`` keeps the literal Euclidean
    form for comparison;
  * convergence is per column: relative residual ||r_c|| / ||b_c|| <= tol once
    at least ``min_iter`` iterations are done; a converged column is frozen and
    the others continue; an all-zero right-hand side returns zero, converged;
  * a logsumexp argument that is not positive and finite (the paper assumes a
    positive inner product) marks the column as broken down and freezes it.
"""

import numpy as np


def lse_dot(w, z):
    """log(w^T z) by the logsumexp transformation of Sec. 5.2.

    y_i = log|w_i| + log|z_i|, s_i = sign(w_i z_i);
    LSE = y_max + log(sum_i s_i exp(y_i - y_max)).  Terms with w_i z_i = 0
    contribute nothing.  Returns (value, ok); ok is False when the signed sum is
    not positive and finite (w^T z <= 0 has no real logarithm).
    """
    w = np.asarray(w, dtype=np.float64).ravel()
    z = np.asarray(z, dtype=np.float64).ravel()
    nz = (w != 0.0) & (z != 0.0)
    if not np.any(nz):
        return -np.inf, False
    wn, zn = w[nz], z[nz]
    if not (np.all(np.isfinite(wn)) and np.all(np.isfinite(zn))):
        return np.nan, False
    y = np.log(np.abs(wn)) + np.log(np.abs(zn))
    s = np.sign(wn) * np.sign(zn)
    ymax = np.max(y)
    total = np.sum(s * np.exp(y - ymax))
    if not (np.isfinite(total) and total > 0.0):
        return np.nan, False
    return ymax + np.log(total), True


def _col_dots(a, b):
    return np.einsum("ij,ij->j", a, b)


def solve(mvm, B, tol, max_iter, min_iter=0, precond=None, x0=None,
          algo="enhanced", reorth=True, use_lse=True, reorth_inner="P",
          record_history=False):
    """Solve K~ U = B column by column with shared MVMs.

    mvm(V) must return K~ V for an n x R array V; precond(W) must return
    P^{-1} W (the preconditioner function P(.) of Alg. 1/2), None = identity.
    ``max_iter`` is one cap for every column or a sequence of R per-column
    caps: column c is frozen after max_iter[c] iterations (its recurrences
    never involve the other columns, so this equals solving it alone with that
    cap; it is how a device run is matched iteration for iteration).
    Returns (U, stats) with per-column ``iters``, ``rel_res`` (recursive
    residual), ``converged``, ``breakdown`` and optionally ``history``.
    """
    if algo not in ("plain", "enhanced"):
        raise ValueError("algo must be 'plain' or 'enhanced'")
    enhanced = algo == "enhanced"
    do_reorth = enhanced and reorth
    do_lse = enhanced and use_lse
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    n, R = B.shape
    P = precond if precond is not None else (lambda w: np.array(w, copy=True))

    bnorm = np.linalg.norm(B, axis=0)
    zero_rhs = bnorm == 0.0
    safe_bnorm = np.where(zero_rhs, 1.0, bnorm)

    # Initialise (Alg. 1/2): r_0 = K(x_0) - b, z_0 = P(r_0), gamma_0 = r_0^T z_0.
    if x0 is None:
        x = np.zeros((n, R))
        r = -B.copy()
    else:
        x = np.asarray(x0, dtype=np.float64).reshape(n, R).copy()
        r = mvm(x) - B
    x[:, zero_rhs] = 0.0
    r[:, zero_rhs] = 0.0
    z = P(r)
    d = -z

    caps = np.broadcast_to(np.asarray(max_iter, dtype=np.int64), (R,)).copy()
    if np.any(caps < 0):
        raise ValueError("max_iter must be >= 0")
    active = ~zero_rhs & (caps > 0)
    converged = zero_rhs.copy()
    breakdown = np.zeros(R, dtype=bool)
    iters = np.zeros(R, dtype=np.int64)

    def gamma_of(rr, zz):
        """Per-column log gamma (enhanced) or gamma (plain), with validity."""
        val = np.full(R, np.nan)
        ok = np.zeros(R, dtype=bool)
        for c in range(R):
            if do_lse:
                val[c], ok[c] = lse_dot(rr[:, c], zz[:, c])
            else:
                g = float(np.dot(rr[:, c], zz[:, c]))
                val[c], ok[c] = g, bool(np.isfinite(g) and g > 0.0)
        return val, ok

    g, ok = gamma_of(r, z)
    bad = active & ~ok
    breakdown |= bad
    active &= ~bad

    def sqrt_gamma(gv):
        return np.exp(0.5 * gv) if do_lse else np.sqrt(np.abs(gv))

    basis_u, basis_w = [], []
    if do_reorth:
        sg = np.where(active, sqrt_gamma(g), 1.0)
        if reorth_inner == "P":
            basis_u.append(r / sg)
            basis_w.append(z / sg)
        else:
            nr = np.linalg.norm(r, axis=0)
            basis_u.append(r / np.where(nr > 0, nr, 1.0))

    history = []
    rel = np.linalg.norm(r, axis=0) / safe_bnorm
    if record_history:
        history.append(rel.copy())
    newly = active & (0 >= min_iter) & (rel <= tol)
    converged |= newly
    active &= ~newly

    k = 0
    while k < caps.max() and np.any(active):
        q = mvm(d)                                   # K(d_k)
        # alpha_k (Alg. 1: exp(log gamma_k - LSE(d_k^T K d_k)); Alg. 2: ratio)
        alpha = np.zeros(R)
        for c in np.flatnonzero(active):
            if do_lse:
                ld, okc = lse_dot(d[:, c], q[:, c])
                if okc:
                    alpha[c] = np.exp(g[c] - ld)
            else:
                dq = float(np.dot(d[:, c], q[:, c]))
                okc = bool(np.isfinite(dq) and dq > 0.0)
                if okc:
                    alpha[c] = g[c] / dq
            if not okc or not np.isfinite(alpha[c]):
                alpha[c] = 0.0
                breakdown[c] = True
                active[c] = False
        x += alpha[None, :] * d                     # x_{k+1} = x_k + alpha_k d_k
        r += alpha[None, :] * q                     # r_{k+1} = r_k + alpha_k K(d_k)
        k += 1
        iters[active] = k

        if do_reorth:                               # Gram-Schmidt against u_0..u_k
            cols = active
            if reorth_inner == "P":
                for uj, wj in zip(basis_u, basis_w):
                    coef = _col_dots(wj, r)
                    r[:, cols] -= coef[cols][None, :] * uj[:, cols]
            else:
                for uj in basis_u:
                    coef = _col_dots(uj, r)
                    r[:, cols] -= coef[cols][None, :] * uj[:, cols]

        rel_now = np.linalg.norm(r, axis=0) / safe_bnorm
        rel = np.where(active, rel_now, rel)
        if record_history:
            history.append(rel.copy())
        newly = active & (k >= min_iter) & (rel <= tol)
        converged |= newly
        active &= ~newly
        active &= k < caps                          # per-column iteration caps
        if not np.any(active):
            break

        z = P(r)                                    # z_{k+1} = P(r_{k+1})
        g_new, okg = gamma_of(r, z)
        bad = active & ~okg
        breakdown |= bad
        active &= ~bad
        if do_lse:                                  # beta_{k+1} = exp(lg_{k+1} - lg_k)
            with np.errstate(invalid="ignore"):
                beta = np.exp(np.where(active, g_new - g, 0.0))
        else:
            beta = np.where(active, g_new / np.where(active, g, 1.0), 0.0)
        dn = -z + beta[None, :] * d                 # d_{k+1} = -z_{k+1} + beta d_k
        d = np.where(active[None, :], dn, d)
        g = np.where(active, g_new, g)
        if do_reorth:
            if reorth_inner == "P":
                sg = np.where(active, sqrt_gamma(g), 1.0)
                basis_u.append(r / sg)
                basis_w.append(z / sg)
            else:
                nr = np.linalg.norm(r, axis=0)
                basis_u.append(r / np.where(nr > 0, nr, 1.0))

    stats = {
        "iters": iters,
        "rel_res": rel,
        "converged": converged,
        "breakdown": breakdown,
    }
    if record_history:
        stats["history"] = np.array(history)
    return x, stats


def true_relative_residual(mvm, B, U):
    """||b_c - K~ u_c|| / ||b_c|| per column (0 for a zero column solved by 0)."""
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    res = np.linalg.norm(B - mvm(np.asarray(U, dtype=np.float64).reshape(B.shape)), axis=0)
    bn = np.linalg.norm(B, axis=0)
    return np.where(bn > 0, res / np.where(bn > 0, bn, 1.0), res)
