"""Kernel matrix x multi-vector products (oracle; test infrastructure only).

Sec. 5.1, Eq. (mvm): (K~ v)_i = a^2 sum_j k(x_i, x_j) v_j + s^2 v_i, where the
noise term exists only when the row and column point sets are the same set
(K~ = a^2 K + s^2 I, Sec. 2.2 with the outputscale of Eq. mvm).  For many
right-hand sides (mBCG, App. A) V is an n2 x R matrix.

``kmvm`` is the plain definition in float64, blocked over output rows only so
that memory stays bounded; ``rows`` restricts the output to a subset of rows
(each output row depends only on its own point), which is how very large
problems are checked on sampled rows.

``kmvm_fp16_emulated`` models a float16-operand product with float32-or-better
accumulation (Sec. 5.1: blocks in half precision, block sums in single; App. B
"block summation").  Rounding model, stated so a test can compare a device
implementation against it bit-for-bit up to accumulation order:
  * x_hat = fp16(fp32(x) / fp32(l))            (inputs divided by the
    lengthscale in float32, then rounded to binary16, round-to-nearest-even)
  * r^2 from x_hat exactly (float64)           (so r^2(x, x) = 0 exactly)
  * k_hat = fp16(k(r^2))                        (kernel tile entries in half)
  * v_hat = fp16(fp32(v) * s_c)                 (per-column input scale s_c)
  * out = a^2 * (sum_j k_hat v_hat) / s_c + s^2 v   (float64 accumulation)
Column scales (Sec. 5.1 overflow discussion): mode 0 uses the power of two
s_c = 2^(15 - e_c) where max_j |v_jc| = f * 2^e_c, f in [0.5, 1), so that the
largest scaled entry lies in [2^14, 2^15); an all-zero column uses s_c = 1.
Mode 1 is the paper's s_c = n2^(-1/2) for every column, formed in float64 and
rounded once to float32.
"""

import numpy as np

from .kernels import kfun, lengthscale_vector, scaled_sqdist


def _row_blocks(n1, n2, d, budget_bytes=1 << 27):
    per_row = max(1, n2 * max(d, 1) * 8)
    b = max(1, min(n1, budget_bytes // per_row))
    return range(0, n1, b), b


def kmvm(X1, X2, V, kind, lengthscale, outputscale, noise, add_noise, rows=None):
    """float64 out = a^2 K(X1[rows], X2) V + [add_noise] s^2 V[rows]."""
    X1 = np.asarray(X1, dtype=np.float64)
    X2 = np.asarray(X2, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    if V.ndim == 1:
        V = V[:, None]
    if rows is None:
        rows = np.arange(X1.shape[0])
    rows = np.asarray(rows, dtype=np.int64)
    if add_noise and X1.shape[0] != X2.shape[0]:
        raise ValueError("the noise term needs the same point set on both sides")
    out = np.empty((rows.size, V.shape[1]), dtype=np.float64)
    starts, b = _row_blocks(rows.size, X2.shape[0], X2.shape[1])
    for s in starts:
        rr = rows[s:s + b]
        Kb = outputscale * kfun(kind, scaled_sqdist(X1[rr], X2, lengthscale))
        out[s:s + b] = Kb @ V
    if add_noise:
        out += noise * V[rows]
    return out


def quantize_inputs_fp16(X, lengthscale):
    """x_hat = fp16(fp32(x) / fp32(l)) as float64 values."""
    X32 = np.asarray(X, dtype=np.float32)
    ls32 = lengthscale_vector(lengthscale, X32.shape[1]).astype(np.float32)
    return (X32 / ls32).astype(np.float16).astype(np.float64)


def column_scales(V, n2, scale_mode):
    """Per-column input scale s_c (see module docstring)."""
    V32 = np.asarray(V, dtype=np.float32)
    if V32.ndim == 1:
        V32 = V32[:, None]
    R = V32.shape[1]
    if scale_mode == 1:
        return np.full(R, np.float32(1.0 / np.sqrt(float(n2))), dtype=np.float32)
    s = np.ones(R, dtype=np.float32)
    for c in range(R):
        m = float(np.max(np.abs(V32[:, c]))) if V32.shape[0] else 0.0
        if m > 0.0:
            _, e = np.frexp(m)
            s[c] = np.float32(np.ldexp(1.0, 15 - int(e)))
    return s


def kmvm_fp16_emulated(X1, X2, V, kind, lengthscale, outputscale, noise, add_noise,
                       scale_mode=0, rows=None):
    """float16-operand product with exact accumulation (model of Sec. 5.1)."""
    V32 = np.asarray(V, dtype=np.float32)
    if V32.ndim == 1:
        V32 = V32[:, None]
    n2 = np.asarray(X2).shape[0]
    X1h = quantize_inputs_fp16(X1, lengthscale)
    X2h = quantize_inputs_fp16(X2, lengthscale)
    if rows is None:
        rows = np.arange(X1h.shape[0])
    rows = np.asarray(rows, dtype=np.int64)
    s = column_scales(V32, n2, scale_mode)
    Vh = (V32 * s[None, :]).astype(np.float16).astype(np.float64)
    ones = np.ones(X1h.shape[1])
    out = np.empty((rows.size, V32.shape[1]), dtype=np.float64)
    starts, b = _row_blocks(rows.size, n2, X1h.shape[1])
    for st in starts:
        rr = rows[st:st + b]
        Kh = kfun(kind, scaled_sqdist(X1h[rr], X2h, ones)).astype(np.float16)
        out[st:st + b] = Kh.astype(np.float64) @ Vh
    out = outputscale * out / s.astype(np.float64)[None, :]
    if add_noise:
        out += noise * V32.astype(np.float64)[rows]
    return out
