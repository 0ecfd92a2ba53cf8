"""Number-format variants of the kernel-matrix product (oracle; test
infrastructure only: nothing outside tests/, the smoke check and the CPU
baseline of the benchmark may import it).

bfloat16 operands (Sec. 2.1 names bfloat16 as the 16-bit format that keeps
binary32's 8-bit exponent and so its range, with an 8-bit significand
(7 stored bits) instead of binary16's 11; the conclusion reports binary16 as
the easier format for CG).  ``round_bf16`` rounds a real to the nearest
bfloat16, ties to even, directly from float64 (no intermediate float32):
  x = m 2^e with m in [0.5, 1); quantum q = 2^max(e - 8, -133) (2^-133 is the
  smallest subnormal); bf16(x) = rint(x / q) q; |bf16(x)| >= 2^128 is inf.
``kmvm_bf16_emulated`` is the bfloat16 counterpart of
kmvm.kmvm_fp16_emulated, with the same rounding model:
  * x_hat = bf16(fp32(x) / fp32(l))
  * r^2 from x_hat exactly (float64), k_hat = bf16(k(r^2))
  * v_hat = bf16(fp32(v) s_c), s_c the column scale of kmvm.column_scales
    (for mode 0 a power of two: bfloat16 has float32's range, so this s_c
    changes nothing unless a value would leave that range)
  * out = a^2 (sum_j k_hat v_hat) / s_c + s^2 v, accumulated in float64.

Half-precision summation schemes (Sec. 5.1 and Fig. 4; App. B, summation
approaches): the accuracy ablations of the product whose entries AND sums are
binary16.  Entries and right-hand sides follow the binary16 model of
kmvm_fp16_emulated (x_hat = fp16(x / l), k_hat = fp16(k(r^2)),
v_hat = fp16(v s_c)); every term is the binary16 product
p_j = fp16(k_hat_j * v_hat_j), and the terms of one output entry are summed in
column order j = 0, 1, ..., n2 - 1:
  * 'block_half':   columns in consecutive blocks of `block` (the last one
    shorter); each block sum is a sequential binary16 sum of its terms, and the
    block sums are added sequentially in binary16;
  * 'block_single': block sums as above; they are added sequentially in
    float32 and the total is rounded back to binary16;
  * 'kahan_half':   one compensated (Kahan) sum over all terms with every
    operation in binary16: y = p - c, t = s + y, c = (t - s) - y, s = t.
The binary16 total T then gives out = a^2 T / s_c + s^2 v (float64).  Each
binary16 (or float32) operation is rounded once to nearest-even: numpy forms a
binary16 sum or product in binary32 and rounds it to binary16, which is the
correctly rounded result because binary32 carries at least 2*11 + 2 bits.
The float32 steps of 'block_single' are numpy float32 additions.
The default scale is the paper's s_c = n2^(-1/2) (scale_mode 1): with the
power-of-two scale of mode 0 a binary16 sum would overflow after a few terms.
The paper gives no block length; the default of 32 columns is the length at
which binary16 block sums added in float32 reach the accuracy Fig. 4b reports
(below 0.1% mean relative error) on positive right-hand sides.
"""

import numpy as np

from .kernels import kfun, lengthscale_vector, scaled_sqdist
from .kmvm import column_scales, quantize_inputs_fp16

BF16_MAX = (2.0 - 2.0 ** -7) * 2.0 ** 127
BF16_MIN_NORMAL = 2.0 ** -126
BF16_MIN_SUBNORMAL = 2.0 ** -133
BF16_UNIT_ROUNDOFF = 2.0 ** -8

SCHEMES = ("block_half", "block_single", "kahan_half")


def round_bf16(x):
    """Nearest bfloat16 (ties to even) of each value, as float64."""
    x = np.asarray(x, dtype=np.float64)
    out = np.array(x, dtype=np.float64, copy=True)
    fin = np.isfinite(x) & (x != 0.0)
    if np.any(fin):
        xf = x[fin]
        _, e = np.frexp(xf)
        qe = np.maximum(e - 8, -133)
        r = np.ldexp(np.rint(np.ldexp(xf, -qe)), qe)
        r = np.where(np.abs(r) >= 2.0 ** 128, np.copysign(np.inf, xf), r)
        out[fin] = r
    return out


def quantize_inputs_bf16(X, lengthscale):
    """x_hat = bf16(fp32(x) / fp32(l)) as float64 values."""
    X32 = np.asarray(X, dtype=np.float32)
    ls32 = lengthscale_vector(lengthscale, X32.shape[1]).astype(np.float32)
    return round_bf16((X32 / ls32).astype(np.float64))


def _row_blocks(n1, n2, budget_bytes=1 << 27):
    b = max(1, min(n1, budget_bytes // max(1, n2 * 8)))
    return range(0, n1, b), b


def kmvm_bf16_emulated(X1, X2, V, kind, lengthscale, outputscale, noise, add_noise,
                       scale_mode=0, rows=None):
    """bfloat16-operand product with exact accumulation (module docstring)."""
    V32 = np.asarray(V, dtype=np.float32)
    if V32.ndim == 1:
        V32 = V32[:, None]
    n2 = np.asarray(X2).shape[0]
    X1h = quantize_inputs_bf16(X1, lengthscale)
    X2h = quantize_inputs_bf16(X2, lengthscale)
    if rows is None:
        rows = np.arange(X1h.shape[0])
    rows = np.asarray(rows, dtype=np.int64)
    s = column_scales(V32, n2, scale_mode)
    Vh = round_bf16((V32 * s[None, :]).astype(np.float64))
    ones = np.ones(X1h.shape[1])
    out = np.empty((rows.size, V32.shape[1]), dtype=np.float64)
    starts, b = _row_blocks(rows.size, n2)
    for st in starts:
        rr = rows[st:st + b]
        Kh = round_bf16(kfun(kind, scaled_sqdist(X1h[rr], X2h, ones)))
        out[st:st + b] = Kh @ Vh
    out = outputscale * out / s.astype(np.float64)[None, :]
    if add_noise:
        out += noise * V32.astype(np.float64)[rows]
    return out


def half_terms(X1, X2, V, kind, lengthscale, scale_mode=1, rows=None):
    """Binary16 terms p[i, j, c] = fp16(k_hat_ij v_hat_jc) and the scales s_c."""
    V32 = np.asarray(V, dtype=np.float32)
    if V32.ndim == 1:
        V32 = V32[:, None]
    n2 = np.asarray(X2).shape[0]
    X1h = quantize_inputs_fp16(X1, lengthscale)
    X2h = quantize_inputs_fp16(X2, lengthscale)
    if rows is not None:
        X1h = X1h[np.asarray(rows, dtype=np.int64)]
    s = column_scales(V32, n2, scale_mode)
    Vh = (V32 * s[None, :]).astype(np.float16)
    Kh = kfun(kind, scaled_sqdist(X1h, X2h, np.ones(X1h.shape[1]))).astype(np.float16)
    P = Kh[:, :, None] * Vh[None, :, :]
    assert P.dtype == np.float16
    return P, s


def half_sum(P, scheme, block=32):
    """Sum the binary16 terms P[:, j, :] over j by `scheme` (module docstring).

    Returns the binary16 totals as float64."""
    if scheme not in SCHEMES:
        raise ValueError(f"unknown summation scheme {scheme!r}")
    if block < 1:
        raise ValueError("block must be >= 1")
    n1, n2, R = P.shape
    if scheme == "kahan_half":
        s = np.zeros((n1, R), np.float16)
        c = np.zeros((n1, R), np.float16)
        for j in range(n2):
            y = P[:, j, :] - c
            t = s + y
            c = (t - s) - y
            s = t
        return s.astype(np.float64)
    tot_h = np.zeros((n1, R), np.float16)
    tot_f = np.zeros((n1, R), np.float32)
    for j0 in range(0, n2, block):
        bs = np.zeros((n1, R), np.float16)
        for j in range(j0, min(n2, j0 + block)):
            bs = bs + P[:, j, :]
        if scheme == "block_half":
            tot_h = tot_h + bs
        else:
            tot_f = tot_f + bs.astype(np.float32)
    if scheme == "block_half":
        return tot_h.astype(np.float64)
    return tot_f.astype(np.float16).astype(np.float64)


def kmvm_fp16_summation(X1, X2, V, kind, lengthscale, outputscale, noise, add_noise, scheme,
                        block=32, scale_mode=1, rows=None):
    """Product with binary16 entries, terms and sums (module docstring)."""
    P, s = half_terms(X1, X2, V, kind, lengthscale, scale_mode, rows)
    T = half_sum(P, scheme, block)
    out = outputscale * T / s.astype(np.float64)[None, :]
    if add_noise:
        V32 = np.asarray(V, dtype=np.float32)
        if V32.ndim == 1:
            V32 = V32[:, None]
        rr = np.arange(V32.shape[0]) if rows is None else np.asarray(rows, dtype=np.int64)
        out += noise * V32.astype(np.float64)[rr]
    return out


class Operator16:
    """K~ as the 16-bit product applies it, as a dense operator for CG runs on
    small problems (the reference of a 16-bit solve's matched-iteration
    parity: Alg. 1 driven by this operator sees the same rounding model as the
    device product, so what remains between the two is float32 arithmetic).

    fmt "fp16" follows kmvm.kmvm_fp16_emulated and "bf16" kmvm_bf16_emulated:
    the kernel matrix of the rounded inputs x_hat is rounded to the format
    once (K_hat), and every application rounds its right-hand side:
      mvm(V) = a^2 (K_hat v_hat) / s_c + s^2 fp32(V),
      v_hat = round(fp32(V) s_c), s_c the column scales of kmvm.column_scales
    (for bf16 with the power-of-two scale of mode 0, which leaves bfloat16
    values unchanged).  Accumulation in float64.  Memory: n^2 float64.
    """

    def __init__(self, X, kind, lengthscale, outputscale, noise, fmt="fp16", scale_mode=0,
                 block=1000):
        if fmt not in ("fp16", "bf16"):
            raise ValueError("fmt must be 'fp16' or 'bf16'")
        self.fmt, self.scale_mode = fmt, scale_mode
        self.a2, self.s2 = float(outputscale), float(noise)
        Xh = (quantize_inputs_fp16(X, lengthscale) if fmt == "fp16"
              else quantize_inputs_bf16(X, lengthscale))
        n = Xh.shape[0]
        ones = np.ones(Xh.shape[1])
        self.K = np.empty((n, n))
        for s in range(0, n, block):
            k = kfun(kind, scaled_sqdist(Xh[s:s + block], Xh, ones))
            self.K[s:s + block] = (k.astype(np.float16).astype(np.float64) if fmt == "fp16"
                                   else round_bf16(k))

    def __call__(self, V):
        V = np.asarray(V, dtype=np.float64)
        one = V.ndim == 1
        V32 = (V[:, None] if one else V).astype(np.float32)
        s = column_scales(V32, V32.shape[0], self.scale_mode).astype(np.float64)
        scaled = (V32 * s.astype(np.float32)[None, :])
        Vh = (scaled.astype(np.float16).astype(np.float64) if self.fmt == "fp16"
              else round_bf16(scaled.astype(np.float64)))
        out = self.a2 * (self.K @ Vh) / s[None, :] + self.s2 * V32.astype(np.float64)
        return out[:, 0] if one else out
