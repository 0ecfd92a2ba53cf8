"""Finite-precision support of stationary kernels (oracle; test infrastructure only).

Sec. 4.1 and App. C: a kernel value below the smallest representable value eps
of a number format is exactly zero in that format, so the kernel has compact
support.  App. C solves k(d) < eps for the distance d at lengthscale l:
  Matern-1/2: exp(-d/l) < eps            ->  d > -l log eps
  RBF:        exp(-d^2 / (2 l^2)) < eps  ->  d > l sqrt(-2 log eps)
(The worked example of Sec. 4.1 divides by l instead of multiplying; the App. C
form is the one that follows from the inequality.)

IEEE binary16 constants (Sec. 2.1 prints them garbled; the standard values are
used): largest finite 65504, smallest normal 2^-14, smallest subnormal 2^-24,
unit round-off 2^-11.

Truncated product (Sec. 4.1, Fig. 2c; the appendix figure on the error of sparsified products):
drop, for every output point, the data points whose kernel value is not
representable in half precision, mu_trunc = K(x*, X_close) v_close.  Under
round-to-nearest-even a binary16 value rounds to zero exactly when it is at
most half the smallest subnormal, 2^-25, so "not representable" is taken as
k <= 2^-25 (FP16_ZERO_THRESHOLD): below the paper's eps = 2^-24 cut-off a
value still rounds up to 2^-24.  `zero_radius` is the scaled distance where
the kernel reaches that threshold; `kmvm_fp16_truncated` applies the
binary16 emulation of kmvm.py to the kept pairs only.
"""

import numpy as np

from .kernels import RBF, MATERN12, MATERN32, MATERN52, kfun, lengthscale_vector, scaled_sqdist
from .kmvm import column_scales, quantize_inputs_fp16

FP16_MAX = 65504.0
FP16_MIN_NORMAL = 2.0 ** -14
FP16_MIN_SUBNORMAL = 2.0 ** -24
FP16_UNIT_ROUNDOFF = 2.0 ** -11
FP16_ZERO_THRESHOLD = 2.0 ** -25


def cutoff_distance(kind_name, lengthscale, eps):
    """Distance beyond which the unit-outputscale kernel value is < eps."""
    le = -np.log(eps)
    if kind_name == "matern12":
        return lengthscale * le
    if kind_name == "rbf":
        return lengthscale * np.sqrt(2.0 * le)
    raise ValueError("closed form only for 'rbf' and 'matern12'")


def zero_radius(kind, threshold=FP16_ZERO_THRESHOLD):
    """Scaled distance r at which the unit-outputscale kernel value equals
    `threshold` (closed form for RBF and Matern-1/2, bisection otherwise)."""
    le = -np.log(threshold)
    if kind == RBF:
        return float(np.sqrt(2.0 * le))
    if kind == MATERN12:
        return float(le)
    lo, hi = 0.0, 1.0
    while kfun(kind, hi * hi) > threshold:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if kfun(kind, mid * mid) > threshold:
            lo = mid
        else:
            hi = mid
    return hi


def kmvm_fp16_truncated(X1, X2, V, kind, lengthscale, outputscale, noise, add_noise,
                        scale_mode=0):
    """Binary16-emulated product over the kept pairs only (per output row, the
    column points closer than zero_radius in the rounded scaled coordinates);
    returns (out, number of kept pairs).  Same rounding model as
    kmvm.kmvm_fp16_emulated."""
    V32 = np.asarray(V, dtype=np.float32)
    if V32.ndim == 1:
        V32 = V32[:, None]
    n2 = np.asarray(X2).shape[0]
    A = quantize_inputs_fp16(X1, lengthscale)
    Bq = quantize_inputs_fp16(X2, lengthscale)
    s = column_scales(V32, n2, scale_mode)
    Vh = (V32 * s[None, :]).astype(np.float16).astype(np.float64)
    R = zero_radius(kind)
    ones = np.ones(A.shape[1])
    out = np.zeros((A.shape[0], V32.shape[1]))
    kept = 0
    for i in range(A.shape[0]):
        r2 = scaled_sqdist(A[i:i + 1], Bq, ones)[0]
        close = np.nonzero(r2 < R * R)[0]
        kept += close.size
        Kh = kfun(kind, r2[close]).astype(np.float16)
        out[i] = Kh.astype(np.float64) @ Vh[close]
    out = outputscale * out / s.astype(np.float64)[None, :]
    if add_noise:
        out += noise * V32.astype(np.float64)
    return out, kept
