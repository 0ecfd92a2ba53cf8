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
"""

import numpy as np

FP16_MAX = 65504.0
FP16_MIN_NORMAL = 2.0 ** -14
FP16_MIN_SUBNORMAL = 2.0 ** -24
FP16_UNIT_ROUNDOFF = 2.0 ** -11


def cutoff_distance(kind_name, lengthscale, eps):
    """Distance beyond which the unit-outputscale kernel value is < eps."""
    le = -np.log(eps)
    if kind_name == "matern12":
        return lengthscale * le
    if kind_name == "rbf":
        return lengthscale * np.sqrt(2.0 * le)
    raise ValueError("closed form only for 'rbf' and 'matern12'")
