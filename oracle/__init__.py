"""Plain, slow, obviously-correct CPU oracle for the low-precision GP solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything under ``oracle/``; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.

Everything is float64 NumPy unless a function says it emulates a lower
precision.  Each function cites the passage of Maddox, Potapczynski & Wilson,
"Low-Precision Arithmetic for Fast Gaussian Processes" (UAI 2022) it follows.

Modules
  kernels   covariance functions and scaled distances (App. C; Matern-5/2 and
            -3/2 from the textbook form, Rasmussen & Williams ch. 4)
  kmvm      the kernel matrix x multi-vector product (Sec. 5.1, Eq. mvm) and
            its float16-operand emulation (Sec. 5.1 block summation)
  direct    dense Cholesky solve of (a^2 K + s^2 I) U = B (Sec. 2.2)
  cg        standard preconditioned CG (App. A, Alg. 2) and the
            enhanced-stability CG (Sec. 5.2, Alg. 1), both batched over
            right-hand-side columns as in mBCG (App. A)
  pivchol   rank-k pivoted Cholesky and the Woodbury preconditioner
            (Sec. 5.2, Eq. woodbury)
  support   finite-precision support cut-offs (Sec. 4.1, App. C)
  train     negative log marginal likelihood and its gradient (Sec. 2.2),
            the pseudo-loss gradient estimator (Sec. 5.3), the App. C priors,
            Adam, and the SplitMix64 probe generator
  precision bfloat16 rounding and the bfloat16-operand product (Sec. 2.1),
            and the binary16 summation schemes: block sums in half or
            single, Kahan's sum in half (Sec. 5.1, Fig. 4; App. B)

Parity status: every function here is pinned by a CPU test in
``tests/test_oracle_*.py`` against closed forms, library routines, brute force
or values the paper prints; none is "parity unpinned".
"""

from . import kernels, kmvm, direct, cg, pivchol, support, train, precision  # noqa: F401
