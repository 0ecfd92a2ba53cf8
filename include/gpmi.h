/*
 * gpmi.h -- C ABI of the MI355X (gfx950) low-precision Gaussian-process solver.
 *
 * Method: Maddox, Potapczynski & Wilson, "Low-Precision Arithmetic for Fast
 * Gaussian Processes", UAI 2022.  The library computes, without ever storing
 * the kernel matrix, the product (a^2 K(X1,X2) + s^2 I) V (Sec. 5.1, Eq. mvm)
 * and solves (a^2 K + s^2 I) U = B by conjugate gradients, either the standard
 * preconditioned form (App. A, Alg. 2) or the enhanced-stability form (Sec.
 * 5.2, Alg. 1: log-scale step sizes via logsumexp, re-orthogonalisation),
 * optionally preconditioned by a rank-k pivoted Cholesky factor through the
 * Woodbury identity (Sec. 5.2, Eq. woodbury).
 *
 * Conventions shared by every entry point:
 *  - Every call returns a gp_status; nothing throws across the ABI.  On any
 *    error the message is available from gp_last_error() (per host thread).
 *    On GP_ERR_ARG no output has been touched.
 *  - Matrices are row-major, float32, and DEVICE pointers unless a comment
 *    says "host".  The caller owns all memory it passes; the library owns the
 *    opaque handles it returns and its own workspaces.
 *  - Streams are HIP streams passed as void* (NULL = the default stream).
 *    Launches are asynchronous on that stream unless a comment says the call
 *    synchronises.
 *  - Library workspaces are cached per device and stream: calls issued on
 *    the same stream are safe; concurrent calls on one stream from several
 *    host threads race.
 */
#ifndef GPMI_H
#define GPMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gp_status;
#define GP_OK 0
#define GP_PENDING 1
#define GP_ERR_ARG (-1)
#define GP_ERR_NOMEM (-2)
#define GP_ERR_HIP (-3)
#define GP_ERR_NOT_PD (-4)
#define GP_ERR_BREAKDOWN (-5)
#define GP_ERR_TOO_LARGE (-6)
#define GP_ERR_UNKNOWN_TICKET (-7)

/* Covariance function (App. C; Matern-5/2 and -3/2 in the textbook
 * half-integer form, r^2 = sum_m ((x_m - x'_m)/l_m)^2):
 *   RBF        exp(-r^2/2)
 *   MATERN52   (1 + sqrt5 r + 5 r^2/3) exp(-sqrt5 r)
 *   MATERN12   exp(-r)
 *   MATERN32   (1 + sqrt3 r) exp(-sqrt3 r)                               */
#define GP_KERNEL_RBF 0
#define GP_KERNEL_MATERN52 1
#define GP_KERNEL_MATERN12 2
#define GP_KERNEL_MATERN32 3

/* Arithmetic of the kernel-matrix product (Sec. 5.1).
 *   GP_PREC_FP32: float32 inputs, kernel entries and accumulation.
 *   GP_PREC_FP16: inputs divided by the lengthscale are rounded to binary16,
 *                 the kernel tile entries and the scaled right-hand sides are
 *                 binary16 matrix-core operands, every product and sum is
 *                 accumulated in float32 ("block summation in single
 *                 precision"), and the output is float32.                     */
#define GP_PREC_FP32 0
#define GP_PREC_FP16 1

/* Hyperparameters (Sec. 2.2 and Eq. mvm): kernel kind, lengthscale(s),
 * outputscale a^2 and noise s^2.  lengthscale is a HOST array of 1 value
 * (isotropic, ard = 0) or d values (ARD, ard = 1).  Requirements: every
 * lengthscale finite and > 0, a^2 finite and > 0, s^2 finite and >= 0
 * (> 0 for solves and preconditioners).                                       */
typedef struct gp_kernel {
  int32_t kind;
  int32_t ard;
  const float* lengthscale;
  float outputscale;
  float noise;
} gp_kernel;

/* Message describing the last error on the calling host thread ("" if none). */
const char* gp_last_error(void);

/* Library version string, e.g. "gpmi 0.1.0 gfx950". */
const char* gp_version(void);

/*
 * gp_kmvm -- out = a^2 K(X1, X2) V + [add_noise] s^2 V          (Eq. mvm)
 *
 *  X1   n1 x d  points of the output rows
 *  X2   n2 x d  points of the summed columns
 *  V    n2 x r  right-hand sides
 *  out  n1 x r  result; must not overlap V, X1 or X2
 *  add_noise    1 adds s^2 V; requires X1 == X2 and n1 == n2 (the same set)
 *  precision    GP_PREC_FP32 or GP_PREC_FP16
 *  scale_mode   FP16 only: 0 scales column c of V by the power of two that
 *               puts max|v_c| in [2^14, 2^15) before rounding it to binary16,
 *               1 uses the paper's n2^(-1/2) (Sec. 5.1); the scale is undone
 *               on the float32 accumulator, so both give the same product up
 *               to rounding.
 *  Limits: 1 <= d <= 64, r >= 1, n1, n2 >= 0 (n1 == 0 is a no-op, n2 == 0
 *  gives out = [add_noise] s^2 V).  Asynchronous on `stream`.
 *  Errors: GP_ERR_ARG (shapes, hyperparameters, null pointers, aliasing),
 *  GP_ERR_NOMEM (workspace), GP_ERR_HIP (launch failure).
 *  FP16 inputs whose |x/l| or squared norm exceeds the binary16 range give
 *  non-finite outputs.
 */
gp_status gp_kmvm(const gp_kernel* k, const float* X1, int64_t n1, const float* X2,
                  int64_t n2, int32_t d, const float* V, int32_t r, float* out,
                  int32_t add_noise, int32_t precision, int32_t scale_mode, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GPMI_H */
