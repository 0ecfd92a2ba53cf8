// gp_true_residual_rows: rows of the float64-accumulated true residual
// b - K~ u (the solver's exit check, on a subset of rows).

#include <algorithm>

#include "internal.h"

namespace gpmi {
namespace {

// Xs[t] = X[rows[t]] (d floats per point).
__global__ void gather_points_kernel(const float* __restrict__ X, int d,
                                     const int64_t* __restrict__ rows, int64_t nrows,
                                     float* __restrict__ Xs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrows * d) return;
  const int64_t t = e / d;
  const int m = (int)(e % d);
  Xs[e] = X[rows[t] * d + m];
}

// res[t][c] = b[i][c] - (a2 * sum_x part[x][t][c] + s2 * u[i][c]), i = rows[t]
__global__ void residual_rows_kernel(const double* __restrict__ part, int nsplit, int64_t nrows,
                                     int r, const int64_t* __restrict__ rows,
                                     const float* __restrict__ B, const float* __restrict__ U,
                                     float a2, float s2, double* __restrict__ res) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrows * r) return;
  const int64_t t = e / r;
  const int c = (int)(e % r);
  const int64_t i = rows[t];
  double kx = 0.0;
  for (int x = 0; x < nsplit; ++x) kx += part[(int64_t)x * nrows * r + e];
  res[e] = (double)B[i * r + c] - ((double)a2 * kx + (double)s2 * (double)U[i * r + c]);
}

// Every row index must lie in [0, n): checked on the device, the result
// counted in *bad (the host reads it before anything else is launched).
__global__ void check_rows_kernel(const int64_t* __restrict__ rows, int64_t nrows, int64_t n,
                                  int* bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nrows && (rows[t] < 0 || rows[t] >= n)) atomicAdd(bad, 1);
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

}  // namespace
}  // namespace gpmi

using namespace gpmi;

extern "C" gp_status gp_true_residual_rows(const gp_kernel* k, const float* X, int64_t n,
                                           int32_t d, const float* B, const float* U, int32_t r,
                                           const int64_t* rows, int64_t nrows, double* res,
                                           void* stream) {
  clear_error();
  KParams kp;
  GP_TRY(check_kernel(k, d, false, &kp));
  if (n < 1) return set_error(GP_ERR_ARG, "n=%lld must be >= 1", (long long)n);
  if (r < 1 || r > cg::kMaxR) return set_error(GP_ERR_ARG, "r=%d outside [1, %d]", r, cg::kMaxR);
  if (nrows < 0) return set_error(GP_ERR_ARG, "nrows=%lld must be >= 0", (long long)nrows);
  if (nrows == 0) return GP_OK;
  if (!X || !B || !U || !rows || !res) return set_error(GP_ERR_ARG, "NULL array argument");
  const size_t rb = (size_t)nrows * r * 8;
  if (overlaps(res, rb, X, (size_t)n * d * 4) || overlaps(res, rb, B, (size_t)n * r * 4) ||
      overlaps(res, rb, U, (size_t)n * r * 4) || overlaps(res, rb, rows, (size_t)nrows * 8))
    return set_error(GP_ERR_ARG, "res overlaps an input");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nsplit = valu::choose_splits64(nrows, n, d);
  const size_t bytes = ((size_t)nrows * d * 4 + 255) / 256 * 256 +
                       ((size_t)nsplit * nrows * r * 8 + 255) / 256 * 256 + 256;
  Arena ar;
  GP_TRY(workspace_get(s, bytes, &ar));
  float* Xs = ar.take<float>((size_t)nrows * d);
  double* part = ar.take<double>((size_t)nsplit * nrows * r);
  int* bad = ar.take<int>(1);
  if (!Xs || !part || !bad) return set_error(GP_ERR_NOMEM, "internal: workspace sizing");
  zero_int_kernel<<<1, 1, 0, s>>>(bad);
  GP_HIP(hipGetLastError());
  check_rows_kernel<<<(unsigned)ceil_div(nrows, 256), 256, 0, s>>>(rows, nrows, n, bad);
  GP_HIP(hipGetLastError());
  int hbad = 0;
  GP_HIP(hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));
  if (hbad) return set_error(GP_ERR_ARG, "%d row indices outside [0, %lld)", hbad, (long long)n);
  gather_points_kernel<<<(unsigned)ceil_div(nrows * d, 256), 256, 0, s>>>(X, d, rows, nrows, Xs);
  GP_HIP(hipGetLastError());
  GP_TRY(valu::launch_partial(kp, Xs, nrows, X, n, U, r, part, true, nsplit, nullptr, s));
  residual_rows_kernel<<<(unsigned)ceil_div(nrows * r, 256), 256, 0, s>>>(
      part, nsplit, nrows, r, rows, B, U, kp.a2, kp.s2, res);
  GP_HIP(hipGetLastError());
  return GP_OK;
}
