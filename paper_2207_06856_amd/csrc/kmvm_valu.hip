// Kernel matrix x multi-vector product on the vector ALUs with float32 kernel
// entries (Eq. mvm).  Two accumulations:
//   float32 -- the single-precision product (the plain-CG baseline and the
//              small solves where matrix cores cannot be filled);
//   float64 -- every product k(x_i, x_j) v_j summed in double, used for the
//              periodic true-residual check of the solver; the float64 sums
//              run on v_mfma_f64_16x16x4f64 (mfma64_rows) while the vector
//              units compute the float32 entries.
// float32: one thread owns output rows; column points (already divided by the
// lengthscale) and right-hand sides stream through LDS in stages of 64.
// A grid of (row block, column split) work groups writes partial sums that a
// fixed-order reduction adds up.

#include <math.h>

#include "device_common.h"
#include "internal.h"
#include "valu_tile.h"

namespace gpmi {
namespace valu {


template <int KIND, int DM, int RT, int RPT, typename AccT>
__global__ __launch_bounds__(256) void kmvm_valu_kernel(const float* __restrict__ X1, int64_t n1,
                                                        const float* __restrict__ X2, int64_t n2,
                                                        const float* __restrict__ V, int r, int c0,
                                                        KParams kp, AccT* __restrict__ part,
                                                        int nsplit, const int* __restrict__ live) {
  __shared__ float sX[JT][DM];
  __shared__ AccT sV[JT][RT];
  if (live && *live == 0) return;
  const int split = blockIdx.x % nsplit;
  const int64_t row_blk = (int64_t)(blockIdx.x / nsplit) * kRowsPerBlock * RPT;
  const int64_t nstage = ceil_div(n2, JT);
  const int64_t sb = split * nstage / nsplit;
  const int64_t se = (split + 1) * nstage / nsplit;
  valu_rows<KIND, DM, RT, RPT, AccT>(X1, n1, X2, n2, V, r, c0, kp.d, kp.ls,
                                     part + (int64_t)split * n1 * r, row_blk, sb, se, sX, sV);
}

template <int KIND, int DM>
__global__ __launch_bounds__(256) void kmvm_f64_kernel(const float* __restrict__ X1, int64_t n1,
                                                       const float* __restrict__ X2, int64_t n2,
                                                       const float* __restrict__ V, int r, int c0,
                                                       KParams kp, double* __restrict__ part,
                                                       int nsplit, const int* __restrict__ live) {
  __shared__ float sX[JT64][DM + 1];
  __shared__ double sV[JT64][16];
  if (live && *live == 0) return;
  const int split = blockIdx.x % nsplit;
  const int64_t row_blk = (int64_t)(blockIdx.x / nsplit) * f64_rows<DM>();
  const int64_t nstage = ceil_div(n2, JT64);
  const int64_t sb = split * nstage / nsplit;
  const int64_t se = (split + 1) * nstage / nsplit;
  mfma64_rows<KIND, DM>(X1, n1, X2, n2, V, r, c0, kp.d, kp.ls, part + (int64_t)split * n1 * r,
                        row_blk, sb, se, sX, sV);
}

template <int KIND, int DM>
static gp_status launch_f64(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                            int64_t n2, const float* V, int r, double* part, int nsplit,
                            const int* live, hipStream_t s) {
  const int64_t blocks = ceil_div(n1, (int64_t)f64_rows<DM>()) * nsplit;
  for (int c0 = 0; c0 < r; c0 += 16) {
    kmvm_f64_kernel<KIND, DM><<<(unsigned)blocks, 256, 0, s>>>(X1, n1, X2, n2, V, r, c0, kp, part,
                                                               nsplit, live);
    GP_HIP(hipGetLastError());
  }
  return GP_OK;
}

template <int DM>
constexpr int rows_per_thread() {
  return DM <= 16 ? 4 : 1;
}

template <int KIND, int DM, int RT>
static gp_status launch_t(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                          int64_t n2, const float* V, int r, void* part, bool acc64, int nsplit,
                          const int* live, hipStream_t s) {
  constexpr int RPT = rows_per_thread<DM>();
  if (acc64) return launch_f64<KIND, DM>(kp, X1, n1, X2, n2, V, r, static_cast<double*>(part), nsplit, live, s);
  const int64_t blocks = ceil_div(n1, (int64_t)kRowsPerBlock * RPT) * nsplit;
  for (int c0 = 0; c0 < r; c0 += RT) {
    kmvm_valu_kernel<KIND, DM, RT, RPT, float><<<(unsigned)blocks, kRowsPerBlock, 0, s>>>(
        X1, n1, X2, n2, V, r, c0, kp, static_cast<float*>(part), nsplit, live);
    GP_HIP(hipGetLastError());
  }
  return GP_OK;
}

template <int KIND, int DM>
static gp_status launch_r(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                          int64_t n2, const float* V, int r, void* part, bool acc64, int nsplit,
                          const int* live, hipStream_t s) {
  if (r <= 1) return launch_t<KIND, DM, 1>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
  if (r <= 4) return launch_t<KIND, DM, 4>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
  if (r <= 8) return launch_t<KIND, DM, 8>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
  return launch_t<KIND, DM, 16>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
}

template <int KIND>
static gp_status launch_d(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                          int64_t n2, const float* V, int r, void* part, bool acc64, int nsplit,
                          const int* live, hipStream_t s) {
  const int d = kp.d;
  if (d <= 4) return launch_r<KIND, 4>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
  if (d <= 8) return launch_r<KIND, 8>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
  if (d <= 16) return launch_r<KIND, 16>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
  if (d <= 32) return launch_r<KIND, 32>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
  return launch_r<KIND, 64>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
}

gp_status launch_partial(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                         int64_t n2, const float* V, int r, void* part, bool acc64, int nsplit,
                         const int* live, hipStream_t s) {
  if (n1 == 0 || r == 0) return GP_OK;
  switch (kp.kind) {
    case GP_KERNEL_RBF:
      return launch_d<GP_KERNEL_RBF>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
    case GP_KERNEL_MATERN52:
      return launch_d<GP_KERNEL_MATERN52>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
    case GP_KERNEL_MATERN12:
      return launch_d<GP_KERNEL_MATERN12>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
    case GP_KERNEL_MATERN32:
      return launch_d<GP_KERNEL_MATERN32>(kp, X1, n1, X2, n2, V, r, part, acc64, nsplit, live, s);
  }
  return set_error(GP_ERR_ARG, "unknown kernel kind %d", kp.kind);
}

__global__ void reduce32_kernel(const float* __restrict__ part, int nsplit, int64_t n1, int r,
                                float a2, float s2, const float* __restrict__ V,
                                float* __restrict__ out, const int* __restrict__ live) {
  if (live && *live == 0) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = n1 * r;
  if (e >= total) return;
  float acc = 0.0f;
  for (int x = 0; x < nsplit; ++x) acc += part[(int64_t)x * total + e];
  float o = a2 * acc;
  if (V) o = fmaf(s2, V[e], o);
  out[e] = o;
}

gp_status launch_reduce32(const float* part, int nsplit, int64_t n1, int r, float a2, float s2,
                          const float* V, float* out, const int* live, hipStream_t s) {
  const int64_t total = n1 * r;
  if (total == 0) return GP_OK;
  reduce32_kernel<<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(part, nsplit, n1, r, a2, s2, V,
                                                                 out, live);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

int choose_splits64(int64_t n1, int64_t n2, int d) {
  const int64_t rblocks = ceil_div(n1, (int64_t)f64_rows_for(d));
  const int64_t nstage = ceil_div(n2, JT64);
  int64_t want = ceil_div(1024, std::max<int64_t>(rblocks, 1));
  want = std::min<int64_t>(want, 64);
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, nstage));
}

int choose_splits(int64_t n1, int64_t n2, int d) {
  const int64_t rblocks = ceil_div(n1, (int64_t)kRowsPerBlock * (d <= 16 ? 4 : 1));
  const int64_t nstage = ceil_div(n2, JT);
  int64_t want = ceil_div(1024, std::max<int64_t>(rblocks, 1));
  want = std::min<int64_t>(want, 64);
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, nstage));
}

}  // namespace valu
}  // namespace gpmi
