// Kernel matrix x multi-vector product on the vector ALUs with float32 kernel
// entries (Eq. mvm).  Two accumulations:
//   float32 -- the single-precision product (the plain-CG baseline and the
//              small solves where matrix cores cannot be filled);
//   float64 -- every product k(x_i, x_j) v_j summed in double, used for the
//              true-residual check of the solver (kmvm_f64_kernel below).
// float32: one thread owns output rows; column points (already divided by the
// lengthscale) and right-hand sides stream through LDS in stages of 64.
// A grid of (row block, column split) work groups writes partial sums that a
// fixed-order reduction adds up.

#include <math.h>

#include <algorithm>

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

// ---- float64 accumulation (true residual) -------------------------------------
// aug64_rows (valu_tile.h): squared distances from augmented float64 vectors
// and every product summed on v_mfma_f64_16x16x4f64.  One work group (4 waves,
// up to 4 subtiles of 16 rows each) covers aug_rows(T) rows against the
// column stages of its split; the float64 partial sums of the split go to
// part[split][i][c].
template <int KIND, int T>
__global__ __launch_bounds__(256) void kmvm_f64_kernel(const float* __restrict__ X1, int64_t n1,
                                                       const float* __restrict__ X2, int64_t n2,
                                                       const float* __restrict__ V, int r, int c0,
                                                       KParams kp, double* __restrict__ part,
                                                       int nsplit, const int* __restrict__ live) {
  __shared__ Aug64Lds<T> sm;
  if (live && *live == 0) return;
  const int split = blockIdx.x % nsplit;
  const int64_t row_blk = (int64_t)(blockIdx.x / nsplit) * aug_rows(T);
  const int64_t nstage = ceil_div(n2, (int64_t)JT64);
  const int64_t sb = split * nstage / nsplit;
  const int64_t se = (split + 1) * nstage / nsplit;
  aug64_rows<KIND, T>(X1, n1, X2, n2, V, r, c0, kp.d, kp.ls, part + (int64_t)split * n1 * r,
                      row_blk, sb, se, sm);
}

template <int KIND, int T>
static gp_status launch_f64_t(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                              int64_t n2, const float* V, int r, double* part, int nsplit,
                              const int* live, hipStream_t s) {
  const int64_t blocks = ceil_div(n1, (int64_t)aug_rows(T)) * nsplit;
  for (int c0 = 0; c0 < r; c0 += 16) {
    kmvm_f64_kernel<KIND, T><<<(unsigned)blocks, 256, 0, s>>>(X1, n1, X2, n2, V, r, c0, kp, part,
                                                              nsplit, live);
    GP_HIP(hipGetLastError());
  }
  return GP_OK;
}

template <int KIND>
static gp_status launch_f64(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                            int64_t n2, const float* V, int r, double* part, int nsplit,
                            const int* live, hipStream_t s) {
#define GP_F64_CASE(TT) \
  case TT: return launch_f64_t<KIND, TT>(kp, X1, n1, X2, n2, V, r, part, nsplit, live, s);
  switch (aug_slices_inst(kp.d)) {
    GP_F64_CASE(1) GP_F64_CASE(2) GP_F64_CASE(3) GP_F64_CASE(4) GP_F64_CASE(5) GP_F64_CASE(6)
    GP_F64_CASE(7) GP_F64_CASE(8) GP_F64_CASE(10) GP_F64_CASE(12) GP_F64_CASE(14)
    GP_F64_CASE(17)
  }
#undef GP_F64_CASE
  return set_error(GP_ERR_ARG, "d=%d outside the float64 product's range", kp.d);
}

// Work groups resident per compute unit for the float64 product of dimension d
// (RBF instantiation; the other kernels use the same tile).
static int f64_blocks_per_cu(int d) {
  const void* f = nullptr;
#define GP_F64_FN(TT) \
  case TT: f = reinterpret_cast<const void*>(&kmvm_f64_kernel<GP_KERNEL_RBF, TT>); break;
  switch (aug_slices_inst(d)) {
    GP_F64_FN(1) GP_F64_FN(2) GP_F64_FN(3) GP_F64_FN(4) GP_F64_FN(5) GP_F64_FN(6)
    GP_F64_FN(7) GP_F64_FN(8) GP_F64_FN(10) GP_F64_FN(12) GP_F64_FN(14) GP_F64_FN(17)
  }
#undef GP_F64_FN
  int nb = 0;
  if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 256, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 4;
  }
  return std::max(1, nb);
}

template <int DM>
constexpr int rows_per_thread() {
  return DM <= 16 ? 4 : 1;
}

template <int KIND, int DM, int RT, int RPT>
static gp_status launch_rows(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                             int64_t n2, const float* V, int r, void* part, int nsplit,
                             const int* live, hipStream_t s) {
  const int64_t blocks = ceil_div(n1, (int64_t)kRowsPerBlock * RPT) * nsplit;
  for (int c0 = 0; c0 < r; c0 += RT) {
    kmvm_valu_kernel<KIND, DM, RT, RPT, float><<<(unsigned)blocks, kRowsPerBlock, 0, s>>>(
        X1, n1, X2, n2, V, r, c0, kp, static_cast<float*>(part), nsplit, live);
    GP_HIP(hipGetLastError());
  }
  return GP_OK;
}

// Work groups below which a launch with several rows per thread leaves most
// SIMDs without a wave (one work group of 4 waves per compute unit at best).
constexpr int64_t kSmallGrid = 256;

// Rows per thread: RPT rows reuse each column point read from LDS, but a
// small problem (the 2000-point plain solve: 2 row blocks x 32 splits = 64
// work groups of 4 waves) then leaves three SIMDs in four without a wave;
// below kSmallGrid work groups every thread owns one row instead (256 work
// groups there).  A row's sums are the same either
// way (same column order, same split boundaries), so the results are too.
template <int KIND, int DM, int RT>
static gp_status launch_t(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                          int64_t n2, const float* V, int r, void* part, bool acc64, int nsplit,
                          const int* live, hipStream_t s) {
  constexpr int RPT = rows_per_thread<DM>();
  (void)acc64;
  if constexpr (RPT > 1) {
    if (ceil_div(n1, (int64_t)kRowsPerBlock * RPT) * nsplit < kSmallGrid)
      return launch_rows<KIND, DM, RT, 1>(kp, X1, n1, X2, n2, V, r, part, nsplit, live, s);
  }
  return launch_rows<KIND, DM, RT, RPT>(kp, X1, n1, X2, n2, V, r, part, nsplit, live, s);
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
  if (acc64) {
    double* p64 = static_cast<double*>(part);
    switch (kp.kind) {
      case GP_KERNEL_RBF:
        return launch_f64<GP_KERNEL_RBF>(kp, X1, n1, X2, n2, V, r, p64, nsplit, live, s);
      case GP_KERNEL_MATERN52:
        return launch_f64<GP_KERNEL_MATERN52>(kp, X1, n1, X2, n2, V, r, p64, nsplit, live, s);
      case GP_KERNEL_MATERN12:
        return launch_f64<GP_KERNEL_MATERN12>(kp, X1, n1, X2, n2, V, r, p64, nsplit, live, s);
      case GP_KERNEL_MATERN32:
        return launch_f64<GP_KERNEL_MATERN32>(kp, X1, n1, X2, n2, V, r, p64, nsplit, live, s);
    }
    return set_error(GP_ERR_ARG, "unknown kernel kind %d", kp.kind);
  }
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
  const float acc = ordered_split_sum(part + e, nsplit, total, 0.0f);
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
  // Column splits s in [1, 64] by the launch's rounds per unit of work,
  // ceil(blocks / resident) / s with blocks = row blocks x s: a grid just above
  // a multiple of the resident work groups leaves most compute units idle for
  // its last round.  The fewest splits within 1% of the best cost are taken
  // (each split adds an n1 x r float64 partial to write and to reduce).
  const int64_t rblocks = ceil_div(std::max<int64_t>(n1, 1), (int64_t)aug_rows(aug_slices_inst(d)));
  const int64_t nstage = ceil_div(std::max<int64_t>(n2, 1), (int64_t)JT64);
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    cus = 256;
  }
  const int64_t resident = (int64_t)cus * f64_blocks_per_cu(d);
  const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(64, nstage));
  double best_cost = 1e300;
  for (int64_t sp = 1; sp <= smax; ++sp)
    best_cost = std::min(best_cost, (double)ceil_div(rblocks * sp, resident) / (double)sp);
  for (int64_t sp = 1; sp <= smax; ++sp)
    if ((double)ceil_div(rblocks * sp, resident) / (double)sp <= best_cost * 1.01) return (int)sp;
  return 1;
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
