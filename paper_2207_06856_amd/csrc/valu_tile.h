// Device-side body of the vector-ALU kernel-matrix product (float32 kernel
// entries, float32 or float64 accumulation), shared by the single-problem and
// batched kernels.
#pragma once

#include "device_common.h"
#include "internal.h"

namespace gpmi {
namespace valu {

constexpr int JT = kStageCols;

// DM: padded dimension held in registers; RT: right-hand sides per launch;
// RPT: output rows per thread (the column point and right-hand sides read from
// LDS are reused for all of them).  One work group: rows row_blk + t + q*256
// (q < RPT) against column stages [sb, se); partial sums go to
// P[i * r + c] for c in [c0, c0 + RT) (P already offset to the split).
template <int KIND, int DM, int RT, int RPT, typename AccT>
__device__ __forceinline__ void valu_rows(const float* __restrict__ X1, int64_t n1,
                                          const float* __restrict__ X2, int64_t n2,
                                          const float* __restrict__ V, int r, int c0, int d,
                                          const float* __restrict__ ls, AccT* __restrict__ P,
                                          int64_t row_blk, int64_t sb, int64_t se,
                                          float (*sX)[DM], AccT (*sV)[RT]) {
  const int64_t row0 = row_blk + threadIdx.x;
  const int rc = min(RT, r - c0);
  float a[RPT][DM];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t i = row0 + q * kRowsPerBlock;
#pragma unroll
    for (int m = 0; m < DM; ++m) a[q][m] = (i < n1 && m < d) ? X1[i * d + m] / ls[m] : 0.0f;
  }
  AccT acc[RPT][RT];
#pragma unroll
  for (int q = 0; q < RPT; ++q)
#pragma unroll
    for (int c = 0; c < RT; ++c) acc[q][c] = AccT(0);

  for (int64_t st = sb; st < se; ++st) {
    const int64_t j0 = st * JT;
    __syncthreads();
    for (int e = threadIdx.x; e < JT * DM; e += blockDim.x) {
      const int jj = e / DM, m = e % DM;
      const int64_t j = j0 + jj;
      sX[jj][m] = (j < n2 && m < d) ? X2[j * d + m] / ls[m] : 0.0f;
    }
    for (int e = threadIdx.x; e < JT * RT; e += blockDim.x) {
      const int jj = e / RT, c = e % RT;
      const int64_t j = j0 + jj;
      sV[jj][c] = (j < n2 && c < rc) ? AccT(V[j * r + c0 + c]) : AccT(0);
    }
    __syncthreads();
    const int jn = (int)min<int64_t>(JT, n2 - j0);
    for (int jj = 0; jj < jn; ++jj) {
      float b[DM];
#pragma unroll
      for (int m = 0; m < DM; ++m) b[m] = sX[jj][m];
      AccT v[RT];
#pragma unroll
      for (int c = 0; c < RT; ++c) v[c] = sV[jj][c];
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        float r2 = 0.0f;
#pragma unroll
        for (int m = 0; m < DM; ++m) {
          const float t = a[q][m] - b[m];
          r2 = fmaf(t, t, r2);
        }
        const AccT k = AccT(kval32<KIND>(r2));
#pragma unroll
        for (int c = 0; c < RT; ++c) acc[q][c] += k * v[c];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t i = row0 + q * kRowsPerBlock;
    if (i < n1) {
      AccT* Pi = P + i * r + c0;
#pragma unroll
      for (int c = 0; c < RT; ++c)
        if (c < rc) Pi[c] = acc[q][c];
    }
  }
}

// ---- float64 accumulation on the matrix cores (true residual) ----------------
// float32 kernel entries (kval32_direct: the same function as valu_rows'
// entries to within the float32 error of r^2, on the hardware transcendentals
// with a one-multiplication argument), summed in float64 by
// v_mfma_f64_16x16x4f64: a wave owns NSUB subtiles of 16 rows; for every 4
// columns each lane computes the one entry k(x_i, x_j) its A-operand slot
// holds (row i = lane % 16 of the subtile, column j = lane / 16 of the four)
// and the 16 x 16 x 4 product adds K_{16x4} V_{4x16} into the subtile's
// float64 accumulator.  The products of float32 values are exact in float64,
// so the only rounding is float64 summation (in a different order than a
// row-by-row loop).  Lane layouts (A: lane l holds A[l%16][l/16]; B: B[l/16][l%16];
// D: lane l, element v holds D[l/16 + 4v][l%16] -- rows interleaved, unlike the
// float32 16x16 forms) were checked against a host product on the device.
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int JT64 = 64;                       // columns per LDS stage

template <int DM>
__host__ __device__ constexpr int f64_subtiles() { return DM <= 16 ? 4 : DM <= 32 ? 2 : 1; }
// rows per 256-thread work group
template <int DM>
__host__ __device__ constexpr int f64_rows() { return 4 * 16 * f64_subtiles<DM>(); }
__host__ __device__ inline int f64_rows_for(int d) { return d <= 16 ? 256 : d <= 32 ? 128 : 64; }

// One work group (256 threads): rows [row_blk, row_blk + f64_rows<DM>()) against
// column stages [sb, se) of JT64 columns, right-hand sides [c0, c0 + 16) of V
// (row stride r); float64 partial sums to P[i * r + c].
template <int KIND, int DM>
__device__ __forceinline__ void mfma64_rows(const float* __restrict__ X1, int64_t n1,
                                            const float* __restrict__ X2, int64_t n2,
                                            const float* __restrict__ V, int r, int c0, int d,
                                            const float* __restrict__ ls, double* __restrict__ P,
                                            int64_t row_blk, int64_t sb, int64_t se,
                                            float (*sX)[DM + 1], double (*sV)[16]) {
  constexpr int NSUB = f64_subtiles<DM>();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int rc = min(16, r - c0);
  const int64_t row0 = row_blk + (int64_t)wave * 16 * NSUB;
  float a[NSUB][DM];
#pragma unroll
  for (int q = 0; q < NSUB; ++q) {
    const int64_t i = row0 + 16 * q + l16;
#pragma unroll
    for (int m = 0; m < DM; ++m) a[q][m] = (i < n1 && m < d) ? X1[i * d + m] / ls[m] : 0.0f;
  }
  d4 acc[NSUB];
#pragma unroll
  for (int q = 0; q < NSUB; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t st = sb; st < se; ++st) {
    const int64_t j0 = st * JT64;
    __syncthreads();
    for (int e = threadIdx.x; e < JT64 * DM; e += blockDim.x) {
      const int jj = e / DM, m = e % DM;
      const int64_t j = j0 + jj;
      sX[jj][m] = (j < n2 && m < d) ? X2[j * d + m] / ls[m] : 0.0f;
    }
    for (int e = threadIdx.x; e < JT64 * 16; e += blockDim.x) {
      const int jj = e / 16, c = e % 16;
      const int64_t j = j0 + jj;
      sV[jj][c] = (j < n2 && c < rc) ? (double)V[j * r + c0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 2
    for (int kb = 0; kb < JT64 / 4; ++kb) {
      const int jj = 4 * kb + g;
      float b[DM];
#pragma unroll
      for (int m = 0; m < DM; ++m) b[m] = sX[jj][m];
      const double bv = sV[jj][l16];
#pragma unroll
      for (int q = 0; q < NSUB; ++q) {
        float r2 = 0.0f;
#pragma unroll
        for (int m = 0; m < DM; ++m) {
          const float t = a[q][m] - b[m];
          r2 = fmaf(t, t, r2);
        }
        const double kv = (double)kval32_direct<KIND>(r2);
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(kv, bv, acc[q], 0, 0, 0);
      }
    }
  }
  if (l16 < rc) {
#pragma unroll
    for (int q = 0; q < NSUB; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = row0 + 16 * q + g + 4 * v;
        if (i < n1) P[i * r + c0 + l16] = acc[q][v];
      }
  }
}

}  // namespace valu
}  // namespace gpmi
