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
// Squared distances from augmented float64 vectors on the matrix cores: with
// a = x_i / l and b = x_j / l (float64), the row vector (a, 1, |a|^2) and the
// column vector (-2b, |b|^2, 1) have the dot product |a - b|^2, which
// v_mfma_f64_16x16x4f64 forms from exact float64 products (error of order
// 1e-16 |a|^2, far below the float32 rounding of the entry).  The kernel value
// k = f(r^2) is evaluated in float32 (kval32_direct), and every product
// k(x_i, x_j) v_j is summed in float64 by a second v_mfma_f64_16x16x4f64: the
// products of float32 values are exact in float64, so the only rounding after
// the entry is float64 summation.  The augmented width d + 2 is padded to 4T.
//
// Lane layouts (wave of 64, l16 = lane % 16, g = lane / 16; A: lane holds
// A[l16][g]; B: B[g][l16]; D: lane l, element v holds D[g + 4v][l16], checked
// against a host product on the device): the distance MFMA takes A[j][k] =
// column slice (lane: column l16, slot 4t + g) and B[k][i] = row slice (lane:
// row l16, slot 4t + g); its element v of lane l is r^2(row l16, column
// g + 4v).  That is already the A layout of the product MFMA for the column
// order (g + 4v): lane l supplies k(row l16, column g + 4v) and the B operand
// takes v_j of column g + 4v, right-hand side l16.  The product's element v of
// lane l is row g + 4v, right-hand side l16.
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int JT64 = 64;                       // columns per LDS stage

__host__ __device__ constexpr int aug_slices_of(int d) { return (d + 2 + 3) / 4; }
// the instantiated slice counts: exact up to T = 8 (d <= 30), padded above
__host__ __device__ constexpr int aug_slices_inst(int d) {
  return aug_slices_of(d) <= 8 ? aug_slices_of(d) : aug_slices_of(d) <= 10 ? 10
         : aug_slices_of(d) <= 12 ? 12 : aug_slices_of(d) <= 14 ? 14 : 17;
}
__host__ __device__ constexpr int aug_subtiles(int t) { return t <= 5 ? 4 : t <= 9 ? 2 : 1; }
// rows per 256-thread work group
__host__ __device__ constexpr int aug_rows(int t) { return 64 * aug_subtiles(t); }

// LDS of one work group: column slices (slot-major, sA[slot * JT64 + column]),
// right-hand sides as float64, the reciprocal lengthscales.
template <int T>
struct Aug64Lds {
  double A[4 * T * JT64];
  double V[JT64][16];
  double inv[kMaxDim];
};

// One work group (256 threads): rows [row_blk, row_blk + aug_rows(T)) against
// column stages [sb, se) of JT64 columns, right-hand sides [c0, c0 + 16) of V
// (row stride r); float64 partial sums to P[i * r + c].  All threads of the
// group must call it (it synchronises).
template <int KIND, int T>
__device__ __forceinline__ void aug64_rows(const float* __restrict__ X1, int64_t n1,
                                           const float* __restrict__ X2, int64_t n2,
                                           const float* __restrict__ V, int r, int c0, int d,
                                           const float* __restrict__ ls, double* __restrict__ P,
                                           int64_t row_blk, int64_t sb, int64_t se,
                                           Aug64Lds<T>& sm) {
  constexpr int NSUB = aug_subtiles(T);
  constexpr int W = 4 * T;
  __syncthreads();
  for (int m = threadIdx.x; m < d; m += blockDim.x) sm.inv[m] = 1.0 / (double)ls[m];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int64_t row0 = row_blk + (int64_t)wave * 16 * NSUB;
  const int rc = min(16, r - c0);

  // row slices (a, 1, |a|^2, 0 ...): lane holds slots 4t + g of row l16
  double ra[NSUB][T];
#pragma unroll
  for (int q = 0; q < NSUB; ++q) {
    const int64_t i = row0 + 16 * q + l16;
    double nrm = 0.0;
    if (i < n1)
      for (int m = 0; m < d; ++m) {
        const double a = (double)X1[i * d + m] * sm.inv[m];
        nrm = fma(a, a, nrm);
      }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int k = 4 * t + g;
      double v = 0.0;
      if (i < n1) v = k < d ? (double)X1[i * d + k] * sm.inv[k] : k == d ? 1.0 : k == d + 1 ? nrm : 0.0;
      ra[q][t] = v;
    }
  }
  d4 acc[NSUB];
#pragma unroll
  for (int q = 0; q < NSUB; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};

  for (int64_t st = sb; st < se; ++st) {
    const int64_t j0 = st * JT64;
    const int jn = (int)min<int64_t>(JT64, n2 - j0);
    __syncthreads();
    // column coordinates of the stage (contiguous in X2): slot m <- -2 b_m
    for (int e = threadIdx.x; e < JT64 * d; e += blockDim.x) {
      const int jj = e / d, m = e - jj * d;
      sm.A[m * JT64 + jj] = jj < jn ? -2.0 * ((double)X2[j0 * d + e] * sm.inv[m]) : 0.0;
    }
    for (int e = threadIdx.x; e < JT64 * 16; e += blockDim.x) {
      const int jj = e >> 4, c = e & 15;
      sm.V[jj][c] = (jj < jn && c < rc) ? (double)V[(j0 + jj) * r + c0 + c] : 0.0;
    }
    __syncthreads();
    // slots d, d + 1 (|b|^2, 1) and the zero padding; a padded column is all
    // zero, so its distance is 0, its entry finite, and its right-hand side 0
    if (threadIdx.x < JT64) {
      const int jj = threadIdx.x;
      double nb = 0.0;
      for (int m = 0; m < d; ++m) {
        const double b = 0.5 * sm.A[m * JT64 + jj];
        nb = fma(b, b, nb);
      }
      const bool in = jj < jn;
      for (int k = d; k < W; ++k) sm.A[k * JT64 + jj] = !in ? 0.0 : k == d ? nb : k == d + 1 ? 1.0 : 0.0;
    }
    __syncthreads();
#pragma unroll 1
    for (int jb = 0; jb < JT64 / 16; ++jb) {
      double at[T];
#pragma unroll
      for (int t = 0; t < T; ++t) at[t] = sm.A[(4 * t + g) * JT64 + 16 * jb + l16];
      double vb[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) vb[v] = sm.V[16 * jb + g + 4 * v][l16];
#pragma unroll
      for (int q = 0; q < NSUB; ++q) {
        d4 r2 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < T; ++t) r2 = __builtin_amdgcn_mfma_f64_16x16x4f64(at[t], ra[q][t], r2, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // r^2 of a pair at (nearly) zero distance can come out a few float64
          // ulps below zero: harmless in the exponential, clamped before a root
          float r2f = (float)r2[v];
          if constexpr (KIND != GP_KERNEL_RBF) r2f = r2f > 0.0f ? r2f : 0.0f;
          const double kv = (double)kval32_direct<KIND>(r2f);
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(kv, vb[v], acc[q], 0, 0, 0);
        }
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
