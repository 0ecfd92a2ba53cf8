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

}  // namespace valu
}  // namespace gpmi
