// Device pieces of the preconditioner apply (Sec. 5.2, Eq. woodbury), shared
// by the single-problem and batched kernels:
//   T = L^T w   skinny product with a huge reduction dimension, on the
//               float32 matrix cores (v_mfma_f32_16x16x4f32);
//   z = s^-2 w - s^-4 L Y   one thread per row, Y staged in LDS.
// L is rank x n (each pivot column contiguous), w and z are n x r.
#pragma once

#include "internal.h"

namespace gpmi {
namespace pc {

typedef float pf4 __attribute__((ext_vector_type(4)));

constexpr int kLtMaxChunks = 1024;  // row chunks of the single-problem L^T w
constexpr int kLtChunkRows = 128;   // rows per chunk of the single-problem L^T w
constexpr int kLtResidentChunks = 512;  // 2 work groups x 256 compute units

// Work group (256 threads): out[m * r + c] = sum_{i0 <= i < i1} L[m][i] w[i][c]
// for m < k, c < r.  Rows go in tiles of 32: the group stages the tile of L
// (k x 32) and of w (32 x r) in LDS with coalesced loads, then wave w runs the
// 16-pivot tiles w, w + 4, ... as 8 steps of a 16x16x4 product per column
// tile.  A operand (lane l): L[tile + l % 16][row], B operand:
// w[row][ctile + l % 16], row = 4 * step + l / 16; D: lane l, element v holds
// pivot tile + 4 * (l / 16) + v, column ctile + l % 16.
constexpr int kLtTile = 32;
struct LtLds {
  float L[kMaxRank][kLtTile + 1];
  float W[kLtTile][64 + 1];
};

__device__ __forceinline__ void lt_chunk_mfma(const float* __restrict__ L, int64_t n, int k,
                                              const float* __restrict__ w, int r, int64_t i0,
                                              int64_t i1, float* __restrict__ out, LtLds& sm) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int kt = (k + 15) / 16, ct = (r + 15) / 16;
  pf4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[a][t] = pf4{0.f, 0.f, 0.f, 0.f};
  // The next tile's staging loads are issued into registers before the
  // current tile's products, so their latency overlaps the matrix work (every
  // load of a tile in flight at once: k * 64 / 256 <= 32 of L and at most 16
  // of w per thread).
  constexpr int kPerL = kMaxRank * kLtTile / 256;
  constexpr int kPerW = kLtTile * 64 / 256;
  float bufL[kPerL], bufW[kPerW];
  auto load_tile = [&](int64_t t0) {
    const int rows = (int)min<int64_t>(kLtTile, i1 - t0);
#pragma unroll
    for (int u = 0; u < kPerL; ++u) {
      const int e = u * 256 + threadIdx.x;
      const int m = e / kLtTile, ii = e % kLtTile;
      bufL[u] = (e < k * kLtTile && ii < rows) ? L[(int64_t)m * n + t0 + ii] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kPerW; ++u) {
      const int e = u * 256 + threadIdx.x;
      const int ii = e / r, c = e % r;
      bufW[u] = (e < kLtTile * r && ii < rows) ? w[(t0 + ii) * r + c] : 0.0f;
    }
  };
  if (i0 < i1) load_tile(i0);
  for (int64_t t0 = i0; t0 < i1; t0 += kLtTile) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPerL; ++u) {
      const int e = u * 256 + threadIdx.x;
      if (e < k * kLtTile) sm.L[e / kLtTile][e % kLtTile] = bufL[u];
    }
#pragma unroll
    for (int u = 0; u < kPerW; ++u) {
      const int e = u * 256 + threadIdx.x;
      if (e < kLtTile * r) sm.W[e / r][e % r] = bufW[u];
    }
    for (int e = threadIdx.x; e < kLtTile * (ct * 16 - r); e += 256) {
      const int span = ct * 16 - r;
      sm.W[e / span][r + e % span] = 0.0f;   // zero column padding
    }
    __syncthreads();
    if (t0 + kLtTile < i1) load_tile(t0 + kLtTile);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int mt = wave + 4 * a;
      if (mt < kt) {
        const int m = mt * 16 + l16;
#pragma unroll 4
        for (int st = 0; st < kLtTile / 4; ++st) {
          const int row = 4 * st + g;
          const float av = m < k ? sm.L[m][row] : 0.0f;
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (t < ct)
              acc[a][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, sm.W[row][t * 16 + l16], acc[a][t], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int mt = wave + 4 * a;
    if (mt >= kt) continue;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < ct) {
        const int c = t * 16 + l16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int mm = mt * 16 + 4 * g + v;
          if (mm < k && c < r) out[mm * r + c] = acc[a][t][v];
        }
      }
    }
  }
}

// sum_{g0 <= q < g1} base[q * stride] in float64, in increasing q, with the
// loads issued eight at a time.
__device__ __forceinline__ double sum_strided(const float* __restrict__ base, int64_t stride,
                                              int g0, int g1) {
  double acc = 0.0;
  int q = g0;
  for (; q + 8 <= g1; q += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = base[(int64_t)(q + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (double)v[u];
  }
  for (; q < g1; ++q) acc += (double)base[(int64_t)q * stride];
  return acc;
}

// acc - sum_{t < m} L[t][i] lp[t] in increasing t (one FMA each), with eight
// loads of L in flight ahead of their FMAs.
__device__ __forceinline__ double sub_lrow(const double* __restrict__ L, int64_t n, int64_t i,
                                           const double* __restrict__ lp, int m, double acc) {
  int t = 0;
  for (; t + 8 <= m; t += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = L[(int64_t)(t + u) * n + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fma(-v[u], lp[t + u], acc);
  }
  for (; t < m; ++t) acc = fma(-L[(int64_t)t * n + i], lp[t], acc);
  return acc;
}

// sy[m * rp + c] = Y[m * r + c] (zero for r <= c < rp); rp a multiple of 16.
__device__ __forceinline__ void stage_y(const float* __restrict__ Y, int k, int r, int rp,
                                        float* __restrict__ sy) {
  for (int e = threadIdx.x; e < k * rp; e += blockDim.x) {
    const int m = e / rp, c = e % rp;
    sy[e] = c < r ? Y[m * r + c] : 0.0f;
  }
}

// z[i][c] = s^-2 w[i][c] - s^-4 sum_m L[m][i] Y[m][c] for one row i.
__device__ __forceinline__ void z_row(const float* __restrict__ L, int64_t n, int k,
                                      const float* __restrict__ sy, int rp,
                                      const float* __restrict__ w, float* __restrict__ z, int r,
                                      int64_t i, float inv_s2, float inv_s4) {
  for (int c0 = 0; c0 < rp; c0 += 16) {
    float acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = 0.0f;
    auto step = [&](float l, int m) {
      const pf4* y4 = reinterpret_cast<const pf4*>(sy + m * rp + c0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const pf4 y = y4[q];
        acc[4 * q + 0] = fmaf(l, y[0], acc[4 * q + 0]);
        acc[4 * q + 1] = fmaf(l, y[1], acc[4 * q + 1]);
        acc[4 * q + 2] = fmaf(l, y[2], acc[4 * q + 2]);
        acc[4 * q + 3] = fmaf(l, y[3], acc[4 * q + 3]);
      }
    };
    // sixteen loads of L in flight before their (in-order) accumulation
    int m = 0;
    for (; m + 16 <= k; m += 16) {
      float l[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) l[u] = L[(int64_t)(m + u) * n + i];
#pragma unroll
      for (int u = 0; u < 16; ++u) step(l[u], m + u);
    }
    for (; m < k; ++m) step(L[(int64_t)m * n + i], m);
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int cc = c0 + c;
      if (cc < r) z[i * r + cc] = inv_s2 * w[i * r + cc] - inv_s4 * acc[c];
    }
  }
}

// Cholesky factorisation C = L L^T of a k x k float64 matrix (k <= kMaxRank)
// and its inverse C^-1 = L^-T L^-1, by one work group of at least kMaxRank
// threads with the matrix held in LDS (A, k * k doubles): right-looking
// factorisation (pivot, column scale, trailing update); the lower factor
// inverted in place row by row (row i of L^-1 from the rows above it); then
// C^-1 = (L^-1)^T L^-1, each entry a dot product over the rows below its
// indices (the same terms in the same order for (a, c) and (c, a), so the
// result is exactly symmetric).  *not_pd is set when a pivot is not > 0.
__device__ __forceinline__ void chol_inverse(const double* __restrict__ C,
                                             double* __restrict__ Cinv, int k, double* A,
                                             int* not_pd) {
  const int t = threadIdx.x, nt = blockDim.x;
  for (int e = t; e < k * k; e += nt) A[e] = C[e];
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (t == 0) {
      const double dj = A[j * k + j];
      if (!(dj > 0.0)) *not_pd = 1;
      A[j * k + j] = sqrt(fmax(dj, 1e-300));
    }
    __syncthreads();
    const double piv = A[j * k + j];
    for (int i = j + 1 + t; i < k; i += nt) A[i * k + j] /= piv;
    __syncthreads();
    const int m = k - j - 1;
    for (int e = t; e < m * m; e += nt) {
      const int i = j + 1 + e / m, l = j + 1 + e % m;
      if (l <= i) A[i * k + l] = fma(-A[i * k + j], A[l * k + j], A[i * k + l]);
    }
    __syncthreads();
  }
  // row i of M = L^-1: M_ij = -(sum_{j <= m < i} L_im M_mj) / L_ii (j < i), M_ii = 1 / L_ii
  for (int i = 0; i < k; ++i) {
    const double inv = 1.0 / A[i * k + i];
    double v = 0.0;
    if (t < i) {
      double s = 0.0;
      for (int m = t; m < i; ++m) s = fma(A[i * k + m], A[m * k + t], s);
      v = -s * inv;
    }
    __syncthreads();
    if (t < i) A[i * k + t] = v;
    if (t == i) A[i * k + i] = inv;
    __syncthreads();
  }
  for (int e = t; e < k * k; e += nt) {
    const int a = e / k, c = e % k;
    double s = 0.0;
    for (int b = a > c ? a : c; b < k; ++b) s = fma(A[b * k + a], A[b * k + c], s);
    Cinv[e] = s;
  }
}

}  // namespace pc
}  // namespace gpmi
