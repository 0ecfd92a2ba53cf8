// Gradient of the pseudo-loss (Sec. 5.3, Eq. approx) from the solutions of
// one multi-right-hand-side solve (Eq. cg).
//
// With B = [y, z_1..z_M] and U = K~^{-1} B (both n x r, r = M + 1), Eq. (approx)
// is sum_ij dK~_ij/dtheta W_ij for the n x n matrix
//     W = U C^T,   C = [-u_0 / 2, z_1 / (2M), ..., z_M / (2M)],
// which is never formed: the fused kernel computes 16 x 16 tiles of W on the
// float32 matrix cores (v_mfma_f32_16x16x4f32, contraction over the r columns)
// and, for each entry, the kernel value and its lengthscale derivative from
// direct float32 differences of the scaled points:
//     dk/dl_m = a^2 G(r) (x~_im - x~_jm)^2 / l_m,   x~ = x / l,
//     G = kappa (RBF), 5/3 (1 + sqrt5 r) e^{-sqrt5 r} (Matern-5/2),
//         3 e^{-sqrt3 r} (Matern-3/2), e^{-r} / r (Matern-1/2, 0 at r = 0),
// so every work group accumulates S_m = sum G W (x~_m - x~'_m)^2 (m < d; one
// sum of G W r^2 for an isotropic lengthscale) and S_k = sum kappa W.  The
// noise derivative is the identity (sum_i W_ii) and the outputscale
// derivative is kappa, so
//     dL/dl_m = a^2 S_m / l_m,  dL/da^2 = S_k,  dL/ds^2 = sum_i W_ii.
// Each lane sums its entries in float32 over the columns of its split; lanes,
// waves and work groups are combined in float64 in a fixed order, so the
// result is deterministic.  A row range [i0, i1) restricts the left index i
// (a partition of the rows adds up to the whole gradient).

#include <math.h>

#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace gpmi {
namespace grad {

namespace {

typedef float gf4 __attribute__((ext_vector_type(4)));

constexpr int kStage = 64;        // columns per LDS stage
constexpr int kDiagRows = 4096;   // rows per diagonal-term chunk

// Kernel value kappa and derivative factor G at scaled squared distance r2.
template <int KIND>
__device__ __forceinline__ void kval_deriv(float r2, float& kap, float& G) {
  if constexpr (KIND == GP_KERNEL_RBF) {
    kap = exp_neg_fast(0.5f * r2);
    G = kap;
  } else {
    const float r = __builtin_amdgcn_sqrtf(r2);
    if constexpr (KIND == GP_KERNEL_MATERN12) {
      const float e = exp_neg_fast(r);
      kap = e;
      G = r2 > 0.0f ? e * __builtin_amdgcn_rcpf(r) : 0.0f;
    } else if constexpr (KIND == GP_KERNEL_MATERN32) {
      const float t = 1.7320508075688772f * r;
      const float e = exp_neg_fast(t);
      kap = (1.0f + t) * e;
      G = 3.0f * e;
    } else {
      const float t = 2.23606797749979f * r;
      const float e = exp_neg_fast(t);
      kap = fmaf(t, fmaf(t, 1.0f / 3.0f, 1.0f), 1.0f) * e;
      G = (5.0f / 3.0f) * (1.0f + t) * e;
    }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One work group = 4 waves x NSUB subtiles of 16 rows against the column
// stages of its split.  MFMA lane layouts (v_mfma_f32_16x16x4f32): A operand
// lane l holds A[l % 16][l / 16], B operand B[l / 16][l % 16], result lane l
// element v holds D[4 (l / 16) + v][l % 16].  Here A = U rows (k = column of
// U), B = C^T, so lane l's four results are W[4 (l/16) + v][l % 16].
template <int KIND, int DM, int RP, bool ISO, int NSUB>
__global__ __launch_bounds__(256) void grad_kernel(const float* __restrict__ X,
                                                   const float* __restrict__ U,
                                                   const float* __restrict__ B, int r,
                                                   float inv2m, int64_t n, int64_t i0, int64_t i1,
                                                   KParams kp, double* __restrict__ part,
                                                   int nsplit) {
  constexpr int NS = RP / 4;
  constexpr int NACC = ISO ? 1 : DM;
  __shared__ __align__(16) float sX[kStage][DM];
  __shared__ __align__(16) float sC[kStage][4][NS];   // sC[j][g][s] = C[j][4 s + g]
  __shared__ double sRed[4][NACC + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int d = kp.d;
  const int split = blockIdx.x % nsplit;
  const int64_t rblk = blockIdx.x / nsplit;
  const int64_t roww = i0 + rblk * (64 * NSUB) + (int64_t)wave * 16 * NSUB;

  float ua[NSUB][NS];
  float a[NSUB][4][DM];
#pragma unroll
  for (int q = 0; q < NSUB; ++q) {
    const int64_t ia = roww + 16 * q + l16;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int c = 4 * s + g;
      ua[q][s] = (ia < i1 && c < r) ? U[ia * r + c] : 0.0f;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t id = roww + 16 * q + 4 * g + v;
#pragma unroll
      for (int m = 0; m < DM; ++m) a[q][v][m] = (id < i1 && m < d) ? X[id * d + m] / kp.ls[m] : 0.0f;
    }
  }
  float acc[NACC];
#pragma unroll
  for (int m = 0; m < NACC; ++m) acc[m] = 0.0f;
  float acck = 0.0f;

  const int64_t nstage = ceil_div(n, kStage);
  const int64_t sb = split * nstage / nsplit;
  const int64_t se = (split + 1) * nstage / nsplit;
  for (int64_t st = sb; st < se; ++st) {
    const int64_t j0 = st * kStage;
    __syncthreads();
    for (int e = threadIdx.x; e < kStage * DM; e += 256) {
      const int jj = e / DM, m = e % DM;
      const int64_t j = j0 + jj;
      sX[jj][m] = (j < n && m < d) ? X[j * d + m] / kp.ls[m] : 0.0f;
    }
    for (int e = threadIdx.x; e < kStage * RP; e += 256) {
      const int jj = e / RP, c = e % RP;
      const int64_t j = j0 + jj;
      float val = 0.0f;
      if (j < n && c < r) val = c == 0 ? -0.5f * U[j * r] : inv2m * B[j * r + c];
      sC[jj][c & 3][c >> 2] = val;
    }
    __syncthreads();
#pragma unroll 1
    for (int t = 0; t < kStage / 16; ++t) {
      const int jj = 16 * t + l16;
      float b[DM];
#pragma unroll
      for (int m4 = 0; m4 < DM; m4 += 4) {
        const gf4 x4 = *reinterpret_cast<const gf4*>(&sX[jj][m4]);
        b[m4] = x4[0];
        b[m4 + 1] = x4[1];
        b[m4 + 2] = x4[2];
        b[m4 + 3] = x4[3];
      }
      float cb[NS];
#pragma unroll
      for (int s4 = 0; s4 < NS; s4 += 4) {
        const gf4 c4 = *reinterpret_cast<const gf4*>(&sC[jj][g][s4]);
        cb[s4] = c4[0];
        cb[s4 + 1] = c4[1];
        cb[s4 + 2] = c4[2];
        cb[s4 + 3] = c4[3];
      }
#pragma unroll
      for (int q = 0; q < NSUB; ++q) {
        gf4 W = gf4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < NS; ++s) W = __builtin_amdgcn_mfma_f32_16x16x4f32(ua[q][s], cb[s], W, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float q2[ISO ? 1 : DM];
          float r2 = 0.0f;
#pragma unroll
          for (int m = 0; m < DM; ++m) {
            const float dl = a[q][v][m] - b[m];
            if constexpr (ISO) {
              r2 = fmaf(dl, dl, r2);
            } else {
              q2[m] = dl * dl;
              r2 += q2[m];
            }
          }
          float kap, G;
          kval_deriv<KIND>(r2, kap, G);
          acck = fmaf(kap, W[v], acck);
          const float P = G * W[v];
          if constexpr (ISO) {
            acc[0] = fmaf(P, r2, acc[0]);
          } else {
#pragma unroll
            for (int m = 0; m < DM; ++m) acc[m] = fmaf(P, q2[m], acc[m]);
          }
        }
      }
    }
  }
  // float64 combination: lanes, then the four waves in order
#pragma unroll
  for (int m = 0; m < NACC; ++m) {
    const double s = wave_sum((double)acc[m]);
    if (lane == 0) sRed[wave][m] = s;
  }
  {
    const double s = wave_sum((double)acck);
    if (lane == 0) sRed[wave][NACC] = s;
  }
  __syncthreads();
  if (threadIdx.x <= NACC) {
    const int k = threadIdx.x;
    part[(int64_t)blockIdx.x * (NACC + 1) + k] = ((sRed[0][k] + sRed[1][k]) + sRed[2][k]) + sRed[3][k];
  }
}

// Per chunk of kDiagRows rows: sum_i W_ii and sum_i y_i u_0i, float64.
__global__ __launch_bounds__(256) void diag_kernel(const float* __restrict__ U,
                                                   const float* __restrict__ B, int r, float inv2m,
                                                   int64_t i0, int64_t i1,
                                                   double* __restrict__ dpart) {
  __shared__ double sRed[2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t c0 = i0 + (int64_t)blockIdx.x * kDiagRows;
  const int64_t c1 = std::min<int64_t>(i1, c0 + kDiagRows);
  double w = 0.0, fit = 0.0;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += 256) {
    const float* Ui = U + i * r;
    const float* Bi = B + i * r;
    const double u0 = Ui[0];
    double s = 0.0;
    for (int c = 1; c < r; ++c) s += (double)Ui[c] * (double)Bi[c];
    w += (double)inv2m * s - 0.5 * u0 * u0;
    fit += (double)Bi[0] * u0;
  }
  w = wave_sum(w);
  fit = wave_sum(fit);
  if (lane == 0) {
    sRed[0][wave] = w;
    sRed[1][wave] = fit;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int k = threadIdx.x;
    dpart[2 * (int64_t)blockIdx.x + k] = ((sRed[k][0] + sRed[k][1]) + sRed[k][2]) + sRed[k][3];
  }
}

// One work group: fixed-order float64 sums of the partials and the final
// gradient out[0..nl) = dL/dl, out[nl] = dL/da^2, out[nl + 1] = dL/ds^2,
// out[nl + 2] = 1/2 y^T u_0.
__global__ __launch_bounds__(256) void finish_kernel(const double* __restrict__ part, int nblk,
                                                     int nacc, const double* __restrict__ dpart,
                                                     int nchunk, KParams kp, int ard,
                                                     double* __restrict__ out) {
  __shared__ double sv[256];
  __shared__ double sums[kMaxDim + 3];
  for (int k = 0; k < nacc + 1 + 2; ++k) {
    double acc = 0.0;
    if (k <= nacc) {
      for (int b = threadIdx.x; b < nblk; b += 256) acc += part[(int64_t)b * (nacc + 1) + k];
    } else {
      for (int b = threadIdx.x; b < nchunk; b += 256) acc += dpart[2 * b + (k - nacc - 1)];
    }
    sv[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) sv[threadIdx.x] += sv[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) sums[k] = sv[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double a2 = kp.a2;
    int nl;
    if (ard) {
      nl = kp.d;
      for (int m = 0; m < kp.d; ++m) out[m] = a2 * sums[m] / (double)kp.ls[m];
    } else {
      nl = 1;
      double s = 0.0;
      for (int m = 0; m < nacc; ++m) s += sums[m];
      out[0] = a2 * s / (double)kp.ls[0];
    }
    out[nl] = sums[nacc];
    out[nl + 1] = sums[nacc + 1];
    out[nl + 2] = 0.5 * sums[nacc + 2];
  }
}

template <int DM>
constexpr int nsub_for() { return DM <= 16 ? 2 : 1; }

template <int KIND, int DM, int RP, bool ISO>
gp_status launch_t(const KParams& kp, const float* X, int64_t n, const float* U, const float* B,
                   int r, float inv2m, int64_t i0, int64_t i1, double* part, int nsplit,
                   hipStream_t s) {
  constexpr int NSUB = nsub_for<DM>();
  const int64_t blocks = ceil_div(i1 - i0, (int64_t)64 * NSUB) * nsplit;
  grad_kernel<KIND, DM, RP, ISO, NSUB><<<(unsigned)blocks, 256, 0, s>>>(X, U, B, r, inv2m, n, i0, i1,
                                                                       kp, part, nsplit);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

template <int KIND, int DM>
gp_status launch_r(const KParams& kp, bool iso, const float* X, int64_t n, const float* U,
                   const float* B, int r, float inv2m, int64_t i0, int64_t i1, double* part,
                   int nsplit, hipStream_t s) {
  if (r <= 16) {
    if (iso) return launch_t<KIND, DM, 16, true>(kp, X, n, U, B, r, inv2m, i0, i1, part, nsplit, s);
    return launch_t<KIND, DM, 16, false>(kp, X, n, U, B, r, inv2m, i0, i1, part, nsplit, s);
  }
  if (iso) return launch_t<KIND, DM, 64, true>(kp, X, n, U, B, r, inv2m, i0, i1, part, nsplit, s);
  return launch_t<KIND, DM, 64, false>(kp, X, n, U, B, r, inv2m, i0, i1, part, nsplit, s);
}

template <int KIND>
gp_status launch_d(const KParams& kp, bool iso, const float* X, int64_t n, const float* U,
                   const float* B, int r, float inv2m, int64_t i0, int64_t i1, double* part,
                   int nsplit, hipStream_t s) {
  const int d = kp.d;
  if (d <= 4) return launch_r<KIND, 4>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, s);
  if (d <= 8) return launch_r<KIND, 8>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, s);
  if (d <= 16) return launch_r<KIND, 16>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, s);
  return launch_r<KIND, 32>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, s);
}

int dm_of(int d) { return d <= 4 ? 4 : d <= 8 ? 8 : d <= 16 ? 16 : 32; }

}  // namespace

int64_t row_blocks(int64_t rows, int d) {
  const int dm = dm_of(d);
  return ceil_div(rows, (int64_t)64 * (dm <= 16 ? 2 : 1));
}

int choose_splits(int64_t rows, int64_t n, int d) {
  const int64_t rb = std::max<int64_t>(row_blocks(rows, d), 1);
  const int64_t nstage = std::max<int64_t>(ceil_div(n, kStage), 1);
  int64_t want = ceil_div(4096, rb);
  want = std::min<int64_t>(want, 64);
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, nstage));
}

size_t workspace_bytes(int64_t rows, int64_t n, int d) {
  const int64_t nblk = row_blocks(rows, d) * choose_splits(rows, n, d);
  const int64_t nchunk = ceil_div(std::max<int64_t>(rows, 1), kDiagRows);
  return 8 * (size_t)nblk * (kMaxDim + 1) + 16 * (size_t)nchunk + 1024;
}

gp_status launch(const KParams& kp, bool ard, const float* X, int64_t n, const float* U,
                 const float* B, int r, int64_t i0, int64_t i1, double* out, Arena& ar,
                 hipStream_t s) {
  const int64_t rows = i1 - i0;
  const int nsplit = choose_splits(rows, n, kp.d);
  const int64_t nblk = rows > 0 ? row_blocks(rows, kp.d) * nsplit : 0;
  const int64_t nchunk = ceil_div(rows, kDiagRows);
  const int nacc = ard ? dm_of(kp.d) : 1;
  double* part = ar.take<double>((size_t)std::max<int64_t>(nblk, 1) * (nacc + 1));
  double* dpart = ar.take<double>((size_t)std::max<int64_t>(nchunk, 1) * 2);
  if (!part || !dpart) return set_error(GP_ERR_NOMEM, "internal: gradient workspace sizing");
  const float inv2m = (float)(0.5 / (double)(r - 1));
  const bool iso = !ard;
  if (rows > 0) {
    gp_status st;
    switch (kp.kind) {
      case GP_KERNEL_RBF:
        st = launch_d<GP_KERNEL_RBF>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, s);
        break;
      case GP_KERNEL_MATERN52:
        st = launch_d<GP_KERNEL_MATERN52>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, s);
        break;
      case GP_KERNEL_MATERN32:
        st = launch_d<GP_KERNEL_MATERN32>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, s);
        break;
      case GP_KERNEL_MATERN12:
        st = launch_d<GP_KERNEL_MATERN12>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, s);
        break;
      default:
        return set_error(GP_ERR_ARG, "unknown kernel kind %d", kp.kind);
    }
    GP_TRY(st);
    diag_kernel<<<(unsigned)nchunk, 256, 0, s>>>(U, B, r, inv2m, i0, i1, dpart);
    GP_HIP(hipGetLastError());
  }
  finish_kernel<<<1, 256, 0, s>>>(part, (int)nblk, nacc, dpart, (int)nchunk, kp, ard ? 1 : 0, out);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

}  // namespace grad
}  // namespace gpmi
