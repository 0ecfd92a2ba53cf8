// Gradient of the pseudo-loss (Sec. 5.3, Eq. approx) from the solutions of
// one multi-right-hand-side solve (Eq. cg).
//
// With B = [y, z_1..z_M] and U = K~^{-1} B (both n x r, r = M + 1), Eq. (approx)
// is sum_ij dK~_ij/dtheta W_ij for the n x n matrix
//     W = U C^T,   C = [-u_0 / 2, z_1 / (2M), ..., z_M / (2M)],
// which is never formed.  For each entry the kernel value and its lengthscale
// derivative come from float32 scaled points:
//     dk/dl_m = a^2 G(r) (x~_im - x~_jm)^2 / l_m,   x~ = x / l,
//     G = kappa (RBF), 5/3 (1 + sqrt5 r) e^{-sqrt5 r} (Matern-5/2),
//         3 e^{-sqrt3 r} (Matern-3/2), e^{-r} / r (Matern-1/2, 0 at r = 0),
// so every work group accumulates S_m = sum G W (x~_m - x~'_m)^2 (m < d; one
// sum of G W r^2 for an isotropic lengthscale) and S_k = sum kappa W.  The
// noise derivative is the identity (sum_i W_ii) and the outputscale
// derivative is kappa, so
//     dL/dl_m = a^2 S_m / l_m,  dL/da^2 = S_k,  dL/ds^2 = sum_i W_ii.
//
// Tiles of W come from the binary16 matrix cores (v_mfma_f32_16x16x32_f16)
// on a two-term split of every operand, x = hi + lo with hi = fp16(x) and
// lo = fp16(x - hi), after a power-of-two scale per column pair (U_c times s_c,
// C_c divided by s_c, balancing their largest entries) and one common power
// of two that keeps every operand below 2^15: U_hi C_hi + U_lo C_hi + U_hi C_lo
// carries about 22 bits, and the exact power of two is undone on the float32
// accumulator.  (The float32 matrix cores run at the vector-ALU rate on this
// chip and their work does not overlap the vector work; the binary16 ones do.)
// The scaled squared distance is a float32 matrix-core product of augmented
// vectors [x~_i, |x~_i|^2, 1] . [-2 x~_j, 1, |x~_j|^2] (absolute error a few
// ulps of |x~_i|^2 + |x~_j|^2, clamped at 0); the per-dimension squares
// (x~_im - x~_jm)^2 are direct float32 differences.  Matern-1/2, whose value
// changes to first order in r at r = 0, takes r^2 from those differences too.
// Each lane sums its entries in float32 over the columns of its split; lanes,
// waves and work groups are combined in float64 in a fixed order, so the
// result is deterministic.  A row range [i0, i1) restricts the left index i
// (a partition of the rows adds up to the whole gradient).
//
// Over the whole range the derivative matrices are symmetric, so
// sum_ij dK_ij W_ij = sum over i, j in the same row block of dK_ij W_ij
// + sum over j past the row block of dK_ij (W_ij + W_ji): a row block visits
// only the column stages from its own first row on, and past its own rows the
// tile of W + W^T = U C^T + C U^T takes the mirrored products as well (C rows
// times U columns).  This halves the entries whose derivative terms are
// evaluated.

#include <math.h>

#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace gpmi {
namespace grad {

namespace {

typedef float gf4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int kStage = 64;        // columns per LDS stage
constexpr int kDiagRows = 4096;   // rows per diagonal-term chunk
constexpr int kColmaxRows = 256;  // rows per column-maximum work group

// exp(-x) from the hardware exp2 (v_exp_f32): relative error about
// 1 ulp + x log2(e) 2^-24 ln 2, below 2e-6 for x <= 20 and negligible beside
// the float32 sums it feeds.
__device__ __forceinline__ float exp_neg(float x) {
  return __builtin_amdgcn_exp2f(-1.4426950408889634f * x);
}

// Kernel value kappa and derivative factor G at scaled squared distance r2.
template <int KIND>
__device__ __forceinline__ void kval_deriv(float r2, float& kap, float& G) {
  if constexpr (KIND == GP_KERNEL_RBF) {
    kap = __builtin_amdgcn_exp2f(-0.7213475204444817f * r2);   // exp(-r2 / 2)
    G = kap;
  } else {
    const float r = __builtin_amdgcn_sqrtf(r2);
    if constexpr (KIND == GP_KERNEL_MATERN12) {
      const float e = exp_neg(r);
      kap = e;
      G = r2 > 0.0f ? e * __builtin_amdgcn_rcpf(r) : 0.0f;
    } else if constexpr (KIND == GP_KERNEL_MATERN32) {
      const float t = 1.7320508075688772f * r;
      const float e = exp_neg(t);
      kap = (1.0f + t) * e;
      G = 3.0f * e;
    } else {
      const float t = 2.23606797749979f * r;
      const float e = exp_neg(t);
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

// ---- operand preparation -------------------------------------------------
// C[i][c] = -u_0i / 2 (c = 0) or z_ic / (2M) (c >= 1).
__device__ __forceinline__ float cval(const float* __restrict__ U, const float* __restrict__ B,
                                      int64_t i, int c, int r, float inv2m) {
  return c == 0 ? -0.5f * U[i * r] : inv2m * B[i * r + c];
}

// cmax[c] = max_i |U_ic|, cmax[64 + c] = max_i |C_ic| as float bits (cleared
// to zero before); one work group per kColmaxRows rows, thread t takes column
// t % 64 of every fourth row.
__global__ __launch_bounds__(256) void colmax_kernel(const float* __restrict__ U,
                                                     const float* __restrict__ B, int64_t n, int r,
                                                     float inv2m, uint32_t* __restrict__ cmax) {
  __shared__ uint32_t sm[2 * 64];
  for (int e = threadIdx.x; e < 2 * 64; e += 256) sm[e] = 0u;
  __syncthreads();
  const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * kColmaxRows;
  const int64_t c1 = std::min<int64_t>(n, c0 + kColmaxRows);
  if (c < r) {
    float mu = 0.0f, mc = 0.0f;
    for (int64_t i = c0 + rg; i < c1; i += 4) {
      mu = fmaxf(mu, fabsf(U[i * r + c]));
      mc = fmaxf(mc, fabsf(cval(U, B, i, c, r, inv2m)));
    }
    atomicMax(&sm[c], __float_as_uint(mu));
    atomicMax(&sm[64 + c], __float_as_uint(mc));
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * 64; e += 256)
    if (sm[e]) atomicMax(&cmax[e], sm[e]);
}

// One wave: scl[c] multiplies U_c and scl[64 + c] multiplies C_c, both powers
// of two with the product 2^(2 gam) for every column; scl[128] = 2^(-2 gam).
// Column c gets U_c 2^(e_c + gam), C_c 2^(gam - e_c) with e_c the rounded
// half of log2(max |C_c| / max |U_c|) (balanced largest entries, each within
// 2^0.5 of m_c = sqrt(max |U_c| max |C_c|)), and gam puts the largest m_c at or
// below 2^14.
__global__ void scale_kernel(const uint32_t* __restrict__ cmax, int r, float* __restrict__ scl) {
  __shared__ float sm[64];
  __shared__ int sgam;
  const int c = threadIdx.x;
  int e = 0;
  float m = 0.0f;
  if (c < r) {
    const float mu = __uint_as_float(cmax[c]), mc = __uint_as_float(cmax[64 + c]);
    if (mu > 0.0f && mc > 0.0f) {
      e = (int)rintf(0.5f * log2f(mc / mu));
      m = sqrtf(mu) * sqrtf(mc);
    }
  }
  if (c < 64) sm[c] = m;
  __syncthreads();
  if (c == 0) {
    float mx = 0.0f;
    for (int k = 0; k < 64; ++k) mx = fmaxf(mx, sm[k]);
    const int gam = mx > 0.0f ? 14 - (int)ceilf(log2f(mx)) : 0;
    sgam = max(-60, min(60, gam));
    scl[128] = ldexpf(1.0f, -2 * sgam);
  }
  __syncthreads();
  if (c < 64) {
    scl[c] = c < r ? ldexpf(1.0f, e + sgam) : 0.0f;
    scl[64 + c] = c < r ? ldexpf(1.0f, sgam - e) : 0.0f;
  }
}

// Per row: scaled point x~ = x / l (DM entries, zero padded), its squared norm,
// and the binary16 split H[i][w][c] of the scaled U (w = 0 hi, 1 lo) and C
// (w = 2 hi, 3 lo), zero for c >= r.
template <int DM, int RP>
__global__ __launch_bounds__(256) void split_kernel(const float* __restrict__ X,
                                                    const float* __restrict__ U,
                                                    const float* __restrict__ B, int64_t n, int r,
                                                    float inv2m, KParams kp,
                                                    const float* __restrict__ scl,
                                                    float* __restrict__ Xs, float* __restrict__ nrm,
                                                    _Float16* __restrict__ H) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.0f;
#pragma unroll
  for (int m = 0; m < DM; ++m) {
    const float v = m < kp.d ? X[i * kp.d + m] / kp.ls[m] : 0.0f;
    Xs[i * DM + m] = v;
    acc = fmaf(v, v, acc);
  }
  nrm[i] = acc;
  _Float16* Hi = H + i * 4 * RP;
  for (int c = 0; c < RP; ++c) {
    float u = 0.0f, cc = 0.0f;
    if (c < r) {
      u = U[i * r + c] * scl[c];
      cc = cval(U, B, i, c, r, inv2m) * scl[64 + c];
    }
    const _Float16 uh = (_Float16)u, ch = (_Float16)cc;
    Hi[c] = uh;
    Hi[RP + c] = (_Float16)(u - (float)uh);
    Hi[2 * RP + c] = ch;
    Hi[3 * RP + c] = (_Float16)(cc - (float)ch);
  }
}

// Column-stage data of one work group, staged through registers so that the
// next stage's global loads are in flight while the current stage computes.
template <int DM, int RP>
struct StageRegs {
  static constexpr int NX4 = (kStage * DM / 4 + 255) / 256;     // float4 of x~ per thread
  static constexpr int NH8 = kStage * 4 * RP / 8 / 256;          // 8-half vectors of H per thread
  gf4 x[NX4];
  float nrm;
  h8 hv[NH8];

  __device__ __forceinline__ void load(const float* __restrict__ Xs, const float* __restrict__ nr,
                                       const _Float16* __restrict__ H, int64_t n, int64_t j0) {
#pragma unroll
    for (int k = 0; k < NX4; ++k) {
      const int e = threadIdx.x + 256 * k;            // float4 index within the stage
      const int jj = e / (DM / 4);
      const int64_t j = j0 + jj;
      x[k] = (e < kStage * DM / 4 && j < n)
                 ? *reinterpret_cast<const gf4*>(Xs + j * DM + 4 * (e % (DM / 4)))
                 : gf4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    {
      const int64_t j = j0 + (threadIdx.x & (kStage - 1));
      nrm = j < n ? nr[j] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < NH8; ++k) {
      const int e = threadIdx.x + 256 * k;            // 8-half index within the stage
      const int jj = e / (RP / 2);
      const int64_t j = j0 + jj;
      hv[k] = j < n ? *reinterpret_cast<const h8*>(H + j * 4 * RP + 8 * (e % (RP / 2)))
                    : h8{0, 0, 0, 0, 0, 0, 0, 0};
    }
  }
};

// One work group = 4 waves x NSUB subtiles of 16 rows against the column
// stages of its split.  Lane layouts: v_mfma_f32_16x16x32_f16 A operand lane l
// holds A[l % 16][8 (l / 16) + t] (t < 8), B operand B[8 (l / 16) + t][l % 16];
// v_mfma_f32_16x16x4f32 A lane l holds A[l % 16][l / 16], B B[l / 16][l % 16];
// both leave D[4 (l / 16) + v][l % 16] in lane l, element v.  For 16 columns c
// of U (one chunk), with k = 8 (l / 16) + t (c = k for k < 16, else k - 16):
//   A1 = [U_hi | U_lo] (rows)    B1 = [C_hi ; C_hi] (columns)
//   A2 = [U_hi | C_hi]           B2 = [C_lo ; U_hi]   (second half mirror only)
//   A3 = [C_lo | C_hi]           B3 = [U_hi ; U_lo]   (mirror only)
// so that W~ = U_hi C_hi + U_lo C_hi + U_hi C_lo (+ the same for C U^T).  The
// distance product takes A = augmented rows, B = augmented columns
// (DK = DM + 4: coordinates, norm, one, padding).
template <int KIND, int DM, int RP, bool ISO, int NSUB, bool SYM>
__global__ __launch_bounds__(256) void grad_kernel(const float* __restrict__ Xs,
                                                   const float* __restrict__ nr,
                                                   const _Float16* __restrict__ H,
                                                   const float* __restrict__ scl, int64_t n,
                                                   int64_t i0, int64_t i1,
                                                   double* __restrict__ part, int nsplit) {
  constexpr int NCH = RP / 16;                  // 16-column chunks of U
  constexpr int NACC = ISO ? 1 : DM;
  constexpr int RB = 64 * NSUB;                 // rows per work group
  constexpr bool MR2 = KIND != GP_KERNEL_MATERN12;   // r^2 on the matrix cores
  constexpr int DK = DM + 4;                    // augmented distance operand length
  constexpr int NK = DK / 4;
  constexpr int NW = SYM ? 3 : 2;               // binary16 products per chunk
  __shared__ __align__(16) float sX[kStage][DM];
  __shared__ __align__(16) float sN[kStage];
  __shared__ __align__(16) _Float16 sH[kStage][4 * RP];
  __shared__ double sRed[4][NACC + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int gl = g & 1, gh = g >> 1;
  const int split = blockIdx.x % nsplit;
  const int64_t rblk = blockIdx.x / nsplit;
  const int64_t rowb = i0 + rblk * RB;
  const int64_t roww = rowb + (int64_t)wave * 16 * NSUB;
  const float unscale = scl[128];
  const h8 z8 = h8{0, 0, 0, 0, 0, 0, 0, 0};

  h8 aw[NSUB][NCH][NW];
  float ha[NSUB][MR2 ? NK : 1];
  float a[NSUB][4][DM];
#pragma unroll
  for (int q = 0; q < NSUB; ++q) {
    const int64_t ia = roww + 16 * q + l16;
    const bool in = ia < i1;
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
      const _Float16* Hr = H + ia * 4 * RP + 16 * h + 8 * gl;
      aw[q][h][0] = in ? *reinterpret_cast<const h8*>(Hr + (gh ? 1 : 0) * RP) : z8;
      aw[q][h][1] = in ? *reinterpret_cast<const h8*>(Hr + (gh ? 2 : 0) * RP) : z8;
      if constexpr (SYM) aw[q][h][2] = in ? *reinterpret_cast<const h8*>(Hr + (gh ? 2 : 3) * RP) : z8;
    }
    if constexpr (MR2) {
      // augmented row [x~, |x~|^2, 1, 0, 0] of row ia; this lane supplies k = 4 s + g
#pragma unroll
      for (int s = 0; s < NK; ++s) {
        const int k = 4 * s + g;
        float v = 0.0f;
        if (in) v = k < DM ? Xs[ia * DM + k] : (k == DM ? nr[ia] : (k == DM + 1 ? 1.0f : 0.0f));
        ha[q][s] = v;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t id = roww + 16 * q + 4 * g + v;
#pragma unroll
      for (int m4 = 0; m4 < DM; m4 += 4) {
        const gf4 x4 = id < i1 ? *reinterpret_cast<const gf4*>(Xs + id * DM + m4)
                               : gf4{0.0f, 0.0f, 0.0f, 0.0f};
        a[q][v][m4] = x4[0];
        a[q][v][m4 + 1] = x4[1];
        a[q][v][m4 + 2] = x4[2];
        a[q][v][m4 + 3] = x4[3];
      }
    }
  }
  float acc[NACC];
#pragma unroll
  for (int m = 0; m < NACC; ++m) acc[m] = 0.0f;
  float acck = 0.0f;

  const int64_t nstage = ceil_div(n, kStage);
  // symmetric: stages from the block's first row on (RB is a multiple of kStage)
  const int64_t s0 = SYM ? rowb / kStage : 0;
  const int64_t own_end = SYM ? s0 + RB / kStage : 0;   // stages holding the block's own rows
  const int64_t sb = s0 + split * (nstage - s0) / nsplit;
  const int64_t se = s0 + (split + 1) * (nstage - s0) / nsplit;
  StageRegs<DM, RP> pre;
  if (sb < se) pre.load(Xs, nr, H, n, sb * kStage);
  for (int64_t st = sb; st < se; ++st) {
    const bool mirror = SYM && st >= own_end;
    __syncthreads();                                   // previous stage's reads are done
#pragma unroll
    for (int k = 0; k < StageRegs<DM, RP>::NX4; ++k) {
      const int e = threadIdx.x + 256 * k;
      if (e < kStage * DM / 4)
        *reinterpret_cast<gf4*>(&sX[e / (DM / 4)][4 * (e % (DM / 4))]) = pre.x[k];
    }
    if (threadIdx.x < kStage) sN[threadIdx.x] = pre.nrm;
#pragma unroll
    for (int k = 0; k < StageRegs<DM, RP>::NH8; ++k) {
      const int e = threadIdx.x + 256 * k;
      *reinterpret_cast<h8*>(&sH[e / (RP / 2)][8 * (e % (RP / 2))]) = pre.hv[k];
    }
    __syncthreads();
    if (st + 1 < se) pre.load(Xs, nr, H, n, (st + 1) * kStage);   // in flight meanwhile
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
      float hb[MR2 ? NK : 1];
      if constexpr (MR2) {
        // augmented column [-2 x~, 1, |x~|^2, 0, 0]; this lane supplies k = 4 s + g
#pragma unroll
        for (int s = 0; s < NK; ++s) {
          const int k = 4 * s + g;
          float v = 0.0f;
#pragma unroll
          for (int m = 0; m < DM; ++m) v = k == m ? -2.0f * b[m] : v;
          hb[s] = k == DM ? 1.0f : (k == DM + 1 ? sN[jj] : v);
        }
      }
      h8 bw[NCH][NW];
#pragma unroll
      for (int h = 0; h < NCH; ++h) {
        const _Float16* Hc = &sH[jj][16 * h + 8 * gl];
        bw[h][0] = *reinterpret_cast<const h8*>(Hc + 2 * RP);
        bw[h][1] = (gh && !mirror) ? z8 : *reinterpret_cast<const h8*>(Hc + (gh ? 0 : 3) * RP);
        if constexpr (SYM) bw[h][2] = *reinterpret_cast<const h8*>(Hc + (gh ? 1 : 0) * RP);
      }
#pragma unroll
      for (int q = 0; q < NSUB; ++q) {
        gf4 W = gf4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int h = 0; h < NCH; ++h) {
          W = __builtin_amdgcn_mfma_f32_16x16x32_f16(aw[q][h][0], bw[h][0], W, 0, 0, 0);
          W = __builtin_amdgcn_mfma_f32_16x16x32_f16(aw[q][h][1], bw[h][1], W, 0, 0, 0);
          if constexpr (SYM) {
            if (mirror) W = __builtin_amdgcn_mfma_f32_16x16x32_f16(aw[q][h][2], bw[h][2], W, 0, 0, 0);
          }
        }
        gf4 R2 = gf4{0.0f, 0.0f, 0.0f, 0.0f};
        if constexpr (MR2) {
#pragma unroll
          for (int s = 0; s < NK; ++s) R2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ha[q][s], hb[s], R2, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float w = W[v] * unscale;
          float q2[ISO ? 1 : DM];
          float r2 = 0.0f;
          if constexpr (!ISO) {
#pragma unroll
            for (int m = 0; m < DM; ++m) {
              const float dl = a[q][v][m] - b[m];
              q2[m] = dl * dl;
              if constexpr (!MR2) r2 += q2[m];
            }
          } else if constexpr (!MR2) {
#pragma unroll
            for (int m = 0; m < DM; ++m) {
              const float dl = a[q][v][m] - b[m];
              r2 = fmaf(dl, dl, r2);
            }
          }
          if constexpr (MR2) r2 = __builtin_amdgcn_fmed3f(R2[v], 0.0f, 3.0e38f);   // clamp at 0
          float kap, G;
          kval_deriv<KIND>(r2, kap, G);
          acck = fmaf(kap, w, acck);
          const float P = G * w;
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

// Device scratch of one call.
struct Work {
  float* Xs;          // n x DM scaled points
  float* nr;          // n squared norms
  _Float16* H;        // n x 4 x RP binary16 split of U and C
  uint32_t* cmax;     // 128 column maxima
  float* scl;         // 129 scales
};

template <int KIND, int DM, int RP, bool ISO>
gp_status launch_t(const KParams& kp, const float* X, int64_t n, const float* U, const float* B,
                   int r, float inv2m, int64_t i0, int64_t i1, double* part, int nsplit,
                   const Work& w, hipStream_t s) {
  constexpr int NSUB = nsub_for<DM>();
  GP_TRY(fill_f32(reinterpret_cast<float*>(w.cmax), 128, 0.0f, s));
  colmax_kernel<<<(unsigned)ceil_div(n, kColmaxRows), 256, 0, s>>>(U, B, n, r, inv2m, w.cmax);
  GP_HIP(hipGetLastError());
  scale_kernel<<<1, 64, 0, s>>>(w.cmax, r, w.scl);
  GP_HIP(hipGetLastError());
  split_kernel<DM, RP><<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(X, U, B, n, r, inv2m, kp, w.scl,
                                                                  w.Xs, w.nr, w.H);
  GP_HIP(hipGetLastError());
  const int64_t blocks = ceil_div(i1 - i0, (int64_t)64 * NSUB) * nsplit;
  if (i0 == 0 && i1 == n)
    grad_kernel<KIND, DM, RP, ISO, NSUB, true><<<(unsigned)blocks, 256, 0, s>>>(
        w.Xs, w.nr, w.H, w.scl, n, i0, i1, part, nsplit);
  else
    grad_kernel<KIND, DM, RP, ISO, NSUB, false><<<(unsigned)blocks, 256, 0, s>>>(
        w.Xs, w.nr, w.H, w.scl, n, i0, i1, part, nsplit);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

template <int KIND, int DM>
gp_status launch_r(const KParams& kp, bool iso, const float* X, int64_t n, const float* U,
                   const float* B, int r, float inv2m, int64_t i0, int64_t i1, double* part,
                   int nsplit, const Work& w, hipStream_t s) {
  if (r <= 16) {
    if (iso) return launch_t<KIND, DM, 16, true>(kp, X, n, U, B, r, inv2m, i0, i1, part, nsplit, w, s);
    return launch_t<KIND, DM, 16, false>(kp, X, n, U, B, r, inv2m, i0, i1, part, nsplit, w, s);
  }
  if (iso) return launch_t<KIND, DM, 64, true>(kp, X, n, U, B, r, inv2m, i0, i1, part, nsplit, w, s);
  return launch_t<KIND, DM, 64, false>(kp, X, n, U, B, r, inv2m, i0, i1, part, nsplit, w, s);
}

template <int KIND>
gp_status launch_d(const KParams& kp, bool iso, const float* X, int64_t n, const float* U,
                   const float* B, int r, float inv2m, int64_t i0, int64_t i1, double* part,
                   int nsplit, const Work& w, hipStream_t s) {
  const int d = kp.d;
  if (d <= 4) return launch_r<KIND, 4>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, w, s);
  if (d <= 8) return launch_r<KIND, 8>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, w, s);
  if (d <= 16) return launch_r<KIND, 16>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, w, s);
  return launch_r<KIND, 32>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, w, s);
}

int dm_of(int d) { return d <= 4 ? 4 : d <= 8 ? 8 : d <= 16 ? 16 : 32; }
int rp_of(int r) { return r <= 16 ? 16 : 64; }

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

size_t workspace_bytes(int64_t rows, int64_t n, int d, int r) {
  const int64_t nblk = row_blocks(rows, d) * choose_splits(rows, n, d);
  const int64_t nchunk = ceil_div(std::max<int64_t>(rows, 1), kDiagRows);
  return 8 * (size_t)nblk * (kMaxDim + 1) + 16 * (size_t)nchunk + 4 * (size_t)n * (dm_of(d) + 1) +
         2 * (size_t)n * 4 * rp_of(r) + 4 * 128 + 4 * 129 + 8 * 256;
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
  Work w;
  w.Xs = ar.take<float>((size_t)n * dm_of(kp.d));
  w.nr = ar.take<float>((size_t)n);
  w.H = ar.take<_Float16>((size_t)n * 4 * rp_of(r));
  w.cmax = ar.take<uint32_t>(128);
  w.scl = ar.take<float>(129);
  if (!part || !dpart || !w.Xs || !w.nr || !w.H || !w.cmax || !w.scl)
    return set_error(GP_ERR_NOMEM, "internal: gradient workspace sizing");
  const float inv2m = (float)(0.5 / (double)(r - 1));
  const bool iso = !ard;
  if (rows > 0) {
    gp_status st;
    switch (kp.kind) {
      case GP_KERNEL_RBF:
        st = launch_d<GP_KERNEL_RBF>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, w, s);
        break;
      case GP_KERNEL_MATERN52:
        st = launch_d<GP_KERNEL_MATERN52>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, w, s);
        break;
      case GP_KERNEL_MATERN32:
        st = launch_d<GP_KERNEL_MATERN32>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, w, s);
        break;
      case GP_KERNEL_MATERN12:
        st = launch_d<GP_KERNEL_MATERN12>(kp, iso, X, n, U, B, r, inv2m, i0, i1, part, nsplit, w, s);
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
