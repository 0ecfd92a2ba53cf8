// Binary16 summation schemes of the kernel-matrix product (Sec. 5.1, Fig. 4;
// App. B, summation approaches): accuracy ablations in which the products and
// the sums are binary16 as well, against the production product whose sums are
// float32 (block summation in single precision, on the matrix cores).
//
// The defining property is the order of the rounded operations, so one thread
// owns one output row and walks the columns j = 0 .. n2-1 in order, keeping per
// right-hand-side column either a block sum and a total (block schemes) or a
// sum and its compensation (Kahan).  Column points and binary16 right-hand
// sides are staged through LDS in 128-column stages shared by the 256 rows of a
// work group.  The kernel value is formed in float32 from the binary16 inputs
// and rounded to binary16; every later operation is a single binary16 (or, for
// the block totals of GP_SUM_BLOCK_SINGLE, float32) operation, with fused
// multiply-adds switched off so that k_hat * v_hat is rounded before it is
// added.

#include <math.h>

#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace gpmi {
namespace hsum {

constexpr int kThreads = 256;
constexpr int kStage = 128;
constexpr int kUnroll = 4;

// x_hat = fp16(x / l) as float32 values, rows padded with zeros to DM columns.
__global__ void quant_x_kernel(const float* __restrict__ X, int64_t n, int64_t n_pad, KParams kp,
                               int dm, float* __restrict__ Xh) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_pad * dm) return;
  const int64_t i = t / dm;
  const int m = (int)(t % dm);
  float v = 0.0f;
  if (i < n && m < kp.d) v = (float)(_Float16)(X[i * kp.d + m] / kp.ls[m]);
  Xh[t] = v;
}

template <int KIND, int SCHEME, int RC, int DM>
__global__ __launch_bounds__(kThreads) void hsum_kernel(
    const float* __restrict__ Xh1, int64_t n1, const float* __restrict__ Xh2, int64_t n2,
    const _Float16* __restrict__ Vt, int64_t n2_pad, int rc, int block,
    const float* __restrict__ inv_scale, float a2, float s2, const float* __restrict__ V,
    int64_t ldv, float* __restrict__ out, int64_t ldo) {
#pragma clang fp contract(off)
  __shared__ float sx[kStage * DM];
  __shared__ _Float16 sv[RC * kStage];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kThreads + tid;
  const bool live = i < n1;

  float xi[DM];
#pragma unroll
  for (int m = 0; m < DM; ++m) xi[m] = live ? Xh1[i * DM + m] : 0.0f;

  _Float16 s[RC], c[RC];          // block sum / running sum ; total / compensation
  float tf[RC];                   // float32 total (GP_SUM_BLOCK_SINGLE)
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    s[q] = (_Float16)0.0f;
    c[q] = (_Float16)0.0f;
    tf[q] = 0.0f;
  }
  int cnt = 0;                    // columns in the current block

  for (int64_t j0 = 0; j0 < n2; j0 += kStage) {
    __syncthreads();
    for (int e = tid; e < kStage * DM; e += kThreads) sx[e] = Xh2[j0 * DM + e];
    for (int e = tid; e < RC * kStage; e += kThreads) {
      const int q = e / kStage, jj = e % kStage;
      sv[e] = q < rc ? Vt[(int64_t)q * n2_pad + j0 + jj] : (_Float16)0.0f;
    }
    __syncthreads();
    const int jn = (int)std::min<int64_t>(kStage, n2 - j0);
    // kernel value of column jj (independent across columns)
    auto kvalue = [&](int jj) {
      float r2 = 0.0f;
#pragma unroll
      for (int m = 0; m < DM; ++m) {
        const float t = xi[m] - sx[jj * DM + m];
        r2 = fmaf(t, t, r2);
      }
      return (_Float16)kval32_fast<KIND>(r2);
    };
    // the ordered, rounded accumulation of column jj
    auto accumulate = [&](_Float16 kh, int jj) {
#pragma unroll
      for (int q = 0; q < RC; ++q) {
        const _Float16 p = kh * sv[q * kStage + jj];
        if constexpr (SCHEME == GP_SUM_KAHAN_HALF) {
          const _Float16 y = p - c[q];
          const _Float16 t = s[q] + y;
          c[q] = (t - s[q]) - y;
          s[q] = t;
        } else {
          s[q] = s[q] + p;
        }
      }
      if constexpr (SCHEME != GP_SUM_KAHAN_HALF) {
        if (++cnt == block) {
          cnt = 0;
#pragma unroll
          for (int q = 0; q < RC; ++q) {
            if constexpr (SCHEME == GP_SUM_BLOCK_HALF)
              c[q] = c[q] + s[q];
            else
              tf[q] = tf[q] + (float)s[q];
            s[q] = (_Float16)0.0f;
          }
        }
      }
    };
    // kUnroll kernel values first, then their accumulations in column order:
    // the independent exponentials overlap, the rounded sums keep their order
    int jj = 0;
    for (; jj + kUnroll <= jn; jj += kUnroll) {
      _Float16 kh[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) kh[u] = kvalue(jj + u);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) accumulate(kh[u], jj + u);
    }
    for (; jj < jn; ++jj) accumulate(kvalue(jj), jj);
  }
  if constexpr (SCHEME != GP_SUM_KAHAN_HALF) {
    if (cnt > 0) {
#pragma unroll
      for (int q = 0; q < RC; ++q) {
        if constexpr (SCHEME == GP_SUM_BLOCK_HALF)
          c[q] = c[q] + s[q];
        else
          tf[q] = tf[q] + (float)s[q];
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    if (q >= rc) break;
    float T;
    if constexpr (SCHEME == GP_SUM_KAHAN_HALF)
      T = (float)s[q];
    else if constexpr (SCHEME == GP_SUM_BLOCK_HALF)
      T = (float)c[q];
    else
      T = (float)(_Float16)tf[q];
    float o = (a2 * inv_scale[q]) * T;
    if (V) o = o + s2 * V[i * ldv + q];
    out[i * ldo + q] = o;
  }
}

struct Args {
  const float *Xh1, *Xh2;
  int64_t n1, n2, n2_pad;
  const _Float16* Vt;
  int rc, block;
  const float* inv_scale;
  float a2, s2;
  const float* V;
  int64_t ldv;
  float* out;
  int64_t ldo;
};

template <int KIND, int SCHEME, int RC, int DM>
gp_status launch_t(const Args& a, hipStream_t s) {
  const unsigned blocks = (unsigned)ceil_div(a.n1, kThreads);
  hsum_kernel<KIND, SCHEME, RC, DM><<<blocks, kThreads, 0, s>>>(
      a.Xh1, a.n1, a.Xh2, a.n2, a.Vt, a.n2_pad, a.rc, a.block, a.inv_scale, a.a2, a.s2, a.V, a.ldv,
      a.out, a.ldo);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

template <int KIND, int SCHEME, int RC>
gp_status launch_dm(int dm, const Args& a, hipStream_t s) {
  return dm == 8 ? launch_t<KIND, SCHEME, RC, 8>(a, s) : launch_t<KIND, SCHEME, RC, 64>(a, s);
}

template <int KIND, int SCHEME>
gp_status launch_rc(int rcmax, int dm, const Args& a, hipStream_t s) {
  if (rcmax == 1) return launch_dm<KIND, SCHEME, 1>(dm, a, s);
  if (rcmax == 4) return launch_dm<KIND, SCHEME, 4>(dm, a, s);
  return launch_dm<KIND, SCHEME, 16>(dm, a, s);
}

template <int KIND>
gp_status launch_scheme(int scheme, int rcmax, int dm, const Args& a, hipStream_t s) {
  switch (scheme) {
    case GP_SUM_BLOCK_HALF: return launch_rc<KIND, GP_SUM_BLOCK_HALF>(rcmax, dm, a, s);
    case GP_SUM_BLOCK_SINGLE: return launch_rc<KIND, GP_SUM_BLOCK_SINGLE>(rcmax, dm, a, s);
    default: return launch_rc<KIND, GP_SUM_KAHAN_HALF>(rcmax, dm, a, s);
  }
}

gp_status launch(int kind, int scheme, int rcmax, int dm, const Args& a, hipStream_t s) {
  switch (kind) {
    case GP_KERNEL_RBF: return launch_scheme<GP_KERNEL_RBF>(scheme, rcmax, dm, a, s);
    case GP_KERNEL_MATERN52: return launch_scheme<GP_KERNEL_MATERN52>(scheme, rcmax, dm, a, s);
    case GP_KERNEL_MATERN12: return launch_scheme<GP_KERNEL_MATERN12>(scheme, rcmax, dm, a, s);
    case GP_KERNEL_MATERN32: return launch_scheme<GP_KERNEL_MATERN32>(scheme, rcmax, dm, a, s);
  }
  return set_error(GP_ERR_ARG, "unknown kernel kind %d", kind);
}

}  // namespace hsum
}  // namespace gpmi

using namespace gpmi;

extern "C" gp_status gp_kmvm_summation(const gp_kernel* k, const float* X1, int64_t n1,
                                       const float* X2, int64_t n2, int32_t d, const float* V,
                                       int32_t r, float* out, int32_t add_noise, int32_t scheme,
                                       int32_t block, int32_t scale_mode, void* stream) {
  clear_error();
  KParams kp;
  GP_TRY(check_kernel(k, d, false, &kp));
  if (n1 < 0 || n2 < 0) return set_error(GP_ERR_ARG, "negative point count");
  if (r < 1) return set_error(GP_ERR_ARG, "r=%d must be >= 1", r);
  if (scheme != GP_SUM_BLOCK_HALF && scheme != GP_SUM_BLOCK_SINGLE && scheme != GP_SUM_KAHAN_HALF)
    return set_error(GP_ERR_ARG, "scheme must be GP_SUM_BLOCK_HALF, GP_SUM_BLOCK_SINGLE or GP_SUM_KAHAN_HALF");
  if (scheme != GP_SUM_KAHAN_HALF && (block < 1 || block > (1 << 30)))
    return set_error(GP_ERR_ARG, "block=%d outside [1, 2^30]", block);
  if (scheme == GP_SUM_KAHAN_HALF) block = 1;
  if (scale_mode != 0 && scale_mode != 1) return set_error(GP_ERR_ARG, "scale_mode must be 0 or 1");
  if (n1 > 0 && (!X1 || !out)) return set_error(GP_ERR_ARG, "X1/out is NULL");
  if (n2 > 0 && (!X2 || !V)) return set_error(GP_ERR_ARG, "X2/V is NULL");
  if (add_noise && (X1 != X2 || n1 != n2))
    return set_error(GP_ERR_ARG, "add_noise needs X1 == X2 and n1 == n2");
  const size_t ob = (size_t)n1 * r * 4;
  if (overlaps(out, ob, V, (size_t)n2 * r * 4) || overlaps(out, ob, X1, (size_t)n1 * d * 4) ||
      overlaps(out, ob, X2, (size_t)n2 * d * 4))
    return set_error(GP_ERR_ARG, "out overlaps an input");
  if (n1 == 0) return GP_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n2 == 0) return fill_f32(out, n1 * r, 0.0f, s);

  const int dm = d <= 8 ? 8 : 64;
  const int64_t n1_pad = round_up(n1, hsum::kThreads);
  const int64_t n2_pad = round_up(n2, hsum::kStage);
  constexpr int kRc = 16;
  const size_t bytes = 4 * (size_t)n1_pad * dm + 4 * (size_t)n2_pad * dm +
                       2 * (size_t)kRc * n2_pad + 12 * (size_t)kRc + 8 * 256;
  Arena ar;
  GP_TRY(workspace_get(s, bytes, &ar));
  float* Xh1 = ar.take<float>((size_t)n1_pad * dm);
  float* Xh2 = ar.take<float>((size_t)n2_pad * dm);
  _Float16* Vt = ar.take<_Float16>((size_t)kRc * n2_pad);
  uint32_t* colmax = ar.take<uint32_t>(kRc);
  float* scale = ar.take<float>(kRc);
  float* inv_scale = ar.take<float>(kRc);
  if (!inv_scale) return set_error(GP_ERR_NOMEM, "internal: workspace sizing");

  hsum::quant_x_kernel<<<(unsigned)ceil_div(n1_pad * dm, 256), 256, 0, s>>>(X1, n1, n1_pad, kp, dm,
                                                                            Xh1);
  GP_HIP(hipGetLastError());
  hsum::quant_x_kernel<<<(unsigned)ceil_div(n2_pad * dm, 256), 256, 0, s>>>(X2, n2, n2_pad, kp, dm,
                                                                            Xh2);
  GP_HIP(hipGetLastError());
  const float fs = (float)(1.0 / sqrt((double)n2));
  const float fi = (float)sqrt((double)n2);
  for (int c0 = 0; c0 < r; c0 += kRc) {
    const int rc = std::min(kRc, r - c0);
    const int rcmax = rc == 1 ? 1 : rc <= 4 ? 4 : 16;
    GP_TRY(f16::quant_rhs(V + c0, n2, rc, r, rcmax, n2_pad, scale_mode, fs, fi, colmax, Vt, scale,
                          inv_scale, s));
    hsum::Args a{Xh1, Xh2, n1, n2, n2_pad, Vt, rc, block, inv_scale, kp.a2, kp.s2,
                 add_noise ? V + c0 : nullptr, r, out + c0, r};
    GP_TRY(hsum::launch(kp.kind, scheme, rcmax, dm, a, s));
  }
  return GP_OK;
}
