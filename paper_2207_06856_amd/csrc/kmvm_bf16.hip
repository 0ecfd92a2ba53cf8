// Fused kernel-matrix x multi-vector product with bfloat16 operands (the
// number format of Sec. 2.1 that keeps float32's exponent range with an 8-bit
// significand) on v_mfma_f32_16x16x32_bf16, float32 accumulation.
//
// Same tile loop as the binary16 product (fused_tile.h): the first MFMA forms
// the exponent argument from augmented operand rows, the kernel values are
// rounded to the operand format, the second MFMA multiplies them with the
// right-hand sides.  Two things change with the format:
//   * the inputs x / l are rounded to bfloat16;
//   * the column-side factors alpha * x_hat and beta * ||x_hat||^2 are float32
//     values carried as three bfloat16 parts (8 + 8 + 8 significand bits), so
//     the argument keeps float32 accuracy; a row is
//       side 1 (columns): [p0(ax), p1(ax), p2(ax), p0(bn), p1(bn), p2(bn), 1, 1, 1]
//       side 0 (rows):    [x, x, x, 1, 1, 1, p0(bn), p1(bn), p2(bn)]
//     of width 3d + 6, padded to a multiple of 32 (d <= 64 gives KC <= 7).
// The kernel values themselves have no binary16 underflow: bfloat16 keeps
// values down to 2^-133, so this product has no finite support to exploit.
// The right-hand sides use the column scales of the binary16 product; a
// power-of-two scale leaves every bfloat16 product unchanged.

#include <math.h>

#include "fused_tile.h"
#include "internal.h"

namespace gpmi {
namespace f16 {

typedef Vec<__bf16>::v8 b8;

__device__ __forceinline__ float bf_round(float x) { return (float)(__bf16)x; }

// One thread writes 8 consecutive elements of one augmented row.
__global__ void prep_points_bf16_kernel(const float* __restrict__ X, int64_t n, int64_t n_pad,
                                        KParams kp, int side, int kp_width, float alpha,
                                        float beta, __bf16* __restrict__ out) {
  const int chunks = kp_width / 8;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_pad * chunks) return;
  const int64_t i = t / chunks;
  const int c = (int)(t % chunks);
  b8 o;
  for (int q = 0; q < 8; ++q) o[q] = (__bf16)0.0f;
  if (i < n) {
    const int d = kp.d;
    const float* x = X + i * d;
    float nrm = 0.0f;
    for (int m = 0; m < d; ++m) {
      const float h = bf_round(x[m] / kp.ls[m]);
      nrm = fmaf(h, h, nrm);
    }
    const float bn = beta * nrm;
    const float bn0 = bf_round(bn);
    const float bn1 = bf_round(bn - bn0);
    const float bn2 = bf_round(bn - bn0 - bn1);
    for (int q = 0; q < 8; ++q) {
      const int p = c * 8 + q;
      float v = 0.0f;
      if (p < 3 * d) {
        const int part = p / d, m = p % d;
        const float h = bf_round(x[m] / kp.ls[m]);
        if (side == 0) {
          v = h;
        } else {
          const float ax = alpha * h;
          const float a0 = bf_round(ax);
          const float a1 = bf_round(ax - a0);
          v = part == 0 ? a0 : part == 1 ? a1 : ax - a0 - a1;
        }
      } else if (p < 3 * d + 6) {
        const int e = p - 3 * d;       // 0..5
        const bool norm_slot = side == 1 ? e < 3 : e >= 3;
        if (norm_slot) {
          const int part = e % 3;
          v = part == 0 ? bn0 : part == 1 ? bn1 : bn2;
        } else {
          v = 1.0f;
        }
      }
      o[q] = (__bf16)v;
    }
  }
  *reinterpret_cast<b8*>(out + i * kp_width + c * 8) = o;
}

gp_status prep_points_bf16(const float* X, int64_t n, int64_t n_pad, const KParams& kp, int side,
                           __bf16* out, hipStream_t s) {
  const int w = aug_width_bf16(kp.d);
  const float c = arg_scale(kp.kind);
  const float alpha = kp.kind == GP_KERNEL_RBF ? c : -2.0f * c;
  const float beta = kp.kind == GP_KERNEL_RBF ? -0.5f * c : c;
  const int64_t total = n_pad * (w / 8);
  if (total == 0) return GP_OK;
  prep_points_bf16_kernel<<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(X, n, n_pad, kp, side, w,
                                                                         alpha, beta, out);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

template <int KIND, int KC, int RB>
__global__ __launch_bounds__(256) void kmvm_bf16_main(const __bf16* __restrict__ Xr,
                                                      const __bf16* __restrict__ Xc,
                                                      const __bf16* __restrict__ Vt,
                                                      float* __restrict__ part, int64_t n1_pad,
                                                      int64_t n2_pad, int nsplit,
                                                      const int* __restrict__ live) {
  if (live && *live == 0) return;
  __shared__ __attribute__((aligned(16))) __bf16 sX[2 * x_stage_halfs<KC>()];
  __shared__ __attribute__((aligned(16))) __bf16 sV[2 * v_stage_halfs<RB>()];
  const int split = blockIdx.x % nsplit;
  const int64_t rblk = blockIdx.x / nsplit;
  const int64_t nstage = n2_pad / JT;
  const int64_t sb = split * nstage / nsplit;
  const int64_t se = (split + 1) * nstage / nsplit;
  float* P = part + ((int64_t)split * n1_pad) * (16 * RB);
  fused_rows<KIND, KC, RB, __bf16>(Xr, Xc, Vt, n2_pad, P, rblk * kRowsPerBlock, sb, se, sX, sV);
}

template <int KIND, int KC, int RB>
static gp_status launch_t(const __bf16* Xr, const __bf16* Xc, const __bf16* Vt, float* part,
                          int64_t n1_pad, int64_t n2_pad, int nsplit, const int* live,
                          hipStream_t s) {
  const int64_t blocks = (n1_pad / kRowsPerBlock) * nsplit;
  kmvm_bf16_main<KIND, KC, RB><<<(unsigned)blocks, 256, 0, s>>>(Xr, Xc, Vt, part, n1_pad, n2_pad,
                                                                nsplit, live);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

template <int KIND, int KC>
static gp_status launch_rb(int rb, const __bf16* Xr, const __bf16* Xc, const __bf16* Vt,
                           float* part, int64_t n1_pad, int64_t n2_pad, int nsplit, const int* live,
                           hipStream_t s) {
  switch (rb) {
    case 1: return launch_t<KIND, KC, 1>(Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
    case 2: return launch_t<KIND, KC, 2>(Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
    case 3: return launch_t<KIND, KC, 3>(Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
    case 4: return launch_t<KIND, KC, 4>(Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
  }
  return set_error(GP_ERR_ARG, "internal: unsupported column block count %d", rb);
}

template <int KIND>
static gp_status launch_kc(int kc, int rb, const __bf16* Xr, const __bf16* Xc, const __bf16* Vt,
                           float* part, int64_t n1_pad, int64_t n2_pad, int nsplit, const int* live,
                           hipStream_t s) {
  switch (kc) {
    case 1: return launch_rb<KIND, 1>(rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
    case 2: return launch_rb<KIND, 2>(rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
    case 3: return launch_rb<KIND, 3>(rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
    case 4: return launch_rb<KIND, 4>(rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
    case 5: return launch_rb<KIND, 5>(rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
    case 6: return launch_rb<KIND, 6>(rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
    case 7: return launch_rb<KIND, 7>(rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
  }
  return set_error(GP_ERR_ARG, "internal: unsupported operand width %d", kc * 32);
}

gp_status launch_main_bf16(int kind, int kc, int rb, const __bf16* Xr, const __bf16* Xc,
                           const __bf16* Vt, float* part, int64_t n1_pad, int64_t n2_pad,
                           int nsplit, const int* live, double entries, hipStream_t s) {
  if (n1_pad == 0) return GP_OK;
  void* tok = prof::begin(s);
  gp_status st;
  switch (kind) {
    case GP_KERNEL_RBF:
      st = launch_kc<GP_KERNEL_RBF>(kc, rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
      break;
    case GP_KERNEL_MATERN52:
      st = launch_kc<GP_KERNEL_MATERN52>(kc, rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
      break;
    case GP_KERNEL_MATERN12:
      st = launch_kc<GP_KERNEL_MATERN12>(kc, rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
      break;
    case GP_KERNEL_MATERN32:
      st = launch_kc<GP_KERNEL_MATERN32>(kc, rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, s);
      break;
    default:
      return set_error(GP_ERR_ARG, "unknown kernel kind %d", kind);
  }
  prof::end(tok, s, entries, kind);
  return st;
}

}  // namespace f16
}  // namespace gpmi
