// Fused, never-materialised kernel matrix x multi-vector product on the
// gfx950 matrix cores (Sec. 5.1, Eq. mvm; binary16 tiles with single-precision
// block summation).
//
// For an output-row tile I and a column tile J the product needs
//   S_IJ  = the kernel's exponent argument for every pair (i, j),
//   K_IJ  = kappa(S_IJ) rounded to binary16,
//   acc_I += K_IJ V_J.
// Both contractions run on v_mfma_f32_16x16x32_f16 with float32 accumulation.
// The exponent argument is produced by the first MFMA directly: the operands
// are augmented rows (built once by prep_points) whose dot product is
//   alpha * <x_i, x_j> + beta * (n_i + n_j),        n = ||x_hat||^2,
// with (alpha, beta) = (c, -c/2) for the RBF kernel (so S = -c r^2 / 2 and
// K = exp2(S), c = log2 e) and (-2c, c) for the Matern family (S = c r^2 with
// c = nu' (log2 e)^2, so sqrt|S| is the scaled distance).  The column-side
// factors alpha*x and beta*n are split into binary16 hi + lo pairs so that the
// argument keeps float32 accuracy although the operands are binary16.  This
// leaves one v_exp_f32 (RBF) or one v_sqrt_f32 + one v_exp_f32 (Matern) and a
// packed conversion per entry on the vector units, which bound the kernel.
//
// The accumulator layout of S^T (lane holds column i = lane%16 and rows
// j = 4*(lane/16) + v) is reused, without an LDS round trip, as the A operand
// of K V: two adjacent 16-column subtiles give each lane the 8 reduction
// slots the second MFMA consumes, and the matching rows of V are gathered from
// LDS in the same order.
//
// Work split: a grid of (row block of 256, column split) work groups; the
// column split equals blockIdx % nsplit, so with 8 splits every XCD (work
// groups are dealt round-robin to the 8 XCDs) streams only its own eighth of
// the column points through its L2.  Partial sums are reduced in a fixed
// order by kmvm_reduce, which also applies a^2, the column scale and s^2 V.

#include <math.h>

#include "fused_tile.h"
#include "internal.h"

namespace gpmi {
namespace f16 {

// ---- a1: augmented binary16 operands ------------------------------------
// One thread writes 8 consecutive halfs of one row.  side 0 = row points (B
// operand of the first MFMA), side 1 = column points (A operand).
//   side 1: [hi(alpha x), lo(alpha x), hi(beta n), lo(beta n), 1, 1, 0...]
//   side 0: [x, x, 1, 1, hi(beta n), lo(beta n), 0...]
__global__ void prep_points_kernel(const float* __restrict__ X, int64_t n, int64_t n_pad,
                                   KParams kp, int side, int kp_width, float alpha, float beta,
                                   _Float16* __restrict__ out) {
  const int chunks = kp_width / 8;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_pad * chunks) return;
  const int64_t i = t / chunks;
  const int c = (int)(t % chunks);
  h8 o;
  for (int q = 0; q < 8; ++q) o[q] = (_Float16)0.0f;
  if (i < n) {
    const int d = kp.d;
    const float* x = X + i * d;
    float nrm = 0.0f;
    for (int m = 0; m < d; ++m) {
      const float h = (float)(_Float16)(x[m] / kp.ls[m]);
      nrm = fmaf(h, h, nrm);
    }
    const float bn = beta * nrm;
    const _Float16 bn_hi = (_Float16)bn;
    const _Float16 bn_lo = (_Float16)(bn - (float)bn_hi);
    for (int q = 0; q < 8; ++q) {
      const int p = c * 8 + q;
      _Float16 v = (_Float16)0.0f;
      if (p < 2 * d) {
        const int m = p < d ? p : p - d;
        const float h = (float)(_Float16)(x[m] / kp.ls[m]);
        if (side == 0) {
          v = (_Float16)h;
        } else {
          const float ax = alpha * h;
          const _Float16 hi = (_Float16)ax;
          v = p < d ? hi : (_Float16)(ax - (float)hi);
        }
      } else if (p < 2 * d + 4) {
        const int e = p - 2 * d;       // 0..3
        if (side == 1)
          v = e == 0 ? bn_hi : e == 1 ? bn_lo : (_Float16)1.0f;
        else
          v = e < 2 ? (_Float16)1.0f : e == 2 ? bn_hi : bn_lo;
      }
      o[q] = v;
    }
  }
  *reinterpret_cast<h8*>(out + i * kp_width + c * 8) = o;
}

gp_status prep_points(const float* X, int64_t n, int64_t n_pad, const KParams& kp, int side,
                      _Float16* out, hipStream_t s) {
  const int w = aug_width(kp.d);
  const float c = arg_scale(kp.kind);
  const float alpha = kp.kind == GP_KERNEL_RBF ? c : -2.0f * c;
  const float beta = kp.kind == GP_KERNEL_RBF ? -0.5f * c : c;
  const int64_t total = n_pad * (w / 8);
  if (total == 0) return GP_OK;
  const int threads = 256;
  prep_points_kernel<<<(unsigned)ceil_div(total, threads), threads, 0, s>>>(X, n, n_pad, kp, side,
                                                                            w, alpha, beta, out);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// ---- right-hand-side quantisation -----------------------------------------
__global__ void fill_u32_kernel(uint32_t* p, int n, uint32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Per-column max |v| as float bits (non-negative floats order like uint32).
__global__ void colmax_kernel(const float* __restrict__ V, int64_t n, int r, int64_t ld,
                              uint32_t* __restrict__ colmax) {
  extern __shared__ uint32_t smax[];
  for (int c = threadIdx.x; c < r; c += blockDim.x) smax[c] = 0u;
  __syncthreads();
  const int64_t total = n * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / r;
    const int c = (int)(e % r);
    const uint32_t b = __float_as_uint(fabsf(V[i * ld + c]));
    atomicMax(&smax[c], b);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < r; c += blockDim.x)
    if (smax[c]) atomicMax(&colmax[c], smax[c]);
}

__device__ inline void pow2_scale(uint32_t maxbits, float* s, float* inv) {
  const float m = __uint_as_float(maxbits);
  if (!(m > 0.0f) || !isfinite(m)) {
    *s = 1.0f;
    *inv = 1.0f;
    return;
  }
  int e;
  frexpf(m, &e);                       // m = f 2^e, f in [0.5, 1)
  *s = ldexpf(1.0f, 15 - e);
  *inv = ldexpf(1.0f, e - 15);
}

// Vt[c][i] = T(V[i][c] * s_c) for c < r, i < n; zero padding elsewhere (T is
// binary16 or bfloat16).  A tiled transpose: a work group reads kQRows rows of
// V (all rp columns, row-contiguous) into LDS, then each thread writes eight
// consecutive rows of one column.  rp <= 64.
constexpr int kQRows = 128;
template <typename T>
__global__ __launch_bounds__(256) void quant_kernel(const float* __restrict__ V, int64_t n, int r,
                                                    int64_t ld, int rp, int64_t n_pad,
                                                    int scale_mode, float fixed_scale,
                                                    float fixed_inv,
                                                    const uint32_t* __restrict__ colmax,
                                                    T* __restrict__ Vt, float* __restrict__ scale,
                                                    float* __restrict__ inv_scale,
                                                    const int* __restrict__ live) {
  typedef typename Vec<T>::v8 h8;
  if (live && *live == 0) return;
  __shared__ float sv[kQRows][64 + 1];
  __shared__ float ss[64];
  const int64_t r0 = (int64_t)blockIdx.x * kQRows;
  if ((int)threadIdx.x < rp) {
    const int c = threadIdx.x;
    float sc = 1.0f, inv = 1.0f;
    if (c < r) {
      if (scale_mode == 1) {
        sc = fixed_scale;
        inv = fixed_inv;
      } else {
        pow2_scale(colmax[c], &sc, &inv);
      }
      if (blockIdx.x == 0) {
        scale[c] = sc;
        inv_scale[c] = inv;
      }
    }
    ss[c] = sc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kQRows * rp; e += 256) {
    const int row = e / rp, c = e % rp;
    const int64_t i = r0 + row;
    sv[row][c] = (c < r && i < n) ? V[i * ld + c] * ss[c] : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < (kQRows / 8) * rp; e += 256) {
    const int c = e / (kQRows / 8), q0 = (e % (kQRows / 8)) * 8;
    const int64_t i0 = r0 + q0;
    if (i0 >= n_pad) continue;
    h8 o;
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (T)sv[q0 + q][c];
    *reinterpret_cast<h8*>(Vt + (int64_t)c * n_pad + i0) = o;
  }
}

template <typename T>
static gp_status quant_rhs_t(const float* V, int64_t n, int r, int64_t ld, int rp, int64_t n_pad,
                             int scale_mode, float fixed_scale, float fixed_inv, uint32_t* colmax,
                             T* Vt, float* scale, float* inv_scale, hipStream_t s) {
  if (scale_mode == 0) {
    fill_u32_kernel<<<(unsigned)ceil_div(r, 256), 256, 0, s>>>(colmax, r, 0u);
    GP_HIP(hipGetLastError());
    if (n > 0) {
      const int64_t total = n * r;
      const int blocks = (int)std::min<int64_t>(1024, ceil_div(total, 256));
      colmax_kernel<<<blocks, 256, r * sizeof(uint32_t), s>>>(V, n, r, ld, colmax);
      GP_HIP(hipGetLastError());
    }
  }
  if (rp > 64) return set_error(GP_ERR_ARG, "internal: %d padded right-hand sides (max 64)", rp);
  if (n_pad > 0 && rp > 0) {
    quant_kernel<T><<<(unsigned)ceil_div(n_pad, (int64_t)kQRows), 256, 0, s>>>(
        V, n, r, ld, rp, n_pad, scale_mode, fixed_scale, fixed_inv, colmax, Vt, scale, inv_scale,
        nullptr);
    GP_HIP(hipGetLastError());
  }
  return GP_OK;
}

gp_status quant_rhs(const float* V, int64_t n, int r, int64_t ld, int rp, int64_t n_pad,
                    int scale_mode, float fixed_scale, float fixed_inv, uint32_t* colmax,
                    _Float16* Vt, float* scale, float* inv_scale, hipStream_t s) {
  return quant_rhs_t(V, n, r, ld, rp, n_pad, scale_mode, fixed_scale, fixed_inv, colmax, Vt, scale,
                     inv_scale, s);
}

gp_status quant_rhs(const float* V, int64_t n, int r, int64_t ld, int rp, int64_t n_pad,
                    int scale_mode, float fixed_scale, float fixed_inv, uint32_t* colmax,
                    __bf16* Vt, float* scale, float* inv_scale, hipStream_t s) {
  return quant_rhs_t(V, n, r, ld, rp, n_pad, scale_mode, fixed_scale, fixed_inv, colmax, Vt, scale,
                     inv_scale, s);
}

template <typename T>
static gp_status quant_only_t(const float* V, int64_t n, int r, int64_t ld, int rp, int64_t n_pad,
                              const uint32_t* colmax, T* Vt, float* scale, float* inv_scale,
                              const int* live, hipStream_t s) {
  if (rp > 64) return set_error(GP_ERR_ARG, "internal: %d padded right-hand sides (max 64)", rp);
  if (n_pad == 0 || rp == 0) return GP_OK;
  quant_kernel<T><<<(unsigned)ceil_div(n_pad, (int64_t)kQRows), 256, 0, s>>>(
      V, n, r, ld, rp, n_pad, 0, 1.0f, 1.0f, colmax, Vt, scale, inv_scale, live);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status quant_only(const float* V, int64_t n, int r, int64_t ld, int rp, int64_t n_pad,
                     const uint32_t* colmax, _Float16* Vt, float* scale, float* inv_scale,
                     const int* live, hipStream_t s) {
  return quant_only_t(V, n, r, ld, rp, n_pad, colmax, Vt, scale, inv_scale, live, s);
}

gp_status quant_only(const float* V, int64_t n, int r, int64_t ld, int rp, int64_t n_pad,
                     const uint32_t* colmax, __bf16* Vt, float* scale, float* inv_scale,
                     const int* live, hipStream_t s) {
  return quant_only_t(V, n, r, ld, rp, n_pad, colmax, Vt, scale, inv_scale, live, s);
}

// ---- a2: fused product ------------------------------------------------------
// First position p in [0, cnt) with list[p] >= v (list increasing).
__device__ __forceinline__ int lower_pos(const int* __restrict__ list, int cnt, int64_t v) {
  int lo = 0, hi = cnt;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (list[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// LIST: row block b visits only the stages lists[b * list_ld + p], p < counts[b]
// (increasing), of its split's stage range (the truncated product).
template <int KIND, int KC, int RB, bool LIST>
__global__ __launch_bounds__(256) void kmvm_f16_main(const _Float16* __restrict__ Xr,
                                                     const _Float16* __restrict__ Xc,
                                                     const _Float16* __restrict__ Vt,
                                                     float* __restrict__ part, int64_t n1_pad,
                                                     int64_t n2_pad, int nsplit,
                                                     const int* __restrict__ live,
                                                     const int* __restrict__ lists,
                                                     const int* __restrict__ counts,
                                                     int64_t list_ld) {
  if (live && *live == 0) return;
  __shared__ __attribute__((aligned(16))) _Float16 sX[2 * x_stage_halfs<KC>()];
  __shared__ __attribute__((aligned(16))) _Float16 sV[2 * v_stage_halfs<RB>()];
  const int split = blockIdx.x % nsplit;
  const int64_t rblk = blockIdx.x / nsplit;
  const int64_t nstage = n2_pad / JT;
  const int64_t sb = split * nstage / nsplit;
  const int64_t se = (split + 1) * nstage / nsplit;
  float* P = part + ((int64_t)split * n1_pad) * (16 * RB);
  if constexpr (LIST) {
    const int* li = lists + rblk * list_ld;
    const int cnt = counts[rblk];
    const int pb = lower_pos(li, cnt, sb), pe = lower_pos(li, cnt, se);
    fused_rows<KIND, KC, RB>(Xr, Xc, Vt, n2_pad, P, rblk * kRowsPerBlock, pb, pe, sX, sV, li);
  } else {
    fused_rows<KIND, KC, RB>(Xr, Xc, Vt, n2_pad, P, rblk * kRowsPerBlock, sb, se, sX, sV);
  }
}

template <int KIND, int KC, int RB>
static gp_status launch_t(const _Float16* Xr, const _Float16* Xc, const _Float16* Vt, float* part,
                          int64_t n1_pad, int64_t n2_pad, int nsplit, const int* live,
                          const StageLists* sl, hipStream_t s) {
  const int64_t blocks = (n1_pad / kRowsPerBlock) * nsplit;
  if (sl)
    kmvm_f16_main<KIND, KC, RB, true><<<(unsigned)blocks, 256, 0, s>>>(
        Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl->lists, sl->counts, sl->ld);
  else
    kmvm_f16_main<KIND, KC, RB, false><<<(unsigned)blocks, 256, 0, s>>>(
        Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, nullptr, nullptr, 0);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

template <int KIND, int KC>
static gp_status launch_rb(int rb, const _Float16* Xr, const _Float16* Xc, const _Float16* Vt,
                           float* part, int64_t n1_pad, int64_t n2_pad, int nsplit, const int* live,
                           const StageLists* sl, hipStream_t s) {
  switch (rb) {
    case 1: return launch_t<KIND, KC, 1>(Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
    case 2: return launch_t<KIND, KC, 2>(Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
    case 3: return launch_t<KIND, KC, 3>(Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
    case 4: return launch_t<KIND, KC, 4>(Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
  }
  return set_error(GP_ERR_ARG, "internal: unsupported column block count %d", rb);
}

template <int KIND>
static gp_status launch_kc(int kc, int rb, const _Float16* Xr, const _Float16* Xc,
                           const _Float16* Vt, float* part, int64_t n1_pad, int64_t n2_pad,
                           int nsplit, const int* live, const StageLists* sl, hipStream_t s) {
  switch (kc) {
    case 1: return launch_rb<KIND, 1>(rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
    case 2: return launch_rb<KIND, 2>(rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
    case 3: return launch_rb<KIND, 3>(rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
    case 4: return launch_rb<KIND, 4>(rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
    case 5: return launch_rb<KIND, 5>(rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
  }
  return set_error(GP_ERR_ARG, "internal: unsupported operand width %d", kc * 32);
}

gp_status launch_main(int kind, int kc, int rb, const _Float16* Xr, const _Float16* Xc,
                      const _Float16* Vt, float* part, int64_t n1_pad, int64_t n2_pad, int nsplit,
                      const int* live, double entries, hipStream_t s, const StageLists* sl) {
  if (n1_pad == 0) return GP_OK;
  void* tok = prof::begin(s);
  gp_status st;
  switch (kind) {
    case GP_KERNEL_RBF:
      st = launch_kc<GP_KERNEL_RBF>(kc, rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
      break;
    case GP_KERNEL_MATERN52:
      st = launch_kc<GP_KERNEL_MATERN52>(kc, rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
      break;
    case GP_KERNEL_MATERN12:
      st = launch_kc<GP_KERNEL_MATERN12>(kc, rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
      break;
    case GP_KERNEL_MATERN32:
      st = launch_kc<GP_KERNEL_MATERN32>(kc, rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, live, sl, s);
      break;
    default:
      return set_error(GP_ERR_ARG, "unknown kernel kind %d", kind);
  }
  prof::end(tok, s, entries, kind);
  return st;
}

__global__ void reduce_kernel(const float* __restrict__ part, int nsplit, int64_t n1,
                              int64_t n1_pad, int r, int rp, const float* __restrict__ inv_scale,
                              float a2, float s2, const float* __restrict__ V, int64_t ldv,
                              float* __restrict__ out, int64_t ldo, const int* __restrict__ live) {
  if (live && *live == 0) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n1 * r) return;
  const int64_t i = e / r;
  const int c = (int)(e % r);
  float acc = 0.0f;
  for (int x = 0; x < nsplit; ++x) acc += part[((int64_t)x * n1_pad + i) * rp + c];
  float o = (a2 * inv_scale[c]) * acc;
  if (V) o = fmaf(s2, V[i * ldv + c], o);
  out[i * ldo + c] = o;
}

gp_status launch_reduce(const float* part, int nsplit, int64_t n1, int64_t n1_pad, int r, int rp,
                        const float* inv_scale, float a2, float s2, const float* V, int64_t ldv,
                        float* out, int64_t ldo, const int* live, hipStream_t s) {
  const int64_t total = n1 * r;
  if (total == 0) return GP_OK;
  reduce_kernel<<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(part, nsplit, n1, n1_pad, r, rp,
                                                               inv_scale, a2, s2, V, ldv, out,
                                                               ldo, live);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

int choose_splits(int64_t n1_pad, int64_t n2_pad) {
  const int64_t rblocks = n1_pad / kRowsPerBlock;
  const int64_t nstage = n2_pad / JT;
  // enough work groups for ~8 per CU on 256 CUs, in multiples of the 8 XCDs
  int64_t want = ceil_div(2048, std::max<int64_t>(rblocks, 1));
  want = round_up(std::max<int64_t>(want, 8), 8);
  want = std::min<int64_t>(want, 64);
  const int rule = (int)std::max<int64_t>(1, std::min<int64_t>(want, nstage));
  return tune::f16_splits(n1_pad, n2_pad, rule);
}

}  // namespace f16
}  // namespace gpmi
