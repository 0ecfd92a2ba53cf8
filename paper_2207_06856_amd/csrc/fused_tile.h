// Device-side body of the fused 16-bit kernel-matrix product (binary16 or
// bfloat16 operands), shared by the single-problem kernels and the batched
// kernel.  See kmvm_f16.hip for the
// design; this file holds the tile loop only.
#pragma once

#include <math.h>

#include "internal.h"

namespace gpmi {
namespace f16 {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 16-bit operand vectors of the tile loop: binary16 or bfloat16 elements.
template <typename T>
struct Vec {
  typedef T v8 __attribute__((ext_vector_type(8)));
  typedef T v4 __attribute__((ext_vector_type(4)));
};

// v_mfma_f32_16x16x32_{f16,bf16}: float32 accumulation of 16-bit products.
template <typename T>
__device__ __forceinline__ f4 mfma32(typename Vec<T>::v8 a, typename Vec<T>::v8 b, f4 c) {
  if constexpr (__is_same(T, _Float16))
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr int kWaves = 4;
constexpr int kSub = 4;                      // 16-row subtiles per wave
constexpr int kRowsPerWave = kSub * 16;
static_assert(kWaves * kRowsPerWave == kRowsPerBlock, "row tiling");
constexpr int JT = kStageCols;
constexpr int kVStride = JT + 4;             // LDS row stride (halfs) of the V stage

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// Scale c of the exponent argument per kernel kind (see file comment).
__host__ __device__ inline float arg_scale(int kind) {
  switch (kind) {
    case GP_KERNEL_RBF: return kLog2e;
    case GP_KERNEL_MATERN52: return 5.0f * kLog2e * kLog2e;
    case GP_KERNEL_MATERN12: return kLog2e * kLog2e;
    default: return 3.0f * kLog2e * kLog2e;   // Matern-3/2
  }
}

template <int KIND>
__device__ __forceinline__ float kernel_value(float S) {
  if constexpr (KIND == GP_KERNEL_RBF) {
    return __builtin_amdgcn_exp2f(S);
  } else {
    const float sp = __builtin_amdgcn_sqrtf(fabsf(S));     // scaled distance
    const float e = __builtin_amdgcn_exp2f(-sp);
    if constexpr (KIND == GP_KERNEL_MATERN12) {
      return e;
    } else if constexpr (KIND == GP_KERNEL_MATERN32) {
      return fmaf(sp, kLn2, 1.0f) * e;                      // (1 + sqrt3 r) e^{-sqrt3 r}
    } else {
      // 1 + s + s^2/3 with s = sqrt5 r = sp * ln2
      const float p = fmaf(sp, fmaf(sp, kLn2 * kLn2 / 3.0f, kLn2), 1.0f);
      return p * e;
    }
  }
}

// LDS footprint (halfs) of one buffer of the column-point stage for width KC.
template <int KC>
constexpr int x_stage_halfs() { return JT * (32 * KC + 8); }
template <int RB>
constexpr int v_stage_halfs() { return 16 * RB * kVStride; }

// One work group: rows [row_blk, row_blk + 256) of the row operands Xr (width
// 32*KC), column stages [sb, se) of Xc / Vt (Vt row stride vt_ld), partial sums
// written to P (rows x 16*RB).  sX / sV point at two stage buffers each.  With
// a stage list, positions [sb, se) of slist name the stages instead (in
// increasing order).  T is the operand format (_Float16 or __bf16); the kernel
// values are rounded to it.
template <int KIND, int KC, int RB, typename T = _Float16>
__device__ __forceinline__ void fused_rows(const T* __restrict__ Xr,
                                           const T* __restrict__ Xc,
                                           const T* __restrict__ Vt, int64_t vt_ld,
                                           float* __restrict__ P, int64_t row_blk, int64_t sb,
                                           int64_t se, T* sXb, T* sVb,
                                           const int* __restrict__ slist = nullptr) {
  typedef typename Vec<T>::v8 h8;
  typedef typename Vec<T>::v4 h4;
  constexpr int KP = 32 * KC;          // augmented width (halfs)
  constexpr int XS = KP + 8;           // LDS row stride (halfs), 16 B padding
  constexpr int RP = 16 * RB;
  constexpr int XCH = JT * KP / 8;     // 16-byte chunks per X stage
  constexpr int VCH = RP * JT / 8;     // 16-byte chunks per V stage
  constexpr int XPT = XCH / 256;       // chunks per thread
  constexpr int VPT = VCH / 256;
  constexpr int XB = x_stage_halfs<KC>();
  constexpr int VB = v_stage_halfs<RB>();
  static_assert(XCH % 256 == 0 && VCH % 256 == 0, "stage chunking");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 4;
  const int l16 = lane & 15;
  const int64_t row0 = row_blk + wave * kRowsPerWave;

  h8 bi[kSub][KC];
#pragma unroll
  for (int is = 0; is < kSub; ++is)
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
      bi[is][kc] = *reinterpret_cast<const h8*>(Xr + (row0 + is * 16 + l16) * KP + kc * 32 + g * 8);

  f4 acc[kSub][RB];
#pragma unroll
  for (int is = 0; is < kSub; ++is)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[is][rb] = f4{0.f, 0.f, 0.f, 0.f};

  h8 xreg[XPT];
  h8 vreg[VPT];
  auto gload = [&](int64_t pos) {
    const int64_t j0 = (slist ? (int64_t)slist[pos] : pos) * JT;
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int ch = tid + q * 256;
      const int row = ch / (KP / 8), col = ch % (KP / 8);
      xreg[q] = *reinterpret_cast<const h8*>(Xc + (j0 + row) * KP + col * 8);
    }
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      const int ch = tid + q * 256;
      const int c = ch / (JT / 8), col = ch % (JT / 8);
      vreg[q] = *reinterpret_cast<const h8*>(Vt + (int64_t)c * vt_ld + j0 + col * 8);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int ch = tid + q * 256;
      const int row = ch / (KP / 8), col = ch % (KP / 8);
      *reinterpret_cast<h8*>(&sXb[buf * XB + row * XS + col * 8]) = xreg[q];
    }
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      const int ch = tid + q * 256;
      const int c = ch / (JT / 8), col = ch % (JT / 8);
      T* dst = &sVb[buf * VB + c * kVStride + col * 8];
      *reinterpret_cast<h4*>(dst) = h4{vreg[q][0], vreg[q][1], vreg[q][2], vreg[q][3]};
      *reinterpret_cast<h4*>(dst + 4) = h4{vreg[q][4], vreg[q][5], vreg[q][6], vreg[q][7]};
    }
  };

  if (sb < se) {
    gload(sb);
    lstore(0);
    __syncthreads();
  }
  for (int64_t st = sb; st < se; ++st) {
    const int buf = (int)((st - sb) & 1);
    const bool more = st + 1 < se;
    if (more) gload(st + 1);
    const T* X = sXb + buf * XB;
    const T* Vs = sVb + buf * VB;
#pragma unroll
    for (int jb = 0; jb < JT / 32; ++jb) {
      h8 a0[KC], a1[KC];
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        a0[kc] = *reinterpret_cast<const h8*>(X + (jb * 32 + l16) * XS + kc * 32 + g * 8);
        a1[kc] = *reinterpret_cast<const h8*>(X + (jb * 32 + 16 + l16) * XS + kc * 32 + g * 8);
      }
      h8 bv[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const T* vr = Vs + (rb * 16 + l16) * kVStride + jb * 32 + g * 4;
        const h4 lo = *reinterpret_cast<const h4*>(vr);
        const h4 hi = *reinterpret_cast<const h4*>(vr + 16);
        bv[rb] = h8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      }
#pragma unroll
      for (int is = 0; is < kSub; ++is) {
        f4 s0 = f4{0.f, 0.f, 0.f, 0.f}, s1 = s0;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
          s0 = mfma32<T>(a0[kc], bi[is][kc], s0);
          s1 = mfma32<T>(a1[kc], bi[is][kc], s1);
        }
        h8 kv;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          kv[v] = (T)kernel_value<KIND>(s0[v]);
          kv[4 + v] = (T)kernel_value<KIND>(s1[v]);
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
          acc[is][rb] = mfma32<T>(kv, bv[rb], acc[is][rb]);
      }
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int is = 0; is < kSub; ++is)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        P[(row0 + is * 16 + 4 * g + v) * RP + rb * 16 + l16] = acc[is][rb][v];
}

}  // namespace f16
}  // namespace gpmi
