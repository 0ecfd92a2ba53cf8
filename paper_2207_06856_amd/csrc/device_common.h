// Device helpers shared by the solver kernels: kernel values in float32 and
// float64, and the logsumexp pair arithmetic of Sec. 5.2.
#pragma once

#include <math.h>

#include "internal.h"

namespace gpmi {

// float32 kernel value from the scaled squared distance r^2.
template <int KIND>
__device__ __forceinline__ float kval32(float r2) {
  if constexpr (KIND == GP_KERNEL_RBF) {
    return expf(-0.5f * r2);
  } else {
    const float r = sqrtf(r2);
    if constexpr (KIND == GP_KERNEL_MATERN12) {
      return expf(-r);
    } else if constexpr (KIND == GP_KERNEL_MATERN32) {
      const float t = 1.7320508075688772f * r;
      return (1.0f + t) * expf(-t);
    } else {
      const float t = 2.23606797749979f * r;
      return (1.0f + t + t * t * (1.0f / 3.0f)) * expf(-t);
    }
  }
}

// exp(-x) for x >= 0 from the hardware exp2 (v_exp_f32, about 1 ulp): the
// product x log2(e) is carried as t + err (err from an FMA and the low part of
// the constant), and exp2(-t - err) = exp2(-t) (1 - err ln 2) to first order,
// so the result stays within a few ulps for the arguments where it is not
// negligible.
__device__ __forceinline__ float exp_neg_fast(float x) {
  constexpr float kL2eHi = 1.44269502162933349609375f;      // float32(log2 e)
  constexpr float kL2eLo = 1.925963033500011079e-8f;        // log2 e - kL2eHi
  constexpr float kLn2 = 0.6931471805599453f;
  const float t = x * kL2eHi;
  const float err = fmaf(x, kL2eLo, fmaf(x, kL2eHi, -t));
  const float e = __builtin_amdgcn_exp2f(-t);
  return fmaf(-e * kLn2, err, e);
}

// float32 kernel value from r^2 on the hardware transcendentals (v_exp_f32,
// v_sqrt_f32); same function as kval32 to a few ulps, about half the vector
// instructions.  Used where the entries feed a float64 sum (true residual).
template <int KIND>
__device__ __forceinline__ float kval32_fast(float r2) {
  if constexpr (KIND == GP_KERNEL_RBF) {
    return exp_neg_fast(0.5f * r2);
  } else {
    const float r = __builtin_amdgcn_sqrtf(r2);
    if constexpr (KIND == GP_KERNEL_MATERN12) {
      return exp_neg_fast(r);
    } else if constexpr (KIND == GP_KERNEL_MATERN32) {
      const float t = 1.7320508075688772f * r;
      return (1.0f + t) * exp_neg_fast(t);
    } else {
      const float t = 2.23606797749979f * r;
      return fmaf(t, fmaf(t, 1.0f / 3.0f, 1.0f), 1.0f) * exp_neg_fast(t);
    }
  }
}

// float32 kernel value from r^2 with the exponent argument formed by one
// multiplication and the hardware exp2 / sqrt: RBF 2^(-r^2 log2(e) / 2);
// Matern s' = sqrt(c r^2) is the scaled distance times log2(e) (c = nu' log2(e)^2
// with nu' = 1, 3, 5), k = poly(s' ln 2) 2^(-s').  Its error relative to the
// exact function of r^2 is about |log k| times the float32 unit roundoff, the
// same order as the error that r^2 itself carries when it is summed in float32
// from coordinate differences, so nothing is gained by compensating the
// argument where the entries only feed a sum (the float64 true residual).
template <int KIND>
__device__ __forceinline__ float kval32_direct(float r2) {
  constexpr float kL2e = 1.4426950408889634f;
  constexpr float kLn2f = 0.6931471805599453f;
  if constexpr (KIND == GP_KERNEL_RBF) {
    return __builtin_amdgcn_exp2f(r2 * (-0.5f * kL2e));
  } else if constexpr (KIND == GP_KERNEL_MATERN12) {
    return __builtin_amdgcn_exp2f(-__builtin_amdgcn_sqrtf(r2 * (kL2e * kL2e)));
  } else if constexpr (KIND == GP_KERNEL_MATERN32) {
    const float sp = __builtin_amdgcn_sqrtf(r2 * (3.0f * kL2e * kL2e));
    return fmaf(sp, kLn2f, 1.0f) * __builtin_amdgcn_exp2f(-sp);
  } else {
    const float sp = __builtin_amdgcn_sqrtf(r2 * (5.0f * kL2e * kL2e));
    const float p = fmaf(sp, fmaf(sp, kLn2f * kLn2f / 3.0f, kLn2f), 1.0f);
    return p * __builtin_amdgcn_exp2f(-sp);
  }
}

// float64 kernel value from r^2 (runtime kind).
__device__ inline double kval64(int kind, double r2) {
  r2 = r2 > 0.0 ? r2 : 0.0;
  switch (kind) {
    case GP_KERNEL_RBF: return exp(-0.5 * r2);
    case GP_KERNEL_MATERN12: return exp(-sqrt(r2));
    case GP_KERNEL_MATERN32: {
      const double t = sqrt(3.0 * r2);
      return (1.0 + t) * exp(-t);
    }
    default: {
      const double t = sqrt(5.0 * r2);
      return (1.0 + t + t * t / 3.0) * exp(-t);
    }
  }
}

// ---- logsumexp pairs ----
__device__ __forceinline__ void lse_push(float& m, float& S, float w, float z) {
  if (w == 0.0f || z == 0.0f) return;
  const float y = __logf(fabsf(w)) + __logf(fabsf(z));
  if (!isfinite(y)) {
    S = NAN;
    return;
  }
  const float sg = ((w < 0.0f) != (z < 0.0f)) ? -1.0f : 1.0f;
  if (y > m) {
    S = S * __expf(m - y) + sg;
    m = y;
  } else {
    S += sg * __expf(y - m);
  }
}

__device__ __forceinline__ void lse_merge(float& m, float& S, float m2, float S2) {
  if (isnan(S2)) {
    S = NAN;
    return;
  }
  if (m2 == -INFINITY) return;
  if (m == -INFINITY) {
    if (!isnan(S)) S = S2;
    m = m2;
    return;
  }
  if (m2 > m) {
    S = S * __expf(m - m2) + S2;
    m = m2;
  } else {
    S += S2 * __expf(m2 - m);
  }
}

// log of the merged pair, or NaN if the inner product has no logarithm
__device__ __forceinline__ double lse_value(float m, float S) {
  if (!(S > 0.0f) || !isfinite(S) || m == -INFINITY) return NAN;
  return (double)m + log((double)S);
}

// acc + p[0] + p[stride] + ... + p[(n - 1) stride], added in index order; the
// loads go out eight at a time ahead of their sums, so that a short sum over
// column-split partials waits for one memory latency per eight terms rather
// than one per term (the order of the additions, hence the result, is that
// of the plain loop).
template <typename T>
__device__ __forceinline__ T ordered_split_sum(const T* __restrict__ p, int n, int64_t stride,
                                               T acc) {
  int x = 0;
  for (; x + 8 <= n; x += 8) {
    T t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = p[(int64_t)(x + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += t[u];
  }
  for (; x < n; ++x) acc += p[(int64_t)x * stride];
  return acc;
}


}  // namespace gpmi
