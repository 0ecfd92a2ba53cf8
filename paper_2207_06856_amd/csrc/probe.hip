// Issue-rate and bandwidth probes of the chip (measurement support): the
// rates that the roofline figures of the benchmark are stated against.
//
// Each probe is a loop of one instruction kind with independent dependency
// chains (enough to hide its latency), over a grid that fills every compute
// unit, timed with HIP events around one launch after one warm-up launch:
//   GP_PROBE_EXP     v_exp_f32            lane operations / s
//   GP_PROBE_SQRT    v_sqrt_f32           lane operations / s
//   GP_PROBE_FMA     v_fma_f32 (the build disables packed FP32)   lane FMAs / s
//   GP_PROBE_MFMA_F16_32  v_mfma_f32_16x16x32_f16   FLOP / s (16384 per op)
//   GP_PROBE_MFMA_F16_16  v_mfma_f32_16x16x16_f16   FLOP / s (8192 per op)
//   GP_PROBE_MFMA_F64     v_mfma_f64_16x16x4_f64    FLOP / s (2048 per op)
//   GP_PROBE_COPY    device-to-device copy of 1 GiB     bytes moved (read + write) / s
//   GP_PROBE_MIX_FMA, GP_PROBE_MIX_EXP   per iteration four independent
//                    v_mfma_f32_16x16x32_f16 next to an independent vector
//                    stream sized to take about as long alone (16 v_fma_f32 or
//                    8 v_exp_f32 per lane)   MFMA FLOP / s of the mixed loop
// With GP_PROBE_TWO_WAVES added to the kind, a loop probe runs 2 work groups
// per compute unit (2 waves per SIMD) instead of 8.

#include "internal.h"

namespace gpmi {
namespace probe {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kChains = 8;

__global__ __launch_bounds__(256) void exp_kernel(int64_t iters, float seed, float* out) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = seed + 0.01f * c + 1e-6f * threadIdx.x;
  for (int64_t k = 0; k < iters; ++k)
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_exp2f(-x[c]);
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void sqrt_kernel(int64_t iters, float seed, float* out) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = seed + 0.01f * c + 1e-6f * threadIdx.x;
  for (int64_t k = 0; k < iters; ++k)
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_sqrtf(fabsf(x[c]));
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void fma_kernel(int64_t iters, float seed, float* out) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = seed + 0.01f * c + 1e-6f * threadIdx.x;
  const float a = 0.999f, b = 0.001f;
  for (int64_t k = 0; k < iters; ++k)
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = fmaf(x[c], a, b);
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void mfma32_kernel(int64_t iters, float seed, float* out) {
  h8 a, b;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    a[q] = (_Float16)(seed * 1e-3f * (q + 1));
    b[q] = (_Float16)(1e-3f * (threadIdx.x % 7));
  }
  f4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
  for (int64_t k = 0; k < iters; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[c], 0, 0, 0);
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void mfma16_kernel(int64_t iters, float seed, float* out) {
  h4 a, b;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    a[q] = (_Float16)(seed * 1e-3f * (q + 1));
    b[q] = (_Float16)(1e-3f * (threadIdx.x % 7));
  }
  f4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
  for (int64_t k = 0; k < iters; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, acc[c], 0, 0, 0);
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void mfma64_kernel(int64_t iters, float seed, float* out) {
  const double a = seed * 1e-3, b = 1e-3 * (threadIdx.x % 7);
  d4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t k = 0; k < iters; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

// Four MFMA accumulators and eight vector chains, all independent of each
// other; VK = 0: two FMAs per chain per iteration, VK = 1: one exponential.
template <int VK>
__global__ __launch_bounds__(256) void mix_kernel(int64_t iters, float seed, float* out) {
  h8 a, b;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    a[q] = (_Float16)(seed * 1e-3f * (q + 1));
    b[q] = (_Float16)(1e-3f * (threadIdx.x % 7));
  }
  f4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = seed + 0.01f * c + 1e-6f * threadIdx.x;
  const float fa = 0.999f, fb = 0.001f;
  for (int64_t k = 0; k < iters; ++k) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[c], 0, 0, 0);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float& y = x[2 * c + h];
        if constexpr (VK == 0) {
          y = fmaf(y, fa, fb);
          y = fmaf(y, fa, fb);
        } else {
          y = __builtin_amdgcn_exp2f(-y);
        }
      }
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src,
                                                   float4* __restrict__ dst, int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace probe
}  // namespace gpmi

using namespace gpmi;

extern "C" gp_status gp_probe_rate(int32_t which, int64_t iters, void* stream, double* rate) {
  clear_error();
  if (!rate) return set_error(GP_ERR_ARG, "rate is NULL");
  const bool two_waves = (which & GP_PROBE_TWO_WAVES) != 0;
  which &= ~GP_PROBE_TWO_WAVES;
  if (which < GP_PROBE_EXP || which > GP_PROBE_MIX_EXP) return set_error(GP_ERR_ARG, "unknown probe %d", which);
  if (two_waves && which == GP_PROBE_COPY)
    return set_error(GP_ERR_ARG, "GP_PROBE_TWO_WAVES applies to the loop probes only");
  if (iters < 1 || iters > (int64_t)1 << 24) return set_error(GP_ERR_ARG, "iters outside [1, 2^24]");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0, cus = 0;
  GP_HIP(hipGetDevice(&dev));
  GP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // 8 (or 2) groups of 4 waves per compute unit
  const int blocks = cus * (two_waves ? 2 : 8);
  const int threads = 256;
  float* out = nullptr;
  void* buf = nullptr;
  const int64_t copy_bytes = (int64_t)1 << 30;
  GP_HIP(hipMalloc(&out, sizeof(float) * blocks * threads));
  if (which == GP_PROBE_COPY && hipMalloc(&buf, 2 * copy_bytes) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(out);
    return set_error(GP_ERR_NOMEM, "cannot allocate the copy buffers");
  }
  hipEvent_t e0, e1;
  GP_HIP(hipEventCreate(&e0));
  GP_HIP(hipEventCreate(&e1));
  auto launch = [&]() {
    switch (which) {
      case GP_PROBE_EXP: probe::exp_kernel<<<blocks, threads, 0, s>>>(iters, 0.3f, out); break;
      case GP_PROBE_SQRT: probe::sqrt_kernel<<<blocks, threads, 0, s>>>(iters, 0.3f, out); break;
      case GP_PROBE_FMA: probe::fma_kernel<<<blocks, threads, 0, s>>>(iters, 0.3f, out); break;
      case GP_PROBE_MFMA_F16_32: probe::mfma32_kernel<<<blocks, threads, 0, s>>>(iters, 0.3f, out); break;
      case GP_PROBE_MFMA_F16_16: probe::mfma16_kernel<<<blocks, threads, 0, s>>>(iters, 0.3f, out); break;
      case GP_PROBE_MFMA_F64: probe::mfma64_kernel<<<blocks, threads, 0, s>>>(iters, 0.3f, out); break;
      case GP_PROBE_MIX_FMA: probe::mix_kernel<0><<<blocks, threads, 0, s>>>(iters, 0.3f, out); break;
      case GP_PROBE_MIX_EXP: probe::mix_kernel<1><<<blocks, threads, 0, s>>>(iters, 0.3f, out); break;
      default: {
        const int64_t n4 = copy_bytes / 16;
        const float4* src = static_cast<const float4*>(buf);
        float4* dst = reinterpret_cast<float4*>(static_cast<char*>(buf) + copy_bytes);
        for (int64_t k = 0; k < iters; ++k) probe::copy_kernel<<<cus * 16, 256, 0, s>>>(src, dst, n4);
      }
    }
  };
  launch();
  gp_status st = GP_OK;
  if (hipGetLastError() != hipSuccess) st = set_error(GP_ERR_HIP, "probe launch failed");
  float ms = 0.0f;
  if (st == GP_OK) {
    (void)hipEventRecord(e0, s);
    launch();
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      st = set_error(GP_ERR_HIP, "probe timing failed");
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (buf) (void)hipFree(buf);
  if (st != GP_OK) return st;
  const double secs = ms * 1e-3;
  const double lanes = (double)blocks * threads;
  const double waves = lanes / 64.0;
  double work = 0.0;
  switch (which) {
    case GP_PROBE_EXP:
    case GP_PROBE_SQRT:
    case GP_PROBE_FMA: work = lanes * probe::kChains * (double)iters; break;
    case GP_PROBE_MFMA_F16_32:
    case GP_PROBE_MIX_FMA:
    case GP_PROBE_MIX_EXP: work = waves * 4.0 * (double)iters * 16384.0; break;
    case GP_PROBE_MFMA_F16_16: work = waves * 4.0 * (double)iters * 8192.0; break;
    case GP_PROBE_MFMA_F64: work = waves * 4.0 * (double)iters * 2048.0; break;
    default: work = 2.0 * (double)copy_bytes * (double)iters; break;
  }
  *rate = secs > 0.0 ? work / secs : 0.0;
  return GP_OK;
}
