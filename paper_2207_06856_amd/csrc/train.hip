// Training-step device kernels: Rademacher probes from a counter-based
// generator, and the Adam update of the hyperparameters (App. C).
//
// Probes (Sec. 2.2 Hutchinson estimate, Sec. 5.3): SplitMix64 (Steele, Lea &
// Flood, OOPSLA 2014) used counter-style, value k = mix(seed + (k + 1) * gamma)
// with gamma = 0x9E3779B97F4A7C15, sign from the top bit.
//
// Optimiser: the positive hyperparameters are softplus of raw values (the
// noise adds its floor of 1e-4), the objective is (L - sum log priors) / n
// with Gamma(shape, rate) priors (3, 6) on every lengthscale, (2, 0.15) on the
// outputscale and (1.1, 0.05) on the noise; Adam (Kingma & Ba 2015) with bias
// correction updates the raw values.  One thread per parameter, float64.

#include <math.h>

#include "internal.h"

namespace gpmi {
namespace train {

namespace {

__device__ __forceinline__ uint64_t splitmix(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void rademacher_kernel(uint64_t seed, uint64_t first, int64_t rows, int cols,
                                  float* __restrict__ out, int64_t ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols;
  const int c = (int)(e % cols);
  const uint64_t z = splitmix(seed, first + (uint64_t)e);
  out[i * ld + c] = (z >> 63) ? -1.0f : 1.0f;
}

__device__ __forceinline__ double softplus(double x) {
  return x > 0.0 ? x + log1p(exp(-x)) : log1p(exp(x));
}

__device__ __forceinline__ double sigmoid(double x) {
  if (x >= 0.0) return 1.0 / (1.0 + exp(-x));
  const double e = exp(x);
  return e / (1.0 + e);
}

constexpr double kNoiseFloor = 1e-4;

__device__ __forceinline__ double constrained(double raw, bool noise) {
  return softplus(raw) + (noise ? kNoiseFloor : 0.0);
}

__global__ void adam_kernel(DevState* st, int nl, double n, AdamOpts o) {
  const int p = threadIdx.x;
  const int np = nl + 2;
  if (p < np) {
    const double th = st->theta[p];
    double g = st->grad[p];
    if (o.priors) {
      double alpha, beta;
      if (p < nl) {
        alpha = 3.0;
        beta = 6.0;
      } else if (p == nl) {
        alpha = 2.0;
        beta = 0.15;
      } else {
        alpha = 1.1;
        beta = 0.05;
      }
      g -= (alpha - 1.0) / th - beta;   // d/dtheta of log Gamma(theta; alpha, beta)
    }
    g = g / n * sigmoid(st->raw[p]);
    const double t = (double)(st->step + 1);
    const double m = o.beta1 * st->m[p] + (1.0 - o.beta1) * g;
    const double v = o.beta2 * st->v[p] + (1.0 - o.beta2) * g * g;
    const double mhat = m / (1.0 - pow(o.beta1, t));
    const double vhat = v / (1.0 - pow(o.beta2, t));
    const double raw = st->raw[p] - o.lr * mhat / (sqrt(vhat) + o.eps);
    st->m[p] = m;
    st->v[p] = v;
    st->raw[p] = raw;
    st->rgrad[p] = g;
    st->theta[p] = constrained(raw, p == nl + 1);
  }
  __syncthreads();
  if (p == 0) st->step += 1;
}

__global__ void theta_kernel(DevState* st, int nl) {
  const int p = threadIdx.x;
  if (p < nl + 2) st->theta[p] = constrained(st->raw[p], p == nl + 1);
}

}  // namespace

gp_status launch_rademacher(uint64_t seed, uint64_t first, int64_t rows, int cols, float* out,
                            int64_t ld, hipStream_t s) {
  const int64_t total = rows * cols;
  if (total == 0) return GP_OK;
  rademacher_kernel<<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(seed, first, rows, cols, out, ld);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_adam(DevState* st, int nl, int64_t n, const AdamOpts& o, hipStream_t s) {
  adam_kernel<<<1, 64, 0, s>>>(st, nl, (double)n, o);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_theta(DevState* st, int nl, hipStream_t s) {
  theta_kernel<<<1, 64, 0, s>>>(st, nl);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

}  // namespace train
}  // namespace gpmi
