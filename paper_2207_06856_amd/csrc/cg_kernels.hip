// Step kernels of the batched (one step size per right-hand-side column)
// conjugate-gradients solve: the standard recurrence of App. A Alg. 2 and the
// enhanced-stability recurrence of Sec. 5.2 / Alg. 1.
//
// Vectors are n x r row-major float32.  Per-column reductions over the n rows
// run in a fixed grid of blocks that write partial results; a one-block launch
// then merges the partials in block order, so results are deterministic, and
// finishes the scalar work of the step (step sizes, masks, convergence) in
// device memory.  The host only polls the number of active columns every few
// iterations.
//
// Logsumexp inner products (Sec. 5.2): for w^T z > 0,
//   log(w^T z) = y_max + log(sum_i s_i exp(y_i - y_max)),
//   y_i = log|w_i| + log|z_i|,  s_i = sign(w_i z_i).
// Each thread keeps a running pair (m, S) = (max y, sum s exp(y - m)); pairs
// merge as (max(m1, m2), S1 exp(m1 - m) + S2 exp(m2 - m)), which equals the
// two-pass form up to rounding.  A pair whose S is not positive and finite
// means the logarithm does not exist: the column breaks down and is frozen.

#include <math.h>

#include "device_common.h"
#include "internal.h"

namespace gpmi {
namespace cg {

Dims make_dims(int64_t n, int r) {
  Dims dm;
  dm.n = n;
  dm.r = r;
  int p = 1;
  while (p < r) p <<= 1;
  dm.rp2 = p;
  const int64_t rows_per_pass = 256 / p;
  int64_t want = ceil_div(n, rows_per_pass * 4);
  // two work groups' worth of rows go to one (8 per thread), whose reduction
  // kernels then merge in the same launch: a small solve is launch-bound
  if (want <= 2) want = 1;
  dm.grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, kMaxBlocks));
  return dm;
}

// Every reduction runs as two launches: a grid of work groups writes one
// partial per group and column, then a single work group merges the partials
// (a kernel boundary makes them visible; an in-kernel "last group merges"
// scheme would need a device-scope fence per group, which on this chip writes
// back the whole L2 of the group's XCD).
//
// Parallel fixed-order merge of nparts partials: thread t takes column
// t % rp2 and partials g = t / rp2, t / rp2 + 256/rp2, ...; the per-thread
// results are then tree-reduced over the row lanes.  Partial g of column c
// sits at index g * kMaxR + c.
template <class T, class Op>
__device__ __forceinline__ T lastblock_sum(const T* part, int nparts, T* buf, int rp2, int r, T zero,
                                           Op op) {
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  T acc = zero;
  if (c < r) {
    // loads issued 32 at a time (one round trip for up to 512 partials at 16
    // row lanes), combined in the same (increasing) order
    int g = ty;
    for (; g + 31 * tys < nparts; g += 32 * tys) {
      T v[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) v[u] = part[(g + u * tys) * kMaxR + c];
#pragma unroll
      for (int u = 0; u < 32; ++u) acc = op(acc, v[u]);
    }
    for (; g < nparts; g += tys) acc = op(acc, part[g * kMaxR + c]);
  }
  buf[threadIdx.x] = acc;
  for (int s = 128; s >= rp2; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) buf[threadIdx.x] = op(buf[threadIdx.x], buf[threadIdx.x + s]);
  }
  __syncthreads();
  return buf[threadIdx.x % rp2];
}

// The same for logsumexp pairs.
__device__ __forceinline__ void lastblock_lse(const float* pm, const float* ps, int nparts, float* bm,
                                              float* bs, int rp2, int r, float* m_out, float* s_out) {
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  float M = -INFINITY, S = 0.0f;
  if (c < r) {
    int g = ty;
    for (; g + 31 * tys < nparts; g += 32 * tys) {
      float vm[32], vs[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        vm[u] = pm[(g + u * tys) * kMaxR + c];
        vs[u] = ps[(g + u * tys) * kMaxR + c];
      }
#pragma unroll
      for (int u = 0; u < 32; ++u) lse_merge(M, S, vm[u], vs[u]);
    }
    for (; g < nparts; g += tys) lse_merge(M, S, pm[g * kMaxR + c], ps[g * kMaxR + c]);
  }
  bm[threadIdx.x] = M;
  bs[threadIdx.x] = S;
  for (int s = 128; s >= rp2; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) {
      float m1 = bm[threadIdx.x], s1 = bs[threadIdx.x];
      lse_merge(m1, s1, bm[threadIdx.x + s], bs[threadIdx.x + s]);
      bm[threadIdx.x] = m1;
      bs[threadIdx.x] = s1;
    }
  }
  __syncthreads();
  *m_out = bm[threadIdx.x % rp2];
  *s_out = bs[threadIdx.x % rp2];
}

// Column-wise tree reduction in LDS over the 256/rp2 row lanes of a block.
// After it, thread t < rp2 holds column t's result in buf[t].
template <class T, class Op>
__device__ __forceinline__ void block_colreduce(T* buf, int rp2, Op op) {
  for (int s = 128; s >= rp2; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) buf[threadIdx.x] = op(buf[threadIdx.x], buf[threadIdx.x + s]);
  }
  __syncthreads();
}

// ---- init ---------------------------------------------------------------------
// ||b_c||^2, activity masks, zero right-hand sides solved by zero.
__global__ void init_state_kernel(State* st, const float* __restrict__ B, int64_t n, int r, int rp2,
                                  double* __restrict__ pd) {
  __shared__ double sb[256];
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  double acc = 0.0;
  if (c < r)
    for (int64_t i = (int64_t)blockIdx.x * tys + ty; i < n; i += (int64_t)gridDim.x * tys) {
      const double b = B[i * r + c];
      acc += b * b;
    }
  sb[threadIdx.x] = acc;
  block_colreduce(sb, rp2, [](double a, double b) { return a + b; });
  if ((int)threadIdx.x < r) pd[blockIdx.x * kMaxR + threadIdx.x] = sb[threadIdx.x];
}

__global__ void init_state_finish(State* st, int r, int rp2, const double* __restrict__ pd, int nparts) {
  __shared__ double sb[256];
  const double b2all = lastblock_sum(pd, nparts, sb, rp2, r, 0.0, [](double a, double b) { return a + b; });
  if ((int)threadIdx.x < kMaxR) {
    const int cc = threadIdx.x;
    const double b2 = cc < r ? b2all : 0.0;
    // a zero right-hand side is solved by zero; a non-finite one cannot be solved
    const bool finite = isfinite(b2);
    const bool live = cc < r && finite && b2 > 0.0;
    st->bnorm2[cc] = b2;
    st->active[cc] = live ? 1 : 0;
    st->converged[cc] = (cc < r && finite && b2 == 0.0) ? 1 : 0;
    st->breakdown[cc] = (cc < r && !finite) ? 1 : 0;
    st->iters[cc] = 0;
    st->alpha[cc] = 0.0;
    st->beta[cc] = 0.0;
    st->lg[cc] = 0.0;
    st->inv_sqrt_g[cc] = 0.0f;
    st->rel[cc] = live ? 1.0f : 0.0f;
    st->true_rel[cc] = 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int na = 0;
    for (int cc = 0; cc < r; ++cc) na += st->active[cc];
    st->nactive = na;
    st->k = 0;
    st->nbasis = 0;
    st->append_slot = 0;
  }
}

gp_status init_state(State* st, const float* B, int64_t n, int r, double* pd, hipStream_t s,
                     const Dims& dm) {
  init_state_kernel<<<dm.grid, 256, 0, s>>>(st, B, n, r, dm.rp2, pd);
  GP_HIP(hipGetLastError());
  init_state_finish<<<1, 256, 0, s>>>(st, r, dm.rp2, pd, dm.grid);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// r = K x0 - b (q holds K x0) or r = -b, x = 0; zero columns get x = r = 0.
__global__ void init_residual_kernel(const float* __restrict__ B, const float* __restrict__ q,
                                     float* __restrict__ x, float* __restrict__ rr, int x0_given,
                                     const State* __restrict__ st, int64_t n, int r) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * r) return;
  const int c = (int)(e % r);
  if (!st->active[c]) {          // zero or non-finite right-hand side
    x[e] = 0.0f;
    rr[e] = 0.0f;
    return;
  }
  if (x0_given) {
    rr[e] = q[e] - B[e];
  } else {
    x[e] = 0.0f;
    rr[e] = -B[e];
  }
}

gp_status init_residual(const float* B, const float* q, float* x, float* rr, bool x0_given,
                        const State* st, const Dims& dm, hipStream_t s) {
  const int64_t total = dm.n * dm.r;
  init_residual_kernel<<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(B, q, x, rr, x0_given ? 1 : 0,
                                                                      st, dm.n, dm.r);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// ---- a3: alpha_k from d_k^T K d_k --------------------------------------------
template <bool LSE>
__device__ __forceinline__ void dq_merge(State* st, int r, int rp2, const float* __restrict__ pm,
                                         const float* __restrict__ ps,
                                         const double* __restrict__ pd, int nparts);

template <bool LSE>
__global__ void dq_kernel(const float* __restrict__ d, const float* __restrict__ q, State* st,
                          int64_t n, int r, int rp2, float* __restrict__ pm,
                          float* __restrict__ ps, double* __restrict__ pd) {
  if (st->nactive == 0) return;
  __shared__ float sm[256];
  __shared__ float ss[256];
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  float m = -INFINITY, S = 0.0f;
  auto push = [&](float a, float b) {
    if (LSE)
      lse_push(m, S, a, b);
    else
      S = fmaf(a, b, S);
  };
  if (c < r) {
    // the loads of four rows in flight before their (in-order) pushes
    const int64_t stride = (int64_t)gridDim.x * tys;
    int64_t i = (int64_t)blockIdx.x * tys + ty;
    for (; i + 3 * stride < n; i += 4 * stride) {
      float a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = d[(i + u * stride) * r + c];
        b[u] = q[(i + u * stride) * r + c];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) push(a[u], b[u]);
    }
    for (; i < n; i += stride) push(d[i * r + c], q[i * r + c]);
  }
  if (LSE) {
    sm[threadIdx.x] = m;
    ss[threadIdx.x] = S;
    for (int s = 128; s >= rp2; s >>= 1) {
      __syncthreads();
      if ((int)threadIdx.x < s) {
        float m1 = sm[threadIdx.x], S1 = ss[threadIdx.x];
        lse_merge(m1, S1, sm[threadIdx.x + s], ss[threadIdx.x + s]);
        sm[threadIdx.x] = m1;
        ss[threadIdx.x] = S1;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < r) {
      pm[blockIdx.x * kMaxR + threadIdx.x] = sm[threadIdx.x];
      ps[blockIdx.x * kMaxR + threadIdx.x] = ss[threadIdx.x];
    }
  } else {
    ss[threadIdx.x] = S;
    block_colreduce(ss, rp2, [](float a, float b) { return a + b; });
    if ((int)threadIdx.x < r) pd[blockIdx.x * kMaxR + threadIdx.x] = ss[threadIdx.x];
  }
  // a grid of one work group merges its own partial here instead of in a
  // second launch (the barrier makes the partial's stores visible to the
  // group; every thread read nactive above, before the merge rewrites it)
  if (gridDim.x == 1) {
    __syncthreads();
    dq_merge<LSE>(st, r, rp2, pm, ps, pd, 1);
  }
}

template <bool LSE>
__device__ __forceinline__ void dq_merge(State* st, int r, int rp2, const float* __restrict__ pm,
                                         const float* __restrict__ ps,
                                         const double* __restrict__ pd, int nparts) {
  __shared__ float sm[256];
  __shared__ float ss[256];
  __shared__ double sdb[256];
  float M = -INFINITY, T = 0.0f;
  double dqv = 0.0;
  if (LSE)
    lastblock_lse(pm, ps, nparts, sm, ss, rp2, r, &M, &T);
  else
    dqv = lastblock_sum(pd, nparts, sdb, rp2, r, 0.0, [](double a, double b) { return a + b; });
  // the r <= 64 columns are the lanes of wave 0: the bookkeeping is done per
  // lane and the active count by a ballot, with no serial pass over State
  if (threadIdx.x < 64) {
    const int cc = threadIdx.x;
    const int k = st->k + 1;
    int act = 0;
    if (cc < r) {
      double alpha = 0.0;
      act = st->active[cc];
      if (act) {
        bool ok;
        if (LSE) {
          const double ld = lse_value(M, T);
          ok = isfinite(ld);
          if (ok) alpha = exp(st->lg[cc] - ld);
        } else {
          ok = isfinite(dqv) && dqv > 0.0;
          if (ok) alpha = st->lg[cc] / dqv;
        }
        if (!ok || !isfinite(alpha)) {
          alpha = 0.0;
          st->breakdown[cc] = 1;
          st->active[cc] = 0;
          act = 0;
        }
      }
      st->alpha[cc] = alpha;
      if (act) st->iters[cc] = k;
    }
    const uint64_t live = __ballot(act != 0);
    if (cc == 0) {
      st->k = k;
      st->nactive = __popcll(live);
    }
  }
}

template <bool LSE>
__global__ void dq_finish(State* st, int r, int rp2, const float* __restrict__ pm,
                          const float* __restrict__ ps, const double* __restrict__ pd, int nparts) {
  if (st->nactive == 0) return;
  dq_merge<LSE>(st, r, rp2, pm, ps, pd, nparts);
}

gp_status dq_step(const float* d, const float* q, State* st, bool lse, float* pm, float* ps,
                  double* pd, const Dims& dm, hipStream_t s) {
  if (lse) {
    dq_kernel<true><<<dm.grid, 256, 0, s>>>(d, q, st, dm.n, dm.r, dm.rp2, pm, ps, pd);
    GP_HIP(hipGetLastError());
    if (dm.grid > 1) dq_finish<true><<<1, 256, 0, s>>>(st, dm.r, dm.rp2, pm, ps, pd, dm.grid);
  } else {
    dq_kernel<false><<<dm.grid, 256, 0, s>>>(d, q, st, dm.n, dm.r, dm.rp2, pm, ps, pd);
    GP_HIP(hipGetLastError());
    if (dm.grid > 1) dq_finish<false><<<1, 256, 0, s>>>(st, dm.r, dm.rp2, pm, ps, pd, dm.grid);
  }
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// ---- a4: x += alpha d, r += alpha K d (active columns) -------------------------
__global__ void update_kernel(float* __restrict__ x, float* __restrict__ rr,
                              const float* __restrict__ d, const float* __restrict__ q,
                              const State* __restrict__ st, int64_t n, int r) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * r) return;
  const int c = (int)(e % r);
  if (!st->active[c]) return;
  const float a = (float)st->alpha[c];
  x[e] = fmaf(a, d[e], x[e]);
  rr[e] = fmaf(a, q[e], rr[e]);
}

gp_status update_step(float* x, float* rr, const float* d, const float* q, const State* st,
                      const Dims& dm, hipStream_t s) {
  const int64_t total = dm.n * dm.r;
  update_kernel<<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(x, rr, d, q, st, dm.n, dm.r);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// ---- a5: one classical Gram-Schmidt pass in the preconditioner inner product --
// coef[j][c] = w_j[:, c]^T r[:, c] for the stored pairs j < nbasis, then
// r[:, c] -= sum_j coef[j][c] u_j[:, c] for active columns.  Two passes (CGS2)
// equal Alg. 1's modified Gram-Schmidt sweep in exact arithmetic.
// The coefficients are a batched skinny product: work group (chunk, j) reduces
// one row chunk of w_j against r; a second kernel adds the chunks in order.
int reorth_chunks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(kReorthChunks, ceil_div(n, 1024)));
}

// VEC = 4 moves four adjacent right-hand-side columns per access (r % 4 == 0).
template <int VEC>
struct Vec;
template <>
struct Vec<1> {
  typedef float T;
  static __device__ __forceinline__ float get(const T& v, int) { return v; }
  static __device__ __forceinline__ T fma(T a, T b, T c) { return fmaf(a, b, c); }
  static __device__ __forceinline__ T zero() { return 0.0f; }
};
template <>
struct Vec<4> {
  typedef float4 T;
  static __device__ __forceinline__ float get(const T& v, int q) {
    return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w;
  }
  static __device__ __forceinline__ T fma(T a, T b, T c) {
    return make_float4(fmaf(a.x, b.x, c.x), fmaf(a.y, b.y, c.y), fmaf(a.z, b.z, c.z),
                       fmaf(a.w, b.w, c.w));
  }
  static __device__ __forceinline__ T zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
};

// Block (chunk, j), chunk-major: the blocks of one row chunk are adjacent, so
// its slice of r is read from HBM once and then served from cache.
template <int VEC>
__global__ void reorth_coef_kernel(const float* __restrict__ W, const float* __restrict__ rr,
                                   const State* __restrict__ st, int64_t n, int r, int rq2,
                                   int nchunk, int jmax, float* __restrict__ pcoef) {
  typedef typename Vec<VEC>::T VT;
  if (st->nactive == 0) return;
  const int chunk = blockIdx.x / jmax;
  const int j = blockIdx.x % jmax;
  if (j >= st->nbasis) return;
  __shared__ float sb[VEC][256];
  const int rq = r / VEC;                  // column groups per row
  const int cq = threadIdx.x % rq2;
  const int ty = threadIdx.x / rq2;
  const int tys = 256 / rq2;
  const int64_t nr = n * r;
  const int64_t i0 = chunk * n / nchunk, i1 = (chunk + 1) * n / nchunk;
  const VT* Wj = reinterpret_cast<const VT*>(W + j * nr);
  const VT* R4 = reinterpret_cast<const VT*>(rr);
  VT acc = Vec<VEC>::zero();
  if (cq < rq) {
    // loads four rows ahead of their (in-order) accumulation
    int64_t i = i0 + ty;
    for (; i + 3 * tys < i1; i += 4 * tys) {
      VT w[4], v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        w[u] = Wj[(i + u * tys) * rq + cq];
        v[u] = R4[(i + u * tys) * rq + cq];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = Vec<VEC>::fma(w[u], v[u], acc);
    }
    for (; i < i1; i += tys) acc = Vec<VEC>::fma(Wj[i * rq + cq], R4[i * rq + cq], acc);
  }
#pragma unroll
  for (int q = 0; q < VEC; ++q) sb[q][threadIdx.x] = Vec<VEC>::get(acc, q);
  for (int s2 = 128; s2 >= rq2; s2 >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s2)
#pragma unroll
      for (int q = 0; q < VEC; ++q) sb[q][threadIdx.x] += sb[q][threadIdx.x + s2];
  }
  __syncthreads();
  if ((int)threadIdx.x < rq)
#pragma unroll
    for (int q = 0; q < VEC; ++q)
      pcoef[((int64_t)j * nchunk + chunk) * kMaxR + threadIdx.x * VEC + q] = sb[q][threadIdx.x];
}

// coef[j][c] = sum over chunks of pcoef[j][chunk][c]: eight threads per entry
// each add an eighth of the chunks in order (loads eight at a time), and the
// eight partial sums are added in a fixed order.
constexpr int kSumLanes = 8;
__global__ void reorth_sum_kernel(const float* __restrict__ pcoef, const State* __restrict__ st,
                                  int r, int nchunk, int max_basis, float* __restrict__ coef) {
  if (st->nactive == 0) return;
  __shared__ float red[256];
  const int e = blockIdx.x * (256 / kSumLanes) + threadIdx.x / kSumLanes;
  const int q = threadIdx.x % kSumLanes;
  const int j = e / r, c = e % r;
  const bool live = j < st->nbasis && j < max_basis;
  float acc = 0.0f;
  if (live) {
    const float* base = pcoef + (int64_t)j * nchunk * kMaxR + c;
    const int g0 = q * nchunk / kSumLanes, g1 = (q + 1) * nchunk / kSumLanes;
    int g = g0;
    for (; g + 8 <= g1; g += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = base[(int64_t)(g + u) * kMaxR];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; g < g1; ++g) acc += base[(int64_t)g * kMaxR];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (live && q == 0) {
    float t = red[threadIdx.x];
#pragma unroll
    for (int u = 1; u < kSumLanes; ++u) t += red[threadIdx.x + u];
    coef[j * kMaxR + c] = t;
  }
}

template <int VEC>
__global__ void reorth_apply_kernel(const float* __restrict__ U, float* __restrict__ rr,
                                    const State* __restrict__ st, const float* __restrict__ coef,
                                    int64_t n, int r) {
  typedef typename Vec<VEC>::T VT;
  if (st->nactive == 0) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // group of VEC columns
  const int64_t nq = n * r / VEC;
  if (e >= nq) return;
  const int c0 = (int)((e * VEC) % r);
  bool any = false;
#pragma unroll
  for (int q = 0; q < VEC; ++q) any |= st->active[c0 + q] != 0;
  if (!any) return;
  const int nb = st->nbasis;
  const VT* U4 = reinterpret_cast<const VT*>(U);
  VT v = reinterpret_cast<const VT*>(rr)[e];
  float out[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q) out[q] = Vec<VEC>::get(v, q);
#pragma unroll 8
  for (int j = 0; j < nb; ++j) {
    const VT u = U4[j * nq + e];
    const VT cf = *reinterpret_cast<const VT*>(coef + j * kMaxR + c0);
#pragma unroll
    for (int q = 0; q < VEC; ++q) out[q] = fmaf(-Vec<VEC>::get(cf, q), Vec<VEC>::get(u, q), out[q]);
  }
#pragma unroll
  for (int q = 0; q < VEC; ++q)
    if (st->active[c0 + q]) rr[e * VEC + q] = out[q];
}

gp_status reorth_pass(const float* U, const float* W, float* rr, State* st, float* pcoef,
                      float* coef, int max_basis, int jmax, const Dims& dm, hipStream_t s) {
  jmax = std::max(1, std::min(jmax, max_basis));
  const int nchunk = reorth_chunks(dm.n);
  const bool v4 = dm.r % 4 == 0;
  const int rq = v4 ? dm.r / 4 : dm.r;
  int rq2 = 1;
  while (rq2 < rq) rq2 <<= 1;
  if (v4)
    reorth_coef_kernel<4><<<(unsigned)(nchunk * jmax), 256, 0, s>>>(W, rr, st, dm.n, dm.r, rq2,
                                                                     nchunk, jmax, pcoef);
  else
    reorth_coef_kernel<1><<<(unsigned)(nchunk * jmax), 256, 0, s>>>(W, rr, st, dm.n, dm.r, rq2,
                                                                     nchunk, jmax, pcoef);
  GP_HIP(hipGetLastError());
  reorth_sum_kernel<<<(unsigned)ceil_div((int64_t)jmax * dm.r, 256 / kSumLanes), 256, 0, s>>>(
      pcoef, st, dm.r, nchunk, jmax, coef);
  GP_HIP(hipGetLastError());
  const int64_t total = dm.n * dm.r / (v4 ? 4 : 1);
  if (v4)
    reorth_apply_kernel<4><<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(U, rr, st, coef, dm.n,
                                                                          dm.r);
  else
    reorth_apply_kernel<1><<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(U, rr, st, coef, dm.n,
                                                                          dm.r);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// ---- a5 in two sweeps: CGS2 through the basis Gram matrix ------------------------
// Two classical passes read the basis four times per iteration (w^T r, then
// r -= U c, twice).  With the Gram matrix G = W^T U of the stored pairs (G is
// symmetric: w_j = P(u_j) with the symmetric preconditioner P), the second
// pass's coefficients follow from the first pass's without another sweep:
//   c2 = W^T (r - U c1) = c1 - G c1,   r <- r - U (c1 + c2) = r - U (2 c1 - G c1).
// G gains one column per iteration: the coefficient sweep of an iteration also
// forms w_j^T u_new for the pair appended at the end of the previous iteration
// (one extra vector stream), and the symmetric entry fills the matching row.
// In exact arithmetic this is CGS2; in floating point it leaves out the second
// pass's correction of the first pass's own rounding in r (of order 1e-7 |r|),
// which the first pass does not amplify here because r is already nearly
// orthogonal to the basis (|c1| << |r|).

// Block (chunk, j): partials of w_j^T r and w_j^T u_new over one row chunk.
template <int VEC>
__global__ void gram_coef_kernel(const float* __restrict__ W, const float* __restrict__ U,
                                 const float* __restrict__ rr, const State* __restrict__ st,
                                 int64_t n, int r, int rq2, int nchunk, int jmax,
                                 float* __restrict__ pcoef, float* __restrict__ pgram) {
  typedef typename Vec<VEC>::T VT;
  if (st->nactive == 0) return;
  const int chunk = blockIdx.x / jmax;
  const int j = blockIdx.x % jmax;
  const int nb = st->nbasis;
  if (j >= nb) return;
  __shared__ float sb[VEC][256];
  __shared__ float sg[VEC][256];
  const int rq = r / VEC;
  const int cq = threadIdx.x % rq2;
  const int ty = threadIdx.x / rq2;
  const int tys = 256 / rq2;
  const int64_t nr = n * r;
  const int64_t i0 = chunk * n / nchunk, i1 = (chunk + 1) * n / nchunk;
  const VT* Wj = reinterpret_cast<const VT*>(W + j * nr);
  const VT* Un = reinterpret_cast<const VT*>(U + (int64_t)(nb - 1) * nr);
  const VT* R4 = reinterpret_cast<const VT*>(rr);
  VT acc = Vec<VEC>::zero(), accg = Vec<VEC>::zero();
  if (cq < rq) {
    int64_t i = i0 + ty;
    for (; i + 3 * tys < i1; i += 4 * tys) {
      VT w[4], v[4], u[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t e = (i + k * tys) * rq + cq;
        w[k] = Wj[e];
        v[k] = R4[e];
        u[k] = Un[e];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        acc = Vec<VEC>::fma(w[k], v[k], acc);
        accg = Vec<VEC>::fma(w[k], u[k], accg);
      }
    }
    for (; i < i1; i += tys) {
      const int64_t e = i * rq + cq;
      acc = Vec<VEC>::fma(Wj[e], R4[e], acc);
      accg = Vec<VEC>::fma(Wj[e], Un[e], accg);
    }
  }
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    sb[q][threadIdx.x] = Vec<VEC>::get(acc, q);
    sg[q][threadIdx.x] = Vec<VEC>::get(accg, q);
  }
  for (int s2 = 128; s2 >= rq2; s2 >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s2)
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        sb[q][threadIdx.x] += sb[q][threadIdx.x + s2];
        sg[q][threadIdx.x] += sg[q][threadIdx.x + s2];
      }
  }
  __syncthreads();
  if ((int)threadIdx.x < rq)
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      const int64_t o = ((int64_t)j * nchunk + chunk) * kMaxR + threadIdx.x * VEC + q;
      pcoef[o] = sb[q][threadIdx.x];
      pgram[o] = sg[q][threadIdx.x];
    }
}

// c1[j][c] and the new Gram column G[j][nb-1] = G[nb-1][j] (entry (j, k) of
// column c at gram[(j * max_basis + k) * r + c]): chunk partials added in
// order, eight lanes per entry as in reorth_sum_kernel.
__global__ void gram_sum_kernel(const float* __restrict__ pcoef, const float* __restrict__ pgram,
                                const State* __restrict__ st, int r, int nchunk, int max_basis,
                                float* __restrict__ c1, float* __restrict__ gram) {
  if (st->nactive == 0) return;
  __shared__ float red[2][256];
  const int e = blockIdx.x * (256 / kSumLanes) + threadIdx.x / kSumLanes;
  const int q = threadIdx.x % kSumLanes;
  const int j = e / r, c = e % r;
  const int nb = st->nbasis;
  const bool live = j < nb && j < max_basis;
  float a = 0.0f, b = 0.0f;
  if (live) {
    const int64_t base = (int64_t)j * nchunk * kMaxR + c;
    const int g0 = q * nchunk / kSumLanes, g1 = (q + 1) * nchunk / kSumLanes;
    int g = g0;
    for (; g + 8 <= g1; g += 8) {
      float va[8], vb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        va[u] = pcoef[base + (int64_t)(g + u) * kMaxR];
        vb[u] = pgram[base + (int64_t)(g + u) * kMaxR];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a += va[u];
        b += vb[u];
      }
    }
    for (; g < g1; ++g) {
      a += pcoef[base + (int64_t)g * kMaxR];
      b += pgram[base + (int64_t)g * kMaxR];
    }
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  if (live && q == 0) {
    float ta = red[0][threadIdx.x], tb = red[1][threadIdx.x];
#pragma unroll
    for (int u = 1; u < kSumLanes; ++u) {
      ta += red[0][threadIdx.x + u];
      tb += red[1][threadIdx.x + u];
    }
    c1[j * kMaxR + c] = ta;
    const int m = nb - 1;
    gram[((int64_t)j * max_basis + m) * r + c] = tb;
    gram[((int64_t)m * max_basis + j) * r + c] = tb;
  }
}

// coef[j][c] = 2 c1[j][c] - sum_k G[j][k][c] c1[k][c] in float64: work group
// (column c, 32 consecutive j), eight lanes per j each summing an eighth of the
// k range in order (eight loads in flight), combined in lane order.
constexpr int kGramLanes = 8;
__global__ void gram_apply_coef_kernel(const float* __restrict__ c1, const float* __restrict__ gram,
                                       const State* __restrict__ st, int r, int max_basis,
                                       float* __restrict__ coef) {
  if (st->nactive == 0) return;
  __shared__ double red[256];
  const int c = blockIdx.x % r;
  const int j = (blockIdx.x / r) * (256 / kGramLanes) + threadIdx.x / kGramLanes;
  const int q = threadIdx.x % kGramLanes;
  const int nb = min(st->nbasis, max_basis);
  double acc = 0.0;
  if (j < nb) {
    const float* Gj = gram + (int64_t)j * max_basis * r + c;
    const int k0 = q * nb / kGramLanes, k1 = (q + 1) * nb / kGramLanes;
    int k = k0;
    for (; k + 8 <= k1; k += 8) {
      float g[8], v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        g[u] = Gj[(int64_t)(k + u) * r];
        v[u] = c1[(k + u) * kMaxR + c];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = fma((double)g[u], (double)v[u], acc);
    }
    for (; k < k1; ++k) acc = fma((double)Gj[(int64_t)k * r], (double)c1[k * kMaxR + c], acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (j < nb && q == 0) {
    double t = red[threadIdx.x];
#pragma unroll
    for (int u = 1; u < kGramLanes; ++u) t += red[threadIdx.x + u];
    coef[j * kMaxR + c] = (float)(2.0 * (double)c1[j * kMaxR + c] - t);
  }
}

gp_status reorth_gram(const float* U, const float* W, float* rr, State* st, float* pcoef,
                      float* pgram, float* c1, float* gram, float* coef, int max_basis, int jmax,
                      const Dims& dm, hipStream_t s) {
  jmax = std::max(1, std::min(jmax, max_basis));
  const int nchunk = reorth_chunks(dm.n);
  const bool v4 = dm.r % 4 == 0;
  const int rq = v4 ? dm.r / 4 : dm.r;
  int rq2 = 1;
  while (rq2 < rq) rq2 <<= 1;
  if (v4)
    gram_coef_kernel<4><<<(unsigned)(nchunk * jmax), 256, 0, s>>>(W, U, rr, st, dm.n, dm.r, rq2,
                                                                   nchunk, jmax, pcoef, pgram);
  else
    gram_coef_kernel<1><<<(unsigned)(nchunk * jmax), 256, 0, s>>>(W, U, rr, st, dm.n, dm.r, rq2,
                                                                   nchunk, jmax, pcoef, pgram);
  GP_HIP(hipGetLastError());
  gram_sum_kernel<<<(unsigned)ceil_div((int64_t)jmax * dm.r, 256 / kSumLanes), 256, 0, s>>>(
      pcoef, pgram, st, dm.r, nchunk, max_basis, c1, gram);
  GP_HIP(hipGetLastError());
  gram_apply_coef_kernel<<<(unsigned)(dm.r * ceil_div(jmax, 256 / kGramLanes)), 256, 0, s>>>(
      c1, gram, st, dm.r, max_basis, coef);
  GP_HIP(hipGetLastError());
  const int64_t total = dm.n * dm.r / (v4 ? 4 : 1);
  if (v4)
    reorth_apply_kernel<4><<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(U, rr, st, coef, dm.n,
                                                                          dm.r);
  else
    reorth_apply_kernel<1><<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(U, rr, st, coef, dm.n,
                                                                          dm.r);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// ---- a7 (scalars): ||r||, gamma_{k+1}, beta, convergence ------------------------
template <bool LSE>
__device__ __forceinline__ void rz_merge(State* st, int r, int rp2, int init, double tol, int min_iter,
                                         const float* __restrict__ pm,
                                         const float* __restrict__ ps,
                                         const double* __restrict__ pd, int nparts,
                                         float* __restrict__ history,
                                         uint32_t* __restrict__ colmax, int rp);

template <bool LSE>
__global__ void rz_kernel(const float* __restrict__ rr, const float* __restrict__ z, State* st,
                          int64_t n, int r, int rp2, int init, float* __restrict__ pm,
                          float* __restrict__ ps, double* __restrict__ pd, double tol,
                          int min_iter, float* __restrict__ history,
                          uint32_t* __restrict__ colmax, int rp) {
  if (!init && st->nactive == 0) return;
  __shared__ float sm[256];
  __shared__ float ss[256];
  __shared__ float sq[256];
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  float m = -INFINITY, S = 0.0f, q2 = 0.0f;
  auto push = [&](float a, float b) {
    q2 = fmaf(a, a, q2);
    if (LSE)
      lse_push(m, S, a, b);
    else
      S = fmaf(a, b, S);
  };
  if (c < r) {
    const int64_t stride = (int64_t)gridDim.x * tys;
    int64_t i = (int64_t)blockIdx.x * tys + ty;
    for (; i + 3 * stride < n; i += 4 * stride) {
      float a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = rr[(i + u * stride) * r + c];
        b[u] = z[(i + u * stride) * r + c];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) push(a[u], b[u]);
    }
    for (; i < n; i += stride) push(rr[i * r + c], z[i * r + c]);
  }
  sm[threadIdx.x] = m;
  ss[threadIdx.x] = S;
  sq[threadIdx.x] = q2;
  for (int s = 128; s >= rp2; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) {
      if (LSE) {
        float m1 = sm[threadIdx.x], S1 = ss[threadIdx.x];
        lse_merge(m1, S1, sm[threadIdx.x + s], ss[threadIdx.x + s]);
        sm[threadIdx.x] = m1;
        ss[threadIdx.x] = S1;
      } else {
        ss[threadIdx.x] += ss[threadIdx.x + s];
      }
      sq[threadIdx.x] += sq[threadIdx.x + s];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < r) {
    const int64_t o = (int64_t)blockIdx.x * kMaxR + threadIdx.x;
    pm[o] = sm[threadIdx.x];
    ps[o] = ss[threadIdx.x];
    pd[o] = sq[threadIdx.x];
  }
  // a grid of one work group merges its own partial (as in dq_kernel)
  if (gridDim.x == 1) {
    __syncthreads();
    rz_merge<LSE>(st, r, rp2, init, tol, min_iter, pm, ps, pd, 1, history, colmax, rp);
  }
}

template <bool LSE>
__device__ __forceinline__ void rz_merge(State* st, int r, int rp2, int init, double tol, int min_iter,
                                         const float* __restrict__ pm,
                                         const float* __restrict__ ps,
                                         const double* __restrict__ pd, int nparts,
                                         float* __restrict__ history,
                                         uint32_t* __restrict__ colmax, int rp) {
  __shared__ float sm[256];
  __shared__ float ss[256];
  __shared__ double sdb[256];
  const int k = st->k;
  const double rr2 = lastblock_sum(pd, nparts, sdb, rp2, r, 0.0, [](double a, double b) { return a + b; });
  float M = -INFINITY, T = 0.0f;
  float dotf = 0.0f;
  if (LSE)
    lastblock_lse(pm, ps, nparts, sm, ss, rp2, r, &M, &T);
  else
    dotf = lastblock_sum(ps, nparts, ss, rp2, r, 0.0f, [](float a, float b) { return a + b; });
  const double dot = dotf;
  int act = 0;
  if ((int)threadIdx.x < r) {
    const int cc = threadIdx.x;
    double g = NAN;
    bool ok;
    if (LSE) {
      g = lse_value(M, T);
      ok = isfinite(g);
    } else {
      g = dot;
      ok = isfinite(dot) && dot > 0.0;
    }
    act = st->active[cc];
    float relc = st->rel[cc];
    if (act) {
      const double rel = sqrt(rr2 / st->bnorm2[cc]);
      relc = (float)rel;
      st->rel[cc] = relc;
      if (k >= min_iter && rel <= tol) {
        st->converged[cc] = 1;
        st->active[cc] = 0;
        act = 0;
      } else if (!ok) {
        st->breakdown[cc] = 1;
        st->active[cc] = 0;
        act = 0;
      } else {
        if (!init) st->beta[cc] = LSE ? exp(g - st->lg[cc]) : g / st->lg[cc];
        st->lg[cc] = g;
        st->inv_sqrt_g[cc] = (float)(LSE ? exp(-0.5 * g) : 1.0 / sqrt(g));
      }
    }
    if (history) history[(int64_t)k * r + cc] = relc;
  }
  for (int cc = threadIdx.x; cc < rp; cc += blockDim.x) colmax[cc] = 0u;
  // the r <= 64 columns are the lanes of wave 0: active count by a ballot
  if (threadIdx.x < 64) {
    const uint64_t live = __ballot(act != 0);
    if (threadIdx.x == 0) {
      st->nactive = __popcll(live);
      st->append_slot = st->nbasis;
    }
  }
}

template <bool LSE>
__global__ void rz_finish(State* st, int r, int rp2, int init, double tol, int min_iter,
                          const float* __restrict__ pm, const float* __restrict__ ps,
                          const double* __restrict__ pd, int nparts, float* __restrict__ history,
                          uint32_t* __restrict__ colmax, int rp) {
  if (!init && st->nactive == 0) return;
  rz_merge<LSE>(st, r, rp2, init, tol, min_iter, pm, ps, pd, nparts, history, colmax, rp);
}

gp_status rz_step(const float* rr, const float* z, State* st, bool lse, bool init, double tol,
                  int min_iter, float* pm, float* ps, double* pd, float* history,
                  uint32_t* colmax, int rp, const Dims& dm, hipStream_t s) {
  if (lse) {
    rz_kernel<true><<<dm.grid, 256, 0, s>>>(rr, z, st, dm.n, dm.r, dm.rp2, init ? 1 : 0, pm, ps, pd,
                                             tol, min_iter, history, colmax, rp);
    GP_HIP(hipGetLastError());
    if (dm.grid > 1)
      rz_finish<true><<<1, 256, 0, s>>>(st, dm.r, dm.rp2, init ? 1 : 0, tol, min_iter, pm, ps,
                                        pd, dm.grid, history, colmax, rp);
  } else {
    rz_kernel<false><<<dm.grid, 256, 0, s>>>(rr, z, st, dm.n, dm.r, dm.rp2, init ? 1 : 0, pm, ps, pd,
                                              tol, min_iter, history, colmax, rp);
    GP_HIP(hipGetLastError());
    if (dm.grid > 1)
      rz_finish<false><<<1, 256, 0, s>>>(st, dm.r, dm.rp2, init ? 1 : 0, tol, min_iter, pm, ps,
                                         pd, dm.grid, history, colmax, rp);
  }
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// ---- a7 (vectors): d = -z + beta d, basis append, column max for requantisation
__global__ void direction_kernel(const float* __restrict__ z, float* __restrict__ d,
                                 const float* __restrict__ rr, float* __restrict__ U,
                                 float* __restrict__ W, State* st, int init, int reorth,
                                 uint32_t* __restrict__ colmax, int64_t n, int r, int rp2) {
  if (st->nactive == 0) return;
  __shared__ uint32_t smax[kMaxR];
  for (int c = threadIdx.x; c < kMaxR; c += blockDim.x) smax[c] = 0u;
  __syncthreads();
  // thread (row lane, column): fixed column, its scalars and running max in registers
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  const int64_t nr = n * r;
  const int slot = st->append_slot;
  uint32_t mx = 0u;
  if (c < r) {
    const bool act = st->active[c] != 0;
    const float beta = (float)st->beta[c];
    const float sg = st->inv_sqrt_g[c];
    float* Us = U ? U + slot * nr : nullptr;
    float* Ws = W ? W + slot * nr : nullptr;
    const int64_t stride = (int64_t)gridDim.x * tys;
    auto row = [&](int64_t e, float dv, float zv, float rv) {
      if (act) {
        dv = init ? -zv : fmaf(beta, dv, -zv);
        d[e] = dv;
        if (reorth) {
          Us[e] = rv * sg;
          if (Ws) Ws[e] = zv * sg;
        }
      }
      mx = max(mx, __float_as_uint(fabsf(dv)));
    };
    // four rows' loads in flight before their updates
    int64_t i = (int64_t)blockIdx.x * tys + ty;
    for (; i + 3 * stride < n; i += 4 * stride) {
      float dv[4], zv[4], rv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t e = (i + u * stride) * r + c;
        dv[u] = d[e];
        zv[u] = act ? z[e] : 0.0f;
        rv[u] = act && reorth ? rr[e] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) row((i + u * stride) * r + c, dv[u], zv[u], rv[u]);
    }
    for (; i < n; i += stride) {
      const int64_t e = i * r + c;
      row(e, d[e], act ? z[e] : 0.0f, act && reorth ? rr[e] : 0.0f);
    }
    if (mx) atomicMax(&smax[c], mx);
  }
  __syncthreads();
  for (int cc = threadIdx.x; cc < r; cc += blockDim.x)
    if (smax[cc]) atomicMax(&colmax[cc], smax[cc]);
  // the appended basis vector counts from the next re-orthogonalisation on
  // (no block of this kernel reads nbasis)
  if (reorth && blockIdx.x == 0 && threadIdx.x == 0) st->nbasis = slot + 1;
}

gp_status direction_step(const float* z, float* d, const float* rr, float* U, float* W,
                         State* st, bool init, bool reorth, uint32_t* colmax, const Dims& dm,
                         hipStream_t s) {
  const int64_t rows_per_pass = 256 / dm.rp2;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(512, ceil_div(dm.n, rows_per_pass * 4)));
  direction_kernel<<<blocks, 256, 0, s>>>(z, d, rr, U, W, st, init ? 1 : 0, reorth ? 1 : 0, colmax,
                                          dm.n, dm.r, dm.rp2);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// ---- a8: true residual from float64-accumulated partial products -------------------
__global__ void true_res_kernel(const double* __restrict__ part, int nsplit,
                                const float* __restrict__ B, const float* __restrict__ x,
                                float a2, float s2, State* st, int64_t n, int r, int rp2,
                                double* __restrict__ pd) {
  __shared__ double sb[256];
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  const int64_t nr = n * r;
  double acc = 0.0;
  if (c < r)
    for (int64_t i = (int64_t)blockIdx.x * tys + ty; i < n; i += (int64_t)gridDim.x * tys) {
      const int64_t e = i * r + c;
      const double kx = ordered_split_sum(part + e, nsplit, nr, 0.0);
      const double res = (double)B[e] - ((double)a2 * kx + (double)s2 * (double)x[e]);
      acc += res * res;
    }
  sb[threadIdx.x] = acc;
  block_colreduce(sb, rp2, [](double a, double b) { return a + b; });
  if ((int)threadIdx.x < r) pd[blockIdx.x * kMaxR + threadIdx.x] = sb[threadIdx.x];
}

__global__ void true_res_finish(State* st, int r, int rp2, const double* __restrict__ pd, int nparts) {
  __shared__ double sb[256];
  const double t = lastblock_sum(pd, nparts, sb, rp2, r, 0.0, [](double a, double b) { return a + b; });
  if ((int)threadIdx.x < r) {
    const int cc = threadIdx.x;
    const double b2 = st->bnorm2[cc];
    st->true_rel[cc] = b2 > 0.0 ? sqrt(t / b2) : sqrt(t);
  }
}

gp_status true_residual_finish(const double* part, int nsplit, const float* B, const float* x,
                               float a2, float s2, State* st, double* pd, const Dims& dm,
                               hipStream_t s) {
  true_res_kernel<<<dm.grid, 256, 0, s>>>(part, nsplit, B, x, a2, s2, st, dm.n, dm.r, dm.rp2, pd);
  GP_HIP(hipGetLastError());
  true_res_finish<<<1, 256, 0, s>>>(st, dm.r, dm.rp2, pd, dm.grid);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

}  // namespace cg
}  // namespace gpmi
