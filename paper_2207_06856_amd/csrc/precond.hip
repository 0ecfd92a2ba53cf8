// Rank-k pivoted Cholesky preconditioner (Sec. 5.2, "Preconditioning";
// Eq. woodbury).
//
// Build (float64 throughout):
//   diag = a^2 (a stationary kernel has a constant diagonal);
//   step m: p = argmax diag (lowest index on ties); stop if diag[p] <= 1e-12 a^2;
//           col_i = a^2 k(x_i, x_p);  L[m][i] = (col_i - sum_{m'<m} L[m'][i] L[m'][p]) / sqrt(diag[p]);
//           diag_i -= L[m][i]^2.
//   One launch per step computes the column, updates the diagonal and writes
//   per-group argmax partials; a one-group launch merges them and picks the
//   next pivot, so the host enqueues all k steps back to back.
//   C = I + s^-2 L^T L (k x k) is formed, factorised by Cholesky and inverted
//   explicitly (the inner system of Eq. woodbury, solved directly in float64).
// Apply:  P^{-1} w = s^-2 w - s^-4 L C^{-1} L^T w, with L^T w and L y from a
// float32 copy of L and C^{-1} applied in float64.
//
// L is stored rank x n (each pivot column contiguous in n), so per-row loops
// over the rank read coalesced memory.

#include <math.h>

#include <vector>

#include "device_common.h"
#include "internal.h"
#include "precond_tile.h"

namespace gpmi {
namespace pc {

constexpr int kBlocks = 1024;

struct BuildState {
  double dmax;           // residual diagonal at the current pivot
  int64_t pivot;         // current pivot
  int rank;              // columns built so far
  int stop;              // 1 once the residual diagonal is exhausted
  double trace;          // sum of the residual diagonal after the last step
  int not_pd;
  unsigned pad;
};

// (value, index) argmax with the lowest index winning ties; NaN never wins.
__device__ inline bool better(double v, int64_t i, double bv, int64_t bi) {
  if (isnan(v)) return false;
  if (isnan(bv)) return true;
  return v > bv || (v == bv && i < bi);
}

// Work-group argmax (lowest index on ties) and sum of the residual diagonal.
__device__ void argmax_partial(const double* __restrict__ diag, int64_t n, double* __restrict__ pv,
                               int64_t* __restrict__ pi, double* __restrict__ psum) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  __shared__ double ssum[256];
  double bv = -INFINITY, sum = 0.0;
  int64_t bi = INT64_MAX;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = diag[i];
    sum += v;
    if (better(v, i, bv, bi)) {
      bv = v;
      bi = i;
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  ssum[threadIdx.x] = sum;
  for (int s = 128; s > 0; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) {
      if (better(sv[threadIdx.x + s], si[threadIdx.x + s], sv[threadIdx.x], si[threadIdx.x])) {
        sv[threadIdx.x] = sv[threadIdx.x + s];
        si[threadIdx.x] = si[threadIdx.x + s];
      }
      ssum[threadIdx.x] += ssum[threadIdx.x + s];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = sv[0];
    pi[blockIdx.x] = si[0];
    psum[blockIdx.x] = ssum[0];
  }
}

// Fixed-order merge of nparts argmax partials by one work group of 256
// threads: the largest residual diagonal (lowest index on ties), its index and
// the residual trace, returned to every thread.
__device__ __forceinline__ void merge_partials(const double* __restrict__ pv,
                                               const int64_t* __restrict__ pi,
                                               const double* __restrict__ psum, int nparts,
                                               double* v_out, int64_t* idx_out, double* tot_out) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  __shared__ double ssum[256];
  double v = -INFINITY, tot = 0.0;
  int64_t idx = INT64_MAX;
  for (int g = threadIdx.x; g < nparts; g += blockDim.x) {
    tot += psum[g];
    if (better(pv[g], pi[g], v, idx)) {
      v = pv[g];
      idx = pi[g];
    }
  }
  sv[threadIdx.x] = v;
  si[threadIdx.x] = idx;
  ssum[threadIdx.x] = tot;
  for (int s = 128; s > 0; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) {
      if (better(sv[threadIdx.x + s], si[threadIdx.x + s], sv[threadIdx.x], si[threadIdx.x])) {
        sv[threadIdx.x] = sv[threadIdx.x + s];
        si[threadIdx.x] = si[threadIdx.x + s];
      }
      ssum[threadIdx.x] += ssum[threadIdx.x + s];
    }
  }
  __syncthreads();
  *v_out = sv[0];
  *idx_out = si[0];
  *tot_out = ssum[0];
  __syncthreads();
}

// One work group: the merge, the pivot of step next_m and the stop rule.  Used
// once before the first step and once after the last (trace and stop); the
// steps in between merge their predecessor's partials themselves.
__global__ void select_kernel(BuildState* bs, const double* __restrict__ pv,
                              const int64_t* __restrict__ pi, const double* __restrict__ psum,
                              int nparts, int64_t* piv_out, int next_m, int rank, double stop_abs) {
  if (bs->stop) return;
  double v, tot;
  int64_t idx;
  merge_partials(pv, pi, psum, nparts, &v, &idx, &tot);
  if (threadIdx.x == 0) {
    bs->trace = tot;
    if (next_m >= rank || !(v > stop_abs) || idx == INT64_MAX) {
      bs->stop = 1;
    } else {
      bs->dmax = v;
      bs->pivot = idx;
      piv_out[next_m] = idx;
    }
  }
}

__global__ void init_kernel(double* __restrict__ diag, int64_t n, double a2, double* pv,
                            int64_t* pi, double* psum) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    diag[i] = a2;
  __syncthreads();
  argmax_partial(diag, n, pv, pi, psum);
}

// Step m of the factorisation.  For m > 0 every work group first merges the
// partials of step m - 1 (pv_in, in the fixed order of select_kernel, so all
// groups find the same pivot; group 0 records it, the trace and the stop);
// for m = 0 the pivot comes from select_kernel.  The step writes its own
// partials to the other buffer (pv), which no group of this launch reads.
__global__ void step_kernel(const float* __restrict__ X, int64_t n, KParams kp, int m,
                            double* __restrict__ L, double* __restrict__ diag, BuildState* bs,
                            const double* __restrict__ pv_in, const int64_t* __restrict__ pi_in,
                            const double* __restrict__ psum_in, int nparts, int64_t* piv_out,
                            double stop_abs, double* pv, int64_t* pi, double* psum) {
  // The stop flag can be set by group 0 of this same launch (after its merge
  // below), so one thread reads it and the whole group follows that reading:
  // waves of one group must never disagree, or the exited ones leave their
  // slots of the merge's LDS reduction unwritten.  A group that sees the flag
  // set here returns as a whole; one that does not reaches the same stop
  // decision from its own merge of the same partials.
  __shared__ int stop_seen;
  if (threadIdx.x == 0) stop_seen = __atomic_load_n(&bs->stop, __ATOMIC_RELAXED);
  __syncthreads();
  if (stop_seen) return;
  __shared__ double lp[kMaxRank];
  __shared__ double xp[kMaxDim];
  int64_t p;
  double dmax;
  if (m == 0) {
    p = bs->pivot;
    dmax = bs->dmax;
  } else {
    double tot;
    merge_partials(pv_in, pi_in, psum_in, nparts, &dmax, &p, &tot);
    const bool stop = !(dmax > stop_abs) || p == INT64_MAX;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
      bs->trace = tot;
      if (stop) {
        bs->stop = 1;
      } else {
        bs->dmax = dmax;
        bs->pivot = p;
        piv_out[m] = p;
      }
    }
    if (stop) return;
  }
  const double inv_sq = 1.0 / sqrt(dmax);
  const int d = kp.d;
  for (int t = threadIdx.x; t < m; t += blockDim.x) lp[t] = L[(int64_t)t * n + p];
  for (int t = threadIdx.x; t < d; t += blockDim.x) xp[t] = (double)X[p * d + t] / (double)kp.ls[t];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double r2 = 0.0;
    for (int t = 0; t < d; ++t) {
      const double df = (double)X[i * d + t] / (double)kp.ls[t] - xp[t];
      r2 = fma(df, df, r2);
    }
    double acc = (double)kp.a2 * kval64(kp.kind, r2);
    acc = sub_lrow(L, n, i, lp, m, acc);
    const double l = acc * inv_sq;
    L[(int64_t)m * n + i] = l;
    diag[i] = fma(-l, l, diag[i]);
  }
  __syncthreads();
  if (threadIdx.x == 0 && blockIdx.x == 0) bs->rank = m + 1;
  argmax_partial(diag, n, pv, pi, psum);
}

// Partial L^T L on the float64 matrix cores (v_mfma_f64_16x16x4f64): work
// group b takes rows [b n / nsplit, (b + 1) n / nsplit) of all k factor columns,
// stages them 64 rows at a time in LDS (each element of L read once), and the
// four waves share the 16 x 16 tiles (ta <= tb) of the k x k result.  Lane
// layouts: A lane l holds A[l % 16][l / 16], B lane l holds B[l / 16][l % 16],
// result lane l element v holds D[l / 16 + 4 v][l % 16].  Both triangles of the
// partial are written (an off-diagonal tile also fills its mirror).
constexpr int kSyrkRows = 64;
__global__ __launch_bounds__(256) void syrk_kernel(const double* __restrict__ L, int64_t n, int k,
                                                   int nsplit, double* __restrict__ part) {
  typedef double sd4 __attribute__((ext_vector_type(4)));
  constexpr int kMaxTiles = kMaxRank / 16;
  constexpr int kMaxPairs = kMaxTiles * (kMaxTiles + 1) / 2;
  __shared__ double sl[kMaxRank][kSyrkRows + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int tk = (k + 15) / 16;
  const int npair = tk * (tk + 1) / 2;
  const int64_t i0 = blockIdx.x * n / nsplit, i1 = (blockIdx.x + 1) * n / nsplit;
  sd4 acc[(kMaxPairs + 3) / 4];
#pragma unroll
  for (int q = 0; q < (kMaxPairs + 3) / 4; ++q) acc[q] = sd4{0.0, 0.0, 0.0, 0.0};
  for (int64_t c0 = i0; c0 < i1; c0 += kSyrkRows) {
    __syncthreads();
    for (int e = threadIdx.x; e < tk * 16 * kSyrkRows; e += 256) {
      const int m = e / kSyrkRows, cc = e % kSyrkRows;
      const int64_t i = c0 + cc;
      sl[m][cc] = (m < k && i < i1) ? L[(int64_t)m * n + i] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (kMaxPairs + 3) / 4; ++q) {
      const int p = wave + 4 * q;
      if (p < npair) {
        // pair index -> (ta, tb), ta <= tb, row by row of the upper triangle
        int ta = 0, rem = p;
        while (rem >= tk - ta) {
          rem -= tk - ta;
          ++ta;
        }
        const int tb = ta + rem;
#pragma unroll 4
        for (int st = 0; st < kSyrkRows / 4; ++st) {
          const int cc = 4 * st + g;
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(sl[ta * 16 + l16][cc], sl[tb * 16 + l16][cc],
                                                        acc[q], 0, 0, 0);
        }
      }
    }
  }
  double* out = part + (int64_t)blockIdx.x * k * k;
#pragma unroll
  for (int q = 0; q < (kMaxPairs + 3) / 4; ++q) {
    const int p = wave + 4 * q;
    if (p >= npair) continue;
    int ta = 0, rem = p;
    while (rem >= tk - ta) {
      rem -= tk - ta;
      ++ta;
    }
    const int tb = ta + rem;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = ta * 16 + g + 4 * v, b = tb * 16 + l16;
      if (a < k && b < k) {
        out[a * k + b] = acc[q][v];
        if (ta != tb) out[b * k + a] = acc[q][v];   // a diagonal tile holds both itself
      }
    }
  }
}

__global__ void form_c_kernel(const double* __restrict__ part, int nsplit, int k, double inv_s2,
                              double* __restrict__ C) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * k) return;
  const double acc = ordered_split_sum(part + e, nsplit, (int64_t)k * k, 0.0);
  C[e] = (e / k == e % k ? 1.0 : 0.0) + inv_s2 * acc;
}

// Cholesky of C and explicit inverse into Cinv (chol_inverse); one work group
// of 1024 threads (the per-entry operation sequences do not depend on the
// group size, so the result is the same as with any other size >= kMaxRank).
constexpr int kCholThreads = 1024;
__global__ __launch_bounds__(kCholThreads) void chol_inv_kernel(const double* __restrict__ C,
                                                       double* __restrict__ Cinv, int k,
                                                       BuildState* bs) {
  __shared__ double A[kMaxRank * kMaxRank];
  chol_inverse(C, Cinv, k, A, &bs->not_pd);
}

__global__ void to_f32_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ---- apply ----------------------------------------------------------------
// T = L^T w on the matrix cores (precond_tile.h): one work group per row chunk
// writes a k x r float32 partial; lt_sum adds the chunk partials in chunk order
// in float64 (four threads per entry, fixed split, fixed combination) and
// lt_solve applies C^{-1} in float64 (Y = C^{-1} T, stored as float32 for the
// second product).  z = s^-2 w - s^-4 L Y with one thread per row.
// The chunk count stops at twice the CU count (the chunks also fix how the
// float32 partials group the rows, so the count does not follow the occupancy):
// one round of longer chunks instead of a second, partly empty round.
int lt_chunks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(kLtResidentChunks, ceil_div(n, kLtChunkRows)));
}

__global__ __launch_bounds__(256) void lt_partial_kernel(const float* __restrict__ L32,
                                                         const float* __restrict__ w, int64_t n,
                                                         int k, int r, int nchunk,
                                                         float* __restrict__ part,
                                                         const int* __restrict__ live) {
  if (live && *live == 0) return;
  __shared__ LtLds sm;
  const int64_t i0 = blockIdx.x * n / nchunk, i1 = (blockIdx.x + 1) * n / nchunk;
  lt_chunk_mfma(L32, n, k, w, r, i0, i1, part + (int64_t)blockIdx.x * k * r, sm);
}

// Sixteen threads per entry, each adding a sixteenth of the chunk partials in
// chunk order; the sixteen float64 sums are added in a fixed order.
constexpr int kLtSumLanes = 16;
__global__ void lt_sum_kernel(const float* __restrict__ part, int k, int r, int nchunk,
                              double* __restrict__ T64, const int* __restrict__ live) {
  if (live && *live == 0) return;
  __shared__ double red[256];
  const int o = blockIdx.x * (256 / kLtSumLanes) + threadIdx.x / kLtSumLanes;
  const int q = threadIdx.x % kLtSumLanes;
  const int kr = k * r;
  double acc = 0.0;
  if (o < kr)
    acc = sum_strided(part + o, (int64_t)kr, q * nchunk / kLtSumLanes,
                      (q + 1) * nchunk / kLtSumLanes);
  red[threadIdx.x] = acc;
  __syncthreads();
  if (q == 0 && o < kr) {
    double t = red[threadIdx.x];
#pragma unroll
    for (int u = 1; u < kLtSumLanes; ++u) t += red[threadIdx.x + u];
    T64[o] = t;
  }
}

__global__ void lt_solve_kernel(const double* __restrict__ T64, const double* __restrict__ Cinv,
                                int k, int r, float* __restrict__ Y32, const int* __restrict__ live) {
  if (live && *live == 0) return;
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= k * r) return;
  const int a = o / r, c = o % r;
  double acc = 0.0;
#pragma unroll 8
  for (int b = 0; b < k; ++b) acc = fma(Cinv[a * k + b], T64[b * r + c], acc);
  Y32[o] = (float)acc;
}

// Two threads per row, each taking eight of every sixteen right-hand sides:
// twice the waves of one thread per row, so twice the L loads in flight (the
// pair's loads of L[m][i] are one address).
__global__ void z_kernel(const float* __restrict__ L32, const float* __restrict__ Y32,
                         const float* __restrict__ w, float* __restrict__ z, int64_t n, int k,
                         int r, float inv_s2, float inv_s4, const int* __restrict__ live) {
  if (live && *live == 0) return;
  __shared__ __attribute__((aligned(16))) float sy[kMaxRank * 64];
  const int rp = (r + 15) & ~15;
  stage_y(Y32, k, r, rp, sy);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 2) + threadIdx.x / 2;
  const int h = threadIdx.x & 1;
  if (i >= n) return;
  for (int c0 = 8 * h; c0 < rp; c0 += 16) {
    float acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0f;
    auto step = [&](float l, int m) {
      const pf4* y4 = reinterpret_cast<const pf4*>(sy + m * rp + c0);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const pf4 y = y4[q];
        acc[4 * q + 0] = fmaf(l, y[0], acc[4 * q + 0]);
        acc[4 * q + 1] = fmaf(l, y[1], acc[4 * q + 1]);
        acc[4 * q + 2] = fmaf(l, y[2], acc[4 * q + 2]);
        acc[4 * q + 3] = fmaf(l, y[3], acc[4 * q + 3]);
      }
    };
    int m = 0;
    for (; m + 16 <= k; m += 16) {
      float l[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) l[u] = L32[(int64_t)(m + u) * n + i];
#pragma unroll
      for (int u = 0; u < 16; ++u) step(l[u], m + u);
    }
    for (; m < k; ++m) step(L32[(int64_t)m * n + i], m);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cc = c0 + c;
      if (cc < r) z[i * r + cc] = inv_s2 * w[i * r + cc] - inv_s4 * acc[c];
    }
  }
}

__global__ void scale_kernel(const float* __restrict__ w, float* __restrict__ z, int64_t total,
                             float inv_s2, const int* __restrict__ live) {
  if (live && *live == 0) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < total) z[e] = inv_s2 * w[e];
}

gp_status apply(const gp_precond* P, const float* rr, float* z, const cg::Dims& dm,
                const int* live, hipStream_t s) {
  const int64_t total = dm.n * dm.r;
  const float inv_s2 = 1.0f / P->kp.s2;
  if (P->rank == 0) {
    scale_kernel<<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(rr, z, total, inv_s2, live);
    GP_HIP(hipGetLastError());
    return GP_OK;
  }
  const int nchunk = lt_chunks(dm.n);
  const int kr = P->rank * dm.r;
  float* part = reinterpret_cast<float*>(P->scratch);
  double* T64 = P->scratch + (size_t)kLtMaxChunks * kMaxRank * 64 / 2;
  lt_partial_kernel<<<(unsigned)nchunk, 256, 0, s>>>(P->L32, rr, dm.n, P->rank, dm.r, nchunk, part,
                                                     live);
  GP_HIP(hipGetLastError());
  lt_sum_kernel<<<(unsigned)ceil_div(kr, 256 / kLtSumLanes), 256, 0, s>>>(part, P->rank, dm.r,
                                                                         nchunk, T64, live);
  GP_HIP(hipGetLastError());
  lt_solve_kernel<<<(unsigned)ceil_div(kr, 256), 256, 0, s>>>(T64, P->Cinv, P->rank, dm.r, P->Y32,
                                                              live);
  GP_HIP(hipGetLastError());
  z_kernel<<<(unsigned)ceil_div(dm.n, 128), 256, 0, s>>>(P->L32, P->Y32, rr, z, dm.n, P->rank,
                                                         dm.r, inv_s2, inv_s2 * inv_s2, live);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

}  // namespace pc
}  // namespace gpmi

using namespace gpmi;
using namespace gpmi::pc;

// Callers make sure no queued work uses the handle's buffers any more.
static void free_precond(gp_precond* P) {
  if (!P) return;
  block_cache_put(P->device, P->block, P->block_bytes);
  delete[] P->piv_host;
  delete P;
}

extern "C" gp_status gp_pivchol_precond(const gp_kernel* k, const float* X, int64_t n, int32_t d,
                                        int32_t rank, gp_precond** out, void* stream) {
  clear_error();
  if (!out) return set_error(GP_ERR_ARG, "out is NULL");
  KParams kp;
  GP_TRY(check_kernel(k, d, true, &kp));
  if (n < 1) return set_error(GP_ERR_ARG, "n=%lld must be >= 1", (long long)n);
  if (!X) return set_error(GP_ERR_ARG, "X is NULL");
  if (rank < 0 || rank > kMaxRank || rank > n)
    return set_error(GP_ERR_ARG, "rank=%d outside [0, min(n, %d)]", rank, kMaxRank);
  hipStream_t s = static_cast<hipStream_t>(stream);
  gp_precond* P = new gp_precond();
  *P = gp_precond{};
  GP_HIP(hipGetDevice(&P->device));
  P->n = n;
  P->d = d;
  P->kp = kp;
  P->piv_host = new int64_t[rank > 0 ? rank : 1];
  const int kr = rank > 0 ? rank : 1;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(kBlocks, ceil_div(n, 256)));
  const int tiles = (kr + 15) / 16;
  const int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(256, ceil_div(n, 8 * kSyrkRows)));
  // the handle's buffers, carved from one block (reused across handles of
  // the same size)
  auto r256 = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t scratch_n = (size_t)kLtMaxChunks * kMaxRank * 64 / 2 + (size_t)kMaxRank * 64;
  P->block_bytes = r256(sizeof(double) * (size_t)kr * n) + r256(sizeof(float) * (size_t)kr * n) +
                   r256(sizeof(double) * (size_t)kr * kr) + r256(sizeof(int64_t) * kr) +
                   r256(sizeof(double) * scratch_n) + r256(sizeof(float) * (size_t)kMaxRank * 64);
  bool ok = block_cache_get(P->block_bytes, &P->block) == GP_OK;
  if (ok) {
    Arena blk;
    blk.base = static_cast<char*>(P->block);
    blk.cap = P->block_bytes;
    P->L64 = blk.take<double>((size_t)kr * n);
    P->L32 = blk.take<float>((size_t)kr * n);
    P->Cinv = blk.take<double>((size_t)kr * kr);
    P->piv_dev = blk.take<int64_t>(kr);
    P->scratch = blk.take<double>(scratch_n);
    P->Y32 = blk.take<float>((size_t)kMaxRank * 64);
    ok = P->L64 && P->L32 && P->Cinv && P->piv_dev && P->scratch && P->Y32;
  }
  if (!ok) {
    (void)hipGetLastError();
    free_precond(P);
    return set_error(GP_ERR_NOMEM, "cannot allocate the rank-%d factor for n=%lld", rank,
                     (long long)n);
  }
  // build scratch (diag, partials, C, state) from the stream's workspace: the
  // build runs on stream s and synchronises it before returning, so later
  // users of the workspace are ordered after it
  const size_t ws = r256(sizeof(double) * n) + 4 * r256(sizeof(double) * kBlocks) +
                    2 * r256(sizeof(int64_t) * kBlocks) +
                    r256(sizeof(double) * (size_t)nsplit * kr * kr) +
                    r256(sizeof(double) * (size_t)kr * kr) + r256(sizeof(BuildState)) + 256;
  Arena ar;
  {
    const gp_status wst = workspace_get(s, ws, &ar);
    if (wst != GP_OK) {
      free_precond(P);
      return wst;
    }
  }
  double* diag = ar.take<double>(n);
  double* pv[2] = {ar.take<double>(kBlocks), ar.take<double>(kBlocks)};
  int64_t* pi[2] = {ar.take<int64_t>(kBlocks), ar.take<int64_t>(kBlocks)};
  double* psum[2] = {ar.take<double>(kBlocks), ar.take<double>(kBlocks)};
  double* sy = ar.take<double>((size_t)nsplit * kr * kr);
  double* C = ar.take<double>((size_t)kr * kr);
  BuildState* bs = ar.take<BuildState>(1);
  if (!diag || !pv[0] || !pv[1] || !pi[0] || !pi[1] || !psum[0] || !psum[1] || !sy || !C || !bs) {
    free_precond(P);
    return set_error(GP_ERR_NOMEM, "internal: preconditioner build workspace too small");
  }
  gp_status st = GP_OK;
  auto run = [&]() -> gp_status {
    GP_HIP(hipMemsetAsync(bs, 0, sizeof(BuildState), s));
    const double stop_abs = 1e-12 * (double)kp.a2;
    // partials of step m - 1 (init: m = 0) live in buffer m % 2
    init_kernel<<<grid, 256, 0, s>>>(diag, n, kp.a2, pv[0], pi[0], psum[0]);
    GP_HIP(hipGetLastError());
    select_kernel<<<1, 256, 0, s>>>(bs, pv[0], pi[0], psum[0], grid, P->piv_dev, 0, rank,
                                    stop_abs);
    GP_HIP(hipGetLastError());
    for (int m = 0; m < rank; ++m) {
      const int bi = m % 2, bo = (m + 1) % 2;
      step_kernel<<<grid, 256, 0, s>>>(X, n, kp, m, P->L64, diag, bs, pv[bi], pi[bi], psum[bi],
                                       grid, P->piv_dev, stop_abs, pv[bo], pi[bo], psum[bo]);
      GP_HIP(hipGetLastError());
    }
    select_kernel<<<1, 256, 0, s>>>(bs, pv[rank % 2], pi[rank % 2], psum[rank % 2], grid,
                                    P->piv_dev, rank, rank, stop_abs);
    GP_HIP(hipGetLastError());
    BuildState hb;
    GP_HIP(hipMemcpyAsync(&hb, bs, sizeof hb, hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    P->rank = hb.rank;
    P->trace_residual = hb.trace;
    if (P->rank > 0) {
      GP_HIP(hipMemcpy(P->piv_host, P->piv_dev, sizeof(int64_t) * P->rank, hipMemcpyDeviceToHost));
      const int kk = P->rank;
      syrk_kernel<<<nsplit, 256, 0, s>>>(P->L64, n, kk, nsplit, sy);
      GP_HIP(hipGetLastError());
      form_c_kernel<<<(kk * kk + 255) / 256, 256, 0, s>>>(sy, nsplit, kk, 1.0 / (double)kp.s2, C);
      GP_HIP(hipGetLastError());
      chol_inv_kernel<<<1, kCholThreads, 0, s>>>(C, P->Cinv, kk, bs);
      GP_HIP(hipGetLastError());
      const int64_t tot = (int64_t)kk * n;
      to_f32_kernel<<<(unsigned)ceil_div(tot, 256), 256, 0, s>>>(P->L64, P->L32, tot);
      GP_HIP(hipGetLastError());
      GP_HIP(hipMemcpyAsync(&hb, bs, sizeof hb, hipMemcpyDeviceToHost, s));
      GP_HIP(hipStreamSynchronize(s));
      if (hb.not_pd)
        return set_error(GP_ERR_NOT_PD, "inner matrix I + L^T L / s^2 is not positive definite");
    }
    (void)tiles;
    return GP_OK;
  };
  st = run();
  if (st != GP_OK) {
    (void)hipStreamSynchronize(s);
    free_precond(P);
    return st;
  }
  *out = P;
  return GP_OK;
}

extern "C" gp_status gp_precond_apply(const gp_precond* P, const float* Rm, int32_t r, float* Z,
                                      void* stream) {
  clear_error();
  if (!P) return set_error(GP_ERR_ARG, "preconditioner is NULL");
  if (r < 1 || r > cg::kMaxR) return set_error(GP_ERR_ARG, "r=%d outside [1, %d]", r, cg::kMaxR);
  if (!Rm || !Z) return set_error(GP_ERR_ARG, "NULL input/output");
  if (overlaps(Rm, (size_t)P->n * r * 4, Z, (size_t)P->n * r * 4))
    return set_error(GP_ERR_ARG, "Z overlaps the input");
  const cg::Dims dm = cg::make_dims(P->n, r);
  return apply(P, Rm, Z, dm, nullptr, static_cast<hipStream_t>(stream));
}

extern "C" gp_status gp_precond_info(const gp_precond* P, int32_t* rank_used, int64_t* pivots,
                                     double* trace_residual) {
  clear_error();
  if (!P) return set_error(GP_ERR_ARG, "preconditioner is NULL");
  if (rank_used) *rank_used = P->rank;
  if (pivots)
    for (int m = 0; m < P->rank; ++m) pivots[m] = P->piv_host[m];
  if (trace_residual) *trace_residual = P->trace_residual;
  return GP_OK;
}

extern "C" gp_status gp_precond_destroy(gp_precond* P) {
  clear_error();
  if (!P) return GP_OK;
  (void)hipDeviceSynchronize();
  free_precond(P);
  return GP_OK;
}
