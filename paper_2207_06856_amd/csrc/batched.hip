// Device kernels of the batched solve: every kernel covers the whole batch
// through a segment table (one Seg per problem) and a chunk table (row ranges
// of at most kChunkRows rows of one problem).  The fused product runs one work
// group per (problem, row block, column split) item from a table sorted
// longest-first; reductions write per-chunk partials that a per-problem
// finish kernel merges in chunk order, so a problem's result does not depend
// on which other problems share the batch.  A problem whose columns are all
// frozen makes every later launch skip its work.

#include <math.h>

#include "batched.h"
#include "device_common.h"
#include "fused_tile.h"
#include "valu_tile.h"

namespace gpmi {
namespace bt {

using cg::kMaxR;
using cg::State;

__device__ __forceinline__ int pow2_at_least(int r) {
  int p = 1;
  while (p < r) p <<= 1;
  return p;
}

// largest p with start[p] <= v (start non-decreasing, start[0] = 0)
__device__ __forceinline__ int find_seg(const int64_t* start, int nprob, int64_t v) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= v)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ---- a1: augmented operands -------------------------------------------------
// Thread per (padded row, 8-half chunk) of the concatenated operands of one side.
__global__ void prep_kernel(const Seg* __restrict__ segs, int nprob, const int64_t* __restrict__ start,
                            int64_t total_rows, int side, int max_chunks,
                            _Float16* __restrict__ out, const int64_t* __restrict__ xoff) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total_rows * max_chunks) return;
  const int64_t row = t / max_chunks;
  const int ch = (int)(t % max_chunks);
  const int p = find_seg(start, nprob, row);
  const Seg& sg = segs[p];
  const int w = sg.w;
  if (ch * 8 >= w) return;
  const int64_t i = row - start[p];
  const float c = f16::arg_scale(sg.kind);
  const float alpha = sg.kind == GP_KERNEL_RBF ? c : -2.0f * c;
  const float beta = sg.kind == GP_KERNEL_RBF ? -0.5f * c : c;
  f16::h8 o;
  for (int q = 0; q < 8; ++q) o[q] = (_Float16)0.0f;
  if (i < sg.n) {
    const int d = sg.d;
    const float* x = sg.X + i * d;
    float nrm = 0.0f;
    for (int m = 0; m < d; ++m) {
      const float h = (float)(_Float16)(x[m] / sg.ls[m]);
      nrm = fmaf(h, h, nrm);
    }
    const float bn = beta * nrm;
    const _Float16 bn_hi = (_Float16)bn;
    const _Float16 bn_lo = (_Float16)(bn - (float)bn_hi);
    for (int q = 0; q < 8; ++q) {
      const int pp = ch * 8 + q;
      _Float16 v = (_Float16)0.0f;
      if (pp < 2 * d) {
        const int m = pp < d ? pp : pp - d;
        const float h = (float)(_Float16)(x[m] / sg.ls[m]);
        if (side == 0) {
          v = (_Float16)h;
        } else {
          const float ax = alpha * h;
          const _Float16 hi = (_Float16)ax;
          v = pp < d ? hi : (_Float16)(ax - (float)hi);
        }
      } else if (pp < 2 * d + 4) {
        const int e = pp - 2 * d;
        if (side == 1)
          v = e == 0 ? bn_hi : e == 1 ? bn_lo : (_Float16)1.0f;
        else
          v = e < 2 ? (_Float16)1.0f : e == 2 ? bn_hi : bn_lo;
      }
      o[q] = v;
    }
  }
  *reinterpret_cast<f16::h8*>(out + xoff[p] + i * w + ch * 8) = o;
}

// ---- right-hand-side quantisation ------------------------------------------------
// Thread per (problem, column < rp, 8-row group of the padded column side).
__global__ void quant_kernel(const Seg* __restrict__ segs, int nprob,
                             const int64_t* __restrict__ qstart, int64_t total, int rp,
                             const float* __restrict__ V, const uint32_t* __restrict__ colmax,
                             int scale_mode, _Float16* __restrict__ Vt, float* __restrict__ scale,
                             float* __restrict__ inv_scale, const int* __restrict__ live) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int p = find_seg(qstart, nprob, t);
  if (live && live[p] == 0) return;
  const Seg& sg = segs[p];
  const int64_t local = t - qstart[p];
  const int64_t groups = sg.n_pad_c / 8;
  const int c = (int)(local / groups);
  const int64_t i0 = (local % groups) * 8;
  float s = 1.0f, inv = 1.0f;
  if (c < sg.r) {
    if (scale_mode == 1) {
      s = (float)(1.0 / sqrt((double)sg.n));
      inv = (float)sqrt((double)sg.n);
    } else {
      const float m = __uint_as_float(colmax[p * kMaxR + c]);
      if (m > 0.0f && isfinite(m)) {
        int e;
        frexpf(m, &e);
        s = ldexpf(1.0f, 15 - e);
        inv = ldexpf(1.0f, e - 15);
      }
    }
    if (i0 == 0) {
      scale[p * kMaxR + c] = s;
      inv_scale[p * kMaxR + c] = inv;
    }
  }
  f16::h8 o;
  const float* v = V + sg.vec_off;
  for (int q = 0; q < 8; ++q) {
    const int64_t i = i0 + q;
    o[q] = (c < sg.r && i < sg.n) ? (_Float16)(v[i * sg.r + c] * s) : (_Float16)0.0f;
  }
  *reinterpret_cast<f16::h8*>(Vt + sg.vt_off + (int64_t)c * sg.n_pad_c + i0) = o;
}

// Column maxima of |V| per problem (for quantising an arbitrary V, e.g. x0).
__global__ void colmax_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                              const float* __restrict__ V, uint32_t* __restrict__ colmax) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  const int r = sg.r;
  __shared__ uint32_t smax[kMaxR];
  for (int c = threadIdx.x; c < kMaxR; c += blockDim.x) smax[c] = 0u;
  __syncthreads();
  const float* v = V + sg.vec_off;
  for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x)
    atomicMax(&smax[e % r], __float_as_uint(fabsf(v[e])));
  __syncthreads();
  for (int c = threadIdx.x; c < r; c += blockDim.x)
    if (smax[c]) atomicMax(&colmax[ck.p * kMaxR + c], smax[c]);
}

__global__ void fill_live_kernel(int* live, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nprob) live[p] = 1;
}

__global__ void zero_u32_kernel(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---- a2: fused product over work items ---------------------------------------------
template <int RB>
__global__ __launch_bounds__(256) void fused_kernel(const Seg* __restrict__ segs,
                                                    const Item* __restrict__ items,
                                                    const _Float16* __restrict__ Xr,
                                                    const _Float16* __restrict__ Xc,
                                                    const int64_t* __restrict__ xr_off,
                                                    const int64_t* __restrict__ xc_off,
                                                    const _Float16* __restrict__ Vt,
                                                    float* __restrict__ part,
                                                    const int* __restrict__ live) {
  __shared__ __attribute__((aligned(16))) _Float16 sX[2 * f16::x_stage_halfs<2>()];
  __shared__ __attribute__((aligned(16))) _Float16 sV[2 * f16::v_stage_halfs<RB>()];
  const Item it = items[blockIdx.x];
  if (live && live[it.p] == 0) return;
  const Seg& sg = segs[it.p];
  const int64_t nstage = sg.n_pad_c / f16::JT;
  const int64_t sb = it.split * nstage / sg.nsplit;
  const int64_t se = (it.split + 1) * nstage / sg.nsplit;
  float* P = part + sg.part_off + (int64_t)it.split * sg.n_pad_r * (16 * RB);
  const _Float16* xr = Xr + xr_off[it.p];
  const _Float16* xc = Xc + xc_off[it.p];
  const _Float16* vt = Vt + sg.vt_off;
  const int64_t rb0 = it.rblk * f16::kRowsPerBlock;
  switch (sg.kind * 2 + (sg.kc - 1)) {
    case 0: f16::fused_rows<0, 1, RB>(xr, xc, vt, sg.n_pad_c, P, rb0, sb, se, sX, sV); break;
    case 1: f16::fused_rows<0, 2, RB>(xr, xc, vt, sg.n_pad_c, P, rb0, sb, se, sX, sV); break;
    case 2: f16::fused_rows<1, 1, RB>(xr, xc, vt, sg.n_pad_c, P, rb0, sb, se, sX, sV); break;
    case 3: f16::fused_rows<1, 2, RB>(xr, xc, vt, sg.n_pad_c, P, rb0, sb, se, sX, sV); break;
    case 4: f16::fused_rows<2, 1, RB>(xr, xc, vt, sg.n_pad_c, P, rb0, sb, se, sX, sV); break;
    case 5: f16::fused_rows<2, 2, RB>(xr, xc, vt, sg.n_pad_c, P, rb0, sb, se, sX, sV); break;
    case 6: f16::fused_rows<3, 1, RB>(xr, xc, vt, sg.n_pad_c, P, rb0, sb, se, sX, sV); break;
    default: f16::fused_rows<3, 2, RB>(xr, xc, vt, sg.n_pad_c, P, rb0, sb, se, sX, sV); break;
  }
}

// out = a^2 inv_scale * sum of split partials + s^2 V; block per chunk.
__global__ void reduce_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                              const float* __restrict__ part, int rp,
                              const float* __restrict__ inv_scale, const float* __restrict__ V,
                              float* __restrict__ out, const int* __restrict__ live) {
  const Chunk ck = chunks[blockIdx.x];
  if (live && live[ck.p] == 0) return;
  const Seg& sg = segs[ck.p];
  const int r = sg.r;
  const float* P = part + sg.part_off;
  const int64_t stride = sg.n_pad_r * rp;
  for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x) {
    const int64_t i = e / r;
    const int c = (int)(e % r);
    float acc = 0.0f;
    for (int x = 0; x < sg.nsplit; ++x) acc += P[x * stride + i * rp + c];
    const int64_t g = sg.vec_off + e;
    out[g] = fmaf(sg.s2, V[g], (sg.a2 * inv_scale[ck.p * kMaxR + c]) * acc);
  }
}

// ---- per-column reductions -----------------------------------------------------
// Chunk partials of (LSE pair or dot) of a, b and optionally of a.a.
template <bool LSE>
__global__ void colred_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                              const float* __restrict__ A, const float* __restrict__ Bv,
                              const int* __restrict__ live, float* __restrict__ pm,
                              float* __restrict__ ps, double* __restrict__ pq) {
  const Chunk ck = chunks[blockIdx.x];
  if (live[ck.p] == 0) return;
  const Seg& sg = segs[ck.p];
  const int r = sg.r;
  const int rp2 = pow2_at_least(r);
  __shared__ float sm[256];
  __shared__ float ss[256];
  __shared__ float sq[256];
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  float m = -INFINITY, S = 0.0f, q2 = 0.0f;
  const float* a = A + sg.vec_off;
  const float* b = Bv + sg.vec_off;
  if (c < r)
    for (int64_t i = ck.i0 + ty; i < ck.i1; i += tys) {
      const float x = a[i * r + c], y = b[i * r + c];
      q2 = fmaf(x, x, q2);
      if (LSE)
        lse_push(m, S, x, y);
      else
        S = fmaf(x, y, S);
    }
  sm[threadIdx.x] = m;
  ss[threadIdx.x] = S;
  sq[threadIdx.x] = q2;
  for (int s2 = 128; s2 >= rp2; s2 >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s2) {
      if (LSE) {
        float m1 = sm[threadIdx.x], S1 = ss[threadIdx.x];
        lse_merge(m1, S1, sm[threadIdx.x + s2], ss[threadIdx.x + s2]);
        sm[threadIdx.x] = m1;
        ss[threadIdx.x] = S1;
      } else {
        ss[threadIdx.x] += ss[threadIdx.x + s2];
      }
      sq[threadIdx.x] += sq[threadIdx.x + s2];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < r) {
    const int64_t o = (int64_t)blockIdx.x * kMaxR + threadIdx.x;
    pm[o] = sm[threadIdx.x];
    ps[o] = ss[threadIdx.x];
    if (pq) pq[o] = sq[threadIdx.x];
  }
}

__device__ __forceinline__ void merge_chunks(const Seg& sg, int c, bool lse, const float* pm,
                                             const float* ps, const double* pq, double* logval,
                                             bool* ok, double* q2) {
  float M = -INFINITY, T = 0.0f;
  double dot = 0.0, qq = 0.0;
  for (int k = 0; k < sg.nchunk; ++k) {
    const int64_t o = (int64_t)(sg.chunk0 + k) * kMaxR + c;
    if (lse)
      lse_merge(M, T, pm[o], ps[o]);
    else
      dot += (double)ps[o];
    if (pq) qq += pq[o];
  }
  if (lse) {
    *logval = lse_value(M, T);
    *ok = isfinite(*logval);
  } else {
    *logval = dot;
    *ok = isfinite(dot) && dot > 0.0;
  }
  *q2 = qq;
}

// alpha_k for every active column; block per problem, thread per column.
__global__ void dq_finish_kernel(const Seg* __restrict__ segs, State* __restrict__ st, int* live,
                                 int lse, const float* __restrict__ pm,
                                 const float* __restrict__ ps) {
  const int p = blockIdx.x;
  if (live[p] == 0) return;
  const Seg& sg = segs[p];
  State& S = st[p];
  const int c = threadIdx.x;
  if (c < sg.r) {
    double alpha = 0.0;
    if (S.active[c]) {
      double lv, q2;
      bool ok;
      merge_chunks(sg, c, lse != 0, pm, ps, nullptr, &lv, &ok, &q2);
      if (ok) alpha = lse ? exp(S.lg[c] - lv) : S.lg[c] / lv;
      if (!ok || !isfinite(alpha)) {
        alpha = 0.0;
        S.breakdown[c] = 1;
        S.active[c] = 0;
      }
    }
    S.alpha[c] = alpha;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int k = S.k + 1;
    S.k = k;
    int na = 0;
    for (int cc = 0; cc < sg.r; ++cc) {
      na += S.active[cc];
      if (S.active[cc]) S.iters[cc] = k;
    }
    S.nactive = na;
    live[p] = na;
  }
}

// gamma_{k+1}, beta, convergence; block per problem.  init = 1 at initialisation.
__global__ void rz_finish_kernel(const Seg* __restrict__ segs, State* __restrict__ st, int* live,
                                 int lse, int init, double tol, int min_iter,
                                 const float* __restrict__ pm, const float* __restrict__ ps,
                                 const double* __restrict__ pq, uint32_t* __restrict__ colmax,
                                 float* __restrict__ history, int max_iter) {
  const int p = blockIdx.x;
  if (!init && live[p] == 0) return;
  const Seg& sg = segs[p];
  State& S = st[p];
  const int c = threadIdx.x;
  const int k = S.k;
  if (c < sg.r) {
    double g, q2;
    bool ok;
    merge_chunks(sg, c, lse != 0, pm, ps, pq, &g, &ok, &q2);
    if (S.active[c]) {
      const double rel = sqrt(q2 / S.bnorm2[c]);
      S.rel[c] = (float)rel;
      if (k >= min_iter && rel <= tol) {
        S.converged[c] = 1;
        S.active[c] = 0;
      } else if (!ok) {
        S.breakdown[c] = 1;
        S.active[c] = 0;
      } else {
        if (!init) S.beta[c] = lse ? exp(g - S.lg[c]) : g / S.lg[c];
        S.lg[c] = g;
        S.inv_sqrt_g[c] = (float)(lse ? exp(-0.5 * g) : 1.0 / sqrt(g));
      }
    }
    if (history && k <= max_iter) history[((int64_t)p * (max_iter + 1) + k) * kMaxR + c] = S.rel[c];
  }
  if (c < kMaxR) colmax[p * kMaxR + c] = 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    int na = 0;
    for (int cc = 0; cc < sg.r; ++cc) na += S.active[cc];
    S.nactive = na;
    S.append_slot = S.nbasis;
    live[p] = na;
  }
}

// ||b||^2 per column, masks; block per problem after colred over B.
__global__ void init_finish_kernel(const Seg* __restrict__ segs, State* __restrict__ st, int* live,
                                   const double* __restrict__ pq) {
  const int p = blockIdx.x;
  const Seg& sg = segs[p];
  State& S = st[p];
  const int c = threadIdx.x;
  if (c < kMaxR) {
    double b2 = 0.0;
    if (c < sg.r)
      for (int k = 0; k < sg.nchunk; ++k) b2 += pq[(int64_t)(sg.chunk0 + k) * kMaxR + c];
    const bool finite = isfinite(b2);
    const bool act = c < sg.r && finite && b2 > 0.0;
    S.bnorm2[c] = b2;
    S.active[c] = act ? 1 : 0;
    S.converged[c] = (c < sg.r && finite && b2 == 0.0) ? 1 : 0;
    S.breakdown[c] = (c < sg.r && !finite) ? 1 : 0;
    S.iters[c] = 0;
    S.alpha[c] = 0.0;
    S.beta[c] = 0.0;
    S.lg[c] = 0.0;
    S.inv_sqrt_g[c] = 0.0f;
    S.rel[c] = act ? 1.0f : 0.0f;
    S.true_rel[c] = 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int na = 0;
    for (int cc = 0; cc < sg.r; ++cc) na += S.active[cc];
    S.nactive = na;
    S.k = 0;
    S.nbasis = 0;
    S.append_slot = 0;
    live[p] = na;
  }
}

// Elementwise steps; block per chunk.
// mode 0: r = q - b (x0 given) or r = -b, x = 0; frozen columns x = r = 0
__global__ void init_residual_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                                     const State* __restrict__ st, const float* __restrict__ B,
                                     const float* __restrict__ q, float* __restrict__ X,
                                     float* __restrict__ R, int x0_given) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  const State& S = st[ck.p];
  const int r = sg.r;
  for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x) {
    const int c = (int)(e % r);
    const int64_t g = sg.vec_off + e;
    if (!S.active[c]) {
      X[g] = 0.0f;
      R[g] = 0.0f;
    } else if (x0_given) {
      R[g] = q[g] - B[g];
    } else {
      X[g] = 0.0f;
      R[g] = -B[g];
    }
  }
}

__global__ void update_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                              const State* __restrict__ st, const int* __restrict__ live,
                              float* __restrict__ X, float* __restrict__ R,
                              const float* __restrict__ D, const float* __restrict__ Q) {
  const Chunk ck = chunks[blockIdx.x];
  if (live[ck.p] == 0) return;
  const Seg& sg = segs[ck.p];
  const State& S = st[ck.p];
  const int r = sg.r;
  for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x) {
    const int c = (int)(e % r);
    if (!S.active[c]) continue;
    const int64_t g = sg.vec_off + e;
    const float a = (float)S.alpha[c];
    X[g] = fmaf(a, D[g], X[g]);
    R[g] = fmaf(a, Q[g], R[g]);
  }
}

// d = -z + beta d (init: d = -z), basis append, column maxima of |d|.
__global__ void direction_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                                 const State* __restrict__ st, const int* __restrict__ live,
                                 const float* __restrict__ Z, float* __restrict__ D,
                                 const float* __restrict__ R, float* __restrict__ Ub,
                                 float* __restrict__ Wb, int init, int reorth,
                                 uint32_t* __restrict__ colmax) {
  const Chunk ck = chunks[blockIdx.x];
  if (live[ck.p] == 0) return;
  const Seg& sg = segs[ck.p];
  const State& S = st[ck.p];
  const int r = sg.r;
  __shared__ uint32_t smax[kMaxR];
  for (int c = threadIdx.x; c < kMaxR; c += blockDim.x) smax[c] = 0u;
  __syncthreads();
  const int64_t nr = sg.n * r;
  const int slot = S.append_slot;
  for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x) {
    const int c = (int)(e % r);
    const int64_t g = sg.vec_off + e;
    float dv = D[g];
    if (S.active[c]) {
      const float zv = Z[g];
      dv = init ? -zv : fmaf((float)S.beta[c], dv, -zv);
      D[g] = dv;
      if (reorth) {
        const float sgm = S.inv_sqrt_g[c];
        Ub[sg.basis_off + slot * nr + e] = R[g] * sgm;
        if (Wb) Wb[sg.basis_off + slot * nr + e] = zv * sgm;
      }
    }
    atomicMax(&smax[c], __float_as_uint(fabsf(dv)));
  }
  __syncthreads();
  for (int c = threadIdx.x; c < r; c += blockDim.x)
    if (smax[c]) atomicMax(&colmax[ck.p * kMaxR + c], smax[c]);
}

__global__ void bump_basis_kernel(State* __restrict__ st, const int* __restrict__ live, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob || live[p] == 0) return;
  st[p].nbasis = st[p].append_slot + 1;
}

// ---- a5: re-orthogonalisation ----------------------------------------------------
// Work group (chunk, group of kJGroup basis vectors): chunk partials of w_j^T r.
__global__ void reorth_coef_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                                   const State* __restrict__ st, const int* __restrict__ live,
                                   const float* __restrict__ W, const float* __restrict__ R,
                                   int max_basis, int jgroups, float* __restrict__ pcoef) {
  const int ci = blockIdx.x / jgroups;
  const int j0 = (blockIdx.x % jgroups) * kJGroup;
  const Chunk ck = chunks[ci];
  if (live[ck.p] == 0) return;
  const int nb = st[ck.p].nbasis;
  if (j0 >= nb) return;
  const Seg& sg = segs[ck.p];
  const int r = sg.r;
  const int rp2 = pow2_at_least(r);
  __shared__ float sb[kJGroup][256];
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  const int64_t nr = sg.n * r;
  const int jn = min(kJGroup, nb - j0);
  const float* Wb = W + sg.basis_off + (int64_t)j0 * nr;
  const float* Rv = R + sg.vec_off;
  float acc[kJGroup];
#pragma unroll
  for (int q = 0; q < kJGroup; ++q) acc[q] = 0.0f;
  if (c < r)
    for (int64_t i = ck.i0 + ty; i < ck.i1; i += tys) {
      const float rv = Rv[i * r + c];
#pragma unroll
      for (int q = 0; q < kJGroup; ++q)
        if (q < jn) acc[q] = fmaf(Wb[q * nr + i * r + c], rv, acc[q]);
    }
#pragma unroll
  for (int q = 0; q < kJGroup; ++q) sb[q][threadIdx.x] = acc[q];
  for (int s2 = 128; s2 >= rp2; s2 >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s2)
#pragma unroll
      for (int q = 0; q < kJGroup; ++q) sb[q][threadIdx.x] += sb[q][threadIdx.x + s2];
  }
  __syncthreads();
  if ((int)threadIdx.x < r)
    for (int q = 0; q < jn; ++q)
      pcoef[((int64_t)ci * max_basis + j0 + q) * kMaxR + threadIdx.x] = sb[q][threadIdx.x];
}

// coef[p][j][c] = sum over the problem's chunks in order; block per problem.
__global__ void reorth_sum_kernel(const Seg* __restrict__ segs, const State* __restrict__ st,
                                  const int* __restrict__ live, const float* __restrict__ pcoef,
                                  int max_basis, float* __restrict__ coef) {
  const int p = blockIdx.x;
  if (live[p] == 0) return;
  const Seg& sg = segs[p];
  const int nb = st[p].nbasis;
  for (int e = threadIdx.x; e < nb * sg.r; e += blockDim.x) {
    const int j = e / sg.r, c = e % sg.r;
    float acc = 0.0f;
    for (int k = 0; k < sg.nchunk; ++k)
      acc += pcoef[((int64_t)(sg.chunk0 + k) * max_basis + j) * kMaxR + c];
    coef[((int64_t)p * max_basis + j) * kMaxR + c] = acc;
  }
}

// coefficients staged in LDS when they fit (USE_LDS), else read from global
template <bool USE_LDS>
__global__ void reorth_apply_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                                    const State* __restrict__ st, const int* __restrict__ live,
                                    const float* __restrict__ U, const float* __restrict__ coef,
                                    int max_basis, float* __restrict__ R) {
  const Chunk ck = chunks[blockIdx.x];
  if (live[ck.p] == 0) return;
  const Seg& sg = segs[ck.p];
  const State& S = st[ck.p];
  const int r = sg.r;
  const int nb = S.nbasis;
  const int64_t nr = sg.n * r;
  extern __shared__ float scf_lds[];       // nb x r coefficients
  const float* cf = coef + (int64_t)ck.p * max_basis * kMaxR;
  if (USE_LDS) {
    for (int e = threadIdx.x; e < nb * r; e += blockDim.x) scf_lds[e] = cf[(e / r) * kMaxR + e % r];
    __syncthreads();
  }
  auto scf_at = [&](int j, int c) { return USE_LDS ? scf_lds[j * r + c] : cf[j * kMaxR + c]; };
  const float* Ub = U + sg.basis_off;
  for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x) {
    const int c = (int)(e % r);
    if (!S.active[c]) continue;
    float v = R[sg.vec_off + e];
    int j = 0;
    for (; j + 8 <= nb; j += 8) {
      float u[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) u[q] = Ub[(j + q) * nr + e];
#pragma unroll
      for (int q = 0; q < 8; ++q) v = fmaf(-scf_at(j + q, c), u[q], v);
    }
    for (; j < nb; ++j) v = fmaf(-scf_at(j, c), Ub[j * nr + e], v);
    R[sg.vec_off + e] = v;
  }
}

// ---- a6: preconditioner apply ----------------------------------------------------
constexpr int kLtRows = 64;
__global__ __launch_bounds__(256) void lt_partial_kernel(const Seg* __restrict__ segs,
                                                         const Chunk* __restrict__ chunks,
                                                         const int* __restrict__ live,
                                                         const float* __restrict__ L32,
                                                         const float* __restrict__ Wv,
                                                         float* __restrict__ part) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  if (live[ck.p] == 0 || sg.rank == 0) return;
  __shared__ float sL[pc::kMaxRank][kLtRows + 1];
  __shared__ float sW[kLtRows][kMaxR + 1];
  const int k = sg.rank, r = sg.r;
  const int nout = k * r;
  constexpr int kPer = pc::kMaxRank * kMaxR / 256;   // outputs per thread at most
  float acc[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) acc[q] = 0.0f;
  const float* L = L32 + sg.l_off;
  const float* w = Wv + sg.vec_off;
  for (int64_t t0 = ck.i0; t0 < ck.i1; t0 += kLtRows) {
    const int rows = (int)min<int64_t>(kLtRows, ck.i1 - t0);
    __syncthreads();
    for (int e = threadIdx.x; e < k * kLtRows; e += 256) {
      const int m = e / kLtRows, ii = e % kLtRows;
      sL[m][ii] = ii < rows ? L[(int64_t)m * sg.n + t0 + ii] : 0.0f;
    }
    for (int e = threadIdx.x; e < kLtRows * r; e += 256) {
      const int ii = e / r, c = e % r;
      sW[ii][c] = ii < rows ? w[(t0 + ii) * r + c] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int o = threadIdx.x + q * 256;
      if (o < nout) {
        const int m = o / r, c = o % r;
        float a2 = acc[q];
        for (int ii = 0; ii < kLtRows; ++ii) a2 = fmaf(sL[m][ii], sW[ii][c], a2);
        acc[q] = a2;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int o = threadIdx.x + q * 256;
    if (o < nout) {
      const int m = o / r, c = o % r;
      part[((int64_t)blockIdx.x * pc::kMaxRank + m) * kMaxR + c] = acc[q];
    }
  }
}

// T = sum of chunk partials, Y = C^{-1} T (float64); block per problem.
__global__ void lt_finish_kernel(const Seg* __restrict__ segs, const int* __restrict__ live,
                                 const float* __restrict__ part, const double* __restrict__ Cinv,
                                 float* __restrict__ Y32) {
  const int p = blockIdx.x;
  const Seg& sg = segs[p];
  if (live[p] == 0 || sg.rank == 0) return;
  __shared__ double sT[pc::kMaxRank * 16];
  const int k = sg.rank, r = sg.r;
  for (int c0 = 0; c0 < r; c0 += 16) {
    const int cn = min(16, r - c0);
    __syncthreads();
    for (int o = threadIdx.x; o < k * cn; o += blockDim.x) {
      const int m = o / cn, c = o % cn;
      double acc = 0.0;
      for (int ch = 0; ch < sg.nchunk; ++ch)
        acc += part[((int64_t)(sg.chunk0 + ch) * pc::kMaxRank + m) * kMaxR + c0 + c];
      sT[o] = acc;
    }
    __syncthreads();
    const double* Ci = Cinv + sg.cinv_off;
    for (int o = threadIdx.x; o < k * cn; o += blockDim.x) {
      const int a = o / cn, c = o % cn;
      double acc = 0.0;
      for (int b = 0; b < k; ++b) acc = fma(Ci[a * k + b], sT[b * cn + c], acc);
      Y32[((int64_t)p * pc::kMaxRank + a) * kMaxR + c0 + c] = (float)acc;
    }
  }
}

// z = s^-2 r - s^-4 L y (rank > 0), z = r (rank 0: no preconditioner).
__global__ void z_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                         const int* __restrict__ live, const float* __restrict__ L32,
                         const float* __restrict__ Y32, const float* __restrict__ R,
                         float* __restrict__ Z) {
  const Chunk ck = chunks[blockIdx.x];
  if (live[ck.p] == 0) return;
  const Seg& sg = segs[ck.p];
  const int r = sg.r, k = sg.rank;
  if (k == 0) {
    for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x)
      Z[sg.vec_off + e] = R[sg.vec_off + e];
    return;
  }
  __shared__ float sy[pc::kMaxRank * kMaxR];
  const float* Yp = Y32 + (int64_t)ck.p * pc::kMaxRank * kMaxR;
  for (int e = threadIdx.x; e < k * kMaxR; e += blockDim.x) sy[e] = Yp[e];
  __syncthreads();
  const float inv_s2 = 1.0f / sg.s2;
  const float inv_s4 = inv_s2 * inv_s2;
  const float* L = L32 + sg.l_off;
  for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x) {
    const int64_t i = e / r;
    const int c = (int)(e % r);
    float s = 0.0f;
    for (int m = 0; m < k; ++m) s = fmaf(L[(int64_t)m * sg.n + i], sy[m * kMaxR + c], s);
    Z[sg.vec_off + e] = inv_s2 * R[sg.vec_off + e] - inv_s4 * s;
  }
}

// ---- a8: true residual (float64 accumulation) ------------------------------------
template <int DM>
__device__ __forceinline__ void trueres_rows(const Seg& sg, const Item& it, double* part64,
                                             float* sXraw, double (*sV)[16]) {
  constexpr int RPT = DM <= 16 ? 4 : 1;
  float (*sX)[DM] = reinterpret_cast<float (*)[DM]>(sXraw);
  const int64_t nstage = ceil_div(sg.n, valu::JT);
  const int64_t sb = it.split * nstage / sg.nsplit64;
  const int64_t se = (it.split + 1) * nstage / sg.nsplit64;
  double* P = part64 + sg.part64_off + (int64_t)it.split * sg.n * sg.r;
  const int64_t rb0 = it.rblk * valu::kRowsPerBlock * RPT;
  for (int c0 = 0; c0 < sg.r; c0 += 16) {
    switch (sg.kind) {
      case GP_KERNEL_RBF:
        valu::valu_rows<GP_KERNEL_RBF, DM, 16, RPT, double>(sg.X, sg.n, sg.X, sg.n, sg.U, sg.r, c0,
                                                            sg.d, sg.ls, P, rb0, sb, se, sX, sV);
        break;
      case GP_KERNEL_MATERN52:
        valu::valu_rows<GP_KERNEL_MATERN52, DM, 16, RPT, double>(sg.X, sg.n, sg.X, sg.n, sg.U, sg.r,
                                                                 c0, sg.d, sg.ls, P, rb0, sb, se,
                                                                 sX, sV);
        break;
      case GP_KERNEL_MATERN12:
        valu::valu_rows<GP_KERNEL_MATERN12, DM, 16, RPT, double>(sg.X, sg.n, sg.X, sg.n, sg.U, sg.r,
                                                                 c0, sg.d, sg.ls, P, rb0, sb, se,
                                                                 sX, sV);
        break;
      default:
        valu::valu_rows<GP_KERNEL_MATERN32, DM, 16, RPT, double>(sg.X, sg.n, sg.X, sg.n, sg.U, sg.r,
                                                                 c0, sg.d, sg.ls, P, rb0, sb, se,
                                                                 sX, sV);
        break;
    }
  }
}

__global__ __launch_bounds__(256) void trueres_partial_kernel(const Seg* __restrict__ segs,
                                                              const Item* __restrict__ items,
                                                              double* __restrict__ part64) {
  __shared__ float sX[valu::JT * 32];
  __shared__ double sV[valu::JT][16];
  const Item it = items[blockIdx.x];
  const Seg& sg = segs[it.p];
  switch (trueres_dm_of(sg.d)) {
    case 4: trueres_rows<4>(sg, it, part64, sX, sV); break;
    case 8: trueres_rows<8>(sg, it, part64, sX, sV); break;
    case 16: trueres_rows<16>(sg, it, part64, sX, sV); break;
    default: trueres_rows<32>(sg, it, part64, sX, sV); break;
  }
}

// per-chunk partial of ||b - K~ x||^2 per column
__global__ void trueres_chunk_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                                     const double* __restrict__ part64, double* __restrict__ pq) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  const int r = sg.r;
  const int rp2 = pow2_at_least(r);
  __shared__ double sb[256];
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  const int64_t nr = sg.n * r;
  double acc = 0.0;
  if (c < r)
    for (int64_t i = ck.i0 + ty; i < ck.i1; i += tys) {
      const int64_t e = i * r + c;
      double kx = 0.0;
      for (int s = 0; s < sg.nsplit64; ++s) kx += part64[sg.part64_off + s * nr + e];
      const double res = (double)sg.B[e] - ((double)sg.a2 * kx + (double)sg.s2 * (double)sg.U[e]);
      acc += res * res;
    }
  sb[threadIdx.x] = acc;
  for (int s2 = 128; s2 >= rp2; s2 >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s2) sb[threadIdx.x] += sb[threadIdx.x + s2];
  }
  __syncthreads();
  if ((int)threadIdx.x < r) pq[(int64_t)blockIdx.x * kMaxR + threadIdx.x] = sb[threadIdx.x];
}

__global__ void trueres_finish_kernel(const Seg* __restrict__ segs, State* __restrict__ st,
                                      const double* __restrict__ pq) {
  const int p = blockIdx.x;
  const Seg& sg = segs[p];
  const int c = threadIdx.x;
  if (c >= sg.r) return;
  double t = 0.0;
  for (int k = 0; k < sg.nchunk; ++k) t += pq[(int64_t)(sg.chunk0 + k) * kMaxR + c];
  const double b2 = st[p].bnorm2[c];
  st[p].true_rel[c] = b2 > 0.0 ? sqrt(t / b2) : sqrt(t);
}

// ---- a9: pivoted Cholesky, all problems per step ------------------------------------
__device__ inline bool better(double v, int64_t i, double bv, int64_t bi) {
  if (isnan(v)) return false;
  if (isnan(bv)) return true;
  return v > bv || (v == bv && i < bi);
}

// Chunk argmax / sum of the residual diagonal (after an optional column step m).
__device__ void chunk_argmax(const Chunk& ck, const double* diag, double* pv, int64_t* pi,
                             double* psum) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  __shared__ double ssum[256];
  double bv = -INFINITY, sum = 0.0;
  int64_t bi = INT64_MAX;
  for (int64_t i = ck.i0 + threadIdx.x; i < ck.i1; i += blockDim.x) {
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

__global__ void pc_init_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                               double* __restrict__ diag_all, double* pv, int64_t* pi,
                               double* psum) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  double* diag = diag_all + sg.diag_off;
  for (int64_t i = ck.i0 + threadIdx.x; i < ck.i1; i += blockDim.x) diag[i] = sg.a2;
  __syncthreads();
  chunk_argmax(ck, diag, pv, pi, psum);
}

// Pivot of step m for every problem still running; a problem still running at
// step m has built columns 0..m-1.
__global__ void pc_select_kernel(const Seg* __restrict__ segs, PcState* __restrict__ ps, int m,
                                 const double* __restrict__ pv, const int64_t* __restrict__ pi,
                                 const double* __restrict__ psum, int64_t* __restrict__ piv_all,
                                 int max_rank, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  const Seg& sg = segs[p];
  PcState& S = ps[p];
  if (S.stop) return;
  S.rank = m;
  double v = -INFINITY, tot = 0.0;
  int64_t idx = INT64_MAX;
  for (int k = 0; k < sg.nchunk; ++k) {
    const int g = sg.chunk0 + k;
    tot += psum[g];
    if (better(pv[g], pi[g], v, idx)) {
      v = pv[g];
      idx = pi[g];
    }
  }
  S.trace = tot;
  if (m >= sg.rank || !(v > 1e-12 * (double)sg.a2) || idx == INT64_MAX) {
    S.stop = 1;
  } else {
    S.dmax = v;
    S.pivot = idx;
    piv_all[(int64_t)p * max_rank + m] = idx;
  }
}

__global__ void pc_step_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                               PcState* __restrict__ ps, int m, double* __restrict__ L64,
                               double* __restrict__ diag_all, double* pv, int64_t* pi,
                               double* psum) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  const PcState& S = ps[ck.p];
  if (S.stop) return;
  __shared__ double lp[pc::kMaxRank];
  __shared__ double xp[kMaxDim];
  const int64_t n = sg.n;
  const int64_t p = S.pivot;
  const double inv_sq = 1.0 / sqrt(S.dmax);
  const int d = sg.d;
  double* L = L64 + sg.l_off;
  double* diag = diag_all + sg.diag_off;
  for (int t = threadIdx.x; t < m; t += blockDim.x) lp[t] = L[(int64_t)t * n + p];
  for (int t = threadIdx.x; t < d; t += blockDim.x) xp[t] = (double)sg.X[p * d + t] / (double)sg.ls[t];
  __syncthreads();
  for (int64_t i = ck.i0 + threadIdx.x; i < ck.i1; i += blockDim.x) {
    double r2 = 0.0;
    for (int t = 0; t < d; ++t) {
      const double df = (double)sg.X[i * d + t] / (double)sg.ls[t] - xp[t];
      r2 = fma(df, df, r2);
    }
    double acc = (double)sg.a2 * kval64(sg.kind, r2);
    for (int t = 0; t < m; ++t) acc = fma(-L[(int64_t)t * n + i], lp[t], acc);
    const double l = acc * inv_sq;
    L[(int64_t)m * n + i] = l;
    diag[i] = fma(-l, l, diag[i]);
  }
  __syncthreads();
  chunk_argmax(ck, diag, pv, pi, psum);
}

// C = I + s^-2 L^T L for every problem: block per (problem, 16 x 16 tile).
__global__ void pc_syrk_kernel(const Seg* __restrict__ segs, const PcState* __restrict__ ps,
                               const int4* __restrict__ tiles, const double* __restrict__ L64,
                               double* __restrict__ C) {
  const int4 t = tiles[blockIdx.x];   // (p, ta, tb, -)
  const Seg& sg = segs[t.x];
  const int k = ps[t.x].rank;
  if (t.y * 16 >= k || t.z * 16 >= k) return;
  __shared__ double la[16][65];
  __shared__ double lb[16][65];
  const int a = threadIdx.x / 16, b = threadIdx.x % 16;
  const double* L = L64 + sg.l_off;
  const int64_t n = sg.n;
  double acc = 0.0;
  for (int64_t c0 = 0; c0 < n; c0 += 64) {
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int rr = e / 64, cc = e % 64;
      const int64_t i = c0 + cc;
      const int ra = t.y * 16 + rr, rb = t.z * 16 + rr;
      la[rr][cc] = (i < n && ra < k) ? L[(int64_t)ra * n + i] : 0.0;
      lb[rr][cc] = (i < n && rb < k) ? L[(int64_t)rb * n + i] : 0.0;
    }
    __syncthreads();
    for (int cc = 0; cc < 64; ++cc) acc = fma(la[a][cc], lb[b][cc], acc);
  }
  const int ga = t.y * 16 + a, gb = t.z * 16 + b;
  if (ga < k && gb < k)
    C[sg.cinv_off + ga * k + gb] = (ga == gb ? 1.0 : 0.0) + acc / (double)sg.s2;
}

// Cholesky of C and explicit inverse; block per problem.
__global__ void pc_cholinv_kernel(const Seg* __restrict__ segs, PcState* __restrict__ ps,
                                  double* __restrict__ Call, double* __restrict__ Cinv_all) {
  const int p = blockIdx.x;
  const int k = ps[p].rank;
  if (k == 0) return;
  double* C = Call + segs[p].cinv_off;
  double* Cinv = Cinv_all + segs[p].cinv_off;
  for (int j = 0; j < k; ++j) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const double dj = C[j * k + j];
      if (!(dj > 0.0)) ps[p].not_pd = 1;
      C[j * k + j] = sqrt(fmax(dj, 1e-300));
    }
    __syncthreads();
    const double piv = C[j * k + j];
    for (int i = j + 1 + threadIdx.x; i < k; i += blockDim.x) C[i * k + j] /= piv;
    __syncthreads();
    for (int e = threadIdx.x; e < (k - j - 1) * (k - j - 1); e += blockDim.x) {
      const int i = j + 1 + e / (k - j - 1), l = j + 1 + e % (k - j - 1);
      if (l <= i) C[i * k + l] = fma(-C[i * k + j], C[l * k + j], C[i * k + l]);
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    for (int a = 0; a < k; ++a) {
      double v = a == c ? 1.0 : 0.0;
      for (int b = 0; b < a; ++b) v = fma(-C[a * k + b], Cinv[b * k + c], v);
      Cinv[a * k + c] = v / C[a * k + a];
    }
    for (int a = k - 1; a >= 0; --a) {
      double v = Cinv[a * k + c];
      for (int b = a + 1; b < k; ++b) v = fma(-C[b * k + a], Cinv[b * k + c], v);
      Cinv[a * k + c] = v / C[a * k + a];
    }
  }
}

__global__ void to_f32_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

}  // namespace bt
}  // namespace gpmi

// ---- host launchers ----------------------------------------------------------------
namespace gpmi {
namespace bt {

static inline unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)ceil_div(n, t); }

gp_status launch_prep(const Dev& D, int side, hipStream_t s) {
  const int64_t rows = side == 0 ? D.total_rows_r : D.total_rows_c;
  const int maxch = D.max_w / 8;
  prep_kernel<<<blocks_for(rows * maxch), 256, 0, s>>>(D.segs, D.nprob,
                                                       side == 0 ? D.rowstart : D.colstart, rows,
                                                       side, maxch, side == 0 ? D.Xr : D.Xc,
                                                       side == 0 ? D.xr_off : D.xc_off);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_quant(const Dev& D, const float* V, int scale_mode, const int* live,
                       hipStream_t s) {
  quant_kernel<<<blocks_for(D.qtotal), 256, 0, s>>>(D.segs, D.nprob, D.qstart, D.qtotal, D.rp, V,
                                                    D.colmax, scale_mode, D.Vt, D.scale,
                                                    D.inv_scale, live);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_colmax(const Dev& D, const float* V, hipStream_t s) {
  zero_u32_kernel<<<blocks_for((int64_t)D.nprob * kMaxR), 256, 0, s>>>(D.colmax,
                                                                       (int64_t)D.nprob * kMaxR);
  GP_HIP(hipGetLastError());
  colmax_kernel<<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, V, D.colmax);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_product(const Dev& D, const float* V, float* out, const int* live,
                         hipStream_t s) {
  void* tok = prof::begin(s);
  switch (D.rb) {
    case 1: fused_kernel<1><<<D.nitems, 256, 0, s>>>(D.segs, D.items, D.Xr, D.Xc, D.xr_off, D.xc_off, D.Vt, D.part, live); break;
    case 2: fused_kernel<2><<<D.nitems, 256, 0, s>>>(D.segs, D.items, D.Xr, D.Xc, D.xr_off, D.xc_off, D.Vt, D.part, live); break;
    case 3: fused_kernel<3><<<D.nitems, 256, 0, s>>>(D.segs, D.items, D.Xr, D.Xc, D.xr_off, D.xc_off, D.Vt, D.part, live); break;
    default: fused_kernel<4><<<D.nitems, 256, 0, s>>>(D.segs, D.items, D.Xr, D.Xc, D.xr_off, D.xc_off, D.Vt, D.part, live); break;
  }
  GP_HIP(hipGetLastError());
  prof::end(tok, s, D.entries, -1);
  reduce_kernel<<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, D.part, D.rp, D.inv_scale, V, out,
                                          live);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_colred(const Dev& D, const float* A, const float* B, bool lse, bool with_q2,
                        hipStream_t s) {
  if (lse)
    colred_kernel<true><<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, A, B, D.live, D.pm, D.ps,
                                                  with_q2 ? D.pq : nullptr);
  else
    colred_kernel<false><<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, A, B, D.live, D.pm, D.ps,
                                                   with_q2 ? D.pq : nullptr);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_init(const Dev& D, const float* B, const float* q, bool x0_given, hipStream_t s) {
  // ||b||^2: colred with A = B = b (dot), all problems treated as live
  fill_live_kernel<<<blocks_for(D.nprob), 256, 0, s>>>(D.live, D.nprob);
  GP_HIP(hipGetLastError());
  colred_kernel<false><<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, B, B, D.live, D.pm, D.ps, D.pq);
  GP_HIP(hipGetLastError());
  init_finish_kernel<<<D.nprob, 64, 0, s>>>(D.segs, D.st, D.live, D.pq);
  GP_HIP(hipGetLastError());
  (void)q;
  (void)x0_given;
  return GP_OK;
}

gp_status launch_init_residual(const Dev& D, const float* B, const float* q, float* X, float* R,
                               bool x0_given, hipStream_t s) {
  init_residual_kernel<<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, D.st, B, q, X, R,
                                                 x0_given ? 1 : 0);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_dq(const Dev& D, bool lse, hipStream_t s) {
  GP_TRY(launch_colred(D, D.d, D.q, lse, false, s));
  dq_finish_kernel<<<D.nprob, 64, 0, s>>>(D.segs, D.st, D.live, lse ? 1 : 0, D.pm, D.ps);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_update(const Dev& D, float* X, hipStream_t s) {
  update_kernel<<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, D.st, D.live, X, D.r, D.d, D.q);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_reorth(const Dev& D, hipStream_t s) {
  const float* W = D.Wb ? D.Wb : D.Ub;
  for (int pass = 0; pass < 2; ++pass) {
    const int jgroups = (D.max_basis + kJGroup - 1) / kJGroup;
    reorth_coef_kernel<<<(unsigned)(D.nchunks * jgroups), 256, 0, s>>>(
        D.segs, D.chunks, D.st, D.live, W, D.r, D.max_basis, jgroups, D.pcoef);
    GP_HIP(hipGetLastError());
    reorth_sum_kernel<<<D.nprob, 256, 0, s>>>(D.segs, D.st, D.live, D.pcoef, D.max_basis, D.coef);
    GP_HIP(hipGetLastError());
    const size_t lds = sizeof(float) * D.max_basis * D.max_r;
    if (lds <= 48 * 1024)
      reorth_apply_kernel<true><<<D.nchunks, 256, lds, s>>>(D.segs, D.chunks, D.st, D.live, D.Ub,
                                                             D.coef, D.max_basis, D.r);
    else
      reorth_apply_kernel<false><<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, D.st, D.live, D.Ub,
                                                           D.coef, D.max_basis, D.r);
    GP_HIP(hipGetLastError());
  }
  return GP_OK;
}

gp_status launch_precond(const Dev& D, hipStream_t s) {
  if (D.max_rank > 0) {
    lt_partial_kernel<<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, D.live, D.L32, D.r, D.ltpart);
    GP_HIP(hipGetLastError());
    lt_finish_kernel<<<D.nprob, 256, 0, s>>>(D.segs, D.live, D.ltpart, D.Cinv, D.Y32);
    GP_HIP(hipGetLastError());
  }
  z_kernel<<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, D.live, D.L32, D.Y32, D.r, D.z);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_rz(const Dev& D, bool lse, bool init, double tol, int min_iter, hipStream_t s) {
  GP_TRY(launch_colred(D, D.r, D.z, lse, true, s));
  rz_finish_kernel<<<D.nprob, 64, 0, s>>>(D.segs, D.st, D.live, lse ? 1 : 0, init ? 1 : 0, tol,
                                          min_iter, D.pm, D.ps, D.pq, D.colmax, D.history,
                                          D.max_basis - 1);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_direction(const Dev& D, bool init, bool reorth, hipStream_t s) {
  direction_kernel<<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, D.st, D.live, D.z, D.d, D.r, D.Ub,
                                             D.Wb, init ? 1 : 0, reorth ? 1 : 0, D.colmax);
  GP_HIP(hipGetLastError());
  if (reorth) {
    bump_basis_kernel<<<blocks_for(D.nprob), 256, 0, s>>>(D.st, D.live, D.nprob);
    GP_HIP(hipGetLastError());
  }
  return GP_OK;
}

gp_status launch_true_residual(const Dev& D, hipStream_t s) {
  trueres_partial_kernel<<<D.nitems64, 256, 0, s>>>(D.segs, D.items64, D.part64);
  GP_HIP(hipGetLastError());
  trueres_chunk_kernel<<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, D.part64, D.pq);
  GP_HIP(hipGetLastError());
  trueres_finish_kernel<<<D.nprob, 64, 0, s>>>(D.segs, D.st, D.pq);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_pivchol(const Dev& D, hipStream_t s) {
  if (D.max_rank == 0) return GP_OK;
  pc_init_kernel<<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, D.diag, D.pv, D.pi, D.psum);
  GP_HIP(hipGetLastError());
  for (int m = 0; m <= D.max_rank; ++m) {
    pc_select_kernel<<<blocks_for(D.nprob, 64), 64, 0, s>>>(D.segs, D.pcs, m, D.pv, D.pi, D.psum,
                                                            D.piv, D.max_rank, D.nprob);
    GP_HIP(hipGetLastError());
    if (m == D.max_rank) break;
    pc_step_kernel<<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, D.pcs, m, D.L64, D.diag, D.pv, D.pi,
                                             D.psum);
    GP_HIP(hipGetLastError());
  }
  if (D.ntiles > 0) {
    pc_syrk_kernel<<<D.ntiles, 256, 0, s>>>(D.segs, D.pcs, D.tiles, D.L64, D.C);
    GP_HIP(hipGetLastError());
  }
  pc_cholinv_kernel<<<D.nprob, 256, 0, s>>>(D.segs, D.pcs, D.C, D.Cinv);
  GP_HIP(hipGetLastError());
  if (D.l_total > 0) {
    to_f32_kernel<<<blocks_for(D.l_total), 256, 0, s>>>(D.L64, D.L32, D.l_total);
    GP_HIP(hipGetLastError());
  }
  return GP_OK;
}

}  // namespace bt
}  // namespace gpmi

namespace gpmi {
namespace bt {

// copy the per-problem caller arrays into / out of the concatenated vectors
__global__ void gather_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                              int which, float* __restrict__ dst) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  const float* src = which == 0 ? sg.B : sg.U;
  for (int64_t e = ck.i0 * sg.r + threadIdx.x; e < ck.i1 * sg.r; e += blockDim.x)
    dst[sg.vec_off + e] = src[e];
}

__global__ void scatter_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                               const float* __restrict__ src) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  for (int64_t e = ck.i0 * sg.r + threadIdx.x; e < ck.i1 * sg.r; e += blockDim.x)
    sg.U[e] = src[sg.vec_off + e];
}

gp_status launch_gather(const Dev& D, int which, float* dst, hipStream_t s) {
  gather_kernel<<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, which, dst);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status launch_scatter(const Dev& D, const float* src, hipStream_t s) {
  scatter_kernel<<<D.nchunks, 256, 0, s>>>(D.segs, D.chunks, src);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

}  // namespace bt
}  // namespace gpmi
