// Device kernels for many problems at once.  Elementwise and reduction kernels
// run one work group per row chunk (a Chunk names the problem and its chunk
// index); the fused product runs one work group per (problem, row block, column
// split) item from a table sorted longest-first; per-problem kernels run one
// work group per slot of the launch set's slot list.  Reductions write
// per-chunk partials into the problem's own region and a per-problem kernel
// merges them in chunk order, so a problem's result does not depend on which
// other problems share a launch.  A problem whose columns are all frozen makes
// every later launch skip its work.

#include <math.h>

#include <algorithm>

#include "batched.h"
#include "device_common.h"
#include "fused_tile.h"
#include "precond_tile.h"
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

// ---- a1: augmented operands (Sec. 3 cross-term form) -----------------------------
// Row side [x, x, 1, 1, hi(b|x|^2), lo(b|x|^2)], column side
// [hi(a x), lo(a x), hi(b|x|^2), lo(b|x|^2), 1, 1] with x = X / lengthscale in
// binary16, so that one binary16 product gives the kernel argument.  Both
// sides of a chunk's rows; the last chunk also writes the zero padding.
__global__ void prep_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  const int w = sg.w;
  const int g8 = w / 8;
  const int d = sg.d;
  const float c = f16::arg_scale(sg.kind);
  const float alpha = sg.kind == GP_KERNEL_RBF ? c : -2.0f * c;
  const float beta = sg.kind == GP_KERNEL_RBF ? -0.5f * c : c;
  for (int side = 0; side < 2; ++side) {
    const int64_t npad = side == 0 ? sg.n_pad_r : sg.n_pad_c;
    const int64_t i1 = ck.i1 == sg.n ? npad : ck.i1;
    _Float16* out = side == 0 ? sg.Xr : sg.Xc;
    for (int64_t t = threadIdx.x; t < (i1 - ck.i0) * g8; t += blockDim.x) {
      const int64_t i = ck.i0 + t / g8;
      const int ch = (int)(t % g8);
      f16::h8 o;
      for (int q = 0; q < 8; ++q) o[q] = (_Float16)0.0f;
      if (i < sg.n) {
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
      *reinterpret_cast<f16::h8*>(out + i * w + ch * 8) = o;
    }
  }
}

// ---- right-hand-side quantisation ------------------------------------------------
// Vt[c][i] = binary16(s_c v[i][c]) for the chunk's rows (the last chunk also
// zeroes the padding rows); columns r..rp-1 are zero.  Scale s_c: the power of
// two that puts max|v_c| in [2^14, 2^15) (mode 0) or n^-1/2 (mode 1).
__global__ void quant_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                             int vsel, const uint32_t* __restrict__ colmax, int scale_mode,
                             float* __restrict__ scale, float* __restrict__ inv_scale,
                             const int* __restrict__ live) {
  const Chunk ck = chunks[blockIdx.x];
  if (live && live[ck.p] == 0) return;
  const Seg& sg = segs[ck.p];
  __shared__ float ss[kMaxR];
  const int r = sg.r, rp = sg.rp;
  for (int c = threadIdx.x; c < rp; c += blockDim.x) {
    float s = 1.0f, inv = 1.0f;
    if (c < r) {
      if (scale_mode == 1) {
        s = (float)(1.0 / sqrt((double)sg.n));
        inv = (float)sqrt((double)sg.n);
      } else {
        const float m = __uint_as_float(colmax[ck.p * kMaxR + c]);
        if (m > 0.0f && isfinite(m)) {
          int e;
          frexpf(m, &e);
          s = ldexpf(1.0f, 15 - e);
          inv = ldexpf(1.0f, e - 15);
        }
      }
      if (ck.k == 0) {
        scale[ck.p * kMaxR + c] = s;
        inv_scale[ck.p * kMaxR + c] = inv;
      }
    }
    ss[c] = s;
  }
  __syncthreads();
  const int64_t i1 = ck.i1 == sg.n ? sg.n_pad_c : ck.i1;
  const int64_t groups = (i1 - ck.i0) / 8;
  const float* v = sg.v[vsel];
  for (int64_t t = threadIdx.x; t < rp * groups; t += blockDim.x) {
    const int c = (int)(t / groups);
    const int64_t i0 = ck.i0 + (t % groups) * 8;
    const float s = ss[c];
    f16::h8 o;
    for (int q = 0; q < 8; ++q) {
      const int64_t i = i0 + q;
      o[q] = (c < r && i < sg.n) ? (_Float16)(v[i * r + c] * s) : (_Float16)0.0f;
    }
    *reinterpret_cast<f16::h8*>(sg.Vt + (int64_t)c * sg.n_pad_c + i0) = o;
  }
}

// Column maxima of |v| per problem (for quantising an arbitrary vector, e.g. x0).
__global__ void colmax_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                              int vsel, uint32_t* __restrict__ colmax) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  const int r = sg.r;
  __shared__ uint32_t smax[kMaxR];
  for (int c = threadIdx.x; c < kMaxR; c += blockDim.x) smax[c] = 0u;
  __syncthreads();
  const float* v = sg.v[vsel];
  for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x)
    atomicMax(&smax[e % r], __float_as_uint(fabsf(v[e])));
  __syncthreads();
  for (int c = threadIdx.x; c < r; c += blockDim.x)
    if (smax[c]) atomicMax(&colmax[ck.p * kMaxR + c], smax[c]);
}

// live[p] = 1 and colmax[p][:] = 0 for the slots of the set
__global__ void select_kernel(const int* __restrict__ plist, int nsel, int* __restrict__ live,
                              uint32_t* __restrict__ colmax, int set_live) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsel * kMaxR) return;
  const int p = plist[t / kMaxR];
  colmax[p * kMaxR + t % kMaxR] = 0u;
  if (set_live && t % kMaxR == 0) live[p] = 1;
}

// ---- a2: fused product over work items ---------------------------------------------
template <int KIND, int KC, int RBMAX>
__device__ __forceinline__ void fused_any_rb(const Seg& sg, const Item& it, _Float16* sX,
                                             _Float16* sV) {
  const int64_t nstage = sg.n_pad_c / f16::JT;
  const int64_t sb = it.split * nstage / sg.nsplit;
  const int64_t se = (it.split + 1) * nstage / sg.nsplit;
  float* P = sg.part + (int64_t)it.split * sg.n_pad_r * sg.rp;
  const int64_t rb0 = it.rblk * f16::kRowsPerBlock;
  if constexpr (RBMAX >= 4) {
    if (sg.rb == 4) {
      f16::fused_rows<KIND, KC, 4>(sg.Xr, sg.Xc, sg.Vt, sg.n_pad_c, P, rb0, sb, se, sX, sV);
      return;
    }
    if (sg.rb == 3) {
      f16::fused_rows<KIND, KC, 3>(sg.Xr, sg.Xc, sg.Vt, sg.n_pad_c, P, rb0, sb, se, sX, sV);
      return;
    }
  }
  if constexpr (RBMAX >= 2) {
    if (sg.rb == 2) {
      f16::fused_rows<KIND, KC, 2>(sg.Xr, sg.Xc, sg.Vt, sg.n_pad_c, P, rb0, sb, se, sX, sV);
      return;
    }
  }
  f16::fused_rows<KIND, KC, 1>(sg.Xr, sg.Xc, sg.Vt, sg.n_pad_c, P, rb0, sb, se, sX, sV);
}

template <int RBMAX>
__global__ __launch_bounds__(256) void fused_kernel(const Seg* __restrict__ segs,
                                                    const Item* __restrict__ items,
                                                    const int* __restrict__ live) {
  __shared__ __attribute__((aligned(16))) _Float16 sX[2 * f16::x_stage_halfs<2>()];
  __shared__ __attribute__((aligned(16))) _Float16 sV[2 * f16::v_stage_halfs<RBMAX>()];
  const Item it = items[blockIdx.x];
  if (live && live[it.p] == 0) return;
  const Seg& sg = segs[it.p];
  switch (sg.kind * 2 + (sg.kc - 1)) {
    case 0: fused_any_rb<0, 1, RBMAX>(sg, it, sX, sV); break;
    case 1: fused_any_rb<0, 2, RBMAX>(sg, it, sX, sV); break;
    case 2: fused_any_rb<1, 1, RBMAX>(sg, it, sX, sV); break;
    case 3: fused_any_rb<1, 2, RBMAX>(sg, it, sX, sV); break;
    case 4: fused_any_rb<2, 1, RBMAX>(sg, it, sX, sV); break;
    case 5: fused_any_rb<2, 2, RBMAX>(sg, it, sX, sV); break;
    case 6: fused_any_rb<3, 1, RBMAX>(sg, it, sX, sV); break;
    default: fused_any_rb<3, 2, RBMAX>(sg, it, sX, sV); break;
  }
}

// Persistent form: a grid sized to the resident capacity of the chip pulls
// items from the longest-first table through an atomic counter (reset by
// reset_counter_kernel before each launch), so the work groups that finish
// early take the remaining items; every group exits once the counter passes
// the table.  Items write disjoint partial sums, so results do not depend on
// which group takes which item.
template <int RBMAX>
__global__ __launch_bounds__(256) void fused_persistent_kernel(const Seg* __restrict__ segs,
                                                               const Item* __restrict__ items,
                                                               int nitems,
                                                               const int* __restrict__ live,
                                                               int* __restrict__ counter) {
  __shared__ __attribute__((aligned(16))) _Float16 sX[2 * f16::x_stage_halfs<2>()];
  __shared__ __attribute__((aligned(16))) _Float16 sV[2 * f16::v_stage_halfs<RBMAX>()];
  __shared__ int s_item;
  for (;;) {
    __syncthreads();   // the previous item is done with LDS and s_item
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = s_item;
    if (idx >= nitems) break;
    const Item it = items[idx];
    if (live && live[it.p] == 0) continue;
    const Seg& sg = segs[it.p];
    switch (sg.kind * 2 + (sg.kc - 1)) {
      case 0: fused_any_rb<0, 1, RBMAX>(sg, it, sX, sV); break;
      case 1: fused_any_rb<0, 2, RBMAX>(sg, it, sX, sV); break;
      case 2: fused_any_rb<1, 1, RBMAX>(sg, it, sX, sV); break;
      case 3: fused_any_rb<1, 2, RBMAX>(sg, it, sX, sV); break;
      case 4: fused_any_rb<2, 1, RBMAX>(sg, it, sX, sV); break;
      case 5: fused_any_rb<2, 2, RBMAX>(sg, it, sX, sV); break;
      case 6: fused_any_rb<3, 1, RBMAX>(sg, it, sX, sV); break;
      default: fused_any_rb<3, 2, RBMAX>(sg, it, sX, sV); break;
    }
  }
}

__global__ void reset_counter_kernel(int* counter) { *counter = 0; }

// out = a^2 inv_scale * sum of split partials + s^2 v; block per chunk.
__global__ void reduce_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                              const float* __restrict__ inv_scale, int vsel, int osel,
                              const int* __restrict__ live) {
  const Chunk ck = chunks[blockIdx.x];
  if (live && live[ck.p] == 0) return;
  const Seg& sg = segs[ck.p];
  const int r = sg.r;
  const float* P = sg.part;
  const int64_t stride = sg.n_pad_r * sg.rp;
  const float* V = sg.v[vsel];
  float* out = sg.v[osel];
  for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x) {
    const int64_t i = e / r;
    const int c = (int)(e % r);
    float acc = 0.0f;
    for (int x = 0; x < sg.nsplit; ++x) acc += P[x * stride + i * sg.rp + c];
    out[e] = fmaf(sg.s2, V[e], (sg.a2 * inv_scale[ck.p * kMaxR + c]) * acc);
  }
}

// ---- per-column reductions -----------------------------------------------------
// Chunk partials of (LSE pair or dot) of a, b and optionally of a.a.
template <bool LSE>
__global__ void colred_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                              int asel, int bsel, const int* __restrict__ live, int with_q2) {
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
  const float* a = sg.v[asel];
  const float* b = sg.v[bsel];
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
    const int64_t o = (int64_t)ck.k * r + threadIdx.x;
    sg.pm[o] = sm[threadIdx.x];
    sg.ps[o] = ss[threadIdx.x];
    if (with_q2) sg.pq[o] = sq[threadIdx.x];
  }
}

__device__ __forceinline__ void merge_chunks(const Seg& sg, int c, bool lse, bool with_q2,
                                             double* logval, bool* ok, double* q2) {
  float M = -INFINITY, T = 0.0f;
  double dot = 0.0, qq = 0.0;
  // loads issued eight chunks at a time, merged in chunk order
  int k = 0;
  for (; k + 8 <= sg.nchunk; k += 8) {
    float vm[8], vs[8];
    double vq[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t o = (int64_t)(k + u) * sg.r + c;
      vm[u] = lse ? sg.pm[o] : 0.0f;
      vs[u] = sg.ps[o];
      vq[u] = with_q2 ? sg.pq[o] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (lse)
        lse_merge(M, T, vm[u], vs[u]);
      else
        dot += (double)vs[u];
      if (with_q2) qq += vq[u];
    }
  }
  for (; k < sg.nchunk; ++k) {
    const int64_t o = (int64_t)k * sg.r + c;
    if (lse)
      lse_merge(M, T, sg.pm[o], sg.ps[o]);
    else
      dot += (double)sg.ps[o];
    if (with_q2) qq += sg.pq[o];
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
__global__ void dq_finish_kernel(const Seg* __restrict__ segs, const int* __restrict__ plist,
                                 State* __restrict__ st, int* live, int lse) {
  const int p = plist[blockIdx.x];
  if (live[p] == 0) return;
  const Seg& sg = segs[p];
  State& S = st[p];
  const int c = threadIdx.x;
  const int k = S.k + 1;
  int act = 0;
  if (c < sg.r) {
    double alpha = 0.0;
    act = S.active[c];
    if (act) {
      double lv, q2;
      bool ok;
      merge_chunks(sg, c, lse != 0, false, &lv, &ok, &q2);
      if (ok) alpha = lse ? exp(S.lg[c] - lv) : S.lg[c] / lv;
      if (!ok || !isfinite(alpha)) {
        alpha = 0.0;
        S.breakdown[c] = 1;
        S.active[c] = 0;
        act = 0;
      }
    }
    S.alpha[c] = alpha;
    if (act) S.iters[c] = k;
  }
  // one wave, a lane per column: the active count by a ballot
  const uint64_t alive = __ballot(act != 0);
  if (c == 0) {
    const int na = __popcll(alive);
    S.k = k;
    S.nactive = na;
    live[p] = na;
  }
}

// gamma_{k+1}, beta, convergence, iteration limit; block per problem.
// init = 1 at initialisation.
__global__ void rz_finish_kernel(const Seg* __restrict__ segs, const int* __restrict__ plist,
                                 State* __restrict__ st, int* live, int lse, int init,
                                 uint32_t* __restrict__ colmax) {
  const int p = plist[blockIdx.x];
  if (!init && live[p] == 0) return;
  const Seg& sg = segs[p];
  State& S = st[p];
  const int c = threadIdx.x;
  const int k = S.k;
  int act = 0;
  if (c < sg.r) {
    double g, q2;
    bool ok;
    merge_chunks(sg, c, lse != 0, true, &g, &ok, &q2);
    act = S.active[c];
    if (act) {
      const double rel = sqrt(q2 / S.bnorm2[c]);
      S.rel[c] = (float)rel;
      if (k >= sg.min_iter && rel <= sg.tol) {
        S.converged[c] = 1;
        S.active[c] = 0;
        act = 0;
      } else if (!ok) {
        S.breakdown[c] = 1;
        S.active[c] = 0;
        act = 0;
      } else if (k >= sg.max_iter) {
        S.active[c] = 0;
        act = 0;
      } else {
        if (!init) S.beta[c] = lse ? exp(g - S.lg[c]) : g / S.lg[c];
        S.lg[c] = g;
        S.inv_sqrt_g[c] = (float)(lse ? exp(-0.5 * g) : 1.0 / sqrt(g));
      }
    }
  }
  if (c < kMaxR) colmax[p * kMaxR + c] = 0u;
  // one wave, a lane per column: the active count by a ballot
  const uint64_t alive = __ballot(act != 0);
  if (c == 0) {
    const int na = __popcll(alive);
    S.nactive = na;
    S.append_slot = S.nbasis;
    live[p] = na;
  }
}

// ||b||^2 per column, masks; block per problem after colred over b.
__global__ void init_finish_kernel(const Seg* __restrict__ segs, const int* __restrict__ plist,
                                   State* __restrict__ st, int* live) {
  const int p = plist[blockIdx.x];
  const Seg& sg = segs[p];
  State& S = st[p];
  const int c = threadIdx.x;
  if (c < kMaxR) {
    double b2 = 0.0;
    if (c < sg.r)
      for (int k = 0; k < sg.nchunk; ++k) b2 += sg.pq[(int64_t)k * sg.r + c];
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
// r = q - b (x0 given) or r = -b, x = 0; frozen columns x = r = 0
__global__ void init_residual_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                                     const State* __restrict__ st, int x0_given) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  const State& S = st[ck.p];
  const int r = sg.r;
  const float* B = sg.v[VB];
  const float* q = sg.v[VQ];
  float* X = sg.v[VX];
  float* R = sg.v[VR];
  for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x) {
    const int c = (int)(e % r);
    if (!S.active[c]) {
      X[e] = 0.0f;
      R[e] = 0.0f;
    } else if (x0_given) {
      R[e] = q[e] - B[e];
    } else {
      X[e] = 0.0f;
      R[e] = -B[e];
    }
  }
}

__global__ void update_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                              const State* __restrict__ st, const int* __restrict__ live) {
  const Chunk ck = chunks[blockIdx.x];
  if (live[ck.p] == 0) return;
  const Seg& sg = segs[ck.p];
  const State& S = st[ck.p];
  const int r = sg.r;
  float* X = sg.v[VX];
  float* R = sg.v[VR];
  const float* D = sg.v[VD];
  const float* Q = sg.v[VQ];
  for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x) {
    const int c = (int)(e % r);
    if (!S.active[c]) continue;
    const float a = (float)S.alpha[c];
    X[e] = fmaf(a, D[e], X[e]);
    R[e] = fmaf(a, Q[e], R[e]);
  }
}

// d = -z + beta d (init: d = -z), basis append, column maxima of |d|.
__global__ void direction_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                                 const State* __restrict__ st, const int* __restrict__ live,
                                 int init, int reorth, uint32_t* __restrict__ colmax) {
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
  const float* Z = sg.v[VZ];
  const float* R = sg.v[VR];
  float* D = sg.v[VD];
  // thread (row lane, column): fixed column, its scalars and running max in registers
  const int rp2 = pow2_at_least(r);
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  if (c < r) {
    const bool act = S.active[c] != 0;
    const float beta = (float)S.beta[c];
    const float sgm = S.inv_sqrt_g[c];
    float* Us = reorth ? sg.Ub + slot * nr : nullptr;
    float* Ws = (reorth && sg.Wb) ? sg.Wb + slot * nr : nullptr;
    uint32_t mx = 0u;
    for (int64_t i = ck.i0 + ty; i < ck.i1; i += tys) {
      const int64_t e = i * r + c;
      float dv = D[e];
      if (act) {
        const float zv = Z[e];
        dv = init ? -zv : fmaf(beta, dv, -zv);
        D[e] = dv;
        if (Us) {
          Us[e] = R[e] * sgm;
          if (Ws) Ws[e] = zv * sgm;
        }
      }
      mx = max(mx, __float_as_uint(fabsf(dv)));
    }
    if (mx) atomicMax(&smax[c], mx);
  }
  __syncthreads();
  for (int cc = threadIdx.x; cc < r; cc += blockDim.x)
    if (smax[cc]) atomicMax(&colmax[ck.p * kMaxR + cc], smax[cc]);
}

__global__ void bump_basis_kernel(const int* __restrict__ plist, int nsel, State* __restrict__ st,
                                  const int* __restrict__ live) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsel) return;
  const int p = plist[t];
  if (live[p] == 0) return;
  st[p].nbasis = st[p].append_slot + 1;
}

// ---- a5: re-orthogonalisation ----------------------------------------------------
// CGS2 from one coefficient sweep and one update sweep per iteration, as in the
// single-problem solver: with G = W^T U the Gram matrix of the problem's stored
// pairs (symmetric: w_j = P(u_j)), the second pass's coefficients are
// c1 - G c1, so r <- r - U (2 c1 - G c1).  The coefficient sweep also forms
// w_j^T u_new for the pair appended at the end of the previous iteration, which
// gives G's new column (and, by symmetry, row).
// Work group (chunk, group of kJGroup basis vectors): chunk partials of
// w_j^T r and w_j^T u_new.
__global__ void reorth_coef_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                                   const State* __restrict__ st, const int* __restrict__ live,
                                   int jgroups) {
  const int ci = blockIdx.x / jgroups;
  const int j0 = (blockIdx.x % jgroups) * kJGroup;
  const Chunk ck = chunks[ci];
  if (live[ck.p] == 0) return;
  const int nb = st[ck.p].nbasis;
  if (j0 >= nb) return;
  const Seg& sg = segs[ck.p];
  const int r = sg.r;
  const int rp2 = pow2_at_least(r);
  const int mb = sg.max_iter + 1;
  __shared__ float sb[kJGroup][256];
  __shared__ float sgm[kJGroup][256];
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  const int64_t nr = sg.n * r;
  const int jn = min(kJGroup, nb - j0);
  const float* Wb = (sg.Wb ? sg.Wb : sg.Ub) + (int64_t)j0 * nr;
  const float* Un = sg.Ub + (int64_t)(nb - 1) * nr;
  const float* Rv = sg.v[VR];
  float acc[kJGroup], accg[kJGroup];
#pragma unroll
  for (int q = 0; q < kJGroup; ++q) acc[q] = accg[q] = 0.0f;
  if (c < r)
    for (int64_t i = ck.i0 + ty; i < ck.i1; i += tys) {
      const float rv = Rv[i * r + c], uv = Un[i * r + c];
#pragma unroll
      for (int q = 0; q < kJGroup; ++q)
        if (q < jn) {
          const float w = Wb[q * nr + i * r + c];
          acc[q] = fmaf(w, rv, acc[q]);
          accg[q] = fmaf(w, uv, accg[q]);
        }
    }
#pragma unroll
  for (int q = 0; q < kJGroup; ++q) {
    sb[q][threadIdx.x] = acc[q];
    sgm[q][threadIdx.x] = accg[q];
  }
  for (int s2 = 128; s2 >= rp2; s2 >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s2)
#pragma unroll
      for (int q = 0; q < kJGroup; ++q) {
        sb[q][threadIdx.x] += sb[q][threadIdx.x + s2];
        sgm[q][threadIdx.x] += sgm[q][threadIdx.x + s2];
      }
  }
  __syncthreads();
  if ((int)threadIdx.x < r)
    for (int q = 0; q < jn; ++q) {
      const int64_t o = ((int64_t)ck.k * mb + j0 + q) * r + threadIdx.x;
      sg.pcoef[o] = sb[q][threadIdx.x];
      sg.pgram[o] = sgm[q][threadIdx.x];
    }
}

// c1[j][c] and G's new column / row = sums over the problem's chunks in order;
// grid (slot, 256 entries).
__global__ void reorth_sum_kernel(const Seg* __restrict__ segs, const int* __restrict__ plist,
                                  const State* __restrict__ st, const int* __restrict__ live) {
  const int p = plist[blockIdx.x];
  if (live[p] == 0) return;
  const Seg& sg = segs[p];
  const int nb = st[p].nbasis;
  const int r = sg.r;
  const int mb = sg.max_iter + 1;
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e >= nb * r) return;
  const int j = e / r, c = e % r;
  const int64_t off = (int64_t)j * r + c;
  const int64_t stride = (int64_t)mb * r;
  float acc = 0.0f, accg = 0.0f;
  int k = 0;
  for (; k + 8 <= sg.nchunk; k += 8) {
    float v[8], w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      v[u] = sg.pcoef[off + (k + u) * stride];
      w[u] = sg.pgram[off + (k + u) * stride];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      acc += v[u];
      accg += w[u];
    }
  }
  for (; k < sg.nchunk; ++k) {
    acc += sg.pcoef[off + k * stride];
    accg += sg.pgram[off + k * stride];
  }
  sg.c1[e] = acc;
  const int m = nb - 1;
  sg.gram[((int64_t)j * mb + m) * r + c] = accg;
  sg.gram[((int64_t)m * mb + j) * r + c] = accg;
}

// coef[j][c] = 2 c1[j][c] - sum_k G[j][k][c] c1[k][c] in float64 (k in order):
// grid (slot, 32 entries (j, c) per group, eight lanes each over fixed eighths
// of k, combined in lane order).
constexpr int kGramLanes = 8;
__global__ void reorth_gram_kernel(const Seg* __restrict__ segs, const int* __restrict__ plist,
                                   const State* __restrict__ st, const int* __restrict__ live) {
  const int p = plist[blockIdx.x];
  if (live[p] == 0) return;
  const Seg& sg = segs[p];
  const int nb = st[p].nbasis;
  const int r = sg.r;
  const int mb = sg.max_iter + 1;
  __shared__ double red[256];
  const int e = blockIdx.y * (256 / kGramLanes) + threadIdx.x / kGramLanes;
  const int q = threadIdx.x % kGramLanes;
  const bool on = e < nb * r;
  const int j = on ? e / r : 0, c = on ? e % r : 0;
  double acc = 0.0;
  if (on) {
    const float* Gj = sg.gram + (int64_t)j * mb * r + c;
    const int k0 = q * nb / kGramLanes, k1 = (q + 1) * nb / kGramLanes;
    for (int k = k0; k < k1; ++k) acc = fma((double)Gj[(int64_t)k * r], (double)sg.c1[k * r + c], acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (on && q == 0) {
    double t = red[threadIdx.x];
#pragma unroll
    for (int u = 1; u < kGramLanes; ++u) t += red[threadIdx.x + u];
    sg.coef[e] = (float)(2.0 * (double)sg.c1[e] - t);
  }
}

// r -= sum_j coef[j] u_j; coefficients staged in LDS when they fit (USE_LDS).
template <bool USE_LDS>
__global__ void reorth_apply_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                                    const State* __restrict__ st, const int* __restrict__ live) {
  const Chunk ck = chunks[blockIdx.x];
  if (live[ck.p] == 0) return;
  const Seg& sg = segs[ck.p];
  const State& S = st[ck.p];
  const int r = sg.r;
  const int nb = S.nbasis;
  const int64_t nr = sg.n * r;
  extern __shared__ float scf_lds[];       // nb x r coefficients
  const float* cf = sg.coef;
  if (USE_LDS) {
    for (int e = threadIdx.x; e < nb * r; e += blockDim.x) scf_lds[e] = cf[e];
    __syncthreads();
  }
  auto scf_at = [&](int j, int c) { return USE_LDS ? scf_lds[j * r + c] : cf[j * r + c]; };
  const float* Ub = sg.Ub;
  float* R = sg.v[VR];
  for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x) {
    const int c = (int)(e % r);
    if (!S.active[c]) continue;
    float v = R[e];
    int j = 0;
    for (; j + 8 <= nb; j += 8) {
      float u[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) u[q] = Ub[(j + q) * nr + e];
#pragma unroll
      for (int q = 0; q < 8; ++q) v = fmaf(-scf_at(j + q, c), u[q], v);
    }
    for (; j < nb; ++j) v = fmaf(-scf_at(j, c), Ub[j * nr + e], v);
    R[e] = v;
  }
}

// ---- a6: preconditioner apply (Woodbury form) ---------------------------------------
// chunk partial of L^T r (rank x r) on the matrix cores
__global__ __launch_bounds__(256) void lt_partial_kernel(const Seg* __restrict__ segs,
                                                         const Chunk* __restrict__ chunks,
                                                         const int* __restrict__ live) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  if (live[ck.p] == 0 || sg.rank == 0) return;
  __shared__ pc::LtLds sm;
  pc::lt_chunk_mfma(sg.L32, sg.n, sg.rank, sg.v[VR], sg.r, ck.i0, ck.i1,
                    sg.ltpart + (int64_t)ck.k * sg.rank * sg.r, sm);
}

// T = sum of the chunk partials (float64, chunk order); grid (slot, 64 entries),
// four threads per entry over fixed quarters of the chunks.
__global__ void lt_sum_kernel(const Seg* __restrict__ segs, const int* __restrict__ plist,
                              const int* __restrict__ live) {
  const int p = plist[blockIdx.x];
  const Seg& sg = segs[p];
  if (live[p] == 0 || sg.rank == 0) return;
  const int kr = sg.rank * sg.r;
  if ((int)blockIdx.y * 64 >= kr) return;
  const int o = blockIdx.y * 64 + (threadIdx.x >> 2);
  __shared__ double red[256];
  const int q = threadIdx.x & 3;
  double acc = 0.0;
  if (o < kr)
    acc = pc::sum_strided(sg.ltpart + o, (int64_t)kr, q * sg.nchunk / 4, (q + 1) * sg.nchunk / 4);
  red[threadIdx.x] = acc;
  __syncthreads();
  if (q == 0 && o < kr)
    sg.T64[o] = ((red[threadIdx.x] + red[threadIdx.x + 1]) + red[threadIdx.x + 2]) + red[threadIdx.x + 3];
}

// Y = C^{-1} T (float64), stored as float32; grid (slot, 256 entries).
__global__ void lt_solve_kernel(const Seg* __restrict__ segs, const int* __restrict__ plist,
                                const int* __restrict__ live) {
  const int p = plist[blockIdx.x];
  const Seg& sg = segs[p];
  if (live[p] == 0 || sg.rank == 0) return;
  const int k = sg.rank, r = sg.r;
  const int o = blockIdx.y * 256 + threadIdx.x;
  if (o >= k * r) return;
  const int a = o / r, c = o % r;
  double acc = 0.0;
#pragma unroll 8
  for (int b = 0; b < k; ++b) acc = fma(sg.Cinv[a * k + b], sg.T64[b * r + c], acc);
  sg.Y32[o] = (float)acc;
}

// z = s^-2 r - s^-4 L y (rank > 0), z = r (rank 0: no preconditioner);
// block per chunk, one thread per row.
__global__ void z_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                         const int* __restrict__ live) {
  const Chunk ck = chunks[blockIdx.x];
  if (live[ck.p] == 0) return;
  const Seg& sg = segs[ck.p];
  const int r = sg.r, k = sg.rank;
  const float* R = sg.v[VR];
  float* Z = sg.v[VZ];
  if (k == 0) {
    for (int64_t e = ck.i0 * r + threadIdx.x; e < ck.i1 * r; e += blockDim.x) Z[e] = R[e];
    return;
  }
  __shared__ __attribute__((aligned(16))) float sy[pc::kMaxRank * kMaxR];
  const int rp = (r + 15) & ~15;
  pc::stage_y(sg.Y32, k, r, rp, sy);
  __syncthreads();
  const float inv_s2 = 1.0f / sg.s2;
  const float inv_s4 = inv_s2 * inv_s2;
  for (int64_t i = ck.i0 + threadIdx.x; i < ck.i1; i += blockDim.x)
    pc::z_row(sg.L32, sg.n, k, sy, rp, R, Z, r, i, inv_s2, inv_s4);
}

// ---- a8: true residual (float64 accumulation on the matrix cores) -------------------
// The single-problem routine (valu_tile.h aug64_rows: augmented float64
// distances, float64 sums of every product) on the item's row block and split.
template <int T>
__device__ __forceinline__ void trueres_rows(const Seg& sg, const Item& it, void* smraw) {
  valu::Aug64Lds<T>& sm = *reinterpret_cast<valu::Aug64Lds<T>*>(smraw);
  const int64_t nstage = ceil_div(sg.n, (int64_t)valu::JT64);
  const int64_t sb = it.split * nstage / sg.nsplit64;
  const int64_t se = (it.split + 1) * nstage / sg.nsplit64;
  double* P = sg.part64 + (int64_t)it.split * sg.n * sg.r;
  const int64_t rb0 = it.rblk * valu::aug_rows(T);
  const float* U = sg.v[VX];
  for (int c0 = 0; c0 < sg.r; c0 += 16) {
    switch (sg.kind) {
      case GP_KERNEL_RBF:
        valu::aug64_rows<GP_KERNEL_RBF, T>(sg.X, sg.n, sg.X, sg.n, U, sg.r, c0, sg.d, sg.ls, P,
                                           rb0, sb, se, sm);
        break;
      case GP_KERNEL_MATERN52:
        valu::aug64_rows<GP_KERNEL_MATERN52, T>(sg.X, sg.n, sg.X, sg.n, U, sg.r, c0, sg.d, sg.ls,
                                                P, rb0, sb, se, sm);
        break;
      case GP_KERNEL_MATERN12:
        valu::aug64_rows<GP_KERNEL_MATERN12, T>(sg.X, sg.n, sg.X, sg.n, U, sg.r, c0, sg.d, sg.ls,
                                                P, rb0, sb, se, sm);
        break;
      default:
        valu::aug64_rows<GP_KERNEL_MATERN32, T>(sg.X, sg.n, sg.X, sg.n, U, sg.r, c0, sg.d, sg.ls,
                                                P, rb0, sb, se, sm);
        break;
    }
  }
}

__global__ __launch_bounds__(256) void trueres_partial_kernel(const Seg* __restrict__ segs,
                                                              const Item* __restrict__ items) {
  // one LDS block sized for the widest instantiation (T = 8: d <= 30)
  __shared__ __attribute__((aligned(16))) char sm[sizeof(valu::Aug64Lds<8>)];
  const Item it = items[blockIdx.x];
  const Seg& sg = segs[it.p];
  switch (trueres_slices_of(sg.d)) {
    case 1: trueres_rows<1>(sg, it, sm); break;
    case 2: trueres_rows<2>(sg, it, sm); break;
    case 3: trueres_rows<3>(sg, it, sm); break;
    case 4: trueres_rows<4>(sg, it, sm); break;
    case 5: trueres_rows<5>(sg, it, sm); break;
    case 6: trueres_rows<6>(sg, it, sm); break;
    case 7: trueres_rows<7>(sg, it, sm); break;
    default: trueres_rows<8>(sg, it, sm); break;
  }
}

// per-chunk partial of ||b - K~ x||^2 per column
__global__ void trueres_chunk_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  const int r = sg.r;
  const int rp2 = pow2_at_least(r);
  __shared__ double sb[256];
  const int c = threadIdx.x % rp2;
  const int ty = threadIdx.x / rp2;
  const int tys = 256 / rp2;
  const int64_t nr = sg.n * r;
  const float* B = sg.v[VB];
  const float* U = sg.v[VX];
  double acc = 0.0;
  if (c < r)
    for (int64_t i = ck.i0 + ty; i < ck.i1; i += tys) {
      const int64_t e = i * r + c;
      double kx = 0.0;
      for (int s = 0; s < sg.nsplit64; ++s) kx += sg.part64[s * nr + e];
      const double res = (double)B[e] - ((double)sg.a2 * kx + (double)sg.s2 * (double)U[e]);
      acc += res * res;
    }
  sb[threadIdx.x] = acc;
  for (int s2 = 128; s2 >= rp2; s2 >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s2) sb[threadIdx.x] += sb[threadIdx.x + s2];
  }
  __syncthreads();
  if ((int)threadIdx.x < r) sg.pq[(int64_t)ck.k * r + threadIdx.x] = sb[threadIdx.x];
}

__global__ void trueres_finish_kernel(const Seg* __restrict__ segs, const int* __restrict__ plist,
                                      State* __restrict__ st) {
  const int p = plist[blockIdx.x];
  const Seg& sg = segs[p];
  const int c = threadIdx.x;
  if (c >= sg.r) return;
  double t = 0.0;
  for (int k = 0; k < sg.nchunk; ++k) t += sg.pq[(int64_t)k * sg.r + c];
  const double b2 = st[p].bnorm2[c];
  st[p].true_rel[c] = b2 > 0.0 ? sqrt(t / b2) : sqrt(t);
}

// ---- a9: pivoted Cholesky, all problems of a set per step ----------------------------
__device__ inline bool better(double v, int64_t i, double bv, int64_t bi) {
  if (isnan(v)) return false;
  if (isnan(bv)) return true;
  return v > bv || (v == bv && i < bi);
}

// Chunk argmax (lowest index on ties) and sum of the residual diagonal.
__device__ void chunk_argmax(const Seg& sg, const Chunk& ck) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  __shared__ double ssum[256];
  double bv = -INFINITY, sum = 0.0;
  int64_t bi = INT64_MAX;
  for (int64_t i = ck.i0 + threadIdx.x; i < ck.i1; i += blockDim.x) {
    const double v = sg.diag[i];
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
    sg.pv[ck.k] = sv[0];
    sg.pi[ck.k] = si[0];
    sg.psum[ck.k] = ssum[0];
  }
}

__global__ void pc_init_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  if (sg.rank == 0) return;
  for (int64_t i = ck.i0 + threadIdx.x; i < ck.i1; i += blockDim.x) sg.diag[i] = sg.a2;
  __syncthreads();
  chunk_argmax(sg, ck);
}

// Pivot of step m for every problem still running; a problem still running at
// step m has built columns 0..m-1.
__global__ void pc_select_kernel(const Seg* __restrict__ segs, const int* __restrict__ plist,
                                 int nsel, PcState* __restrict__ ps, int m) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsel) return;
  const int p = plist[t];
  const Seg& sg = segs[p];
  PcState& S = ps[p];
  if (m == 0) {
    S.stop = 0;
    S.not_pd = 0;
    S.trace = 0.0;
  }
  if (S.stop) return;
  S.rank = m;
  if (sg.rank == 0) {
    S.stop = 1;
    return;
  }
  double v = -INFINITY, tot = 0.0;
  int64_t idx = INT64_MAX;
  for (int k = 0; k < sg.nchunk; ++k) {
    tot += sg.psum[k];
    if (better(sg.pv[k], sg.pi[k], v, idx)) {
      v = sg.pv[k];
      idx = sg.pi[k];
    }
  }
  S.trace = tot;
  if (m >= sg.rank || !(v > 1e-12 * (double)sg.a2) || idx == INT64_MAX) {
    S.stop = 1;
  } else {
    S.dmax = v;
    S.pivot = idx;
    sg.piv[m] = idx;
  }
}

__global__ void pc_step_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                               const PcState* __restrict__ ps, int m) {
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
  double* L = sg.L64;
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
    acc = pc::sub_lrow(L, n, i, lp, m, acc);
    const double l = acc * inv_sq;
    L[(int64_t)m * n + i] = l;
    sg.diag[i] = fma(-l, l, sg.diag[i]);
  }
  __syncthreads();
  chunk_argmax(sg, ck);
}

// C = I + s^-2 L^T L for every problem: block per (problem, 16 x 16 tile).
__global__ void pc_syrk_kernel(const Seg* __restrict__ segs, const PcState* __restrict__ ps,
                               const int4* __restrict__ tiles) {
  // tile (p, ta, tb) with ta <= tb; the (tb, ta) tile is its mirror image
  // (the products commute, so the mirrored sums are the same numbers)
  constexpr int kStep = 128;
  const int4 t = tiles[blockIdx.x];
  const Seg& sg = segs[t.x];
  const int k = ps[t.x].rank;
  if (t.y * 16 >= k || t.z * 16 >= k) return;
  __shared__ double la[16][kStep + 1];
  __shared__ double lb[16][kStep + 1];
  const int a = threadIdx.x / 16, b = threadIdx.x % 16;
  const double* L = sg.L64;
  const int64_t n = sg.n;
  // four interleaved partial sums (columns cc = q mod 4), added in a fixed
  // order at the end
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t c0 = 0; c0 < n; c0 += kStep) {
    __syncthreads();
    // the step's 16 staging loads per thread in flight at once
    double va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = u * 256 + (int)threadIdx.x;
      const int rr = e / kStep, cc = e % kStep;
      const int64_t i = c0 + cc;
      const int ra = t.y * 16 + rr, rb = t.z * 16 + rr;
      va[u] = (i < n && ra < k) ? L[(int64_t)ra * n + i] : 0.0;
      vb[u] = (i < n && rb < k) ? L[(int64_t)rb * n + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = u * 256 + (int)threadIdx.x;
      la[e / kStep][e % kStep] = va[u];
      lb[e / kStep][e % kStep] = vb[u];
    }
    __syncthreads();
#pragma unroll 8
    for (int cc = 0; cc < kStep; cc += 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = fma(la[a][cc + q], lb[b][cc + q], acc[q]);
    }
  }
  const double sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  const int ga = t.y * 16 + a, gb = t.z * 16 + b;
  if (ga < k && gb < k) {
    const double v = (ga == gb ? 1.0 : 0.0) + sum / (double)sg.s2;
    sg.C[ga * k + gb] = v;
    if (t.y != t.z) sg.C[gb * k + ga] = v;
  }
}

// Cholesky of C and explicit inverse (pc::chol_inverse); work group per problem.
__global__ __launch_bounds__(256) void pc_cholinv_kernel(const Seg* __restrict__ segs,
                                                         const int* __restrict__ plist,
                                                         PcState* __restrict__ ps) {
  __shared__ double A[pc::kMaxRank * pc::kMaxRank];
  const int p = plist[blockIdx.x];
  const int k = ps[p].rank;
  if (k == 0) return;
  pc::chol_inverse(segs[p].C, segs[p].Cinv, k, A, &ps[p].not_pd);
}

// binary32 copy of the built factor columns, the chunk's rows
__global__ void to_f32_kernel(const Seg* __restrict__ segs, const Chunk* __restrict__ chunks,
                              const PcState* __restrict__ ps) {
  const Chunk ck = chunks[blockIdx.x];
  const Seg& sg = segs[ck.p];
  const int k = ps[ck.p].rank;
  const int64_t rows = ck.i1 - ck.i0;
  for (int64_t t = threadIdx.x; t < k * rows; t += blockDim.x) {
    const int64_t e = (t / rows) * sg.n + ck.i0 + t % rows;
    sg.L32[e] = (float)sg.L64[e];
  }
}

}  // namespace bt
}  // namespace gpmi

// ---- host sequences ----------------------------------------------------------------
namespace gpmi {
namespace bt {

static inline unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)ceil_div(n, t); }

#define BT_LAUNCH_CHECK() GP_HIP(hipGetLastError())

static gp_status launch_quant(const Dev& D, const Tab& T, int vsel, int scale_mode, const int* live,
                              hipStream_t s) {
  quant_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, vsel, D.colmax, scale_mode, D.scale,
                                         D.inv_scale, live);
  BT_LAUNCH_CHECK();
  return GP_OK;
}

// Work groups of the persistent product that fit on the device at once.
template <int RBMAX>
static int persistent_grid() {
  static int cached[8] = {0};   // per device ordinal (first 8)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  const int slot = dev & 7;
  if (cached[slot] == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused_persistent_kernel<RBMAX>, 256, 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      (void)hipGetLastError();
      per_cu = 2;
      cus = 256;
    }
    cached[slot] = std::max(1, per_cu) * std::max(1, cus);
  }
  return cached[slot];
}

template <int RBMAX>
static gp_status launch_fused(const Dev& D, const Tab& T, const int* live, hipStream_t s) {
  if (D.persistent && D.counter) {
    reset_counter_kernel<<<1, 1, 0, s>>>(D.counter);
    BT_LAUNCH_CHECK();
    const int grid = std::min(T.nitems, persistent_grid<RBMAX>());
    fused_persistent_kernel<RBMAX><<<grid, 256, 0, s>>>(D.segs, T.items, T.nitems, live, D.counter);
  } else {
    fused_kernel<RBMAX><<<T.nitems, 256, 0, s>>>(D.segs, T.items, live);
  }
  BT_LAUNCH_CHECK();
  return GP_OK;
}

static gp_status launch_product(const Dev& D, const Tab& T, int vsel, int osel, const int* live,
                                hipStream_t s) {
  void* tok = prof::begin(s);
  if (T.rb <= 1)
    GP_TRY(launch_fused<1>(D, T, live, s));
  else if (T.rb == 2)
    GP_TRY(launch_fused<2>(D, T, live, s));
  else
    GP_TRY(launch_fused<4>(D, T, live, s));
  prof::end(tok, s, T.entries, -1);
  reduce_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, D.inv_scale, vsel, osel, live);
  BT_LAUNCH_CHECK();
  return GP_OK;
}

static gp_status launch_colred(const Dev& D, const Tab& T, int asel, int bsel, bool lse,
                               bool with_q2, hipStream_t s) {
  if (lse)
    colred_kernel<true><<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, asel, bsel, D.live, with_q2 ? 1 : 0);
  else
    colred_kernel<false><<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, asel, bsel, D.live, with_q2 ? 1 : 0);
  BT_LAUNCH_CHECK();
  return GP_OK;
}

static gp_status launch_precond(const Dev& D, const Tab& T, hipStream_t s) {
  if (T.max_rank > 0) {
    lt_partial_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, D.live);
    BT_LAUNCH_CHECK();
    const int kr = T.max_rank * T.max_r;
    lt_sum_kernel<<<dim3(T.nsel, (unsigned)ceil_div(kr, 64)), 256, 0, s>>>(D.segs, T.plist, D.live);
    BT_LAUNCH_CHECK();
    lt_solve_kernel<<<dim3(T.nsel, (unsigned)ceil_div(kr, 256)), 256, 0, s>>>(D.segs, T.plist,
                                                                               D.live);
    BT_LAUNCH_CHECK();
  }
  z_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, D.live);
  BT_LAUNCH_CHECK();
  return GP_OK;
}

static gp_status launch_rz(const Dev& D, const Tab& T, bool lse, bool init, hipStream_t s) {
  GP_TRY(launch_colred(D, T, VR, VZ, lse, true, s));
  rz_finish_kernel<<<T.nsel, 64, 0, s>>>(D.segs, T.plist, D.st, D.live, lse ? 1 : 0, init ? 1 : 0,
                                         D.colmax);
  BT_LAUNCH_CHECK();
  return GP_OK;
}

static gp_status launch_direction(const Dev& D, const Tab& T, bool init, bool reorth,
                                  hipStream_t s) {
  direction_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, D.st, D.live, init ? 1 : 0,
                                             reorth ? 1 : 0, D.colmax);
  BT_LAUNCH_CHECK();
  if (reorth) {
    bump_basis_kernel<<<blocks_for(T.nsel), 256, 0, s>>>(T.plist, T.nsel, D.st, D.live);
    BT_LAUNCH_CHECK();
  }
  return GP_OK;
}

static gp_status launch_reorth(const Dev& D, const Tab& T, hipStream_t s) {
  const int jgroups = (T.max_basis + kJGroup - 1) / kJGroup;
  const size_t lds = sizeof(float) * T.max_basis * T.max_r;
  reorth_coef_kernel<<<(unsigned)(T.nchunks * jgroups), 256, 0, s>>>(D.segs, T.chunks, D.st,
                                                                      D.live, jgroups);
  BT_LAUNCH_CHECK();
  reorth_sum_kernel<<<dim3(T.nsel, (unsigned)ceil_div(T.max_basis * T.max_r, 256)), 256, 0, s>>>(
      D.segs, T.plist, D.st, D.live);
  BT_LAUNCH_CHECK();
  reorth_gram_kernel<<<dim3(T.nsel, (unsigned)ceil_div(T.max_basis * T.max_r, 256 / kGramLanes)),
                       256, 0, s>>>(D.segs, T.plist, D.st, D.live);
  BT_LAUNCH_CHECK();
  if (lds <= 48 * 1024)
    reorth_apply_kernel<true><<<T.nchunks, 256, lds, s>>>(D.segs, T.chunks, D.st, D.live);
  else
    reorth_apply_kernel<false><<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, D.st, D.live);
  BT_LAUNCH_CHECK();
  return GP_OK;
}

gp_status seq_prepare(const Dev& D, const Tab& T, hipStream_t s) {
  if (T.nsel == 0) return GP_OK;
  // occupancy queries of the persistent product, outside any stream capture
  (void)persistent_grid<1>();
  (void)persistent_grid<2>();
  (void)persistent_grid<4>();
  prep_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks);
  BT_LAUNCH_CHECK();
  // pivoted Cholesky: one select + one column step per pivot for the whole set
  pc_init_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks);
  BT_LAUNCH_CHECK();
  for (int m = 0; m <= T.max_rank; ++m) {
    pc_select_kernel<<<blocks_for(T.nsel, 64), 64, 0, s>>>(D.segs, T.plist, T.nsel, D.pcs, m);
    BT_LAUNCH_CHECK();
    if (m == T.max_rank) break;
    pc_step_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, D.pcs, m);
    BT_LAUNCH_CHECK();
  }
  if (T.max_rank > 0) {
    if (T.ntiles > 0) {
      pc_syrk_kernel<<<T.ntiles, 256, 0, s>>>(D.segs, D.pcs, T.tiles);
      BT_LAUNCH_CHECK();
    }
    pc_cholinv_kernel<<<T.nsel, 256, 0, s>>>(D.segs, T.plist, D.pcs);
    BT_LAUNCH_CHECK();
    to_f32_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, D.pcs);
    BT_LAUNCH_CHECK();
  }
  return GP_OK;
}

gp_status seq_start(const Dev& D, const Tab& T, const RunOpts& o, bool x0_given, hipStream_t s) {
  if (T.nsel == 0) return GP_OK;
  // ||b||^2 with every problem of the set live, then the masks
  select_kernel<<<blocks_for((int64_t)T.nsel * kMaxR), 256, 0, s>>>(T.plist, T.nsel, D.live,
                                                                     D.colmax, 1);
  BT_LAUNCH_CHECK();
  colred_kernel<false><<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, VB, VB, D.live, 1);
  BT_LAUNCH_CHECK();
  init_finish_kernel<<<T.nsel, 64, 0, s>>>(D.segs, T.plist, D.st, D.live);
  BT_LAUNCH_CHECK();
  if (x0_given) {
    colmax_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, VX, D.colmax);
    BT_LAUNCH_CHECK();
    GP_TRY(launch_quant(D, T, VX, o.scale_mode, nullptr, s));
    GP_TRY(launch_product(D, T, VX, VQ, nullptr, s));
  }
  init_residual_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, D.st, x0_given ? 1 : 0);
  BT_LAUNCH_CHECK();
  GP_TRY(launch_precond(D, T, s));
  GP_TRY(launch_rz(D, T, o.lse, true, s));
  GP_TRY(launch_direction(D, T, true, o.reorth, s));
  return launch_quant(D, T, VD, o.scale_mode, D.live, s);
}

gp_status seq_iteration(const Dev& D, const Tab& T, const RunOpts& o, hipStream_t s) {
  if (T.nsel == 0) return GP_OK;
  GP_TRY(launch_product(D, T, VD, VQ, D.live, s));
  GP_TRY(launch_colred(D, T, VD, VQ, o.lse, false, s));
  dq_finish_kernel<<<T.nsel, 64, 0, s>>>(D.segs, T.plist, D.st, D.live, o.lse ? 1 : 0);
  BT_LAUNCH_CHECK();
  update_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks, D.st, D.live);
  BT_LAUNCH_CHECK();
  if (o.reorth) GP_TRY(launch_reorth(D, T, s));
  GP_TRY(launch_precond(D, T, s));
  GP_TRY(launch_rz(D, T, o.lse, false, s));
  GP_TRY(launch_direction(D, T, false, o.reorth, s));
  return launch_quant(D, T, VD, o.scale_mode, D.live, s);
}

gp_status seq_true_residual(const Dev& D, const Tab& T, hipStream_t s) {
  if (T.nsel == 0) return GP_OK;
  trueres_partial_kernel<<<T.nitems64, 256, 0, s>>>(D.segs, T.items64);
  BT_LAUNCH_CHECK();
  trueres_chunk_kernel<<<T.nchunks, 256, 0, s>>>(D.segs, T.chunks);
  BT_LAUNCH_CHECK();
  trueres_finish_kernel<<<T.nsel, 64, 0, s>>>(D.segs, T.plist, D.st);
  BT_LAUNCH_CHECK();
  return GP_OK;
}

}  // namespace bt
}  // namespace gpmi
