// Truncated (compact-support) binary16 product (Sec. 4.1, Fig. 2c, App. C).
//
// In binary16 a kernel value below half the smallest subnormal (2^-25)
// rounds to exactly zero, so every pair of points farther apart than a
// kernel-specific radius contributes nothing to the binary16 product: the
// support of the half-precision kernel is finite (Sec. 4.1; App. C gives the
// RBF radius l (-2 log eps)^(1/2) and the Matern-1/2 one -l log eps).  The
// truncated product drops those pairs and is therefore exactly the full
// binary16 product (the paper's zero-error claim).
//
// On the matrix-core tiles the unit of work is a (256-row block, 128-column
// stage) tile, so pairs are dropped a tile at a time:
//   1. both point sets are put in Z-order (interleaved bits of the quantised
//      scaled coordinates, sorted with a device radix sort) so that a block or
//      a stage covers a compact region;
//   2. every row block and column stage gets the bounding box of its points'
//      scaled binary16 coordinates fp16(x / l) -- the values the product's
//      distances are formed from;
//   3. a row block keeps the stages whose box distance is below the radius R
//      at which the kernel value is 2^-26 (half the rounding threshold, which
//      covers the float32 error of the product's distance argument many times
//      over), in increasing order;
//   4. the product runs over the kept stages only; each column split keeps its
//      stage-id range, so the float32 sums see the same nonzero terms in the
//      same order as the product over all stages of the same ordering -- the
//      two agree bit for bit;
//   5. the output rows return to the caller's order.

#include <math.h>

#include <algorithm>
#include <rocprim/device/device_radix_sort.hpp>
#include <vector>

#include "fused_tile.h"
#include "internal.h"

namespace gpmi {
namespace trunc {

namespace {

__global__ void fill_u32_kernel(uint32_t* p, int n, uint32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__device__ __forceinline__ uint32_t ord_of(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float float_of(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// the product's scaled coordinate of point i, dimension m
__device__ __forceinline__ float xh(const float* __restrict__ X, int64_t i, int d, int m,
                                    const KParams& kp) {
  return (float)(_Float16)(X[i * d + m] / kp.ls[m]);
}

// ext[m] = ordered min, ext[kMaxDim + m] = ordered max (cleared to 0xff.. / 0)
__global__ void extent_kernel(const float* __restrict__ X, int64_t n, KParams kp,
                              uint32_t* __restrict__ ext) {
  __shared__ uint32_t lo[kMaxDim], hi[kMaxDim];
  const int d = kp.d;
  for (int m = threadIdx.x; m < d; m += blockDim.x) {
    lo[m] = 0xffffffffu;
    hi[m] = 0u;
  }
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * d;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / d;
    const int m = (int)(e % d);
    const uint32_t o = ord_of(xh(X, i, d, m, kp));
    atomicMin(&lo[m], o);
    atomicMax(&hi[m], o);
  }
  __syncthreads();
  for (int m = threadIdx.x; m < d; m += blockDim.x) {
    atomicMin(&ext[m], lo[m]);
    atomicMax(&ext[kMaxDim + m], hi[m]);
  }
}

// Z-order key: D' = min(d, 63) dimensions, B = min(21, 63 / D') bits each,
// interleaved from the most significant bit down.
__global__ void morton_kernel(const float* __restrict__ X, int64_t n, KParams kp,
                              const uint32_t* __restrict__ ext, uint64_t* __restrict__ key,
                              int* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = kp.d;
  const int dd = d < 63 ? d : 63;
  const int bits = min(21, 63 / dd);
  const float top = (float)((1u << bits) - 1);
  uint32_t q[kMaxDim];
  for (int m = 0; m < dd; ++m) {
    const float lo = float_of(ext[m]), hi = float_of(ext[kMaxDim + m]);
    const float t = hi > lo ? (xh(X, i, d, m, kp) - lo) / (hi - lo) : 0.0f;
    q[m] = (uint32_t)fminf(fmaxf(t * top, 0.0f), top);
  }
  uint64_t k = 0;
  for (int b = bits - 1; b >= 0; --b)
    for (int m = 0; m < dd; ++m) k = (k << 1) | ((q[m] >> b) & 1u);
  key[i] = k;
  idx[i] = (int)i;
}

// dst[i][c] = src[perm[i]][c]
__global__ void gather_kernel(const float* __restrict__ src, const int* __restrict__ perm,
                              int64_t n, int w, float* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * w) return;
  const int64_t i = e / w;
  const int c = (int)(e % w);
  dst[e] = src[(int64_t)perm[i] * w + c];
}

// dst[perm[i]][c] = src[i][c]
__global__ void scatter_kernel(const float* __restrict__ src, const int* __restrict__ perm,
                               int64_t n, int w, float* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * w) return;
  const int64_t i = e / w;
  const int c = (int)(e % w);
  dst[(int64_t)perm[i] * w + c] = src[e];
}

// Box of group b (points [b g, (b + 1) g) of the ordered set): box[b][m] = min,
// box[b][d + m] = max of the scaled binary16 coordinate; one work group per box.
__global__ void box_kernel(const float* __restrict__ Xs, int64_t n, KParams kp, int gsize,
                           float* __restrict__ box) {
  __shared__ uint32_t lo[kMaxDim], hi[kMaxDim];
  const int d = kp.d;
  for (int m = threadIdx.x; m < d; m += blockDim.x) {
    lo[m] = 0xffffffffu;
    hi[m] = 0u;
  }
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * gsize;
  const int64_t i1 = min(n, i0 + gsize);
  for (int64_t e = i0 * d + threadIdx.x; e < i1 * d; e += blockDim.x) {
    const int64_t i = e / d;
    const int m = (int)(e % d);
    const uint32_t o = ord_of(xh(Xs, i, d, m, kp));
    atomicMin(&lo[m], o);
    atomicMax(&hi[m], o);
  }
  __syncthreads();
  for (int m = threadIdx.x; m < d; m += blockDim.x) {
    box[(int64_t)blockIdx.x * 2 * d + m] = float_of(lo[m]);
    box[(int64_t)blockIdx.x * 2 * d + d + m] = float_of(hi[m]);
  }
}

// Row block b: lists[b * nstage + p] = the stages (increasing) whose box is
// within squared distance r2 of the row block's box; counts[b] = how many.
// One work group per row block; stages go in chunks of 256 with a block-wide
// prefix count so the list stays in stage order.
__global__ __launch_bounds__(256) void list_kernel(const float* __restrict__ rbox,
                                                   const float* __restrict__ cbox, int d,
                                                   int64_t nstage, float r2,
                                                   int* __restrict__ lists,
                                                   int* __restrict__ counts) {
  __shared__ int warp_cnt[4];
  __shared__ int base;
  const float* rb = rbox + (int64_t)blockIdx.x * 2 * d;
  int* out = lists + (int64_t)blockIdx.x * nstage;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t j0 = 0; j0 < nstage; j0 += 256) {
    const int64_t j = j0 + threadIdx.x;
    bool keep = false;
    if (j < nstage) {
      const float* cb = cbox + j * 2 * d;
      float acc = 0.0f;
      for (int m = 0; m < d; ++m) {
        const float gap = fmaxf(fmaxf(rb[m] - cb[d + m], cb[m] - rb[d + m]), 0.0f);
        acc = fmaf(gap, gap, acc);
      }
      keep = acc < r2;
    }
    const uint64_t mask = __ballot(keep);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) warp_cnt[wave] = __popcll(mask);
    __syncthreads();
    int off = base;
    for (int w = 0; w < wave; ++w) off += warp_cnt[w];
    if (keep) out[off + before] = (int)j;
    __syncthreads();
    if (threadIdx.x == 0) base += warp_cnt[0] + warp_cnt[1] + warp_cnt[2] + warp_cnt[3];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = base;
}

// Unit-outputscale kernel value as a function of the scaled distance r.
double kval(int kind, double r) {
  switch (kind) {
    case GP_KERNEL_RBF: return exp(-0.5 * r * r);
    case GP_KERNEL_MATERN12: return exp(-r);
    case GP_KERNEL_MATERN32: {
      const double t = sqrt(3.0) * r;
      return (1.0 + t) * exp(-t);
    }
    default: {
      const double t = sqrt(5.0) * r;
      return (1.0 + t + t * t / 3.0) * exp(-t);
    }
  }
}

}  // namespace

// Scaled distance beyond which the kernel value is below 2^-26 (bisection on
// the decreasing closed form).
double radius(int kind) {
  const double target = ldexp(1.0, -26);
  double lo = 0.0, hi = 1.0;
  while (kval(kind, hi) > target) hi *= 2.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (kval(kind, mid) > target)
      lo = mid;
    else
      hi = mid;
  }
  return hi;
}

}  // namespace trunc
}  // namespace gpmi

using namespace gpmi;

namespace {

// Z-order permutation of one point set into perm (n ints); scratch from ar.
gp_status zorder(const float* X, int64_t n, const KParams& kp, int* perm, Arena& ar,
                 hipStream_t s) {
  uint32_t* ext = ar.take<uint32_t>(2 * kMaxDim);
  uint64_t* keys = ar.take<uint64_t>((size_t)n);
  uint64_t* keys2 = ar.take<uint64_t>((size_t)n);
  int* idx = ar.take<int>((size_t)n);
  if (!ext || !keys || !keys2 || !idx) return set_error(GP_ERR_NOMEM, "internal: truncation workspace");
  trunc::fill_u32_kernel<<<1, kMaxDim, 0, s>>>(ext, kMaxDim, 0xffffffffu);
  GP_HIP(hipGetLastError());
  trunc::fill_u32_kernel<<<1, kMaxDim, 0, s>>>(ext + kMaxDim, kMaxDim, 0u);
  GP_HIP(hipGetLastError());
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(n * kp.d, 256)));
  trunc::extent_kernel<<<blocks, 256, 0, s>>>(X, n, kp, ext);
  GP_HIP(hipGetLastError());
  trunc::morton_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(X, n, kp, ext, keys, idx);
  GP_HIP(hipGetLastError());
  size_t tmp_bytes = 0;
  GP_HIP(rocprim::radix_sort_pairs(nullptr, tmp_bytes, keys, keys2, idx, perm, (unsigned)n, 0u, 64u, s));
  void* tmp = ar.take<char>(tmp_bytes);
  if (!tmp) return set_error(GP_ERR_NOMEM, "internal: truncation workspace (sort)");
  GP_HIP(rocprim::radix_sort_pairs(tmp, tmp_bytes, keys, keys2, idx, perm, (unsigned)n, 0u, 64u, s));
  return GP_OK;
}

size_t zorder_bytes(int64_t n) {
  size_t tmp_bytes = 0;
  (void)rocprim::radix_sort_pairs(nullptr, tmp_bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                  (const int*)nullptr, (int*)nullptr, (unsigned)n, 0u, 64u,
                                  (hipStream_t)0);
  return 8 * kMaxDim + 16 * (size_t)n + 4 * (size_t)n + tmp_bytes + 5 * 256;
}

}  // namespace

extern "C" gp_status gp_kmvm_truncated(const gp_kernel* k, const float* X1, int64_t n1,
                                       const float* X2, int64_t n2, int32_t d, const float* V,
                                       int32_t r, float* out, int32_t add_noise, int32_t skip,
                                       gp_trunc_stats* stats, void* stream) {
  clear_error();
  KParams kp;
  GP_TRY(check_kernel(k, d, false, &kp));
  if (n1 < 0 || n2 < 0) return set_error(GP_ERR_ARG, "negative point count");
  if (n1 > INT32_MAX / 2 || n2 > INT32_MAX / 2) return set_error(GP_ERR_ARG, "point count too large");
  if (r < 1) return set_error(GP_ERR_ARG, "r=%d must be >= 1", r);
  if (skip != 0 && skip != 1) return set_error(GP_ERR_ARG, "skip must be 0 or 1");
  if (n1 > 0 && (!X1 || !out)) return set_error(GP_ERR_ARG, "X1/out is NULL");
  if (n2 > 0 && (!X2 || !V)) return set_error(GP_ERR_ARG, "X2/V is NULL");
  const bool same = X1 == X2 && n1 == n2;
  if (add_noise && !same) return set_error(GP_ERR_ARG, "add_noise needs X1 == X2 and n1 == n2");
  const size_t ob = (size_t)n1 * r * 4;
  if (overlaps(out, ob, V, (size_t)n2 * r * 4) || overlaps(out, ob, X1, (size_t)n1 * d * 4) ||
      overlaps(out, ob, X2, (size_t)n2 * d * 4))
    return set_error(GP_ERR_ARG, "out overlaps an input");
  if (stats) *stats = gp_trunc_stats{};
  if (n1 == 0) return GP_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n2 == 0) return fill_f32(out, n1 * r, 0.0f, s);

  const int w = f16::aug_width(d);
  const int kc = w / 32;
  const int64_t n1_pad = round_up(n1, f16::kRowsPerBlock);
  const int64_t n2_pad = round_up(n2, f16::kStageCols);
  const int64_t nrb = n1_pad / f16::kRowsPerBlock, nstage = n2_pad / f16::kStageCols;
  const int rchunk = std::min(r, 64);
  const int rp_max = (int)round_up(rchunk, 16);
  // half the column splits of the full product: a row block keeps only part
  // of its stages, so fewer, longer stage ranges per work group amortise the
  // pipeline start of each group (1M points, 25% of tiles kept: 4 splits
  // 24.7 ms, 8 splits 27.8 ms); skip = 0 uses the same ranges
  const int nsplit = std::max(1, f16::choose_splits(n1_pad, n2_pad) / 2);
  const size_t bytes = zorder_bytes(n1) + (same ? 0 : zorder_bytes(n2)) + 4 * (size_t)(n1 + n2) +
                       4 * (size_t)n1 * d + 4 * (size_t)n2 * d + 4 * (size_t)n2 * r +
                       4 * (size_t)n1 * r + 2 * (size_t)n1_pad * w + 2 * (size_t)n2_pad * w +
                       2 * (size_t)rp_max * n2_pad + 4 * (size_t)nsplit * n1_pad * rp_max +
                       8 * (size_t)(nrb + nstage) * d + 4 * (size_t)nrb * nstage + 4 * (size_t)nrb +
                       12 * (size_t)rp_max + 32 * 256;
  Arena ar;
  GP_TRY(workspace_get(s, bytes, &ar));
  int* perm1 = ar.take<int>((size_t)n1);
  int* perm2 = same ? perm1 : ar.take<int>((size_t)n2);
  float* X1s = ar.take<float>((size_t)n1 * d);
  float* X2s = same ? X1s : ar.take<float>((size_t)n2 * d);
  float* Vs = ar.take<float>((size_t)n2 * r);
  float* outs = ar.take<float>((size_t)n1 * r);
  _Float16* Xr = ar.take<_Float16>((size_t)n1_pad * w);
  _Float16* Xc = ar.take<_Float16>((size_t)n2_pad * w);
  _Float16* Vt = ar.take<_Float16>((size_t)rp_max * n2_pad);
  float* part = ar.take<float>((size_t)nsplit * n1_pad * rp_max);
  float* rbox = ar.take<float>((size_t)nrb * 2 * d);
  float* cbox = ar.take<float>((size_t)nstage * 2 * d);
  int* lists = ar.take<int>((size_t)nrb * nstage);
  int* counts = ar.take<int>((size_t)nrb);
  uint32_t* colmax = ar.take<uint32_t>(rp_max);
  float* scale = ar.take<float>(rp_max);
  float* inv_scale = ar.take<float>(rp_max);
  if (!perm2 || !X2s || !Vs || !outs || !Xr || !Xc || !Vt || !part || !rbox || !cbox || !lists ||
      !counts || !inv_scale)
    return set_error(GP_ERR_NOMEM, "internal: truncation workspace sizing");

  // 1. orderings and ordered copies
  GP_TRY(zorder(X1, n1, kp, perm1, ar, s));
  if (!same) GP_TRY(zorder(X2, n2, kp, perm2, ar, s));
  trunc::gather_kernel<<<(unsigned)ceil_div(n1 * d, 256), 256, 0, s>>>(X1, perm1, n1, d, X1s);
  GP_HIP(hipGetLastError());
  if (!same) {
    trunc::gather_kernel<<<(unsigned)ceil_div(n2 * d, 256), 256, 0, s>>>(X2, perm2, n2, d, X2s);
    GP_HIP(hipGetLastError());
  }
  trunc::gather_kernel<<<(unsigned)ceil_div(n2 * r, 256), 256, 0, s>>>(V, perm2, n2, r, Vs);
  GP_HIP(hipGetLastError());
  GP_TRY(f16::prep_points(X1s, n1, n1_pad, kp, 0, Xr, s));
  GP_TRY(f16::prep_points(X2s, n2, n2_pad, kp, 1, Xc, s));

  // 2-3. boxes and stage lists
  trunc::box_kernel<<<(unsigned)nrb, 256, 0, s>>>(X1s, n1, kp, f16::kRowsPerBlock, rbox);
  GP_HIP(hipGetLastError());
  trunc::box_kernel<<<(unsigned)nstage, 256, 0, s>>>(X2s, n2, kp, f16::kStageCols, cbox);
  GP_HIP(hipGetLastError());
  const double R = trunc::radius(kp.kind);
  const float r2 = skip ? (float)(R * R) : INFINITY;
  trunc::list_kernel<<<(unsigned)nrb, 256, 0, s>>>(rbox, cbox, d, nstage, r2, lists, counts);
  GP_HIP(hipGetLastError());
  f16::StageLists sl{lists, counts, nstage};

  // 4. the product over the kept stages (right-hand sides in chunks of 64)
  for (int c0 = 0; c0 < r; c0 += 64) {
    const int rc = std::min(64, r - c0);
    const int rb = (int)ceil_div(rc, 16);
    const int rp = 16 * rb;
    GP_TRY(f16::quant_rhs(Vs + c0, n2, rc, r, rp, n2_pad, 0, 1.0f, 1.0f, colmax, Vt, scale,
                          inv_scale, s));
    GP_TRY(f16::launch_main(kp.kind, kc, rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, nullptr,
                             (double)n1 * (double)n2, s, &sl));
    GP_TRY(f16::launch_reduce(part, nsplit, n1, n1_pad, rc, rp, inv_scale, kp.a2, kp.s2,
                              add_noise ? Vs + c0 : nullptr, r, outs + c0, r, nullptr, s));
  }
  // 5. back to the caller's row order
  trunc::scatter_kernel<<<(unsigned)ceil_div(n1 * r, 256), 256, 0, s>>>(outs, perm1, n1, r, out);
  GP_HIP(hipGetLastError());
  if (stats) {
    std::vector<int> hc((size_t)nrb);
    GP_HIP(hipMemcpyAsync(hc.data(), counts, 4 * (size_t)nrb, hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    int64_t visited = 0;
    for (int v : hc) visited += v;
    stats->tiles_total = nrb * nstage;
    stats->tiles_visited = visited;
    stats->radius = R;
  }
  return GP_OK;
}
