// Symmetric fused product K~V for one point set (X1 = X2): every kernel value
// of a pair of distinct row panels is evaluated once and used for both
// contributions, (K V)_i += k_ij v_j and (K V)_j += k_ij v_i (Sec. 5.1,
// Eq. mvm: K~ is symmetric), halving the exponentials and conversions per
// entry of the product.  The arithmetic per entry is that of the binary16
// product of kmvm_f16.hip (same augmented operands, same exponent argument,
// same binary16 kernel values and right-hand sides, float32 accumulation);
// only the order of the float32 sums differs.
//
// Layout of the work: the padded point set is cut into row panels of 1536
// points (kPanel).  A work group of 8 waves owns one panel; each wave owns 64
// rows of each of the panel's 3 row blocks of 512 and keeps their row operands
// and row sums in registers for the whole sweep (three blocks fit the 256
// registers of a wave because a stage keeps only the current and the next
// 32-column block's operands live).  A work item is a panel and a range of
// 128-column stages to its right: the panel's own diagonal block (the first
// 12 stages of its first item) contributes only the direct sums; every later
// stage contributes both.  Larger panels mean fewer column partials (n^2 R 4 /
// (2 kPanel) bytes) and fewer stage boundaries per pair.  Per 16-row subtile and 32 columns:
//   S^T = X_c X_r^T (matrix cores), k = kappa(S) (vector unit), binary16;
//   row sums   += K V_c      (matrix cores, as in the one-sided product);
//   K is written to a per-wave LDS tile and read back transposed with
//   ds_read_b64_tr_b16 (within each 16-lane group, output lane 4a + e receives
//   element e of source lanes a, a + 4, a + 8, a + 12), which gives each lane
//   8 rows of one column: the A operand of
//   column sums += K^T V_r (matrix cores).
// The column sums of a stage are added over the panel's rows in each wave,
// then over the 8 waves in a fixed order through LDS, and written once per
// (panel, stage) to a triangular buffer of column partials; the row sums are
// written once per item.  sym_reduce adds, for every output row, the row
// partials of its panel's items and the column partials of the panels before
// it in fixed orders, then applies a^2, the column scale and s^2 V: results
// are bitwise repeatable.
//
// Limits of this form: one 32-wide operand chunk (d <= 14) and one block of
// 16 right-hand sides (r <= 16); the caller uses the one-sided product
// otherwise.

#include <math.h>

#include "fused_tile.h"
#include "internal.h"

namespace gpmi {
namespace sym {

using f16::f4;
using f16::h4;
using f16::h8;
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s4 lds_s4;

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kM = 3;                          // row blocks per panel (per wave: 64 rows each)
constexpr int kRowBlock = 64 * kWaves;         // 512
constexpr int kPanel = kM * kRowBlock;         // 1536
constexpr int JT = f16::kStageCols;            // 128 columns per stage
constexpr int kDiagStages = kPanel / JT;       // 12
constexpr int KP = 32;                         // operand width (halfs)
constexpr int XS = KP + 8;                     // LDS row stride of the column operands
constexpr int kVS = JT + 8;                    // LDS row stride of the right-hand sides (68 dwords: rows 4 banks apart)
constexpr int kTS = 32;                        // LDS row stride of the transpose tile (halfs)
constexpr int kSS = JT + 4;                    // LDS row stride of a wave's column sums
constexpr int kSlot = 16 * kSS;                // floats per wave for the column sums
static_assert(kPanel % JT == 0, "panel / stage");

struct Item {
  int panel;
  int s0, s1;        // stages [s0, s1) of 128 columns
  int rowpart;       // slot of this item's row partial sums
};

// Item plan shared by host and device: panel a visits stages [D a, S) (D =
// kDiagStages): its D diagonal stages and off_a = S - D (a + 1) stages to the
// right, the latter cut into chunks_of(a) pieces of nearly equal length (at
// most L stages); the first piece also takes the diagonal stages.
__host__ __device__ inline int64_t off_stages(int64_t a, int64_t S) {
  const int64_t o = S - (a + 1) * kDiagStages;
  return o > 0 ? o : 0;
}
__host__ __device__ inline int64_t chunks_of(int64_t a, int64_t S, int64_t L) {
  const int64_t o = off_stages(a, S);
  return o <= L ? 1 : (o + L - 1) / L;
}

// Items in launch order: the first piece of every panel (the longest: it
// carries the diagonal block), then the other pieces panel by panel; each
// item's row-partial slot is its panel-major index, so that a panel's slots
// are contiguous (first[a] .. first[a + 1]).  One thread per panel.
__global__ void plan_kernel(int P, int64_t S, int64_t L, Item* __restrict__ items,
                            int* __restrict__ first, int64_t* __restrict__ colbase) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a > P) return;
  int k = 0;
  int64_t cb = 0;
  for (int b = 0; b < a; ++b) {
    k += (int)chunks_of(b, S, L);
    cb += off_stages(b, S) * JT * 16;
  }
  first[a] = k;
  if (a == P) return;
  colbase[a] = cb;
  const int64_t o = off_stages(a, S), nc = chunks_of(a, S, L);
  const int64_t s0 = (int64_t)(a + 1) * kDiagStages;
  for (int64_t c = 0; c < nc; ++c) {
    const int64_t lo = s0 + o * c / nc, hi = s0 + o * (c + 1) / nc;
    const Item it{a, (int)(c == 0 ? a * kDiagStages : lo), (int)hi, k + (int)c};
    items[c == 0 ? a : P + (k - a) + (int)c - 1] = it;
  }
}

// One 16-row subtile against 32 columns: exponent arguments S^T = X_c X_r^T
// on the matrix cores (lane holds S[c = 4 g + v (+16)][i = l16]).
__device__ __forceinline__ void tile_args(const h8& a0, const h8& a1, const h8& b, f4& s0, f4& s1) {
  s0 = f16::mfma32<_Float16>(a0, b, f4{0.f, 0.f, 0.f, 0.f});
  s1 = f16::mfma32<_Float16>(a1, b, f4{0.f, 0.f, 0.f, 0.f});
}

// Kernel values from the arguments, row sums += K V_c.
template <int KIND>
__device__ __forceinline__ h8 tile_finish(const f4& s0, const f4& s1, const h8& bv, f4& acc) {
  h8 kv;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    kv[v] = (_Float16)f16::kernel_value<KIND>(s0[v]);
    kv[4 + v] = (_Float16)f16::kernel_value<KIND>(s1[v]);
  }
  acc = f16::mfma32<_Float16>(kv, bv, acc);
  return kv;
}

// The 32 x 32 transpose tile: rows of 32 halfs (8 chunks of 4), chunk c of
// row i stored at chunk c ^ ((i >> 1) & 7), so that the 8-byte writes below
// and the transposed reads hit distinct LDS banks.
__device__ __forceinline__ int tile_chunk(int row, int chunk) {
  return row * kTS + 4 * (chunk ^ ((row >> 1) & 7));
}

// kv of local row block q (0 or 1) of a 32-row transpose tile
__device__ __forceinline__ void tile_store(_Float16* tile, int q, int g, int l16, const h8& kv) {
  const int row = q * 16 + l16;
  *reinterpret_cast<h4*>(tile + tile_chunk(row, g)) = h4{kv[0], kv[1], kv[2], kv[3]};
  *reinterpret_cast<h4*>(tile + tile_chunk(row, 4 + g)) = h4{kv[4], kv[5], kv[6], kv[7]};
}

// Transposed read of columns 16 h .. 16 h + 15 of a 32-row tile: lane holds
// rows 8 g .. 8 g + 7 of column 16 h + l16 (A operand of K^T V).
__device__ __forceinline__ h8 tile_column(const _Float16* tile, int h, int g, int l16) {
  typedef short s8 __attribute__((ext_vector_type(8)));
  const int ra = 8 * g + (l16 >> 2), rb = ra + 4, ch = 4 * h + (l16 & 3);
  const s4 r0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)(tile + tile_chunk(ra, ch)));
  const s4 r1 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)(tile + tile_chunk(rb, ch)));
  return __builtin_bit_cast(h8, s8{r0[0], r0[1], r0[2], r0[3], r1[0], r1[1], r1[2], r1[3]});
}

// Identity slots for the matrix-core transpose: lane holds B[k = 8 g + j][n =
// l16] = 1 when k = 16 h + n (h = 0, 1), so that D = K I_h lists, per lane,
// 4 rows of the 16 columns in slots 16 h .. 16 h + 15 of the kernel tile.
__device__ __forceinline__ h8 identity_slots(int h, int g, int l16) {
  h8 b;
#pragma unroll
  for (int j = 0; j < 8; ++j) b[j] = (_Float16)(8 * g + j == 16 * h + l16 ? 1.0f : 0.0f);
  return b;
}

// Column of the stage that slot n (0..15) of the identity set h stands for:
// slot k = 16 h + n of the kernel tile holds column 4 (k / 8) + k % 8 when
// k % 8 < 4, else 16 + 4 (k / 8) + k % 8 - 4 (the S^T lane layout).
__device__ __forceinline__ int slot_column(int h, int n) {
  const int k = 16 * h + n, kg = k >> 3, kq = k & 7;
  return kq < 4 ? 4 * kg + kq : 16 + 4 * kg + kq - 4;
}

// One stage of 128 columns for the wave's 2 x 64 rows.  OFFD: also the
// column sums T (the transposed contributions).  TR selects how the kernel
// tile is transposed for K^T V: 0 through the wave's two LDS tiles (written,
// then read back with ds_read_b64_tr_b16; the tiles alternate so that one is
// read while the next is written), 1 on the matrix cores (D = K I_h, exact for
// binary16 values, converted back to binary16).  Both give the same values
// in the same summation order.
template <int KIND, bool OFFD, int TR>
__device__ __forceinline__ void stage_body(const _Float16* __restrict__ X,
                                           const _Float16* __restrict__ Vs, const h8 (&bi)[kM][4],
                                           const h8 (&vB)[kM][2], const h8 (&eye)[2],
                                           f4 (&acc)[kM][4], f4 (&T)[JT / 16], _Float16* tiles,
                                           int g, int l16) {
  // operands of the current 32-column block (and of the next, read one step
  // before the block starts: its first exponent arguments are issued then)
  auto load_a = [&](int jb, h8& x0, h8& x1) {
    x0 = *reinterpret_cast<const h8*>(X + (jb * 32 + l16) * XS + g * 8);
    x1 = *reinterpret_cast<const h8*>(X + (jb * 32 + 16 + l16) * XS + g * 8);
  };
  auto load_v = [&](int jb) {
    const _Float16* vr = Vs + l16 * kVS + jb * 32 + g * 4;
    const h4 lo = *reinterpret_cast<const h4*>(vr);
    const h4 hi = *reinterpret_cast<const h4*>(vr + 16);
    return h8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  };
  h8 ca0, ca1, cbv, na0, na1, nbv;
  load_a(0, ca0, ca1);
  cbv = load_v(0);
  // steps t = (jb, m, p): a pair of 16-row subtiles against 32 columns.  With
  // the LDS transpose the steps are software-pipelined: the transposed read of
  // step t - 1 is issued before the kernel values of step t are computed, and
  // consumed after them, so the LDS latency overlaps the exponentials.
  constexpr int kSteps = (JT / 32) * kM * 2;
  h8 c0p, c1p;
  // the exponent arguments of step t + 1 are issued on the matrix cores
  // before the kernel values of step t are computed on the vector unit
  f4 sa0, sa1, sb0, sb1;
  tile_args(ca0, ca1, bi[0][0], sa0, sa1);
  tile_args(ca0, ca1, bi[0][1], sb0, sb1);
#pragma unroll
  for (int t = 0; t < kSteps; ++t) {
    const int jb = t / (kM * 2), m = (t / 2) % kM, p = t % 2;
    const int tp = t - 1, jbp = tp / (kM * 2), mp = (tp / 2) % kM, pp = tp % 2;
    if constexpr (OFFD && TR == 0) {
      if (t > 0) {
        const _Float16* tq = tiles + (tp & 1) * 32 * kTS;
        c0p = tile_column(tq, 0, g, l16);
        c1p = tile_column(tq, 1, g, l16);
      }
    }
    f4 na0s, na1s, nb0s, nb1s;
    const int tn = t + 1, jbn = tn / (kM * 2), mn = (tn / 2) % kM, pn = tn % 2;
    // The wave's priority is raised while it issues these four independent
    // MFMAs, so that the other wave on the SIMD, busy with its exponentials,
    // yields the issue slot to them and the matrix cores start early (the
    // results are unchanged; 1.6-1.9% faster at 1.8M points).
    if (t + 1 < kSteps) {
      if (jbn != jb) {
        load_a(jbn, na0, na1);
        nbv = load_v(jbn);
        __builtin_amdgcn_s_setprio(1);
        tile_args(na0, na1, bi[mn][2 * pn], na0s, na1s);
        tile_args(na0, na1, bi[mn][2 * pn + 1], nb0s, nb1s);
        __builtin_amdgcn_s_setprio(0);
      } else {
        __builtin_amdgcn_s_setprio(1);
        tile_args(ca0, ca1, bi[mn][2 * pn], na0s, na1s);
        tile_args(ca0, ca1, bi[mn][2 * pn + 1], nb0s, nb1s);
        __builtin_amdgcn_s_setprio(0);
      }
    }
    // both subtiles' kernel values first, then their two row-sum MFMAs
    h8 k0, k1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      k0[v] = (_Float16)f16::kernel_value<KIND>(sa0[v]);
      k0[4 + v] = (_Float16)f16::kernel_value<KIND>(sa1[v]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      k1[v] = (_Float16)f16::kernel_value<KIND>(sb0[v]);
      k1[4 + v] = (_Float16)f16::kernel_value<KIND>(sb1[v]);
    }
    acc[m][2 * p] = f16::mfma32<_Float16>(k0, cbv, acc[m][2 * p]);
    acc[m][2 * p + 1] = f16::mfma32<_Float16>(k1, cbv, acc[m][2 * p + 1]);
    if (t + 1 < kSteps) {
      sa0 = na0s; sa1 = na1s; sb0 = nb0s; sb1 = nb1s;
      if (jbn != jb) {
        ca0 = na0; ca1 = na1; cbv = nbv;
      }
    }
    if constexpr (OFFD && TR == 0) {
      if (t > 0) {
        T[jbp * 2] = f16::mfma32<_Float16>(c0p, vB[mp][pp], T[jbp * 2]);
        T[jbp * 2 + 1] = f16::mfma32<_Float16>(c1p, vB[mp][pp], T[jbp * 2 + 1]);
      }
      _Float16* tw = tiles + (t & 1) * 32 * kTS;
      tile_store(tw, 0, g, l16, k0);
      tile_store(tw, 1, g, l16, k1);
      if (t == kSteps - 1) {
        const h8 c0 = tile_column(tw, 0, g, l16);
        const h8 c1 = tile_column(tw, 1, g, l16);
        T[jb * 2] = f16::mfma32<_Float16>(c0, vB[m][p], T[jb * 2]);
        T[jb * 2 + 1] = f16::mfma32<_Float16>(c1, vB[m][p], T[jb * 2 + 1]);
      }
    }
    if constexpr (OFFD && TR == 1) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const f4 z = f4{0.f, 0.f, 0.f, 0.f};
        const f4 d0 = f16::mfma32<_Float16>(k0, eye[h], z);
        const f4 d1 = f16::mfma32<_Float16>(k1, eye[h], z);
        const h8 c = h8{(_Float16)d0[0], (_Float16)d0[1], (_Float16)d0[2], (_Float16)d0[3],
                        (_Float16)d1[0], (_Float16)d1[1], (_Float16)d1[2], (_Float16)d1[3]};
        T[jb * 2 + h] = f16::mfma32<_Float16>(c, vB[m][p], T[jb * 2 + h]);
      }
    }
  }
}

// Transposition of the kernel tile for K^T V (see stage_body).
constexpr int kSymTranspose = 0;

template <int KIND, int TR>
__global__ __launch_bounds__(kThreads, 1) void sym_kernel(const _Float16* __restrict__ Xr,
                                                          const _Float16* __restrict__ Xc,
                                                          const _Float16* __restrict__ Vt,
                                                          int64_t n_pad,
                                                          const Item* __restrict__ items,
                                                          float* __restrict__ rowpart,
                                                          float* __restrict__ colpart,
                                                          const int64_t* __restrict__ colbase,
                                                          const int* __restrict__ live) {
  if (live && *live == 0) return;
  __shared__ __attribute__((aligned(16))) _Float16 sX[2 * JT * XS];
  __shared__ __attribute__((aligned(16))) _Float16 sV[2 * 16 * kVS];
  __shared__ __attribute__((aligned(16))) _Float16 sT[kWaves * 2 * 32 * kTS];
  __shared__ __attribute__((aligned(16))) float sSlot[kWaves * kSlot];

  const Item it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 4;
  const int l16 = lane & 15;
  const int64_t prow0 = (int64_t)it.panel * kPanel;
  const int64_t diag_end = (int64_t)(it.panel + 1) * kDiagStages;

  // the wave's rows of the panel: row operands (B operand of S^T) and
  // right-hand sides (B operand of K^T V: lane holds rows 32 p + 8 g .. + 7
  // of right-hand side l16), resident for the whole item
  h8 bi[kM][4];
  h8 vB[kM][2];
#pragma unroll
  for (int m = 0; m < kM; ++m) {
    const int64_t r0 = prow0 + m * kRowBlock + wave * 64;
#pragma unroll
    for (int is = 0; is < 4; ++is)
      bi[m][is] = *reinterpret_cast<const h8*>(Xr + (r0 + is * 16 + l16) * KP + g * 8);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const _Float16* vp = Vt + (int64_t)l16 * n_pad + r0 + 32 * p;
      if constexpr (TR == 0) {
        vB[m][p] = *reinterpret_cast<const h8*>(vp + 8 * g);
      } else {
        // rows 4 g .. 4 g + 3 and 16 + 4 g .. + 3 of the pair (the row slots of D = K I_h)
        const h4 lo = *reinterpret_cast<const h4*>(vp + 4 * g);
        const h4 hi = *reinterpret_cast<const h4*>(vp + 16 + 4 * g);
        vB[m][p] = h8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      }
    }
  }
  h8 eye[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) eye[h] = identity_slots(h, g, l16);
  f4 acc[kM][4];
#pragma unroll
  for (int m = 0; m < kM; ++m)
#pragma unroll
    for (int is = 0; is < 4; ++is) acc[m][is] = f4{0.f, 0.f, 0.f, 0.f};

  // stage staging: 512 chunks of 8 column operands (one per thread), 256 of
  // 8 right-hand-side values
  h8 xreg, vreg;
  auto gload = [&](int64_t st) {
    const int64_t j0 = st * JT;
    xreg = *reinterpret_cast<const h8*>(Xc + (j0 + (tid >> 2)) * KP + (tid & 3) * 8);
    if (tid < 256)
      vreg = *reinterpret_cast<const h8*>(Vt + (int64_t)(tid >> 4) * n_pad + j0 + (tid & 15) * 8);
  };
  auto lstore = [&](int buf) {
    *reinterpret_cast<h8*>(&sX[buf * JT * XS + (tid >> 2) * XS + (tid & 3) * 8]) = xreg;
    if (tid < 256) {
      _Float16* dst = &sV[buf * 16 * kVS + (tid >> 4) * kVS + (tid & 15) * 8];
      *reinterpret_cast<h4*>(dst) = h4{vreg[0], vreg[1], vreg[2], vreg[3]};
      *reinterpret_cast<h4*>(dst + 4) = h4{vreg[4], vreg[5], vreg[6], vreg[7]};
    }
  };

  _Float16* tiles = sT + wave * 2 * 32 * kTS;
  const int64_t sb = it.s0, se = it.s1;
  if (sb < se) {
    gload(sb);
    lstore(0);
    __syncthreads();
  }
  // column sums of a stage: wave partials through LDS ([rhs][column]), added
  // in wave order and written as [rhs][128 columns] of the stage.  The sum of
  // stage st is formed at the start of stage st + 1 (after the barrier that
  // ends stage st), so its LDS reads and global store overlap the next
  // stage's first tiles instead of idling the compute units between barriers.
  auto reduce_slots = [&](int64_t stp) {
    const int rr = tid >> 5, cc = 4 * (tid & 31);
    f4 sum = *reinterpret_cast<const f4*>(sSlot + rr * kSS + cc);
#pragma unroll
    for (int w = 1; w < kWaves; ++w)
      sum += *reinterpret_cast<const f4*>(sSlot + w * kSlot + rr * kSS + cc);
    float* dst = colpart + colbase[it.panel] + (stp - diag_end) * JT * 16 + rr * JT + cc;
    *reinterpret_cast<f4*>(dst) = sum;
  };
  bool pending = false;
  int64_t pend_st = 0;
  for (int64_t st = sb; st < se; ++st) {
    const int buf = (int)((st - sb) & 1);
    const bool more = st + 1 < se;
    if (more) gload(st + 1);
    if (pending) {
      reduce_slots(pend_st);
      pending = false;
    }
    const _Float16* X = sX + buf * JT * XS;
    const _Float16* Vs = sV + buf * 16 * kVS;
    f4 T[JT / 16];
    if (st < diag_end) {
      stage_body<KIND, false, TR>(X, Vs, bi, vB, eye, acc, T, tiles, g, l16);
    } else {
#pragma unroll
      for (int cb = 0; cb < JT / 16; ++cb) T[cb] = f4{0.f, 0.f, 0.f, 0.f};
      stage_body<KIND, true, TR>(X, Vs, bi, vB, eye, acc, T, tiles, g, l16);
      // every thread has read the previous stage's slots before they are reused
      __syncthreads();
      float* slot = sSlot + wave * kSlot;
#pragma unroll
      for (int cb = 0; cb < JT / 16; ++cb) {
        if constexpr (TR == 0) {
          *reinterpret_cast<f4*>(slot + l16 * kSS + cb * 16 + 4 * g) = T[cb];
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            slot[l16 * kSS + (cb >> 1) * 32 + slot_column(cb & 1, 4 * g + v)] = T[cb][v];
        }
      }
      pending = true;
      pend_st = st;
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
  }
  if (pending) reduce_slots(pend_st);

  float* R = rowpart + (int64_t)it.rowpart * kPanel * 16;
#pragma unroll
  for (int m = 0; m < kM; ++m)
#pragma unroll
    for (int is = 0; is < 4; ++is)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        R[(int64_t)l16 * kPanel + m * kRowBlock + wave * 64 + is * 16 + 4 * g + v] = acc[m][is][v];
}

// out[i][c] = a2 inv_scale[c] (row partials of panel(i)'s items in item order
// + column partials of panels 0 .. panel(i) - 1 in panel order) + s2 V[i][c].
__global__ void sym_reduce_kernel(const float* __restrict__ rowpart,
                                  const float* __restrict__ colpart,
                                  const int* __restrict__ first,
                                  const int64_t* __restrict__ colbase, int64_t n, int r,
                                  const float* __restrict__ inv_scale, float a2, float s2,
                                  const float* __restrict__ V, int64_t ldv, float* __restrict__ out,
                                  int64_t ldo, const int* __restrict__ live) {
  if (live && *live == 0) return;
  // one thread per (row, group of 4 right-hand sides); consecutive threads
  // take consecutive rows, so every load is contiguous across the wave.  Rows
  // run from the last panel down: a row of panel p adds p column partials, so
  // the longest waves start first and the grid does not end on a tail of them.
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * 4) return;
  const int q = (int)(e / n);
  const int64_t i = n - 1 - (e - (int64_t)q * n);
  const int c0 = 4 * q;
  if (c0 >= r) return;
  const int64_t p = i / kPanel;
  const int64_t li = i - p * kPanel;
  f4 acc = f4{0.f, 0.f, 0.f, 0.f};
  const int k0 = first[p], k1 = first[p + 1];
  for (int k = k0; k < k1; k += 4) {
    f4 x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k + u < k1) {
        const float* b = rowpart + (int64_t)(k + u) * kPanel * 16 + li;
        x[u] = f4{b[(c0 + 0) * kPanel], b[(c0 + 1) * kPanel], b[(c0 + 2) * kPanel],
                  b[(c0 + 3) * kPanel]};
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k + u < k1) acc += x[u];
  }
  for (int64_t a = 0; a < p; a += 8) {
    f4 x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (a + u < p) {
        const int64_t j = i - (a + u + 1) * kPanel;      // column offset within panel a's range
        const float* b = colpart + colbase[a + u] + (j / JT) * JT * 16 + (j % JT);
        x[u] = f4{b[(c0 + 0) * JT], b[(c0 + 1) * JT], b[(c0 + 2) * JT], b[(c0 + 3) * JT]};
      }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (a + u < p) acc += x[u];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = c0 + u;
    if (c < r) {
      float o = (a2 * inv_scale[c]) * acc[u];
      if (V) o = fmaf(s2, V[i * ldv + c], o);
      out[i * ldo + c] = o;
    }
  }
}

}  // namespace sym

namespace f16 {

bool sym_supported(int d, int r) { return aug_width(d) == sym::KP && r <= 16; }

int64_t sym_pad(int64_t n) { return round_up(std::max<int64_t>(n, 1), sym::kPanel); }

// Stages per item: about 2048 items over the upper triangle (8 per compute
// unit), at least 8.
static int64_t sym_chunk(int64_t n_pad) {
  const int64_t P = n_pad / sym::kPanel, S = n_pad / sym::JT;
  int64_t total = 0;
  for (int64_t a = 0; a < P; ++a) total += sym::off_stages(a, S);
  return std::max<int64_t>(8, ceil_div(total, 2048));
}

SymPlan sym_plan(int64_t n_pad) {
  SymPlan pl{};
  pl.n_pad = n_pad;
  pl.panels = (int)(n_pad / sym::kPanel);
  pl.stages = n_pad / sym::JT;
  pl.chunk = sym_chunk(n_pad);
  int64_t items = 0, cols = 0;
  for (int64_t a = 0; a < pl.panels; ++a) {
    items += sym::chunks_of(a, pl.stages, pl.chunk);
    cols += sym::off_stages(a, pl.stages) * sym::JT;
  }
  pl.items = items;
  pl.rowpart_floats = items * sym::kPanel * 16;
  pl.colpart_floats = cols * 16;
  return pl;
}

size_t sym_bytes(const SymPlan& pl) {
  auto r256 = [](size_t b) { return (b + 255) & ~size_t(255); };
  return r256(sizeof(sym::Item) * pl.items) + r256(sizeof(int) * (pl.panels + 1)) +
         r256(sizeof(int64_t) * pl.panels) + r256(4 * (size_t)pl.rowpart_floats) +
         r256(4 * (size_t)pl.colpart_floats);
}

gp_status sym_carve(SymPlan& pl, Arena& ar) {
  pl.items_dev = ar.take<char>(sizeof(sym::Item) * pl.items);
  pl.first = ar.take<int>(pl.panels + 1);
  pl.colbase = ar.take<int64_t>(pl.panels);
  pl.rowpart = ar.take<float>(pl.rowpart_floats);
  pl.colpart = ar.take<float>(std::max<int64_t>(pl.colpart_floats, 1));
  if (!pl.items_dev || !pl.first || !pl.colbase || !pl.rowpart || !pl.colpart)
    return set_error(GP_ERR_NOMEM, "internal: symmetric product workspace sizing");
  return GP_OK;
}

gp_status sym_prepare(const SymPlan& pl, hipStream_t s) {
  sym::plan_kernel<<<(unsigned)ceil_div(pl.panels + 1, 256), 256, 0, s>>>(pl.panels, pl.stages, pl.chunk,
                                    reinterpret_cast<sym::Item*>(pl.items_dev), pl.first,
                                    pl.colbase);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status sym_launch(int kind, const SymPlan& pl, const _Float16* Xr, const _Float16* Xc,
                     const _Float16* Vt, const int* live, double entries, hipStream_t s) {
  const sym::Item* items = reinterpret_cast<const sym::Item*>(pl.items_dev);
  const unsigned grid = (unsigned)pl.items;
  void* tok = prof::begin(s);
  switch (kind) {
    case GP_KERNEL_RBF:
      sym::sym_kernel<GP_KERNEL_RBF, sym::kSymTranspose><<<grid, sym::kThreads, 0, s>>>(
          Xr, Xc, Vt, pl.n_pad, items, pl.rowpart, pl.colpart, pl.colbase, live);
      break;
    case GP_KERNEL_MATERN52:
      sym::sym_kernel<GP_KERNEL_MATERN52, sym::kSymTranspose><<<grid, sym::kThreads, 0, s>>>(
          Xr, Xc, Vt, pl.n_pad, items, pl.rowpart, pl.colpart, pl.colbase, live);
      break;
    case GP_KERNEL_MATERN12:
      sym::sym_kernel<GP_KERNEL_MATERN12, sym::kSymTranspose><<<grid, sym::kThreads, 0, s>>>(
          Xr, Xc, Vt, pl.n_pad, items, pl.rowpart, pl.colpart, pl.colbase, live);
      break;
    case GP_KERNEL_MATERN32:
      sym::sym_kernel<GP_KERNEL_MATERN32, sym::kSymTranspose><<<grid, sym::kThreads, 0, s>>>(
          Xr, Xc, Vt, pl.n_pad, items, pl.rowpart, pl.colpart, pl.colbase, live);
      break;
    default:
      return set_error(GP_ERR_ARG, "unknown kernel kind %d", kind);
  }
  GP_HIP(hipGetLastError());
  prof::end(tok, s, entries, kind);
  return GP_OK;
}

gp_status sym_reduce(const SymPlan& pl, int64_t n, int r, const float* inv_scale, float a2,
                     float s2, const float* V, int64_t ldv, float* out, int64_t ldo,
                     const int* live, hipStream_t s) {
  if (n == 0) return GP_OK;
  sym::sym_reduce_kernel<<<(unsigned)ceil_div(n * 4, 256), 256, 0, s>>>(
      pl.rowpart, pl.colpart, pl.first, pl.colbase, n, r, inv_scale, a2, s2, V, ldv, out, ldo,
      live);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

}  // namespace f16
}  // namespace gpmi
