// Internal declarations shared by the gpmi host code and kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "gpmi.h"

namespace gpmi {

constexpr int kMaxDim = 64;

// Kernel hyperparameters as passed by value to device code.
struct KParams {
  int kind;
  int d;
  float a2;      // outputscale
  float s2;      // noise
  float ls[kMaxDim];
};

// ---- error state (per host thread) ----
gp_status set_error(gp_status st, const char* fmt, ...);
void clear_error();

#define GP_HIP(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      return ::gpmi::set_error(GP_ERR_HIP, "%s failed: %s (%s:%d)", #expr,        \
                               hipGetErrorString(e_), __FILE__, __LINE__);        \
  } while (0)

#define GP_TRY(expr)                 \
  do {                               \
    gp_status s_ = (expr);           \
    if (s_ != GP_OK) return s_;      \
  } while (0)

__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
__host__ __device__ inline int64_t ceil_div(int64_t x, int64_t m) { return (x + m - 1) / m; }

// Bump allocator over one device block; every sub-buffer is 256-byte aligned.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (off + bytes > cap) return nullptr;
    T* p = reinterpret_cast<T*>(base + off);
    off += bytes;
    return p;
  }
};

// Library-owned device workspace cached per (device, stream).  Growing it
// synchronises the stream first so no queued kernel still uses the old block.
gp_status workspace_get(hipStream_t s, size_t bytes, Arena* out);
// Free every per-stream workspace (waits for each device first); bytes freed.
size_t workspace_release();
// Free every cached preconditioner block; bytes freed.
size_t block_cache_release();

// Device blocks returned by long-lived handles, kept per (device, size) for
// the next handle of the same size (at most kBlockCacheBytes in total, beyond
// which blocks are freed), so a handle built and destroyed repeatedly does not
// pay hipMalloc and the device synchronisation of hipFree each time.
// block_cache_put expects no queued work to use the block any more.
constexpr size_t kBlockCacheBytes = size_t(4) << 30;
gp_status block_cache_get(size_t bytes, void** out);
void block_cache_put(int device, void* p, size_t bytes);

// Autotuned launch-shape decisions (tune.cpp); built-in rules until gp_autotune.
namespace tune {
constexpr int kBuckets = GP_TUNE_BUCKETS;
int64_t bucket_rows(int b);
int bucket_of(int64_t n1_pad);
// column splits of the single-problem binary16 product (fallback: built-in rule)
int f16_splits(int64_t n1_pad, int64_t n2_pad, int fallback);
int bt_split_div();      // batched: splits = clamp(stages / div, 1, 8)
bool bt_persistent();    // batched: persistent product launch
}  // namespace tune

// Opt-in launch timing of the fused product (gp_profile_*).
namespace prof {
void* begin(hipStream_t s);                       // nullptr when disabled
void end(void* token, hipStream_t s, double entries, int kind);
}  // namespace prof

// Device fill (usable under stream capture, unlike a memset node).
gp_status fill_f32(float* p, int64_t n, float v, hipStream_t s);

// Validation helpers.
gp_status check_kernel(const gp_kernel* k, int32_t d, bool need_noise, KParams* kp);
bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes);

// ---------------------------------------------------------------------------
// Kernel-matrix product, float16 matrix-core path (a1, a2 of the hot path).
// ---------------------------------------------------------------------------
namespace f16 {
constexpr int kRowsPerBlock = 256;   // 4 waves x 4 subtiles x 16 rows
constexpr int kStageCols = 128;      // columns per LDS stage

// Width (halfs) of the augmented operand rows for dimension d: binary16
// operands carry the column-side factors as hi + lo pairs, bfloat16 operands
// (8-bit significands) as three parts.
inline int aug_width(int d) { return (int)round_up(2 * d + 4, 32); }
inline int aug_width_bf16(int d) { return (int)round_up(3 * d + 6, 32); }

// Prepared operands of one point set: augmented binary16 rows.
gp_status prep_points(const float* X, int64_t n, int64_t n_pad, const KParams& kp, int side,
                      _Float16* out, hipStream_t s);

// Scaled, transposed binary16 copy of V (n x r, row stride ld) as Vt
// (rp x n_pad) and per-column scales.  colmax must hold rp uint32 (cleared
// here).  scale_mode 0: power of two; 1: fixed_scale for every column.
gp_status quant_rhs(const float* V, int64_t n, int r, int64_t ld, int rp, int64_t n_pad,
                    int scale_mode, float fixed_scale, float fixed_inv, uint32_t* colmax,
                    _Float16* Vt, float* scale, float* inv_scale, hipStream_t s);
gp_status quant_rhs(const float* V, int64_t n, int r, int64_t ld, int rp, int64_t n_pad,
                    int scale_mode, float fixed_scale, float fixed_inv, uint32_t* colmax,
                    __bf16* Vt, float* scale, float* inv_scale, hipStream_t s);

// bfloat16 operands: inputs divided by the lengthscale rounded to bfloat16,
// column-side factors in three bfloat16 parts (width aug_width_bf16(d)).
gp_status prep_points_bf16(const float* X, int64_t n, int64_t n_pad, const KParams& kp, int side,
                           __bf16* out, hipStream_t s);

// The fused product with bfloat16 operands (no stage lists).
gp_status launch_main_bf16(int kind, int kc, int rb, const __bf16* Xr, const __bf16* Xc,
                           const __bf16* Vt, float* part, int64_t n1_pad, int64_t n2_pad,
                           int nsplit, const int* live, double entries, hipStream_t s);

// Per-row-block lists of the column stages a truncated product visits.
struct StageLists {
  const int* lists;    // row block b: stage ids lists[b * ld + p], p < counts[b], increasing
  const int* counts;
  int64_t ld;
};

// Main fused product over prepared operands: part[nsplit][n1_pad][rp].
// If live is non-null and *live == 0 the launch does nothing (used by the
// solver once every column is frozen).
// `entries` (n1 x n2 of the unpadded sets) is recorded by the launch timer.
// With stage lists, each row block visits only its listed stages (column
// splits keep their stage-id ranges, so skipping zero tiles leaves every sum
// unchanged).
gp_status launch_main(int kind, int kc, int rb, const _Float16* Xr, const _Float16* Xc,
                      const _Float16* Vt, float* part, int64_t n1_pad, int64_t n2_pad,
                      int nsplit, const int* live, double entries, hipStream_t s,
                      const StageLists* sl = nullptr);

// Quantise V with the per-column maxima already in colmax (no clearing, no
// max pass): the solver's direction kernel produces colmax itself.
gp_status quant_only(const float* V, int64_t n, int r, int64_t ld, int rp, int64_t n_pad,
                     const uint32_t* colmax, _Float16* Vt, float* scale, float* inv_scale,
                     const int* live, hipStream_t s);
gp_status quant_only(const float* V, int64_t n, int r, int64_t ld, int rp, int64_t n_pad,
                     const uint32_t* colmax, __bf16* Vt, float* scale, float* inv_scale,
                     const int* live, hipStream_t s);

// out[i][c] = a2 * inv_scale[c] * sum_x part[x][i][c] + s2 * V[i][c] (V may be
// null); V and out have row strides ldv and ldo.
gp_status launch_reduce(const float* part, int nsplit, int64_t n1, int64_t n1_pad, int r, int rp,
                        const float* inv_scale, float a2, float s2, const float* V, int64_t ldv,
                        float* out, int64_t ldo, const int* live, hipStream_t s);

int choose_splits(int64_t n1_pad, int64_t n2_pad);

// Symmetric product of one point set (kmvm_sym.hip): panels of 1536 points,
// each kernel value of two distinct panels evaluated once for both sides.
// Operands, right-hand sides (rp = 16) and the output use n_pad = sym_pad(n).
struct SymPlan {
  int64_t n_pad;
  int panels;
  int64_t stages;
  int64_t chunk;            // stages per work item
  int64_t items;
  int64_t rowpart_floats;
  int64_t colpart_floats;
  char* items_dev;          // carved by sym_carve
  int* first;
  int64_t* colbase;
  float* rowpart;
  float* colpart;
};
bool sym_supported(int d, int r);   // one 32-wide operand chunk, r <= 16
// smallest point count the solver and gp_kmvm give to the symmetric product
constexpr int64_t kSymMinN = 16384;
int64_t sym_pad(int64_t n);
SymPlan sym_plan(int64_t n_pad);
size_t sym_bytes(const SymPlan& pl);
gp_status sym_carve(SymPlan& pl, Arena& ar);
// writes the item table (once per plan, before the first launch)
gp_status sym_prepare(const SymPlan& pl, hipStream_t s);
gp_status sym_launch(int kind, const SymPlan& pl, const _Float16* Xr, const _Float16* Xc,
                     const _Float16* Vt, const int* live, double entries, hipStream_t s);
gp_status sym_reduce(const SymPlan& pl, int64_t n, int r, const float* inv_scale, float a2,
                     float s2, const float* V, int64_t ldv, float* out, int64_t ldo,
                     const int* live, hipStream_t s);
}  // namespace f16

// ---------------------------------------------------------------------------
// Kernel-matrix product on the vector ALUs: float32 entries, float32 or
// float64 accumulation.
// ---------------------------------------------------------------------------
namespace valu {
constexpr int kRowsPerBlock = 256;
constexpr int kStageCols = 64;
// part is float (acc32) or double (acc64): [nsplit][n1][r]
gp_status launch_partial(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                         int64_t n2, const float* V, int r, void* part, bool acc64, int nsplit,
                         const int* live, hipStream_t s);
gp_status launch_reduce32(const float* part, int nsplit, int64_t n1, int r, float a2, float s2,
                          const float* V, float* out, const int* live, hipStream_t s);
int choose_splits(int64_t n1, int64_t n2, int d);
// column splits of the float64-accumulated product (true residual)
int choose_splits64(int64_t n1, int64_t n2, int d);
}  // namespace valu

// ---------------------------------------------------------------------------
// Conjugate-gradient step kernels (a3-a8 of the hot path).
// ---------------------------------------------------------------------------
namespace cg {
constexpr int kMaxR = 64;
constexpr int kMaxBlocks = 512;
constexpr int kReorthChunks = 256;

// Per-solve scalars, resident in device memory.
struct State {
  double lg[kMaxR];          // log gamma_k (logsumexp mode) or gamma_k
  double alpha[kMaxR];
  double beta[kMaxR];
  double bnorm2[kMaxR];
  double true_rel[kMaxR];
  float inv_sqrt_g[kMaxR];   // 1/sqrt(gamma_k), scale of the appended basis pair
  float rel[kMaxR];          // recursive relative residual
  int active[kMaxR];
  int converged[kMaxR];
  int breakdown[kMaxR];
  int iters[kMaxR];
  int k;                     // iterations done
  int nactive;
  int nbasis;                // basis pairs stored
  int append_slot;           // slot the next direction kernel writes
};

struct Dims {
  int64_t n;
  int r;
  int rp2;                   // power of two >= r
  int grid;                  // blocks of the reductions
};
Dims make_dims(int64_t n, int r);

gp_status init_state(State* st, const float* B, int64_t n, int r, double* pd, hipStream_t s,
                     const Dims& dm);
gp_status init_residual(const float* B, const float* q, float* x, float* rr, bool x0_given,
                        const State* st, const Dims& dm, hipStream_t s);
gp_status dq_step(const float* d, const float* q, State* st, bool lse, float* pm, float* ps,
                  double* pd, const Dims& dm, hipStream_t s);
gp_status update_step(float* x, float* rr, const float* d, const float* q, const State* st,
                      const Dims& dm, hipStream_t s);
// pcoef holds max_basis * reorth_chunks(n) * kMaxR floats.
int reorth_chunks(int64_t n);
// jmax: an upper bound on the stored pairs (<= max_basis); only that many
// coefficient blocks per row chunk are launched.
gp_status reorth_pass(const float* U, const float* W, float* rr, State* st, float* pcoef,
                      float* coef, int max_basis, int jmax, const Dims& dm, hipStream_t s);
// Both CGS2 passes in one coefficient sweep and one update sweep through the
// basis Gram matrix; pgram is sized as pcoef, c1 and coef hold max_basis * kMaxR
// floats, gram max_basis^2 * r floats (written one column per call).
gp_status reorth_gram(const float* U, const float* W, float* rr, State* st, float* pcoef,
                      float* pgram, float* c1, float* gram, float* coef, int max_basis, int jmax,
                      const Dims& dm, hipStream_t s);
gp_status rz_step(const float* rr, const float* z, State* st, bool lse, bool init, double tol,
                  int min_iter, float* pm, float* ps, double* pd, float* history,
                  uint32_t* colmax, int rp, const Dims& dm, hipStream_t s);
gp_status direction_step(const float* z, float* d, const float* rr, float* U, float* W,
                         State* st, bool init, bool reorth, uint32_t* colmax, const Dims& dm,
                         hipStream_t s);
// true residual: res = b - (a2 * sum + s2 * x) from float64 partials; sets st->true_rel
gp_status true_residual_finish(const double* part, int nsplit, const float* B, const float* x,
                               float a2, float s2, State* st, double* pd, const Dims& dm,
                               hipStream_t s);
}  // namespace cg

// ---------------------------------------------------------------------------
// Pivoted-Cholesky preconditioner (a6, a9).
// ---------------------------------------------------------------------------
namespace pc {
constexpr int kMaxRank = 128;
}  // namespace pc

// ---------------------------------------------------------------------------
// Pseudo-loss gradient (Sec. 5.3, Eq. approx) and training step kernels.
// ---------------------------------------------------------------------------
namespace grad {
// Workspace bytes of launch() for a row range of `rows` rows, r columns.
size_t workspace_bytes(int64_t rows, int64_t n, int d, int r);
// out (device, L + 3 doubles): dL/dl.., dL/da^2, dL/ds^2, 1/2 y^T u_0 over
// rows [i0, i1); partial sums are carved from ar.
gp_status launch(const KParams& kp, bool ard, const float* X, int64_t n, const float* U,
                 const float* B, int r, int64_t i0, int64_t i1, double* out, Arena& ar,
                 hipStream_t s);
}  // namespace grad

namespace train {
constexpr int kMaxP = GP_TRAIN_MAX_PARAMS;
// Optimiser state, device resident.
struct DevState {
  double raw[kMaxP];
  double m[kMaxP];
  double v[kMaxP];
  double theta[kMaxP];
  double grad[kMaxP + 1];    // gradient estimate, then 1/2 y^T u_0
  double rgrad[kMaxP];       // objective gradient in raw values
  int step;
};
struct AdamOpts {
  double lr, beta1, beta2, eps;
  bool priors;
};
gp_status launch_rademacher(uint64_t seed, uint64_t first, int64_t rows, int cols, float* out,
                            int64_t ld, hipStream_t s);
// Adam on raw values from st->grad (nl lengthscales, then a^2 and s^2).
gp_status launch_adam(DevState* st, int nl, int64_t n, const AdamOpts& o, hipStream_t s);
// theta = constrained(raw).
gp_status launch_theta(DevState* st, int nl, hipStream_t s);
}  // namespace train

}  // namespace gpmi

// Opaque preconditioner handle of the C ABI.
struct gp_precond {
  int device;
  int64_t n;
  int d;
  int rank;              // rank actually built
  gpmi::KParams kp;
  double* L64;           // rank x n, column-major (each pivot column contiguous)
  float* L32;            // float32 copy for the apply
  double* Cinv;          // rank x rank, inverse of I + s^-2 L^T L
  int64_t* piv_dev;
  int64_t* piv_host;
  double trace_residual;
  double* scratch;       // apply partials
  float* Y32;            // rank x 64
  void* block;           // one device block holding the buffers above
  size_t block_bytes;
};

namespace gpmi {
namespace pc {
// z = P^{-1} r for an n x r block (r <= 64), on stream s; live as for the MVM.
gp_status apply(const gp_precond* P, const float* rr, float* z, const cg::Dims& dm,
                const int* live, hipStream_t s);
}  // namespace pc
}  // namespace gpmi
