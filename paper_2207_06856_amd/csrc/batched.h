// Many independent GP problems (uneven n, d, r, kernel and hyperparameters)
// advanced together, one launch per step for a whole set of problems.
//
// Every problem owns one contiguous device region (its "slot region") that
// holds all of its vectors, binary16 operands, partial sums, basis and
// preconditioner; the problem's Seg record carries pointers into it.  The
// per-problem scalar state lives in slot-indexed arrays (Dev).  A launch set
// (Tab) names some slots plus their row chunks and work items; kernels only
// touch the problems of the set they are launched with.  Both the one-shot
// batched solve and the serving loop drive the same kernels through these
// three structures.
#pragma once

#include <vector>

#include "internal.h"

namespace gpmi {
namespace bt {

constexpr int kChunkRows = 512;    // rows per reduction / elementwise chunk
constexpr int kJGroup = 8;         // basis vectors per re-orthogonalisation work group

// vector selectors (Seg::v)
enum : int { VB = 0, VX = 1, VR = 2, VZ = 3, VD = 4, VQ = 5, kNumVec = 6 };

// One problem, device resident.  All arrays are row-major; "n x r" vectors
// have the r columns of one row adjacent.
struct Seg {
  const float* X;        // n x d points
  float* v[kNumVec];     // n x r: b (read only), x, r, z, d, q
  float* Ub;             // (max_iter + 1) x n x r re-orthogonalisation basis (r / sqrt(gamma))
  float* Wb;             // same for z / sqrt(gamma); NULL without preconditioner
  _Float16* Xr;          // n_pad_r x w augmented row operands
  _Float16* Xc;          // n_pad_c x w augmented column operands
  _Float16* Vt;          // rp x n_pad_c scaled binary16 right-hand sides (column major)
  float* part;           // nsplit x n_pad_r x rp product partial sums
  double* part64;        // nsplit64 x n x r true-residual partial sums
  double* L64;           // rank x n pivoted-Cholesky factor
  float* L32;            // rank x n binary32 copy
  double* C;             // rank x rank I + s^-2 L^T L, then its Cholesky factor
  double* Cinv;          // rank x rank inverse of I + s^-2 L^T L
  double* diag;          // n residual diagonal of the factorisation
  int64_t* piv;          // rank pivots
  double* T64;           // rank x r L^T w
  float* Y32;            // rank x r C^-1 L^T w
  float* coef;           // (max_iter + 1) x r re-orthogonalisation coefficients
  float* pm;             // nchunk x r chunk partials (LSE maximum or dot)
  float* ps;             // nchunk x r (LSE scaled sum)
  double* pq;            // nchunk x r (sum of squares)
  float* pcoef;          // nchunk x (max_iter + 1) x r
  float* pgram;          // nchunk x (max_iter + 1) x r: chunk partials of w_j^T u_new
  float* c1;             // (max_iter + 1) x r first-pass coefficients
  float* gram;           // (max_iter + 1)^2 x r basis Gram matrix w_j^T u_k
  float* ltpart;         // nchunk x rank x r
  double* pv;            // nchunk argmax value
  double* psum;          // nchunk diagonal sum
  int64_t* pi;           // nchunk argmax index
  int64_t n, n_pad_r, n_pad_c;
  double tol;
  int r, rb, rp, d, w, kc, kind, nsplit, nsplit64, rank, nchunk, max_iter, min_iter;
  float a2, s2;
  float ls[kMaxDim];
};

// Row chunk of one problem (reductions and elementwise work); k = chunk index
// within the problem.
struct Chunk {
  int p;
  int k;
  int64_t i0, i1;
};

// Fused-product work item: (problem, row block, column split).
struct Item {
  int p;
  int split;
  int64_t rblk;
};

// Padded point dimension of the true-residual items (4, 8, 16 or 32).
// slices of 4 augmented coordinates of the true-residual product: d + 2
// padded to 4T (batched and served problems have d <= 30, so T <= 8)
__host__ __device__ inline int trueres_slices_of(int d) { return (d + 2 + 3) / 4; }

// Per-problem pivoted-Cholesky build state.
struct PcState {
  double dmax;
  int64_t pivot;
  int rank;
  int stop;
  double trace;
  int not_pd;
  int pad;
};

// Slot-indexed device arrays.
struct Dev {
  int nslots;
  Seg* segs;             // nslots
  cg::State* st;         // nslots
  int* live;             // nslots: number of active columns (0 = nothing to do)
  uint32_t* colmax;      // nslots x kMaxR
  float* scale;          // nslots x kMaxR
  float* inv_scale;      // nslots x kMaxR
  PcState* pcs;          // nslots
  int* counter;          // work counter of the persistent product launch
  bool persistent;       // product as one persistent launch pulling items (else one group per item)
};

// A launch set.
struct Tab {
  int nsel = 0;
  const int* plist = nullptr;      // nsel slots
  int nchunks = 0;
  const Chunk* chunks = nullptr;
  int nitems = 0;
  const Item* items = nullptr;     // longest first
  int nitems64 = 0;
  const Item* items64 = nullptr;
  int ntiles = 0;
  const int4* tiles = nullptr;     // (slot, tile row, tile col, -) of I + s^-2 L^T L
  int rb = 1;                      // largest rb of the set
  int max_rank = 0, max_r = 1, max_basis = 1;
  double entries = 0.0;            // sum of n^2 (logical entries per product)
};

// ---- host side: slot regions and launch sets ---------------------------------------
struct SlotSpec {
  KParams kp;
  int64_t n = 0;
  int d = 0, r = 0, rank = 0, max_iter = 0, min_iter = 0;
  double tol = 0.0;
  bool reorth = true;
  bool own_io = false;   // the region also holds X, b and x (serving); else caller arrays
};

size_t slot_bytes(const SlotSpec& q);
// Lay out a region of slot_bytes(q) bytes at base (256-byte aligned) into g.
void slot_carve(const SlotSpec& q, void* base, Seg* g);

struct HostTab {
  std::vector<int> plist;
  std::vector<Chunk> chunks;
  std::vector<Item> items, items64;
  std::vector<int4> tiles;
  int rb = 1, max_rank = 0, max_r = 1, max_basis = 1;
  double entries = 0.0;
};
void build_tab(const std::vector<Seg>& segs, const std::vector<int>& plist, HostTab* t);
size_t tab_bytes(const HostTab& t);
// Copy the tables into dev (tab_bytes(t) bytes, 256-byte aligned) and fill *out.
gp_status tab_upload(const HostTab& t, void* dev, Tab* out, hipStream_t s);

// ---- device sequences (every call enqueues on s) ---------------------------------
struct RunOpts {
  bool lse = true;
  bool reorth = true;
  int scale_mode = 0;
};
// Operands, preconditioner build (PcState written; ranks may stop early).
gp_status seq_prepare(const Dev& D, const Tab& T, hipStream_t s);
// State and first direction; x0_given: the x vectors hold the initial guess.
gp_status seq_start(const Dev& D, const Tab& T, const RunOpts& o, bool x0_given, hipStream_t s);
// One iteration of every live problem of T.
gp_status seq_iteration(const Dev& D, const Tab& T, const RunOpts& o, hipStream_t s);
// ||b - K~ x|| / ||b|| per column in float64 (State::true_rel).
gp_status seq_true_residual(const Dev& D, const Tab& T, hipStream_t s);

}  // namespace bt
}  // namespace gpmi
