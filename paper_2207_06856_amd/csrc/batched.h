// Batched solve of many independent GP problems (uneven n, d, r, kernel and
// hyperparameters) with one launch per step for the whole batch.
#pragma once

#include "internal.h"

namespace gpmi {
namespace bt {

constexpr int kChunkRows = 512;    // rows per reduction / elementwise chunk
constexpr int kJGroup = 8;         // basis vectors per re-orthogonalisation work group

// One problem, device resident.
struct Seg {
  const float* X;
  const float* B;
  float* U;
  int64_t n;
  int64_t vec_off;     // element offset of the n x r block in the concatenated vectors
  int64_t rowp_off;    // row offset of the row-side operands (rows padded to 256)
  int64_t colp_off;    // row offset of the column-side operands (rows padded to 128)
  int64_t vt_off;      // half offset of the transposed binary16 right-hand sides
  int64_t part_off;    // float offset of the product partial sums
  int64_t basis_off;   // float offset of the re-orthogonalisation basis
  int64_t l_off;       // element offset of the pivoted-Cholesky factor (rank x n)
  int64_t cinv_off;    // element offset of C^{-1} (rank x rank)
  int64_t diag_off;    // element offset of the residual diagonal (n)
  int64_t part64_off;  // double offset of the true-residual partial sums
  int64_t n_pad_r, n_pad_c;
  int r, d, w, kc, kind, nsplit, nsplit64, rank, chunk0, nchunk;
  float a2, s2;
  float ls[kMaxDim];
};

// Row chunk of one problem (reductions and elementwise work).
struct Chunk {
  int p;
  int pad;
  int64_t i0, i1;
};

// Fused-product work item: (problem, row block, column split).
struct Item {
  int p;
  int split;
  int64_t rblk;
};

// Padded dimension of the true-residual items (rows per thread 4 up to 16).
__host__ __device__ inline int trueres_dm_of(int d) { return d <= 4 ? 4 : d <= 8 ? 8 : d <= 16 ? 16 : 32; }

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

// Device buffers and tables of one batched solve.
struct Dev {
  int nprob;
  int nchunks, nitems, nitems64, ntiles;
  int rb, rp, max_w, max_d, max_r, max_rank, max_basis;
  int64_t total_rows_r, total_rows_c, qtotal, l_total;
  double entries;            // sum of n_p^2 (logical entries per batched product)
  Seg* segs;
  Chunk* chunks;
  Item* items;
  Item* items64;
  int4* tiles;
  int64_t *rowstart, *colstart, *xr_off, *xc_off, *qstart;
  // vectors (concatenated n_p x r_p blocks)
  float *b, *x, *r, *z, *d, *q;
  float *Ub, *Wb;
  // product operands
  _Float16 *Xr, *Xc, *Vt;
  float* part;
  uint32_t* colmax;
  float *scale, *inv_scale;
  double* part64;
  // reductions
  float *pm, *ps;
  double* pq;
  float *pcoef, *coef;
  float* history;
  cg::State* st;
  int* live;
  // preconditioners
  double *L64, *C, *Cinv, *diag, *pv, *psum;
  int64_t* pi;
  int64_t* piv;
  float* L32;
  float* ltpart;
  float* Y32;
  PcState* pcs;
};

gp_status launch_prep(const Dev& D, int side, hipStream_t s);
gp_status launch_quant(const Dev& D, const float* V, int scale_mode, const int* live, hipStream_t s);
gp_status launch_colmax(const Dev& D, const float* V, hipStream_t s);
gp_status launch_product(const Dev& D, const float* V, float* out, const int* live, hipStream_t s);
gp_status launch_colred(const Dev& D, const float* A, const float* B, bool lse, bool with_q2,
                        hipStream_t s);
gp_status launch_init(const Dev& D, const float* B, const float* q, bool x0_given, hipStream_t s);
gp_status launch_init_residual(const Dev& D, const float* B, const float* q, float* X, float* R,
                               bool x0_given, hipStream_t s);
gp_status launch_dq(const Dev& D, bool lse, hipStream_t s);
gp_status launch_update(const Dev& D, float* X, hipStream_t s);
gp_status launch_reorth(const Dev& D, hipStream_t s);
gp_status launch_precond(const Dev& D, hipStream_t s);
gp_status launch_rz(const Dev& D, bool lse, bool init, double tol, int min_iter, hipStream_t s);
gp_status launch_direction(const Dev& D, bool init, bool reorth, hipStream_t s);
gp_status launch_true_residual(const Dev& D, hipStream_t s);
gp_status launch_pivchol(const Dev& D, hipStream_t s);
// which = 0: B -> dst, 1: U -> dst
gp_status launch_gather(const Dev& D, int which, float* dst, hipStream_t s);
gp_status launch_scatter(const Dev& D, const float* src, hipStream_t s);

}  // namespace bt
}  // namespace gpmi
