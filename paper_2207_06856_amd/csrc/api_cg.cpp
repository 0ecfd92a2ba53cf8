// gp_cg_solve: host driver of the batched conjugate-gradients solve.
//
// Everything between polls runs on the device: the host enqueues
// `poll_every` iterations of
//   K d -> alpha (a3) -> x, r update (a4) -> re-orthogonalisation (a5, two
//   classical passes) -> z = P(r) (a6) -> gamma, beta, convergence (a7) ->
//   d = -z + beta d, basis append, binary16 requantisation of d (a7)
// and then reads back the number of active columns.  Kernels of an iteration
// enqueued after every column froze return immediately, so overshooting the
// last poll costs only launch latency.

#include <math.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace gpmi {

namespace {
__global__ void zero_words_kernel(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

gp_status zero_words(void* p, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n == 0) return GP_OK;
  zero_words_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(static_cast<uint32_t*>(p), n);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

struct Plan {
  // problem
  KParams kp;
  const float* X;
  const float* B;
  float* U;
  int64_t n;
  int r;
  gp_cg_opts o;
  bool lse, reorth, fp16, bf16;   // fp16: a 16-bit matrix-core product; bf16: its format
  bool sym;                       // binary16 product in its symmetric form (kmvm_sym.hip)
  f16::SymPlan sp;
  cg::Dims dm;
  // 16-bit product (binary16, or bfloat16 in the same buffers)
  int w, kc, rb, rp;
  int64_t n_pad;
  int nsplit16;
  // fp32 product
  int nsplit32;
  int nsplit64;
  int max_basis;
  // buffers
  float *rr, *z, *d, *q;
  float *Ub, *Wb;
  _Float16 *Xr, *Xc, *Vt;
  float* part16;
  uint32_t* colmax;
  float *scale, *inv_scale;
  float* part32;
  double* part64;
  float *pm, *ps;
  double* pd;
  float *pcoef, *coef, *pgram, *c1, *gram;
  float* history;
  cg::State* st;
};

size_t plan_bytes(Plan& p, bool want_history) {
  const int64_t n = p.n;
  const int r = p.r;
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~size_t(255); };
  add(4 * n * r);                              // rr
  if (p.o.P) add(4 * n * r);                   // z
  add(4 * n * r);                              // d
  add(4 * n * r);                              // q
  if (p.reorth) {
    add(4 * (size_t)p.max_basis * n * r);      // U basis
    if (p.o.P) add(4 * (size_t)p.max_basis * n * r);
  }
  if (p.fp16) {
    add(2 * (size_t)p.n_pad * p.w);
    add(2 * (size_t)p.n_pad * p.w);
    add(2 * (size_t)p.rp * p.n_pad);
    if (p.sym)
      b += f16::sym_bytes(p.sp);
    else
      add(4 * (size_t)p.nsplit16 * p.n_pad * p.rp);
    add(4 * 64);
    add(4 * 64);
  } else {
    add(4 * (size_t)p.nsplit32 * n * r);
  }
  add(4 * 64);                                 // column maxima of d
  if (p.o.true_res_every >= 0) add(8 * (size_t)p.nsplit64 * n * r);
  add(4 * cg::kMaxBlocks * cg::kMaxR);
  add(4 * cg::kMaxBlocks * cg::kMaxR);
  add(8 * cg::kMaxBlocks * cg::kMaxR);
  if (p.reorth) {
    add(4 * (size_t)cg::reorth_chunks(n) * p.max_basis * cg::kMaxR);    // pcoef
    add(4 * (size_t)cg::reorth_chunks(n) * p.max_basis * cg::kMaxR);    // pgram
    add(4 * (size_t)p.max_basis * cg::kMaxR);                           // coef
    add(4 * (size_t)p.max_basis * cg::kMaxR);                           // c1
    add(4 * (size_t)p.max_basis * p.max_basis * r);                     // gram
  }
  if (want_history) add(4 * (size_t)(p.o.max_iter + 1) * r);
  add(sizeof(cg::State));
  return b;
}

void plan_carve(Plan& p, Arena& a, bool want_history) {
  const int64_t n = p.n;
  const int r = p.r;
  p.rr = a.take<float>(n * r);
  p.z = p.o.P ? a.take<float>(n * r) : p.rr;
  p.d = a.take<float>(n * r);
  p.q = a.take<float>(n * r);
  p.Ub = p.Wb = nullptr;
  if (p.reorth) {
    p.Ub = a.take<float>((size_t)p.max_basis * n * r);
    p.Wb = p.o.P ? a.take<float>((size_t)p.max_basis * n * r) : nullptr;
  }
  if (p.fp16) {
    p.Xr = a.take<_Float16>((size_t)p.n_pad * p.w);
    p.Xc = a.take<_Float16>((size_t)p.n_pad * p.w);
    p.Vt = a.take<_Float16>((size_t)p.rp * p.n_pad);
    if (p.sym)
      p.part16 = f16::sym_carve(p.sp, a) == GP_OK ? p.sp.rowpart : nullptr;
    else
      p.part16 = a.take<float>((size_t)p.nsplit16 * p.n_pad * p.rp);
    p.scale = a.take<float>(64);
    p.inv_scale = a.take<float>(64);
  } else {
    p.part32 = a.take<float>((size_t)p.nsplit32 * n * r);
  }
  p.colmax = a.take<uint32_t>(64);
  p.part64 = p.o.true_res_every >= 0 ? a.take<double>((size_t)p.nsplit64 * n * r) : nullptr;
  p.pm = a.take<float>(cg::kMaxBlocks * cg::kMaxR);
  p.ps = a.take<float>(cg::kMaxBlocks * cg::kMaxR);
  p.pd = a.take<double>(cg::kMaxBlocks * cg::kMaxR);
  p.pcoef = p.coef = p.pgram = p.c1 = p.gram = nullptr;
  if (p.reorth) {
    p.pcoef = a.take<float>((size_t)cg::reorth_chunks(n) * p.max_basis * cg::kMaxR);
    p.pgram = a.take<float>((size_t)cg::reorth_chunks(n) * p.max_basis * cg::kMaxR);
    p.coef = a.take<float>((size_t)p.max_basis * cg::kMaxR);
    p.c1 = a.take<float>((size_t)p.max_basis * cg::kMaxR);
    p.gram = a.take<float>((size_t)p.max_basis * p.max_basis * r);
  }
  p.history = want_history ? a.take<float>((size_t)(p.o.max_iter + 1) * r) : nullptr;
  p.st = a.take<cg::State>(1);
}

// q = K~ v for the solve's precision; live gates the launches.
__bf16* as_bf16(_Float16* p) { return reinterpret_cast<__bf16*>(p); }

gp_status product(Plan& p, const float* v, float* out, const int* live, hipStream_t s) {
  if (p.sym) {
    GP_TRY(f16::sym_launch(p.kp.kind, p.sp, p.Xr, p.Xc, p.Vt, live, (double)p.n * (double)p.n, s));
    return f16::sym_reduce(p.sp, p.n, p.r, p.inv_scale, p.kp.a2, p.kp.s2, v, p.r, out, p.r, live,
                           s);
  }
  if (p.fp16) {
    if (p.bf16)
      GP_TRY(f16::launch_main_bf16(p.kp.kind, p.kc, p.rb, as_bf16(p.Xr), as_bf16(p.Xc),
                                   as_bf16(p.Vt), p.part16, p.n_pad, p.n_pad, p.nsplit16, live,
                                   (double)p.n * (double)p.n, s));
    else
      GP_TRY(f16::launch_main(p.kp.kind, p.kc, p.rb, p.Xr, p.Xc, p.Vt, p.part16, p.n_pad, p.n_pad,
                              p.nsplit16, live, (double)p.n * (double)p.n, s));
    return f16::launch_reduce(p.part16, p.nsplit16, p.n, p.n_pad, p.r, p.rp, p.inv_scale, p.kp.a2,
                              p.kp.s2, v, p.r, out, p.r, live, s);
  }
  GP_TRY(valu::launch_partial(p.kp, p.X, p.n, p.X, p.n, v, p.r, p.part32, false, p.nsplit32, live,
                              s));
  return valu::launch_reduce32(p.part32, p.nsplit32, p.n, p.r, p.kp.a2, p.kp.s2, v, out, live, s);
}

gp_status quantise(Plan& p, const float* v, bool pow2_from_colmax, const int* live, hipStream_t s) {
  if (!p.fp16) return GP_OK;
  if (p.bf16) {
    __bf16* Vt = as_bf16(p.Vt);
    if (p.o.scale_mode == 1)
      return f16::quant_rhs(v, p.n, p.r, p.r, p.rp, p.n_pad, 1, (float)(1.0 / sqrt((double)p.n)),
                            (float)sqrt((double)p.n), p.colmax, Vt, p.scale, p.inv_scale, s);
    if (pow2_from_colmax)
      return f16::quant_only(v, p.n, p.r, p.r, p.rp, p.n_pad, p.colmax, Vt, p.scale, p.inv_scale,
                             live, s);
    return f16::quant_rhs(v, p.n, p.r, p.r, p.rp, p.n_pad, 0, 1.0f, 1.0f, p.colmax, Vt, p.scale,
                          p.inv_scale, s);
  }
  const float fs = (float)(1.0 / sqrt((double)p.n));
  const float fi = (float)sqrt((double)p.n);
  if (p.o.scale_mode == 1)
    return f16::quant_rhs(v, p.n, p.r, p.r, p.rp, p.n_pad, 1, fs, fi, p.colmax, p.Vt, p.scale,
                          p.inv_scale, s);
  if (pow2_from_colmax)
    return f16::quant_only(v, p.n, p.r, p.r, p.rp, p.n_pad, p.colmax, p.Vt, p.scale, p.inv_scale,
                           live, s);
  return f16::quant_rhs(v, p.n, p.r, p.r, p.rp, p.n_pad, 0, fs, fi, p.colmax, p.Vt, p.scale,
                        p.inv_scale, s);
}

// it: 0-based iteration index (the basis holds at most it + 1 pairs).
gp_status iteration(Plan& p, int it, hipStream_t s) {
  const int* live = &p.st->nactive;
  GP_TRY(product(p, p.d, p.q, live, s));
  GP_TRY(cg::dq_step(p.d, p.q, p.st, p.lse, p.pm, p.ps, p.pd, p.dm, s));
  GP_TRY(cg::update_step(p.U, p.rr, p.d, p.q, p.st, p.dm, s));
  if (p.reorth) {
    const float* W = p.Wb ? p.Wb : p.Ub;
    GP_TRY(cg::reorth_gram(p.Ub, W, p.rr, p.st, p.pcoef, p.pgram, p.c1, p.gram, p.coef,
                           p.max_basis, it + 2, p.dm, s));
  }
  if (p.o.P) GP_TRY(pc::apply(p.o.P, p.rr, p.z, p.dm, live, s));
  GP_TRY(cg::rz_step(p.rr, p.z, p.st, p.lse, false, p.o.tol, p.o.min_iter, p.pm, p.ps, p.pd,
                     p.history, p.colmax, p.rp, p.dm, s));
  GP_TRY(cg::direction_step(p.z, p.d, p.rr, p.Ub, p.Wb, p.st, false, p.reorth, p.colmax, p.dm, s));
  return quantise(p, p.d, true, live, s);
}

gp_status true_residual(Plan& p, hipStream_t s) {
  GP_TRY(valu::launch_partial(p.kp, p.X, p.n, p.X, p.n, p.U, p.r, p.part64, true, p.nsplit64,
                              nullptr, s));
  return cg::true_residual_finish(p.part64, p.nsplit64, p.B, p.U, p.kp.a2, p.kp.s2, p.st, p.pd,
                                  p.dm, s);
}

}  // namespace
}  // namespace gpmi

using namespace gpmi;

extern "C" void gp_cg_default_opts(gp_cg_opts* o) {
  if (!o) return;
  *o = gp_cg_opts{};
  o->tol = 1.0;
  o->max_iter = 100;
  o->min_iter = 10;
  o->algo = GP_CG_ENHANCED;
  o->reorth = 1;
  o->use_lse = 1;
  o->precision = GP_PREC_FP16;
  o->scale_mode = 0;
  o->x0_given = 0;
  o->true_res_every = 0;
  o->poll_every = 10;
  o->P = nullptr;
}

extern "C" gp_status gp_cg_solve(const gp_kernel* k, const float* X, int64_t n, int32_t d,
                                 const float* B, int32_t r, float* U, const gp_cg_opts* o,
                                 gp_cg_stats* stats, void* stream) {
  clear_error();
  Plan p{};
  if (o)
    p.o = *o;
  else
    gp_cg_default_opts(&p.o);
  GP_TRY(check_kernel(k, d, true, &p.kp));
  if (n < 1) return set_error(GP_ERR_ARG, "n=%lld must be >= 1", (long long)n);
  if (r < 1 || r > cg::kMaxR) return set_error(GP_ERR_ARG, "r=%d outside [1, %d]", r, cg::kMaxR);
  if (!X || !B || !U) return set_error(GP_ERR_ARG, "X, B and U must be non-NULL");
  if (!(p.o.tol >= 0.0) || !isfinite(p.o.tol)) return set_error(GP_ERR_ARG, "tol must be finite, >= 0");
  if (p.o.max_iter < 0 || p.o.min_iter < 0) return set_error(GP_ERR_ARG, "negative iteration limit");
  if (p.o.algo != GP_CG_STANDARD && p.o.algo != GP_CG_ENHANCED)
    return set_error(GP_ERR_ARG, "algo must be GP_CG_STANDARD or GP_CG_ENHANCED");
  if (p.o.precision != GP_PREC_FP32 && p.o.precision != GP_PREC_FP16 &&
      p.o.precision != GP_PREC_BF16)
    return set_error(GP_ERR_ARG, "precision must be GP_PREC_FP32, GP_PREC_FP16 or GP_PREC_BF16");
  if (p.o.scale_mode != 0 && p.o.scale_mode != 1) return set_error(GP_ERR_ARG, "scale_mode must be 0 or 1");
  if (p.o.P && (p.o.P->n != n || p.o.P->d != d))
    return set_error(GP_ERR_ARG, "preconditioner was built for n=%lld d=%d",
                     (long long)p.o.P->n, p.o.P->d);
  const size_t vb = (size_t)n * r * 4;
  if (overlaps(U, vb, B, vb) || overlaps(U, vb, X, (size_t)n * d * 4))
    return set_error(GP_ERR_ARG, "U overlaps X or B");
  if (p.o.poll_every <= 0) p.o.poll_every = 10;

  hipStream_t s = static_cast<hipStream_t>(stream);
  p.X = X;
  p.B = B;
  p.U = U;
  p.n = n;
  p.r = r;
  const bool enhanced = p.o.algo == GP_CG_ENHANCED;
  p.lse = enhanced && p.o.use_lse;
  p.reorth = enhanced && p.o.reorth;
  p.fp16 = p.o.precision == GP_PREC_FP16 || p.o.precision == GP_PREC_BF16;
  p.bf16 = p.o.precision == GP_PREC_BF16;
  p.dm = cg::make_dims(n, r);
  p.max_basis = p.o.max_iter + 1;
  p.w = p.bf16 ? f16::aug_width_bf16(d) : f16::aug_width(d);
  p.kc = p.w / 32;
  p.rb = (int)ceil_div(r, 16);
  p.rp = 16 * p.rb;
  p.sym = p.fp16 && !p.bf16 && f16::sym_supported(d, r) && n >= f16::kSymMinN;
  p.n_pad = p.sym ? f16::sym_pad(n) : round_up(n, f16::kRowsPerBlock);
  if (p.sym) p.sp = f16::sym_plan(p.n_pad);
  p.nsplit16 = f16::choose_splits(p.n_pad, p.n_pad);
  p.nsplit32 = valu::choose_splits(n, n, d);
  p.nsplit64 = valu::choose_splits64(n, n, d);
  const bool want_history = stats && stats->history;

  Arena ar;
  gp_status wst = workspace_get(s, plan_bytes(p, want_history), &ar);
  if (wst == GP_ERR_NOMEM && p.sym) {
    // the symmetric product's partial sums (n^2 R 4 / (2 panel) bytes) do not
    // fit: the one-sided product's workspace is O(n)
    clear_error();
    p.sym = false;
    p.n_pad = round_up(n, f16::kRowsPerBlock);
    p.nsplit16 = f16::choose_splits(p.n_pad, p.n_pad);
    wst = workspace_get(s, plan_bytes(p, want_history), &ar);
  }
  GP_TRY(wst);
  plan_carve(p, ar, want_history);
  if (!p.st || (p.fp16 && !p.part16))
    return set_error(GP_ERR_NOMEM, "internal: solver workspace sizing");
  if (p.sym) GP_TRY(f16::sym_prepare(p.sp, s));
  uint32_t* cm = p.colmax;

  // ---- initialisation (Alg. 1/2 "Initialize") ----
  GP_TRY(zero_words(p.st, sizeof(cg::State), s));
  if (p.history) GP_TRY(fill_f32(p.history, (int64_t)(p.o.max_iter + 1) * r, -1.0f, s));
  GP_TRY(cg::init_state(p.st, B, n, r, p.pd, s, p.dm));
  int mvms = 0;
  if (p.bf16) {
    GP_TRY(f16::prep_points_bf16(X, n, p.n_pad, p.kp, 0, as_bf16(p.Xr), s));
    GP_TRY(f16::prep_points_bf16(X, n, p.n_pad, p.kp, 1, as_bf16(p.Xc), s));
  } else if (p.fp16) {
    GP_TRY(f16::prep_points(X, n, p.n_pad, p.kp, 0, p.Xr, s));
    GP_TRY(f16::prep_points(X, n, p.n_pad, p.kp, 1, p.Xc, s));
  }
  if (p.o.x0_given) {
    GP_TRY(quantise(p, U, false, nullptr, s));
    GP_TRY(product(p, U, p.q, nullptr, s));
    ++mvms;
  }
  GP_TRY(cg::init_residual(B, p.q, U, p.rr, p.o.x0_given != 0, p.st, p.dm, s));
  if (p.o.P) GP_TRY(pc::apply(p.o.P, p.rr, p.z, p.dm, nullptr, s));
  GP_TRY(cg::rz_step(p.rr, p.z, p.st, p.lse, true, p.o.tol, p.o.min_iter, p.pm, p.ps, p.pd,
                     p.history, cm, p.rp, p.dm, s));
  GP_TRY(cg::direction_step(p.z, p.d, p.rr, p.Ub, p.Wb, p.st, true, p.reorth, cm, p.dm, s));
  GP_TRY(quantise(p, p.d, true, &p.st->nactive, s));

  // ---- iterations ----
  cg::State hs;
  GP_HIP(hipMemcpyAsync(&hs, p.st, sizeof hs, hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));
  // periodic true residuals: row j after (j + 1) * every launched iterations
  const int every = p.o.true_res_every;
  const int trows = every > 0 ? p.o.max_iter / every : 0;
  std::vector<double> thist((size_t)trows * r, -1.0);
  auto record_true = [&](int launched_now) {
    if (every <= 0 || launched_now % every != 0) return;
    const int row = launched_now / every - 1;
    if (row < 0 || row >= trows) return;
    std::copy(hs.true_rel, hs.true_rel + r, thist.begin() + (size_t)row * r);
  };
  int launched = 0;
  while (launched < p.o.max_iter && hs.nactive > 0) {
    // a chunk ends at every multiple of true_res_every, so the periodic
    // residual is taken exactly every that many iterations
    int chunk = std::min(p.o.poll_every, p.o.max_iter - launched);
    if (every > 0) chunk = std::min(chunk, every - launched % every);
    for (int c = 0; c < chunk; ++c) GP_TRY(iteration(p, launched + c, s));
    launched += chunk;
    const bool periodic = every > 0 && launched % every == 0 && launched < p.o.max_iter;
    if (periodic) GP_TRY(true_residual(p, s));
    GP_HIP(hipMemcpyAsync(&hs, p.st, sizeof hs, hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    if (periodic) record_true(launched);
  }
  if (p.o.true_res_every >= 0) GP_TRY(true_residual(p, s));
  GP_HIP(hipMemcpyAsync(&hs, p.st, sizeof hs, hipMemcpyDeviceToHost, s));
  std::vector<float> hist;
  if (p.history) {
    hist.resize((size_t)(p.o.max_iter + 1) * r);
    GP_HIP(hipMemcpyAsync(hist.data(), p.history, hist.size() * 4, hipMemcpyDeviceToHost, s));
  }
  GP_HIP(hipStreamSynchronize(s));
  mvms += hs.k;
  if (p.o.true_res_every >= 0) record_true(launched);

  int broke = 0;
  for (int c = 0; c < r; ++c) broke += hs.breakdown[c];
  if (stats) {
    for (int c = 0; c < r; ++c) {
      if (stats->iters) stats->iters[c] = hs.iters[c];
      if (stats->rel_res) stats->rel_res[c] = hs.rel[c];
      if (stats->true_rel_res) stats->true_rel_res[c] = p.o.true_res_every >= 0 ? hs.true_rel[c] : -1.0;
      // convergence also requires the float64 true residual, when computed
      const bool true_ok = p.o.true_res_every < 0 || hs.true_rel[c] <= GP_TRUE_RES_SLACK * std::max(p.o.tol, GP_TRUE_RES_FLOOR);
      if (stats->converged) stats->converged[c] = (int8_t)(hs.converged[c] && true_ok);
      if (stats->breakdown) stats->breakdown[c] = (int8_t)hs.breakdown[c];
    }
    if (stats->history) std::copy(hist.begin(), hist.end(), stats->history);
    if (stats->true_history) std::copy(thist.begin(), thist.end(), stats->true_history);
    stats->total_iters = hs.k;
    stats->mvms = mvms;
  }
  if (broke == r) return set_error(GP_ERR_BREAKDOWN, "every column broke down");
  return GP_OK;
}
