// Hyperparameter training behind the C ABI: the gradient estimate of
// Sec. 5.3 (Eq. approx) and the Adam loop of App. C.
//
// One training step = probes drawn on the device, pivoted-Cholesky
// preconditioner for the current hyperparameters, one mBCG solve of
// K~ U = [y, z_1..z_M] (Eq. cg), the fused gradient reduction, and the Adam
// update on the device.  The host only orders the calls and reads back the
// few scalars of the optimiser state after each step.

#include <math.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "internal.h"

using namespace gpmi;

namespace {

int nlen(int d, int ard) { return ard ? d : 1; }

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

gp_status check_grad_args(const gp_kernel* k, int64_t n, int32_t d, const float* X,
                          const float* B, const float* U, int32_t r, KParams* kp) {
  GP_TRY(check_kernel(k, d, false, kp));
  if (d > GP_TRAIN_MAX_DIM) return set_error(GP_ERR_ARG, "d=%d above %d", d, GP_TRAIN_MAX_DIM);
  if (n < 1) return set_error(GP_ERR_ARG, "n must be >= 1");
  if (r < 2 || r > cg::kMaxR) return set_error(GP_ERR_ARG, "r=%d outside [2, 64]", r);
  if (!X || !B || !U) return set_error(GP_ERR_ARG, "X, B and U must be non-NULL");
  return GP_OK;
}

}  // namespace

extern "C" gp_status gp_mll_grad(const gp_kernel* k, const float* X, int64_t n, int32_t d,
                                 const float* B, const float* U, int32_t r, int64_t row_begin,
                                 int64_t row_end, double* grad, void* stream) {
  clear_error();
  KParams kp;
  GP_TRY(check_grad_args(k, n, d, X, B, U, r, &kp));
  if (!grad) return set_error(GP_ERR_ARG, "grad is NULL");
  if (row_begin < 0 || row_end < row_begin || row_end > n)
    return set_error(GP_ERR_ARG, "row range [%lld, %lld) outside [0, %lld]", (long long)row_begin,
                     (long long)row_end, (long long)n);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nl = nlen(d, k->ard);
  Arena ar;
  GP_TRY(workspace_get(s, grad::workspace_bytes(row_end - row_begin, n, d, r) + 8 * (nl + 3) + 256, &ar));
  double* out = ar.take<double>(nl + 3);
  if (!out) return set_error(GP_ERR_NOMEM, "internal: gradient workspace sizing");
  GP_TRY(grad::launch(kp, k->ard != 0, X, n, U, B, r, row_begin, row_end, out, ar, s));
  GP_HIP(hipMemcpyAsync(grad, out, 8 * (size_t)(nl + 3), hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));
  return GP_OK;
}

extern "C" gp_status gp_rademacher(uint64_t seed, uint64_t first, int64_t rows, int32_t cols,
                                   float* out, int64_t ld, void* stream) {
  clear_error();
  if (rows < 0 || cols < 1 || ld < cols) return set_error(GP_ERR_ARG, "need rows >= 0, 1 <= cols <= ld");
  if (rows > 0 && !out) return set_error(GP_ERR_ARG, "out is NULL");
  return train::launch_rademacher(seed, first, rows, cols, out, ld, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------
// Trainer
// ---------------------------------------------------------------------------
struct gp_trainer {
  gp_train_config c;
  hipStream_t s = nullptr;
  int device = 0;
  int64_t n = 0;
  int d = 0, nl = 0, r = 0;
  float* X = nullptr;                 // n x d
  float* B = nullptr;                 // n x r: [y, probes]
  float* U = nullptr;                 // n x r
  train::DevState* st = nullptr;
  train::DevState host{};             // mirror after the last sync
  bool stepped = false;
};

extern "C" void gp_train_default_config(gp_train_config* c) {
  if (!c) return;
  *c = gp_train_config{};
  c->kind = GP_KERNEL_RBF;
  c->ard = 1;
  c->probes = 15;
  c->precond_rank = 100;
  c->use_priors = 1;
  c->lr = 0.1;
  c->beta1 = 0.9;
  c->beta2 = 0.999;
  c->eps = 1e-8;
  c->seed = 0;
  gp_cg_default_opts(&c->cg);
  c->cg.max_iter = 50;
  c->cg.min_iter = 10;
  c->cg.tol = 1.0;
  c->cg.true_res_every = -1;
}

static void release(gp_trainer* t) {
  if (!t) return;
  if (t->X) (void)hipFree(t->X);
  if (t->B) (void)hipFree(t->B);
  if (t->U) (void)hipFree(t->U);
  if (t->st) (void)hipFree(t->st);
  delete t;
}

static gp_status sync_state(gp_trainer* t) {
  GP_HIP(hipMemcpyAsync(&t->host, t->st, sizeof(train::DevState), hipMemcpyDeviceToHost, t->s));
  GP_HIP(hipStreamSynchronize(t->s));
  return GP_OK;
}

extern "C" gp_status gp_trainer_create(const gp_train_config* c, const float* X, const float* y,
                                       int64_t n, int32_t d, const double* theta0, void* stream,
                                       gp_trainer** out) {
  clear_error();
  if (!c || !out) return set_error(GP_ERR_ARG, "config and out must be non-NULL");
  *out = nullptr;
  if (c->kind < GP_KERNEL_RBF || c->kind > GP_KERNEL_MATERN32)
    return set_error(GP_ERR_ARG, "unknown kernel kind %d", c->kind);
  if (d < 1 || d > GP_TRAIN_MAX_DIM) return set_error(GP_ERR_ARG, "d=%d outside [1, %d]", d, GP_TRAIN_MAX_DIM);
  if (n < 1) return set_error(GP_ERR_ARG, "n must be >= 1");
  if (!X || !y) return set_error(GP_ERR_ARG, "X and y must be non-NULL");
  if (c->probes < 1 || c->probes > cg::kMaxR - 1) return set_error(GP_ERR_ARG, "probes=%d outside [1, 63]", c->probes);
  if (c->precond_rank < 0 || c->precond_rank > pc::kMaxRank || c->precond_rank > n)
    return set_error(GP_ERR_ARG, "precond_rank outside [0, min(n, 128)]");
  if (!(c->lr > 0.0) || !(c->beta1 >= 0.0 && c->beta1 < 1.0) || !(c->beta2 >= 0.0 && c->beta2 < 1.0) ||
      !(c->eps >= 0.0))
    return set_error(GP_ERR_ARG, "Adam settings need lr > 0, 0 <= beta < 1, eps >= 0");
  const int nl = nlen(d, c->ard);
  double th[GP_TRAIN_MAX_PARAMS];
  for (int p = 0; p < nl + 2; ++p) th[p] = theta0 ? theta0[p] : (p == nl + 1 ? 2.0 : log(2.0));
  for (int p = 0; p < nl + 2; ++p) {
    const double lo = p == nl + 1 ? 1e-4 : 0.0;
    if (!(isfinite(th[p]) && th[p] > lo))
      return set_error(GP_ERR_ARG, "theta0[%d] must be finite and > %g", p, lo);
  }
  gp_trainer* t = new gp_trainer();
  t->c = *c;
  t->s = static_cast<hipStream_t>(stream);
  t->n = n;
  t->d = d;
  t->nl = nl;
  t->r = c->probes + 1;
  auto fail = [&](gp_status st) {
    release(t);
    return st;
  };
  if (hipGetDevice(&t->device) != hipSuccess) return fail(set_error(GP_ERR_HIP, "hipGetDevice failed"));
  const size_t xb = 4 * (size_t)n * d, vb = 4 * (size_t)n * t->r;
  if (hipMalloc(&t->X, xb) != hipSuccess || hipMalloc(&t->B, vb) != hipSuccess ||
      hipMalloc(&t->U, vb) != hipSuccess || hipMalloc(&t->st, sizeof(train::DevState)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(set_error(GP_ERR_NOMEM, "cannot allocate the trainer's device arrays"));
  }
  train::DevState h{};
  for (int p = 0; p < nl + 2; ++p) {
    const double v = th[p] - (p == nl + 1 ? 1e-4 : 0.0);
    h.raw[p] = v + log(-expm1(-v));   // softplus^-1
  }
  if (hipMemcpyAsync(t->X, X, xb, hipMemcpyDeviceToDevice, t->s) != hipSuccess ||
      hipMemcpy2DAsync(t->B, 4 * (size_t)t->r, y, 4, 4, (size_t)n, hipMemcpyDeviceToDevice, t->s) != hipSuccess ||
      hipMemcpyAsync(t->st, &h, sizeof h, hipMemcpyHostToDevice, t->s) != hipSuccess)
    return fail(set_error(GP_ERR_HIP, "copying the training data failed"));
  gp_status st = train::launch_theta(t->st, nl, t->s);
  if (st == GP_OK) st = sync_state(t);
  if (st != GP_OK) return fail(st);
  *out = t;
  return GP_OK;
}

extern "C" gp_status gp_trainer_step(gp_trainer* t, gp_train_step_info* info) {
  clear_error();
  if (!t) return set_error(GP_ERR_ARG, "trainer is NULL");
  const int nl = t->nl, r = t->r, M = t->c.probes;
  const double t0 = now_s();
  // probes of this step: counter block (step * n + i) * M + c
  GP_TRY(train::launch_rademacher(t->c.seed, (uint64_t)t->host.step * (uint64_t)t->n * (uint64_t)M,
                                  t->n, M, t->B + 1, r, t->s));
  float ls[GP_TRAIN_MAX_DIM];
  for (int m = 0; m < nl; ++m) ls[m] = (float)t->host.theta[m];
  gp_kernel k{t->c.kind, t->c.ard, ls, (float)t->host.theta[nl], (float)t->host.theta[nl + 1]};
  gp_precond* P = nullptr;
  int rank_used = 0;
  if (t->c.precond_rank > 0) {
    GP_TRY(gp_pivchol_precond(&k, t->X, t->n, t->d, t->c.precond_rank, &P, t->s));
    (void)gp_precond_info(P, &rank_used, nullptr, nullptr);
  }
  const double t1 = now_s();
  gp_cg_opts o = t->c.cg;
  o.P = P;
  o.x0_given = 0;
  std::vector<int32_t> iters(r);
  std::vector<float> rel(r);
  std::vector<int8_t> conv(r);
  gp_cg_stats cs{};
  cs.iters = iters.data();
  cs.rel_res = rel.data();
  cs.converged = conv.data();
  gp_status st = gp_cg_solve(&k, t->X, t->n, t->d, t->B, r, t->U, &o, &cs, t->s);
  if (P) (void)gp_precond_destroy(P);
  if (st != GP_OK) return st;
  const double t2 = now_s();
  KParams kp;
  GP_TRY(check_kernel(&k, t->d, false, &kp));
  Arena ar;
  GP_TRY(workspace_get(t->s, grad::workspace_bytes(t->n, t->n, t->d, r), &ar));
  GP_TRY(grad::launch(kp, t->c.ard != 0, t->X, t->n, t->U, t->B, r, 0, t->n, t->st->grad, ar, t->s));
  const train::DevState before = t->host;
  GP_TRY(train::launch_adam(t->st, nl, t->n, train::AdamOpts{t->c.lr, t->c.beta1, t->c.beta2, t->c.eps, t->c.use_priors != 0}, t->s));
  GP_TRY(sync_state(t));
  const double t3 = now_s();
  t->stepped = true;
  if (info) {
    *info = gp_train_step_info{};
    info->step = t->host.step;
    info->cg_iters = cs.total_iters;
    int nc = 0;
    double mr = 0.0;
    for (int c = 0; c < r; ++c) {
      nc += conv[c] != 0;
      mr = std::max(mr, (double)rel[c]);
    }
    info->cg_converged = nc;
    info->precond_rank = rank_used;
    info->max_rel_res = mr;
    for (int p = 0; p < nl + 2; ++p) {
      info->theta[p] = before.theta[p];
      info->grad[p] = t->host.grad[p];
      info->raw_grad[p] = t->host.rgrad[p];
      info->theta_next[p] = t->host.theta[p];
    }
    info->data_fit = t->host.grad[nl + 2];
    info->seconds_precond = t1 - t0;
    info->seconds_solve = t2 - t1;
    info->seconds_grad = t3 - t2;
  }
  return GP_OK;
}

extern "C" gp_status gp_trainer_get_state(gp_trainer* t, gp_train_state* out) {
  clear_error();
  if (!t || !out) return set_error(GP_ERR_ARG, "trainer and out must be non-NULL");
  *out = gp_train_state{};
  out->nparams = t->nl + 2;
  out->step = t->host.step;
  for (int p = 0; p < t->nl + 2; ++p) {
    out->raw[p] = t->host.raw[p];
    out->m[p] = t->host.m[p];
    out->v[p] = t->host.v[p];
    out->theta[p] = t->host.theta[p];
  }
  return GP_OK;
}

extern "C" gp_status gp_trainer_set_state(gp_trainer* t, const gp_train_state* in) {
  clear_error();
  if (!t || !in) return set_error(GP_ERR_ARG, "trainer and state must be non-NULL");
  if (in->nparams != t->nl + 2) return set_error(GP_ERR_ARG, "nparams=%d, trainer has %d", in->nparams, t->nl + 2);
  if (in->step < 0) return set_error(GP_ERR_ARG, "step must be >= 0");
  for (int p = 0; p < t->nl + 2; ++p)
    if (!isfinite(in->raw[p]) || !isfinite(in->m[p]) || !(in->v[p] >= 0.0) || !isfinite(in->v[p]))
      return set_error(GP_ERR_ARG, "state entry %d is not finite (or v < 0)", p);
  train::DevState h = t->host;
  h.step = in->step;
  for (int p = 0; p < t->nl + 2; ++p) {
    h.raw[p] = in->raw[p];
    h.m[p] = in->m[p];
    h.v[p] = in->v[p];
  }
  GP_HIP(hipMemcpyAsync(t->st, &h, sizeof h, hipMemcpyHostToDevice, t->s));
  GP_TRY(train::launch_theta(t->st, t->nl, t->s));
  return sync_state(t);
}

extern "C" gp_status gp_trainer_blocks(gp_trainer* t, float* B_out, float* U_out) {
  clear_error();
  if (!t) return set_error(GP_ERR_ARG, "trainer is NULL");
  if (!t->stepped) return set_error(GP_ERR_ARG, "no step has been taken");
  const size_t vb = 4 * (size_t)t->n * t->r;
  if (B_out) GP_HIP(hipMemcpyAsync(B_out, t->B, vb, hipMemcpyDeviceToDevice, t->s));
  if (U_out) GP_HIP(hipMemcpyAsync(U_out, t->U, vb, hipMemcpyDeviceToDevice, t->s));
  GP_HIP(hipStreamSynchronize(t->s));
  return GP_OK;
}

extern "C" gp_status gp_trainer_destroy(gp_trainer* t) {
  clear_error();
  if (!t) return GP_OK;
  (void)hipStreamSynchronize(t->s);
  release(t);
  return GP_OK;
}
