// Predictive means with a cached solve (Sec. 4.1, the predictive-mean
// experiment: the weights v = K~^{-1} y are solved for once, after which every
// mean is the product K(x*, X) v): gp_model_create solves once and keeps X and
// v on the device; gp_model_predict is one kernel-matrix product against that
// cache, plain or over the finite binary16 support (gp_kmvm_truncated).

#include <math.h>
#include <string.h>

#include <algorithm>

#include "internal.h"

struct gp_model {
  int device = 0;
  gp_kernel k{};
  float ls[gpmi::kMaxDim];
  int64_t n = 0;
  int d = 0;
  float* X = nullptr;      // n x d
  float* v = nullptr;      // n: (a^2 K + s^2 I)^{-1} y
  gp_model_info info{};
};

using namespace gpmi;

namespace {
void release(gp_model* m) {
  if (!m) return;
  if (m->X) (void)hipFree(m->X);
  if (m->v) (void)hipFree(m->v);
  delete m;
}
}  // namespace

extern "C" void gp_model_default_opts(gp_cg_opts* o) {
  if (!o) return;
  gp_cg_default_opts(o);
  o->tol = 1e-2;
  o->max_iter = 1000;
  o->true_res_every = 0;
}

extern "C" gp_status gp_model_create(const gp_kernel* k, const float* X, int64_t n, int32_t d,
                                     const float* y, const gp_cg_opts* o_in, int32_t precond_rank,
                                     void* stream, gp_model** out) {
  clear_error();
  if (!out) return set_error(GP_ERR_ARG, "out is NULL");
  *out = nullptr;
  KParams kp;
  GP_TRY(check_kernel(k, d, true, &kp));
  if (n < 1) return set_error(GP_ERR_ARG, "n must be >= 1");
  if (!X || !y) return set_error(GP_ERR_ARG, "X and y must be non-NULL");
  if (precond_rank < 0 || precond_rank > pc::kMaxRank || precond_rank > n)
    return set_error(GP_ERR_ARG, "precond_rank outside [0, min(n, 128)]");
  gp_cg_opts o;
  if (o_in)
    o = *o_in;
  else
    gp_model_default_opts(&o);
  if (o.P) return set_error(GP_ERR_ARG, "the model builds its own preconditioner; opts.P must be NULL");
  if (o.x0_given) return set_error(GP_ERR_ARG, "opts.x0_given must be 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  gp_model* m = new gp_model();
  GP_HIP(hipGetDevice(&m->device));
  m->n = n;
  m->d = d;
  m->k = *k;
  const int nl = k->ard ? d : 1;
  for (int i = 0; i < nl; ++i) m->ls[i] = k->lengthscale[i];
  m->k.lengthscale = m->ls;
  if (hipMalloc(&m->X, 4 * (size_t)n * d) != hipSuccess || hipMalloc(&m->v, 4 * (size_t)n) != hipSuccess) {
    (void)hipGetLastError();
    release(m);
    return set_error(GP_ERR_NOMEM, "cannot allocate the model's arrays");
  }
  gp_status st = GP_OK;
  if (hipMemcpyAsync(m->X, X, 4 * (size_t)n * d, hipMemcpyDeviceToDevice, s) != hipSuccess)
    st = set_error(GP_ERR_HIP, "copying X failed");
  gp_precond* P = nullptr;
  if (st == GP_OK && precond_rank > 0) st = gp_pivchol_precond(&m->k, m->X, n, d, precond_rank, &P, s);
  int32_t iters = 0;
  float rel = 0.0f;
  double trel = 0.0;
  int8_t conv = 0, brk = 0;
  gp_cg_stats cs{};
  cs.iters = &iters;
  cs.rel_res = &rel;
  cs.true_rel_res = &trel;
  cs.converged = &conv;
  cs.breakdown = &brk;
  if (st == GP_OK) {
    o.P = P;
    st = gp_cg_solve(&m->k, m->X, n, d, y, 1, m->v, &o, &cs, s);
  }
  if (P) (void)gp_precond_destroy(P);
  if (st != GP_OK) {
    release(m);
    return st;
  }
  m->info.n = n;
  m->info.d = d;
  m->info.iters = iters;
  m->info.converged = conv;
  m->info.rel_res = rel;
  m->info.true_rel_res = trel;
  *out = m;
  return GP_OK;
}

extern "C" gp_status gp_model_predict(const gp_model* m, const float* Xs, int64_t ns, float* mu,
                                      int32_t precision, int32_t truncate, void* stream) {
  clear_error();
  if (!m) return set_error(GP_ERR_ARG, "model is NULL");
  if (ns < 0) return set_error(GP_ERR_ARG, "ns must be >= 0");
  if (ns > 0 && (!Xs || !mu)) return set_error(GP_ERR_ARG, "Xs and mu must be non-NULL");
  if (truncate != 0 && truncate != 1) return set_error(GP_ERR_ARG, "truncate must be 0 or 1");
  if (truncate && precision != GP_PREC_FP16)
    return set_error(GP_ERR_ARG, "truncation is a property of the binary16 product (precision FP16)");
  if (truncate)
    return gp_kmvm_truncated(&m->k, Xs, ns, m->X, m->n, m->d, m->v, 1, mu, 0, 1, nullptr, stream);
  return gp_kmvm(&m->k, Xs, ns, m->X, m->n, m->d, m->v, 1, mu, 0, precision, 0, stream);
}

extern "C" gp_status gp_model_info_read(const gp_model* m, gp_model_info* out) {
  clear_error();
  if (!m || !out) return set_error(GP_ERR_ARG, "model and out must be non-NULL");
  *out = m->info;
  return GP_OK;
}

extern "C" gp_status gp_model_weights(const gp_model* m, float* v_out, void* stream) {
  clear_error();
  if (!m || !v_out) return set_error(GP_ERR_ARG, "model and v_out must be non-NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  GP_HIP(hipMemcpyAsync(v_out, m->v, 4 * (size_t)m->n, hipMemcpyDeviceToDevice, s));
  return GP_OK;
}

extern "C" int32_t gp_model_device(const gp_model* m) { return m ? m->device : -1; }

extern "C" gp_status gp_model_destroy(gp_model* m) {
  clear_error();
  if (!m) return GP_OK;
  (void)hipDeviceSynchronize();
  release(m);
  return GP_OK;
}
