// gp_cg_solve_batched: host driver of the batched solve.
//
// Every problem gets a slot region in one workspace; B and U stay in the
// caller's arrays (U is the iterate x).  The host builds one launch set for
// the whole batch, enqueues the preparation (operands and the pivoted-Cholesky
// builds, one launch pair per pivot step for all problems), the start, and
// the iterations.  The `poll_every` iterations between two polls of the
// per-problem activity flags are captured once into a HIP graph and replayed.

#include <math.h>

#include <algorithm>
#include <vector>

#include "batched.h"

using namespace gpmi;
using namespace gpmi::bt;

namespace {

// Slot-indexed arrays for nslots problems carved from an arena.
bool carve_dev(Arena& ar, int nslots, Dev* D) {
  D->nslots = nslots;
  D->segs = ar.take<Seg>(nslots);
  D->st = ar.take<cg::State>(nslots);
  D->live = ar.take<int>(nslots);
  D->colmax = ar.take<uint32_t>((size_t)nslots * cg::kMaxR);
  D->scale = ar.take<float>((size_t)nslots * cg::kMaxR);
  D->inv_scale = ar.take<float>((size_t)nslots * cg::kMaxR);
  D->pcs = ar.take<PcState>(nslots);
  D->counter = ar.take<int>(1);
  D->persistent = tune::bt_persistent();
  return D->counter != nullptr;
}

size_t dev_bytes(int nslots) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(sizeof(Seg) * nslots) + al(sizeof(cg::State) * nslots) + al(4 * (size_t)nslots) +
         3 * al(4 * (size_t)nslots * cg::kMaxR) + al(sizeof(PcState) * nslots) + al(sizeof(int));
}

}  // namespace

extern "C" gp_status gp_cg_solve_batched(int32_t nprob, const gp_problem* probs,
                                         const gp_cg_opts* o_in, gp_cg_stats* stats,
                                         void* stream) {
  clear_error();
  if (nprob < 1 || nprob > 4096) return set_error(GP_ERR_ARG, "nprob=%d outside [1, 4096]", nprob);
  if (!probs) return set_error(GP_ERR_ARG, "problems are NULL");
  gp_cg_opts o;
  if (o_in)
    o = *o_in;
  else
    gp_cg_default_opts(&o);
  if (o.precision != GP_PREC_FP16)
    return set_error(GP_ERR_ARG, "batched solves use the binary16 product (precision FP16)");
  if (o.P) return set_error(GP_ERR_ARG, "batched solves build per-problem preconditioners; P must be NULL");
  if (!(o.tol >= 0.0) || !isfinite(o.tol)) return set_error(GP_ERR_ARG, "tol must be finite, >= 0");
  if (o.max_iter < 0 || o.min_iter < 0) return set_error(GP_ERR_ARG, "negative iteration limit");
  if (o.algo != GP_CG_STANDARD && o.algo != GP_CG_ENHANCED)
    return set_error(GP_ERR_ARG, "algo must be GP_CG_STANDARD or GP_CG_ENHANCED");
  if (o.scale_mode != 0 && o.scale_mode != 1) return set_error(GP_ERR_ARG, "scale_mode must be 0 or 1");
  if (o.poll_every <= 0) o.poll_every = 10;
  const bool enhanced = o.algo == GP_CG_ENHANCED;
  RunOpts ro;
  ro.lse = enhanced && o.use_lse;
  ro.reorth = enhanced && o.reorth;
  ro.scale_mode = o.scale_mode;

  std::vector<SlotSpec> specs(nprob);
  std::vector<Seg> segs(nprob);
  size_t region_total = 0;
  std::vector<size_t> region_off(nprob);
  for (int p = 0; p < nprob; ++p) {
    const gp_problem& q = probs[p];
    SlotSpec& sp = specs[p];
    gp_status st = check_kernel(&q.k, q.d, true, &sp.kp);
    if (st != GP_OK) return set_error(st, "problem %d: %s", p, gp_last_error());
    if (q.d > 30) return set_error(GP_ERR_ARG, "problem %d: batched solves take d <= 30", p);
    if (q.n < 1) return set_error(GP_ERR_ARG, "problem %d: n must be >= 1", p);
    if (q.r < 1 || q.r > cg::kMaxR) return set_error(GP_ERR_ARG, "problem %d: r outside [1, 64]", p);
    if (!q.X || !q.B || !q.U) return set_error(GP_ERR_ARG, "problem %d: NULL array", p);
    if (q.precond_rank < 0 || q.precond_rank > pc::kMaxRank || q.precond_rank > q.n)
      return set_error(GP_ERR_ARG, "problem %d: precond_rank outside [0, min(n, 128)]", p);
    const size_t vb = (size_t)q.n * q.r * 4;
    if (overlaps(q.U, vb, q.B, vb) || overlaps(q.U, vb, q.X, (size_t)q.n * q.d * 4))
      return set_error(GP_ERR_ARG, "problem %d: U overlaps X or B", p);
    sp.n = q.n;
    sp.d = q.d;
    sp.r = q.r;
    sp.rank = q.precond_rank;
    sp.max_iter = o.max_iter;
    sp.min_iter = o.min_iter;
    sp.tol = o.tol;
    sp.reorth = ro.reorth;
    sp.own_io = false;
    region_off[p] = region_total;
    region_total += slot_bytes(sp);
    slot_carve(sp, nullptr, &segs[p]);   // sizes only, for the tables
  }
  std::vector<int> plist(nprob);
  for (int p = 0; p < nprob; ++p) plist[p] = p;
  HostTab ht;
  build_tab(segs, plist, &ht);

  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t tb = tab_bytes(ht);
  Arena ar;
  GP_TRY(workspace_get(s, dev_bytes(nprob) + tb + region_total + 256, &ar));
  Dev D{};
  if (!carve_dev(ar, nprob, &D)) return set_error(GP_ERR_NOMEM, "internal: batched workspace sizing");
  void* tabmem = ar.take<char>(tb);
  char* regions = ar.take<char>(region_total);
  if (!tabmem || !regions) return set_error(GP_ERR_NOMEM, "internal: batched workspace sizing");
  for (int p = 0; p < nprob; ++p) {
    slot_carve(specs[p], regions + region_off[p], &segs[p]);
    segs[p].X = probs[p].X;
    segs[p].v[VB] = const_cast<float*>(probs[p].B);
    segs[p].v[VX] = probs[p].U;
  }
  Tab T;
  GP_TRY(tab_upload(ht, tabmem, &T, s));
  GP_HIP(hipMemcpyAsync(D.segs, segs.data(), sizeof(Seg) * nprob, hipMemcpyHostToDevice, s));

  // ---- preparation: operands and preconditioners ----
  GP_TRY(seq_prepare(D, T, s));
  if (ht.max_rank > 0) {
    std::vector<PcState> hp(nprob);
    GP_HIP(hipMemcpyAsync(hp.data(), D.pcs, sizeof(PcState) * nprob, hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    for (int p = 0; p < nprob; ++p) {
      if (hp[p].not_pd)
        return set_error(GP_ERR_NOT_PD, "problem %d: inner preconditioner matrix not positive definite", p);
      segs[p].rank = hp[p].rank;   // early stop: the rank actually built
    }
    GP_HIP(hipMemcpyAsync(D.segs, segs.data(), sizeof(Seg) * nprob, hipMemcpyHostToDevice, s));
  }
  GP_TRY(seq_start(D, T, ro, o.x0_given != 0, s));

  // ---- iterations: poll_every iterations per captured graph ----
  std::vector<int> live(nprob);
  auto read_live = [&]() -> gp_status {
    GP_HIP(hipMemcpyAsync(live.data(), D.live, 4 * (size_t)nprob, hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    return GP_OK;
  };
  GP_TRY(read_live());
  hipStream_t cs = nullptr;
  hipGraphExec_t exec = nullptr;
  gp_status st = GP_OK;
  int launched = 0;
  auto alive = [&]() { return std::any_of(live.begin(), live.end(), [](int v) { return v > 0; }); };
  while (st == GP_OK && launched < o.max_iter && alive()) {
    const int chunk = std::min(o.poll_every, o.max_iter - launched);
    if (chunk == o.poll_every && !exec) {
      // capture once on a private stream ordered after the caller's stream
      hipEvent_t ev;
      GP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      GP_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      GP_HIP(hipEventRecord(ev, s));
      GP_HIP(hipStreamWaitEvent(cs, ev, 0));
      GP_HIP(hipEventDestroy(ev));
      GP_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      for (int c = 0; c < chunk && st == GP_OK; ++c) st = seq_iteration(D, T, ro, cs);
      hipGraph_t graph = nullptr;
      const hipError_t ce = hipStreamEndCapture(cs, &graph);
      if (st != GP_OK) break;
      if (ce != hipSuccess) {
        st = set_error(GP_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ce));
        break;
      }
      const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        st = set_error(GP_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
        break;
      }
    }
    if (chunk == o.poll_every && exec) {
      const hipError_t le = hipGraphLaunch(exec, s);
      if (le != hipSuccess) {
        st = set_error(GP_ERR_HIP, "graph launch failed: %s", hipGetErrorString(le));
        break;
      }
    } else {
      for (int c = 0; c < chunk && st == GP_OK; ++c) st = seq_iteration(D, T, ro, s);
    }
    launched += chunk;
    if (st == GP_OK) st = read_live();
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (cs) {
    (void)hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
  }
  if (st != GP_OK) return st;

  if (o.true_res_every >= 0) GP_TRY(seq_true_residual(D, T, s));
  std::vector<cg::State> hs(nprob);
  GP_HIP(hipMemcpyAsync(hs.data(), D.st, sizeof(cg::State) * nprob, hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));

  int64_t cols = 0, broke = 0;
  for (int p = 0; p < nprob; ++p) {
    const int r = probs[p].r;
    cols += r;
    for (int c = 0; c < r; ++c) broke += hs[p].breakdown[c];
    if (!stats) continue;
    gp_cg_stats& S = stats[p];
    for (int c = 0; c < r; ++c) {
      if (S.iters) S.iters[c] = hs[p].iters[c];
      if (S.rel_res) S.rel_res[c] = hs[p].rel[c];
      if (S.true_rel_res) S.true_rel_res[c] = o.true_res_every >= 0 ? hs[p].true_rel[c] : -1.0;
      // convergence also requires the float64 true residual, when computed
      const bool true_ok = o.true_res_every < 0 || hs[p].true_rel[c] <= GP_TRUE_RES_SLACK * std::max(o.tol, GP_TRUE_RES_FLOOR);
      if (S.converged) S.converged[c] = (int8_t)(hs[p].converged[c] && true_ok);
      if (S.breakdown) S.breakdown[c] = (int8_t)hs[p].breakdown[c];
    }
    S.total_iters = hs[p].k;
    S.mvms = hs[p].k + (o.x0_given ? 1 : 0);
  }
  if (broke == cols) return set_error(GP_ERR_BREAKDOWN, "every column broke down");
  return GP_OK;
}
