// gp_serve_*: continuous batching of GP solves on one device.
//
// Host side only: a scheduler thread owns the device stream and drives the
// same per-set kernels as the batched solve.  Requests wait in a FIFO queue;
// between rounds the scheduler admits the queue head while a slot and arena
// space are free, prepares and starts the admitted requests together, runs
// iters_per_round iterations over every resident request, and retires the
// ones whose columns have all stopped.  Prediction requests (the second
// request type) have their own FIFO, host thread and stream: each one is a
// single product against a cached model, run as soon as it arrives alongside
// the solve rounds.  Submit / poll / wait / cancel only touch host state
// under one mutex.

#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batched.h"

using namespace gpmi;
using namespace gpmi::bt;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, cap) with coalescing of neighbouring holes.
class FirstFit {
 public:
  explicit FirstFit(uint64_t cap) {
    if (cap) holes_[0] = cap;
  }
  bool take(uint64_t bytes, uint64_t* off) {
    for (auto it = holes_.begin(); it != holes_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const uint64_t rest = it->second - bytes, at = it->first + bytes;
      holes_.erase(it);
      if (rest) holes_[at] = rest;
      return true;
    }
    return false;
  }
  void give(uint64_t off, uint64_t bytes) {
    auto it = holes_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != holes_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      holes_.erase(nx);
    }
    if (it != holes_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        holes_.erase(it);
      }
    }
  }

 private:
  std::map<uint64_t, uint64_t> holes_;
};

enum class RState { Queued, Resident, Done };

struct Req {
  uint64_t ticket = 0;
  bool predict = false;       // a prediction request (pq) rather than a solve (q)
  gp_predict_request pq{};
  gp_request q{};
  SlotSpec spec;
  uint64_t bytes = 0;
  RState state = RState::Queued;
  bool cancel = false;
  int slot = -1;
  uint64_t off = 0;
  gp_result res{};
};

// Device buffer that grows on demand (the scheduler is synchronised when it grows).
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  gp_status ensure(size_t bytes) {
    if (bytes <= cap) return GP_OK;
    const size_t want = std::max(bytes, cap * 2);
    if (p) GP_HIP(hipFree(p));
    p = nullptr;
    cap = 0;
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return set_error(GP_ERR_NOMEM, "table buffer of %zu bytes", want);
    }
    cap = want;
    return GP_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

}  // namespace

struct gp_server {
  gp_serve_config cfg{};
  RunOpts ro;
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  void* devmem = nullptr;
  Dev D{};
  DevBuf tab_join, tab_iter, tab_fin;
  std::vector<Seg> segs;
  std::vector<Req*> slot_req;
  std::vector<int> free_slots;
  FirstFit alloc{0};
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::deque<Req*> pqueue;    // prediction requests, run by the prediction thread
  DevBuf pbuf;                // device copies of test points and means
  hipStream_t pstream = nullptr;
  std::condition_variable cv_pred;
  std::thread pth;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  bool failed = false;
  std::string fail_msg;
  int nresident = 0;
  int64_t submitted = 0, completed = 0, rounds = 0, iterations = 0;
  uint64_t bytes_in_use = 0, peak_bytes = 0;
  double busy = 0.0;
  std::thread th;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  void run();
  gp_status admit(std::vector<Req*>& join, std::vector<int>& resident);
  gp_status finish(const std::vector<int>& slots);
  gp_status predict(const std::vector<Req*>& preds);
  void predict_loop();
  void complete(Req* R, gp_status st, const char* msg);   // mu held
  void release_slot(Req* R);                              // mu held
};

namespace {

size_t dev_bytes(int nslots) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(sizeof(Seg) * nslots) + al(sizeof(cg::State) * nslots) + al(4 * (size_t)nslots) +
         3 * al(4 * (size_t)nslots * cg::kMaxR) + al(sizeof(PcState) * nslots) + al(sizeof(int));
}

void carve_dev(char* base, int nslots, Dev* D) {
  Arena ar;
  ar.base = base;
  ar.cap = dev_bytes(nslots);
  D->nslots = nslots;
  D->segs = ar.take<Seg>(nslots);
  D->st = ar.take<cg::State>(nslots);
  D->live = ar.take<int>(nslots);
  D->colmax = ar.take<uint32_t>((size_t)nslots * cg::kMaxR);
  D->scale = ar.take<float>((size_t)nslots * cg::kMaxR);
  D->inv_scale = ar.take<float>((size_t)nslots * cg::kMaxR);
  D->pcs = ar.take<PcState>(nslots);
  D->counter = ar.take<int>(1);
  D->persistent = false;
}

// Restores the calling thread's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

void gp_server::release_slot(Req* R) {
  alloc.give(R->off, R->bytes);
  bytes_in_use -= R->bytes;
  slot_req[R->slot] = nullptr;
  free_slots.push_back(R->slot);
  --nresident;
  R->slot = -1;
}

void gp_server::complete(Req* R, gp_status st, const char* msg) {
  R->res.status = st;
  R->res.t_finish = now();
  R->res.footprint_bytes = R->bytes;
  if (msg) snprintf(R->res.message, sizeof(R->res.message), "%s", msg);
  R->state = RState::Done;
  ++completed;
  cv_done.notify_all();
}

// Prepare and start newly admitted requests; those that fail are completed.
gp_status gp_server::admit(std::vector<Req*>& join, std::vector<int>& resident) {
  hipStream_t s = stream;
  std::vector<int> plist;
  for (Req* R : join) {
    Seg& g = segs[R->slot];
    slot_carve(R->spec, arena + R->off, &g);
    GP_HIP(hipMemcpyAsync(const_cast<float*>(g.X), R->q.X, sizeof(float) * R->q.n * R->q.d,
                          hipMemcpyHostToDevice, s));
    GP_HIP(hipMemcpyAsync(g.v[VB], R->q.B, sizeof(float) * R->q.n * R->q.r,
                          hipMemcpyHostToDevice, s));
    GP_HIP(hipMemcpyAsync(D.segs + R->slot, &g, sizeof(Seg), hipMemcpyHostToDevice, s));
    plist.push_back(R->slot);
  }
  HostTab ht;
  build_tab(segs, plist, &ht);
  GP_TRY(tab_join.ensure(tab_bytes(ht)));
  Tab T;
  GP_TRY(tab_upload(ht, tab_join.p, &T, s));
  GP_TRY(seq_prepare(D, T, s));
  std::vector<PcState> hp(join.size());
  for (size_t i = 0; i < join.size(); ++i)
    GP_HIP(hipMemcpyAsync(&hp[i], D.pcs + join[i]->slot, sizeof(PcState), hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));
  std::vector<int> ok;
  std::vector<Req*> bad;
  for (size_t i = 0; i < join.size(); ++i) {
    Req* R = join[i];
    if (hp[i].not_pd) {
      bad.push_back(R);
      continue;
    }
    if (segs[R->slot].rank != hp[i].rank) {
      segs[R->slot].rank = hp[i].rank;   // early stop: the rank actually built
      GP_HIP(hipMemcpyAsync(D.segs + R->slot, &segs[R->slot], sizeof(Seg), hipMemcpyHostToDevice, s));
    }
    ok.push_back(R->slot);
  }
  if (!bad.empty()) {
    std::lock_guard<std::mutex> lk(mu);
    for (Req* R : bad) {
      release_slot(R);
      complete(R, GP_ERR_NOT_PD, "inner preconditioner matrix not positive definite");
    }
  }
  if (ok.empty()) return GP_OK;
  if (ok.size() != plist.size()) {
    build_tab(segs, ok, &ht);
    GP_TRY(tab_upload(ht, tab_join.p, &T, s));
  }
  GP_TRY(seq_start(D, T, ro, false, s));
  GP_HIP(hipStreamSynchronize(s));
  resident.insert(resident.end(), ok.begin(), ok.end());
  return GP_OK;
}

// True residual, statistics and copy-out of the given slots; completes them.
gp_status gp_server::finish(const std::vector<int>& slots) {
  hipStream_t s = stream;
  HostTab ht;
  build_tab(segs, slots, &ht);
  GP_TRY(tab_fin.ensure(tab_bytes(ht)));
  Tab T;
  GP_TRY(tab_upload(ht, tab_fin.p, &T, s));
  GP_TRY(seq_true_residual(D, T, s));
  std::vector<cg::State> hs(slots.size());
  for (size_t i = 0; i < slots.size(); ++i) {
    const int p = slots[i];
    const Req* R = slot_req[p];
    GP_HIP(hipMemcpyAsync(&hs[i], D.st + p, sizeof(cg::State), hipMemcpyDeviceToHost, s));
    GP_HIP(hipMemcpyAsync(R->q.U_out, segs[p].v[VX], sizeof(float) * R->q.n * R->q.r,
                          hipMemcpyDeviceToHost, s));
  }
  GP_HIP(hipStreamSynchronize(s));
  std::lock_guard<std::mutex> lk(mu);
  for (size_t i = 0; i < slots.size(); ++i) {
    Req* R = slot_req[slots[i]];
    const cg::State& S = hs[i];
    const int r = R->q.r;
    gp_result& res = R->res;
    res.iters = S.k;
    res.converged = res.breakdown = 0;
    res.max_rel_res = res.max_true_rel_res = 0.0;
    // convergence also requires the float64 true residual (within the slack)
    const double tmax = GP_TRUE_RES_SLACK * std::max(R->q.tol, GP_TRUE_RES_FLOOR);
    for (int c = 0; c < r; ++c) {
      res.converged += (S.converged[c] && S.true_rel[c] <= tmax) ? 1 : 0;
      res.breakdown += S.breakdown[c];
      res.max_rel_res = std::max(res.max_rel_res, (double)S.rel[c]);
      res.max_true_rel_res = std::max(res.max_true_rel_res, S.true_rel[c]);
    }
    if (gp_cg_stats* st = R->q.stats) {
      for (int c = 0; c < r; ++c) {
        if (st->iters) st->iters[c] = S.iters[c];
        if (st->rel_res) st->rel_res[c] = S.rel[c];
        if (st->true_rel_res) st->true_rel_res[c] = S.true_rel[c];
        if (st->converged)
          st->converged[c] = (int8_t)(S.converged[c] && S.true_rel[c] <= tmax);
        if (st->breakdown) st->breakdown[c] = (int8_t)S.breakdown[c];
      }
      st->total_iters = S.k;
      st->mvms = S.k;
    }
    release_slot(R);
    const bool all_broke = res.breakdown == r;
    complete(R, all_broke ? GP_ERR_BREAKDOWN : GP_OK, all_broke ? "every column broke down" : nullptr);
  }
  return GP_OK;
}

// Run the given prediction requests one after another on the prediction
// stream (test points in, binary16 product against the model's cache, means
// out) and complete them.  A request the product rejects completes with its
// error; a device failure is returned (the caller completes the rest).
gp_status gp_server::predict(const std::vector<Req*>& preds) {
  hipStream_t s = pstream;
  for (Req* R : preds) {
    const gp_predict_request& q = R->pq;
    gp_model_info mi{};
    (void)gp_model_info_read(q.model, &mi);
    const size_t xb = 4 * (size_t)q.ns * mi.d, mb = 4 * (size_t)q.ns;
    GP_TRY(pbuf.ensure(xb + mb + 256));
    float* dX = static_cast<float*>(pbuf.p);
    float* dmu = reinterpret_cast<float*>(static_cast<char*>(pbuf.p) + ((xb + 255) & ~size_t(255)));
    GP_HIP(hipMemcpyAsync(dX, q.Xs, xb, hipMemcpyHostToDevice, s));
    const gp_status st = gp_model_predict(q.model, dX, q.ns, dmu, GP_PREC_FP16, q.truncate, s);
    if (st == GP_OK) {
      GP_HIP(hipMemcpyAsync(q.mu_out, dmu, mb, hipMemcpyDeviceToHost, s));
      GP_HIP(hipStreamSynchronize(s));
    } else if (st == GP_ERR_HIP) {
      return st;
    }
    std::lock_guard<std::mutex> lk(mu);
    complete(R, st, st == GP_OK ? nullptr : gp_last_error());
  }
  return GP_OK;
}

void gp_server::predict_loop() {
  (void)hipSetDevice(cfg.device);
  for (;;) {
    std::vector<Req*> preds;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_pred.wait(lk, [&] { return stop || !pqueue.empty(); });
      if (stop) break;
      while (!pqueue.empty()) {
        Req* R = pqueue.front();
        pqueue.pop_front();
        R->state = RState::Resident;
        R->res.t_admit = now();
        preds.push_back(R);
      }
    }
    const gp_status st = predict(preds);
    if (st != GP_OK) {
      std::lock_guard<std::mutex> lk(mu);
      const std::string msg = gp_last_error();
      for (Req* R : preds)
        if (R->state != RState::Done) complete(R, st, msg.c_str());
    }
  }
  // shutdown: whatever is still queued is cancelled
  std::lock_guard<std::mutex> lk(mu);
  for (Req* R : pqueue) complete(R, GP_ERR_CANCELLED, "server stopped");
  pqueue.clear();
}

void gp_server::run() {
  (void)hipSetDevice(cfg.device);
  std::vector<int> resident;   // slots in admission order
  HostTab ht_iter;
  Tab T_iter;
  bool dirty = true;
  std::vector<int> live(cfg.max_slots);
  gp_status st = GP_OK;
  for (;;) {
    std::vector<Req*> join;
    std::vector<Req*> dropped;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !queue.empty() || !resident.empty(); });
      if (stop) break;
      for (int p : resident)
        if (slot_req[p]->cancel) dropped.push_back(slot_req[p]);
      for (Req* R : dropped) {
        resident.erase(std::find(resident.begin(), resident.end(), R->slot));
        release_slot(R);
        complete(R, GP_ERR_CANCELLED, "cancelled");
        dirty = true;
      }
      while (!queue.empty() && !free_slots.empty()) {
        Req* R = queue.front();
        uint64_t off;
        if (!alloc.take(R->bytes, &off)) break;   // first come first served
        queue.pop_front();
        R->off = off;
        R->slot = free_slots.back();
        free_slots.pop_back();
        slot_req[R->slot] = R;
        R->state = RState::Resident;
        R->res.t_admit = now();
        bytes_in_use += R->bytes;
        peak_bytes = std::max(peak_bytes, bytes_in_use);
        ++nresident;
        join.push_back(R);
      }
    }
    const Clock::time_point tr = Clock::now();
    D.persistent = tune::bt_persistent();
    if (!join.empty()) {
      st = admit(join, resident);
      if (st != GP_OK) break;
      dirty = true;
    }
    if (resident.empty()) continue;
    if (dirty) {
      build_tab(segs, resident, &ht_iter);
      st = tab_iter.ensure(tab_bytes(ht_iter));
      if (st == GP_OK) st = tab_upload(ht_iter, tab_iter.p, &T_iter, stream);
      if (st != GP_OK) break;
      dirty = false;
    }
    for (int i = 0; i < cfg.iters_per_round && st == GP_OK; ++i) st = seq_iteration(D, T_iter, ro, stream);
    if (st == GP_OK && hipMemcpyAsync(live.data(), D.live, sizeof(int) * cfg.max_slots,
                                      hipMemcpyDeviceToHost, stream) != hipSuccess)
      st = set_error(GP_ERR_HIP, "activity flags copy failed");
    if (st == GP_OK && hipStreamSynchronize(stream) != hipSuccess)
      st = set_error(GP_ERR_HIP, "stream synchronisation failed");
    if (st != GP_OK) break;
    std::vector<int> done;
    for (int p : resident)
      if (live[p] == 0) done.push_back(p);
    if (!done.empty()) {
      st = finish(done);
      if (st != GP_OK) break;
      resident.erase(std::remove_if(resident.begin(), resident.end(),
                                    [&](int p) { return live[p] == 0; }),
                     resident.end());
      dirty = true;
    }
    std::lock_guard<std::mutex> lk(mu);
    ++rounds;
    iterations += (int64_t)cfg.iters_per_round * (int64_t)(resident.size() + done.size());
    busy += std::chrono::duration<double>(Clock::now() - tr).count();
  }
  // failure or shutdown: complete everything still pending
  std::lock_guard<std::mutex> lk(mu);
  const bool err = st != GP_OK;
  if (err) {
    failed = true;
    fail_msg = gp_last_error();
  }
  for (auto& kv : reqs) {
    Req* R = kv.second.get();
    if (R->state == RState::Done || R->predict) continue;   // predictions: their own thread
    if (R->state == RState::Resident) release_slot(R);
    complete(R, err ? st : GP_ERR_CANCELLED, err ? fail_msg.c_str() : "server stopped");
  }
  queue.clear();
}

extern "C" void gp_serve_default_config(gp_serve_config* c) {
  if (!c) return;
  memset(c, 0, sizeof(*c));
  c->hbm_budget_bytes = 8ull << 30;
  c->max_slots = 64;
  c->device = 0;
  c->iters_per_round = 5;
  c->min_iter = 10;
  c->algo = GP_CG_ENHANCED;
  c->reorth = 1;
  c->use_lse = 1;
  c->scale_mode = 0;
}

extern "C" gp_status gp_serve_create(const gp_serve_config* c, gp_server** out) {
  clear_error();
  if (!c || !out) return set_error(GP_ERR_ARG, "config and out must not be NULL");
  *out = nullptr;
  if (c->max_slots < 1 || c->max_slots > 1024) return set_error(GP_ERR_ARG, "max_slots outside [1, 1024]");
  if (c->iters_per_round < 1) return set_error(GP_ERR_ARG, "iters_per_round must be >= 1");
  if (c->min_iter < 0) return set_error(GP_ERR_ARG, "min_iter must be >= 0");
  if (c->algo != GP_CG_ENHANCED && c->algo != GP_CG_STANDARD)
    return set_error(GP_ERR_ARG, "algo must be GP_CG_STANDARD or GP_CG_ENHANCED");
  if (c->scale_mode != 0 && c->scale_mode != 1) return set_error(GP_ERR_ARG, "scale_mode must be 0 or 1");
  if (c->hbm_budget_bytes < (1ull << 20)) return set_error(GP_ERR_ARG, "hbm_budget_bytes below 1 MiB");
  int ndev = 0;
  GP_HIP(hipGetDeviceCount(&ndev));
  if (c->device < 0 || c->device >= ndev) return set_error(GP_ERR_ARG, "device %d not present", c->device);
  std::unique_ptr<gp_server> S(new gp_server());
  S->cfg = *c;
  const bool enhanced = c->algo == GP_CG_ENHANCED;
  S->ro.lse = enhanced && c->use_lse;
  S->ro.reorth = enhanced && c->reorth;
  S->ro.scale_mode = c->scale_mode;
  DeviceGuard dg(c->device);
  if (hipMalloc(reinterpret_cast<void**>(&S->arena), c->hbm_budget_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(GP_ERR_NOMEM, "arena of %llu bytes", (unsigned long long)c->hbm_budget_bytes);
  }
  const size_t db = dev_bytes(c->max_slots);
  if (hipMalloc(&S->devmem, db) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(S->arena);
    return set_error(GP_ERR_NOMEM, "slot arrays");
  }
  carve_dev(static_cast<char*>(S->devmem), c->max_slots, &S->D);
  if (hipMemset(S->devmem, 0, db) != hipSuccess ||
      hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&S->pstream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(S->devmem);
    (void)hipFree(S->arena);
    return set_error(GP_ERR_HIP, "server set-up failed");
  }
  S->alloc = FirstFit(c->hbm_budget_bytes);
  S->segs.assign(c->max_slots, Seg{});
  S->slot_req.assign(c->max_slots, nullptr);
  for (int p = c->max_slots - 1; p >= 0; --p) S->free_slots.push_back(p);
  S->t0 = Clock::now();
  gp_server* raw = S.get();
  raw->th = std::thread([raw] { raw->run(); });
  raw->pth = std::thread([raw] { raw->predict_loop(); });
  *out = S.release();
  return GP_OK;
}

extern "C" gp_status gp_serve_submit(gp_server* s, const gp_request* q, uint64_t* ticket) {
  clear_error();
  if (!s || !q || !ticket) return set_error(GP_ERR_ARG, "server, request and ticket must not be NULL");
  SlotSpec sp;
  gp_status st = check_kernel(&q->k, q->d, true, &sp.kp);
  if (st != GP_OK) return st;
  if (q->d > 30) return set_error(GP_ERR_ARG, "served requests take d <= 30");
  if (q->n < 1) return set_error(GP_ERR_ARG, "n must be >= 1");
  if (q->r < 1 || q->r > cg::kMaxR) return set_error(GP_ERR_ARG, "r outside [1, 64]");
  if (!q->X || !q->B || !q->U_out) return set_error(GP_ERR_ARG, "NULL array");
  if (!(q->tol >= 0.0) || !isfinite(q->tol)) return set_error(GP_ERR_ARG, "tol must be finite, >= 0");
  if (q->max_iter < 0 || q->max_iter > 100000) return set_error(GP_ERR_ARG, "max_iter outside [0, 100000]");
  if (q->precond_rank < 0 || q->precond_rank > pc::kMaxRank || q->precond_rank > q->n)
    return set_error(GP_ERR_ARG, "precond_rank outside [0, min(n, 128)]");
  sp.n = q->n;
  sp.d = q->d;
  sp.r = q->r;
  sp.rank = q->precond_rank;
  sp.max_iter = q->max_iter;
  sp.min_iter = s->cfg.min_iter;
  sp.tol = q->tol;
  sp.reorth = s->ro.reorth;
  sp.own_io = true;
  const uint64_t bytes = slot_bytes(sp);
  if (bytes > s->cfg.hbm_budget_bytes)
    return set_error(GP_ERR_TOO_LARGE, "request needs %llu bytes, the arena holds %llu",
                     (unsigned long long)bytes, (unsigned long long)s->cfg.hbm_budget_bytes);
  std::unique_ptr<Req> R(new Req());
  R->q = *q;
  R->spec = sp;
  R->bytes = bytes;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop || s->failed)
    return set_error(GP_ERR_STOPPED, "server stopped%s%s", s->failed ? ": " : "", s->fail_msg.c_str());
  R->ticket = s->next_ticket++;
  R->res.t_submit = s->now();
  *ticket = R->ticket;
  s->queue.push_back(R.get());
  s->reqs.emplace(R->ticket, std::move(R));
  ++s->submitted;
  s->cv_work.notify_one();
  return GP_OK;
}

extern "C" gp_status gp_serve_submit_predict(gp_server* s, const gp_predict_request* q,
                                            uint64_t* ticket) {
  clear_error();
  if (!s || !q || !ticket) return set_error(GP_ERR_ARG, "server, request and ticket must not be NULL");
  if (!q->model) return set_error(GP_ERR_ARG, "model is NULL");
  if (gp_model_device(q->model) != s->cfg.device)
    return set_error(GP_ERR_ARG, "the model lives on device %d, the server on %d",
                     gp_model_device(q->model), s->cfg.device);
  if (q->ns < 1) return set_error(GP_ERR_ARG, "ns must be >= 1");
  if (!q->Xs || !q->mu_out) return set_error(GP_ERR_ARG, "NULL array");
  if (q->truncate != 0 && q->truncate != 1) return set_error(GP_ERR_ARG, "truncate must be 0 or 1");
  std::unique_ptr<Req> R(new Req());
  R->predict = true;
  R->pq = *q;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop || s->failed)
    return set_error(GP_ERR_STOPPED, "server stopped%s%s", s->failed ? ": " : "", s->fail_msg.c_str());
  R->ticket = s->next_ticket++;
  R->res.t_submit = s->now();
  *ticket = R->ticket;
  s->pqueue.push_back(R.get());
  s->reqs.emplace(R->ticket, std::move(R));
  ++s->submitted;
  s->cv_pred.notify_one();
  return GP_OK;
}

namespace {
gp_status take_result(gp_server* s, std::unordered_map<uint64_t, std::unique_ptr<Req>>::iterator it,
                      gp_result* res) {
  Req* R = it->second.get();
  if (R->state != RState::Done) return GP_PENDING;
  if (res) *res = R->res;
  const gp_status st = R->res.status;
  s->reqs.erase(it);
  return st;
}
}  // namespace

extern "C" gp_status gp_serve_poll(gp_server* s, uint64_t ticket, gp_result* res) {
  clear_error();
  if (!s) return set_error(GP_ERR_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return set_error(GP_ERR_UNKNOWN_TICKET, "unknown ticket %llu", (unsigned long long)ticket);
  return take_result(s, it, res);
}

extern "C" gp_status gp_serve_wait(gp_server* s, uint64_t ticket, int64_t timeout_ms, gp_result* res) {
  clear_error();
  if (!s) return set_error(GP_ERR_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto done = [&] {
    auto it = s->reqs.find(ticket);
    return it == s->reqs.end() || it->second->state == RState::Done;
  };
  if (timeout_ms < 0)
    s->cv_done.wait(lk, done);
  else
    s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return set_error(GP_ERR_UNKNOWN_TICKET, "unknown ticket %llu", (unsigned long long)ticket);
  return take_result(s, it, res);
}

extern "C" gp_status gp_serve_cancel(gp_server* s, uint64_t ticket) {
  clear_error();
  if (!s) return set_error(GP_ERR_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second->state == RState::Done)
    return set_error(GP_ERR_UNKNOWN_TICKET, "ticket %llu is not pending", (unsigned long long)ticket);
  Req* R = it->second.get();
  if (R->state == RState::Queued) {
    auto& qu = R->predict ? s->pqueue : s->queue;
    qu.erase(std::find(qu.begin(), qu.end(), R));
    s->complete(R, GP_ERR_CANCELLED, "cancelled");
  } else {
    R->cancel = true;
    s->cv_work.notify_one();
  }
  return GP_OK;
}

extern "C" gp_status gp_serve_stats_read(gp_server* s, gp_serve_stats* out) {
  clear_error();
  if (!s || !out) return set_error(GP_ERR_ARG, "server and out must not be NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  out->queued = (int32_t)(s->queue.size() + s->pqueue.size());
  out->resident = s->nresident;
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->rounds = s->rounds;
  out->iterations = s->iterations;
  out->bytes_in_use = s->bytes_in_use;
  out->peak_bytes = s->peak_bytes;
  out->busy_seconds = s->busy;
  out->uptime_seconds = s->now();
  return GP_OK;
}

extern "C" gp_status gp_serve_destroy(gp_server* s) {
  clear_error();
  if (!s) return GP_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->cv_pred.notify_all();
  if (s->th.joinable()) s->th.join();
  if (s->pth.joinable()) s->pth.join();
  {
    DeviceGuard dg(s->cfg.device);
    if (s->stream) {
      (void)hipStreamSynchronize(s->stream);
      (void)hipStreamDestroy(s->stream);
    }
    if (s->pstream) {
      (void)hipStreamSynchronize(s->pstream);
      (void)hipStreamDestroy(s->pstream);
    }
    s->tab_join.release();
    s->tab_iter.release();
    s->tab_fin.release();
    s->pbuf.release();
    if (s->devmem) (void)hipFree(s->devmem);
    if (s->arena) (void)hipFree(s->arena);
  }
  delete s;
  return GP_OK;
}
