// gp_cg_solve_batched: host driver of the batched solve.
//
// The host builds the segment, chunk and work-item tables once, then enqueues
// whole-batch launches: preparation, the per-problem pivoted-Cholesky builds
// (one launch pair per pivot step for all problems), initialisation, and the
// iterations.  The `poll_every` iterations between two polls of the per-problem
// activity flags are captured once into a HIP graph and replayed.

#include <math.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "batched.h"

namespace gpmi {
namespace bt {
namespace {

__global__ void zero_words_kernel(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

gp_status zero_bytes(void* p, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n == 0) return GP_OK;
  zero_words_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(static_cast<uint32_t*>(p), n);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

int splits_for(int64_t n_pad_c) {
  const int64_t stages = n_pad_c / f16::kStageCols;
  return (int)std::max<int64_t>(1, std::min<int64_t>(8, stages / 16));
}

int splits64_for(int64_t n) {
  const int64_t stages = ceil_div(n, valu::kStageCols);
  return (int)std::max<int64_t>(1, std::min<int64_t>(8, stages / 16));
}

struct Host {
  std::vector<Seg> segs;
  std::vector<Chunk> chunks;
  std::vector<Item> items, items64;
  std::vector<int4> tiles;
  std::vector<int64_t> rowstart, colstart, xr_off, xc_off, qstart;
  int64_t vec_total = 0, xr_total = 0, xc_total = 0, vt_total = 0, part_total = 0;
  int64_t basis_total = 0, l_total = 0, cinv_total = 0, diag_total = 0, part64_total = 0;
};

// one iteration of the batched recurrence (a2 -> a7)
gp_status iteration(const Dev& D, const gp_cg_opts& o, bool lse, bool reorth, hipStream_t s) {
  GP_TRY(launch_product(D, D.d, D.q, D.live, s));
  GP_TRY(launch_dq(D, lse, s));
  GP_TRY(launch_update(D, D.x, s));
  if (reorth) GP_TRY(launch_reorth(D, s));
  GP_TRY(launch_precond(D, s));
  GP_TRY(launch_rz(D, lse, false, o.tol, o.min_iter, s));
  GP_TRY(launch_direction(D, false, reorth, s));
  return launch_quant(D, D.d, o.scale_mode, D.live, s);
}

}  // namespace
}  // namespace bt
}  // namespace gpmi

using namespace gpmi;
using namespace gpmi::bt;

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
  const bool lse = enhanced && o.use_lse;
  const bool reorth = enhanced && o.reorth;
  const int max_basis = o.max_iter + 1;

  Host H;
  Dev D{};
  D.nprob = nprob;
  D.max_basis = max_basis;
  int max_r = 1, max_w = 32, max_d = 1, max_rank = 0;
  for (int p = 0; p < nprob; ++p) {
    const gp_problem& q = probs[p];
    KParams kp;
    gp_status st = check_kernel(&q.k, q.d, true, &kp);
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
    max_r = std::max(max_r, q.r);
    max_d = std::max(max_d, q.d);
    max_w = std::max(max_w, f16::aug_width(q.d));
    max_rank = std::max(max_rank, q.precond_rank);
  }
  D.rb = (int)ceil_div(max_r, 16);
  D.rp = 16 * D.rb;
  D.max_w = max_w;
  D.max_d = max_d;
  D.max_r = max_r;
  D.max_rank = max_rank;

  // ---- tables ----
  H.segs.resize(nprob);
  H.rowstart.push_back(0);
  H.colstart.push_back(0);
  H.qstart.push_back(0);
  double entries = 0.0;
  for (int p = 0; p < nprob; ++p) {
    const gp_problem& q = probs[p];
    Seg& g = H.segs[p];
    g = Seg{};
    KParams kp;
    check_kernel(&q.k, q.d, true, &kp);
    g.X = q.X;
    g.B = q.B;
    g.U = q.U;
    g.n = q.n;
    g.r = q.r;
    g.d = q.d;
    g.w = f16::aug_width(q.d);
    g.kc = g.w / 32;
    g.kind = kp.kind;
    g.a2 = kp.a2;
    g.s2 = kp.s2;
    for (int m = 0; m < kMaxDim; ++m) g.ls[m] = kp.ls[m];
    g.rank = q.precond_rank;
    g.n_pad_r = round_up(q.n, f16::kRowsPerBlock);
    g.n_pad_c = round_up(q.n, f16::kStageCols);
    g.nsplit = splits_for(g.n_pad_c);
    g.nsplit64 = splits64_for(q.n);
    g.vec_off = H.vec_total;
    H.vec_total += q.n * q.r;
    H.xr_off.push_back(H.xr_total);
    H.xr_total += g.n_pad_r * g.w;
    H.xc_off.push_back(H.xc_total);
    H.xc_total += g.n_pad_c * g.w;
    H.rowstart.push_back(H.rowstart.back() + g.n_pad_r);
    H.colstart.push_back(H.colstart.back() + g.n_pad_c);
    g.vt_off = H.vt_total;
    H.vt_total += (int64_t)D.rp * g.n_pad_c;
    H.qstart.push_back(H.qstart.back() + (int64_t)D.rp * (g.n_pad_c / 8));
    g.part_off = H.part_total;
    H.part_total += (int64_t)g.nsplit * g.n_pad_r * D.rp;
    g.basis_off = H.basis_total;
    if (reorth) H.basis_total += (int64_t)max_basis * q.n * q.r;
    g.l_off = H.l_total;
    H.l_total += (int64_t)g.rank * q.n;
    g.cinv_off = H.cinv_total;
    H.cinv_total += (int64_t)g.rank * g.rank;
    g.diag_off = H.diag_total;
    H.diag_total += q.n;
    g.part64_off = H.part64_total;
    H.part64_total += (int64_t)g.nsplit64 * q.n * q.r;
    g.chunk0 = (int)H.chunks.size();
    for (int64_t i0 = 0; i0 < q.n; i0 += kChunkRows)
      H.chunks.push_back(Chunk{p, 0, i0, std::min<int64_t>(q.n, i0 + kChunkRows)});
    g.nchunk = (int)H.chunks.size() - g.chunk0;
    for (int64_t rb = 0; rb < g.n_pad_r / f16::kRowsPerBlock; ++rb)
      for (int sp = 0; sp < g.nsplit; ++sp) H.items.push_back(Item{p, sp, rb});
    const int rpt = trueres_dm_of(q.d) <= 16 ? 4 : 1;
    for (int64_t rb = 0; rb < ceil_div(q.n, (int64_t)valu::kRowsPerBlock * rpt); ++rb)
      for (int sp = 0; sp < g.nsplit64; ++sp) H.items64.push_back(Item{p, sp, rb});
    const int tk = (g.rank + 15) / 16;
    for (int a = 0; a < tk; ++a)
      for (int b = 0; b < tk; ++b) H.tiles.push_back(make_int4(p, a, b, 0));
    entries += (double)q.n * (double)q.n;
  }
  H.rowstart.pop_back();
  H.colstart.pop_back();
  const int64_t qtotal = H.qstart.back();
  H.qstart.pop_back();
  // longest work first: stages per item, ties by problem order
  auto cost = [&](const Item& it) {
    const Seg& g = H.segs[it.p];
    const int64_t st = g.n_pad_c / f16::kStageCols;
    return (it.split + 1) * st / g.nsplit - it.split * st / g.nsplit;
  };
  std::stable_sort(H.items.begin(), H.items.end(),
                   [&](const Item& a, const Item& b) { return cost(a) > cost(b); });
  auto cost64 = [&](const Item& it) {
    const Seg& g = H.segs[it.p];
    const int64_t st = ceil_div(g.n, valu::kStageCols);
    return ((it.split + 1) * st / g.nsplit64 - it.split * st / g.nsplit64) *
           (int64_t)trueres_dm_of(g.d) * ceil_div(g.r, 16);
  };
  std::stable_sort(H.items64.begin(), H.items64.end(),
                   [&](const Item& a, const Item& b) { return cost64(a) > cost64(b); });
  D.nchunks = (int)H.chunks.size();
  D.nitems = (int)H.items.size();
  D.nitems64 = (int)H.items64.size();
  D.ntiles = (int)H.tiles.size();
  D.total_rows_r = std::accumulate(H.segs.begin(), H.segs.end(), (int64_t)0,
                                   [](int64_t a, const Seg& g) { return a + g.n_pad_r; });
  D.total_rows_c = std::accumulate(H.segs.begin(), H.segs.end(), (int64_t)0,
                                   [](int64_t a, const Seg& g) { return a + g.n_pad_c; });
  D.qtotal = qtotal;
  D.l_total = H.l_total;
  D.entries = entries;
  const bool any_pc = max_rank > 0;

  // ---- workspace ----
  size_t bytes = 0;
  auto add = [&](size_t b) { bytes += (b + 255) & ~size_t(255); };
  add(sizeof(Seg) * nprob);
  add(sizeof(Chunk) * D.nchunks);
  add(sizeof(Item) * D.nitems);
  add(sizeof(Item) * D.nitems64);
  add(sizeof(int4) * std::max(1, D.ntiles));
  for (int k = 0; k < 5; ++k) add(8 * (size_t)nprob);
  add(4 * (size_t)H.vec_total * 6);                              // b x r z d q
  if (reorth) add(4 * (size_t)H.basis_total * (any_pc ? 2 : 1));
  add(2 * (size_t)H.xr_total);
  add(2 * (size_t)H.xc_total);
  add(2 * (size_t)H.vt_total);
  add(4 * (size_t)H.part_total);
  add(4 * (size_t)nprob * cg::kMaxR * 3);                        // colmax scale inv
  add(8 * (size_t)H.part64_total);
  add(4 * (size_t)D.nchunks * cg::kMaxR * 2);                    // pm ps
  add(8 * (size_t)D.nchunks * cg::kMaxR);                        // pq
  if (reorth) {
    add(4 * (size_t)D.nchunks * max_basis * cg::kMaxR);
    add(4 * (size_t)nprob * max_basis * cg::kMaxR);
  }
  const bool want_hist = false;
  add(sizeof(cg::State) * nprob);
  add(4 * (size_t)nprob);
  add(8 * (size_t)std::max<int64_t>(1, H.l_total));               // L64
  add(4 * (size_t)std::max<int64_t>(1, H.l_total));               // L32
  add(8 * (size_t)std::max<int64_t>(1, H.cinv_total) * 2);        // C Cinv
  add(8 * (size_t)H.diag_total);
  add(8 * (size_t)D.nchunks * 2 + 8 * (size_t)D.nchunks);         // pv psum pi
  add(8 * (size_t)nprob * std::max(1, max_rank));                 // pivots
  add(4 * (size_t)D.nchunks * pc::kMaxRank * cg::kMaxR);          // lt partials
  add(4 * (size_t)nprob * pc::kMaxRank * cg::kMaxR);              // Y32
  add(sizeof(PcState) * nprob);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Arena ar;
  GP_TRY(workspace_get(s, bytes, &ar));
  D.segs = ar.take<Seg>(nprob);
  D.chunks = ar.take<Chunk>(D.nchunks);
  D.items = ar.take<Item>(D.nitems);
  D.items64 = ar.take<Item>(D.nitems64);
  D.tiles = ar.take<int4>(std::max(1, D.ntiles));
  D.rowstart = ar.take<int64_t>(nprob);
  D.colstart = ar.take<int64_t>(nprob);
  D.xr_off = ar.take<int64_t>(nprob);
  D.xc_off = ar.take<int64_t>(nprob);
  D.qstart = ar.take<int64_t>(nprob);
  D.b = ar.take<float>(H.vec_total);
  D.x = ar.take<float>(H.vec_total);
  D.r = ar.take<float>(H.vec_total);
  D.z = ar.take<float>(H.vec_total);
  D.d = ar.take<float>(H.vec_total);
  D.q = ar.take<float>(H.vec_total);
  D.Ub = reorth ? ar.take<float>(H.basis_total) : nullptr;
  D.Wb = (reorth && any_pc) ? ar.take<float>(H.basis_total) : nullptr;
  D.Xr = ar.take<_Float16>(H.xr_total);
  D.Xc = ar.take<_Float16>(H.xc_total);
  D.Vt = ar.take<_Float16>(H.vt_total);
  D.part = ar.take<float>(H.part_total);
  D.colmax = ar.take<uint32_t>((size_t)nprob * cg::kMaxR);
  D.scale = ar.take<float>((size_t)nprob * cg::kMaxR);
  D.inv_scale = ar.take<float>((size_t)nprob * cg::kMaxR);
  D.part64 = ar.take<double>(H.part64_total);
  D.pm = ar.take<float>((size_t)D.nchunks * cg::kMaxR);
  D.ps = ar.take<float>((size_t)D.nchunks * cg::kMaxR);
  D.pq = ar.take<double>((size_t)D.nchunks * cg::kMaxR);
  D.pcoef = reorth ? ar.take<float>((size_t)D.nchunks * max_basis * cg::kMaxR) : nullptr;
  D.coef = reorth ? ar.take<float>((size_t)nprob * max_basis * cg::kMaxR) : nullptr;
  D.history = nullptr;
  (void)want_hist;
  D.st = ar.take<cg::State>(nprob);
  D.live = ar.take<int>(nprob);
  D.L64 = ar.take<double>(std::max<int64_t>(1, H.l_total));
  D.L32 = ar.take<float>(std::max<int64_t>(1, H.l_total));
  D.C = ar.take<double>(std::max<int64_t>(1, H.cinv_total));
  D.Cinv = ar.take<double>(std::max<int64_t>(1, H.cinv_total));
  D.diag = ar.take<double>(H.diag_total);
  D.pv = ar.take<double>(D.nchunks);
  D.psum = ar.take<double>(D.nchunks);
  D.pi = ar.take<int64_t>(D.nchunks);
  D.piv = ar.take<int64_t>((size_t)nprob * std::max(1, max_rank));
  D.ltpart = ar.take<float>((size_t)D.nchunks * pc::kMaxRank * cg::kMaxR);
  D.Y32 = ar.take<float>((size_t)nprob * pc::kMaxRank * cg::kMaxR);
  D.pcs = ar.take<PcState>(nprob);
  if (!D.pcs) return set_error(GP_ERR_NOMEM, "internal: batched workspace sizing");

  GP_HIP(hipMemcpyAsync(D.segs, H.segs.data(), sizeof(Seg) * nprob, hipMemcpyHostToDevice, s));
  GP_HIP(hipMemcpyAsync(D.chunks, H.chunks.data(), sizeof(Chunk) * D.nchunks, hipMemcpyHostToDevice, s));
  GP_HIP(hipMemcpyAsync(D.items, H.items.data(), sizeof(Item) * D.nitems, hipMemcpyHostToDevice, s));
  GP_HIP(hipMemcpyAsync(D.items64, H.items64.data(), sizeof(Item) * D.nitems64, hipMemcpyHostToDevice, s));
  if (D.ntiles)
    GP_HIP(hipMemcpyAsync(D.tiles, H.tiles.data(), sizeof(int4) * D.ntiles, hipMemcpyHostToDevice, s));
  GP_HIP(hipMemcpyAsync(D.rowstart, H.rowstart.data(), 8 * nprob, hipMemcpyHostToDevice, s));
  GP_HIP(hipMemcpyAsync(D.colstart, H.colstart.data(), 8 * nprob, hipMemcpyHostToDevice, s));
  GP_HIP(hipMemcpyAsync(D.xr_off, H.xr_off.data(), 8 * nprob, hipMemcpyHostToDevice, s));
  GP_HIP(hipMemcpyAsync(D.xc_off, H.xc_off.data(), 8 * nprob, hipMemcpyHostToDevice, s));
  GP_HIP(hipMemcpyAsync(D.qstart, H.qstart.data(), 8 * nprob, hipMemcpyHostToDevice, s));

  // ---- initialisation ----
  GP_TRY(zero_bytes(D.st, sizeof(cg::State) * nprob, s));
  GP_TRY(zero_bytes(D.pcs, sizeof(PcState) * nprob, s));
  GP_TRY(zero_bytes(D.colmax, 4 * (size_t)nprob * cg::kMaxR, s));
  GP_TRY(zero_bytes(D.Y32, 4 * (size_t)nprob * pc::kMaxRank * cg::kMaxR, s));
  GP_TRY(launch_prep(D, 0, s));
  GP_TRY(launch_prep(D, 1, s));
  GP_TRY(launch_gather(D, 0, D.b, s));
  if (any_pc) {
    GP_TRY(launch_pivchol(D, s));
    std::vector<PcState> hp(nprob);
    GP_HIP(hipMemcpyAsync(hp.data(), D.pcs, sizeof(PcState) * nprob, hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    for (int p = 0; p < nprob; ++p) {
      if (hp[p].not_pd)
        return set_error(GP_ERR_NOT_PD, "problem %d: inner preconditioner matrix not positive definite", p);
      if (hp[p].rank != H.segs[p].rank) {
        // early stop: record the rank actually built
        H.segs[p].rank = hp[p].rank;
      }
    }
    GP_HIP(hipMemcpyAsync(D.segs, H.segs.data(), sizeof(Seg) * nprob, hipMemcpyHostToDevice, s));
  }
  GP_TRY(launch_init(D, D.b, nullptr, false, s));
  if (o.x0_given) {
    GP_TRY(launch_gather(D, 1, D.x, s));
    GP_TRY(launch_colmax(D, D.x, s));
    GP_TRY(launch_quant(D, D.x, o.scale_mode, nullptr, s));
    GP_TRY(launch_product(D, D.x, D.q, nullptr, s));
  }
  GP_TRY(launch_init_residual(D, D.b, D.q, D.x, D.r, o.x0_given != 0, s));
  GP_TRY(launch_precond(D, s));
  GP_TRY(launch_rz(D, lse, true, o.tol, o.min_iter, s));
  GP_TRY(launch_direction(D, true, reorth, s));
  GP_TRY(launch_quant(D, D.d, o.scale_mode, D.live, s));

  // ---- iterations: poll_every iterations per captured graph ----
  std::vector<int> live(nprob);
  auto any_live = [&]() -> gp_status {
    GP_HIP(hipMemcpyAsync(live.data(), D.live, 4 * (size_t)nprob, hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    return GP_OK;
  };
  GP_TRY(any_live());
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
      for (int c = 0; c < chunk && st == GP_OK; ++c) st = iteration(D, o, lse, reorth, cs);
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
      for (int c = 0; c < chunk && st == GP_OK; ++c) st = iteration(D, o, lse, reorth, s);
    }
    launched += chunk;
    if (st == GP_OK) st = any_live();
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (cs) {
    (void)hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
  }
  if (st != GP_OK) return st;

  GP_TRY(launch_scatter(D, D.x, s));
  if (o.true_res_every >= 0) GP_TRY(launch_true_residual(D, s));
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
      if (S.converged) S.converged[c] = (int8_t)hs[p].converged[c];
      if (S.breakdown) S.breakdown[c] = (int8_t)hs[p].breakdown[c];
    }
    S.total_iters = hs[p].k;
    S.mvms = hs[p].k + (o.x0_given ? 1 : 0);
  }
  if (broke == cols) return set_error(GP_ERR_BREAKDOWN, "every column broke down");
  return GP_OK;
}
