// Autotuner: launch-shape decisions of the binary16 product, measured on the
// device with synthetic operands and installed in a process-wide table.
//
//   single-problem product: column splits per row-count bucket (the split is
//     the XCD-aware column partition of kmvm_f16_main; more splits mean more
//     work groups and more partial-sum traffic);
//   batched product: the per-problem split rule, splits = clamp(stages / div,
//     1, 8), and the launch form (one work group per item, or one persistent
//     launch pulling items from an atomic counter).
//
// Until gp_autotune runs, every lookup returns the built-in rule, so results
// are reproducible run to run; tuned decisions change only the order of the
// float32 partial sums, not what is computed.  With GPMI_TUNE_CACHE set to a
// file path the table is loaded from that file at first use and written by
// gp_autotune.

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <vector>

#include "internal.h"

namespace gpmi {
namespace tune {
namespace {

struct Table {
  int tuned = 0;
  int f16_splits[kBuckets] = {0};   // 0: built-in rule
  double f16_gain[kBuckets] = {0};
  int bt_split_div = 16;
  int bt_persistent = 0;
  double bt_gain = 0.0;
};

std::mutex g_mu;
Table g_table;
bool g_loaded = false;
thread_local const Table* t_override = nullptr;

void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = getenv("GPMI_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  Table t;
  char key[64];
  double v;
  while (fscanf(f, "%63s %lf", key, &v) == 2) {
    int b;
    if (sscanf(key, "f16_splits_%d", &b) == 1 && b >= 0 && b < kBuckets) t.f16_splits[b] = (int)v;
    else if (sscanf(key, "f16_gain_%d", &b) == 1 && b >= 0 && b < kBuckets) t.f16_gain[b] = v;
    else if (!strcmp(key, "bt_split_div")) t.bt_split_div = std::max(1, (int)v);
    else if (!strcmp(key, "bt_persistent")) t.bt_persistent = v != 0.0;
    else if (!strcmp(key, "bt_gain")) t.bt_gain = v;
    else if (!strcmp(key, "tuned")) t.tuned = v != 0.0;
  }
  fclose(f);
  g_table = t;
}

void save_locked() {
  const char* path = getenv("GPMI_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "w");
  if (!f) return;
  fprintf(f, "tuned %d\n", g_table.tuned);
  for (int b = 0; b < kBuckets; ++b)
    fprintf(f, "f16_splits_%d %d\nf16_gain_%d %.6f\n", b, g_table.f16_splits[b], b, g_table.f16_gain[b]);
  fprintf(f, "bt_split_div %d\nbt_persistent %d\nbt_gain %.6f\n", g_table.bt_split_div,
          g_table.bt_persistent, g_table.bt_gain);
  fclose(f);
}

Table snapshot() {
  if (t_override) return *t_override;
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  return g_table;
}

__global__ void hash_fill_kernel(float* p, int64_t n, uint32_t seed, float lo, float hi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t x = (uint32_t)i * 2654435761u ^ seed;
  x ^= x >> 15;
  x *= 2246822519u;
  x ^= x >> 13;
  x *= 3266489917u;
  x ^= x >> 16;
  p[i] = lo + (hi - lo) * (float)(x >> 8) * (1.0f / 16777216.0f);
}

gp_status hash_fill(float* p, int64_t n, uint32_t seed, float lo, float hi, hipStream_t s) {
  hash_fill_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(p, n, seed, lo, hi);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// Smallest device time of one call of f over `reps` timed calls, after one
// warm-up call (the minimum is the least noisy estimate of a kernel's cost).
template <class F>
gp_status time_calls(F f, int reps, hipStream_t s, double* ms_out) {
  GP_TRY(f());
  hipEvent_t a, b;
  GP_HIP(hipEventCreate(&a));
  GP_HIP(hipEventCreate(&b));
  gp_status st = GP_OK;
  double best = 1e30;
  for (int i = 0; i < reps && st == GP_OK; ++i) {
    GP_HIP(hipEventRecord(a, s));
    st = f();
    GP_HIP(hipEventRecord(b, s));
    GP_HIP(hipEventSynchronize(b));
    float ms = 0.0f;
    GP_HIP(hipEventElapsedTime(&ms, a, b));
    best = std::min(best, (double)ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms_out = best;
  return st;
}

// A candidate replaces the built-in rule only when it is this much faster.
constexpr double kMinGain = 1.02;

struct DevBlock {
  void* p = nullptr;
  ~DevBlock() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

int64_t bucket_rows(int b) { return (int64_t)4096 << b; }

int bucket_of(int64_t n1_pad) {
  int b = 0;
  while (b + 1 < kBuckets && bucket_rows(b + 1) <= n1_pad) ++b;
  return b;
}

int f16_splits(int64_t n1_pad, int64_t n2_pad, int fallback) {
  const Table t = snapshot();
  const int v = t.f16_splits[bucket_of(n1_pad)];
  if (v <= 0) return fallback;
  return (int)std::max<int64_t>(1, std::min<int64_t>(v, n2_pad / f16::kStageCols));
}

int bt_split_div() { return snapshot().bt_split_div; }
bool bt_persistent() { return snapshot().bt_persistent != 0; }

}  // namespace tune
}  // namespace gpmi

using namespace gpmi;
using namespace gpmi::tune;

static void fill_info(const Table& t, gp_tune_info* out) {
  if (!out) return;
  memset(out, 0, sizeof(*out));
  out->tuned = t.tuned;
  for (int b = 0; b < kBuckets; ++b) {
    out->f16_splits[b] = t.f16_splits[b];
    out->f16_bucket_rows[b] = bucket_rows(b);
    out->f16_gain[b] = t.f16_gain[b];
  }
  out->batched_split_div = t.bt_split_div;
  out->batched_persistent = t.bt_persistent;
  out->batched_gain = t.bt_gain;
}

extern "C" gp_status gp_tune_get(gp_tune_info* out) {
  clear_error();
  if (!out) return set_error(GP_ERR_ARG, "out is NULL");
  fill_info(snapshot(), out);
  return GP_OK;
}

extern "C" gp_status gp_tune_reset(void) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  g_loaded = true;   // defaults, and do not reload the cache file
  g_table = Table{};
  return GP_OK;
}

extern "C" gp_status gp_tune_set(const gp_tune_info* in) {
  clear_error();
  if (!in) return set_error(GP_ERR_ARG, "in is NULL");
  Table t;
  for (int b = 0; b < kBuckets; ++b) {
    if (in->f16_splits[b] < 0 || in->f16_splits[b] > 64)
      return set_error(GP_ERR_ARG, "f16_splits[%d] = %d outside [0, 64]", b, in->f16_splits[b]);
    t.f16_splits[b] = in->f16_splits[b];
    t.f16_gain[b] = in->f16_gain[b];
  }
  if (in->batched_split_div < 1 || in->batched_split_div > 1024)
    return set_error(GP_ERR_ARG, "batched_split_div outside [1, 1024]");
  t.bt_split_div = in->batched_split_div;
  t.bt_persistent = in->batched_persistent != 0;
  t.bt_gain = in->batched_gain;
  t.tuned = in->tuned != 0;
  std::lock_guard<std::mutex> lk(g_mu);
  g_loaded = true;
  g_table = t;
  return GP_OK;
}

extern "C" gp_status gp_autotune(int32_t max_bucket, void* stream, gp_tune_info* out) {
  clear_error();
  if (max_bucket < 0 || max_bucket >= kBuckets)
    return set_error(GP_ERR_ARG, "max_bucket outside [0, %d]", kBuckets - 1);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Table t = snapshot();

  // ---- single-problem product: splits per bucket (RBF, d = 8, 16 right-hand sides)
  {
    // each bucket is timed at sqrt(2) times its lower edge (its geometric middle)
    const int64_t nmax = bucket_rows(max_bucket) * 3 / 2;
    const int d = 8, r = 16;
    DevBlock mem;
    const size_t bytes = sizeof(float) * ((size_t)nmax * d + 2 * (size_t)nmax * r);
    GP_HIP(hipMalloc(&mem.p, bytes));
    float* X = static_cast<float*>(mem.p);
    float* V = X + (size_t)nmax * d;
    float* O = V + (size_t)nmax * r;
    GP_TRY(hash_fill(X, nmax * d, 17u, -2.0f, 2.0f, s));
    GP_TRY(hash_fill(V, nmax * r, 29u, -1.0f, 1.0f, s));
    float ls = 1.0f;
    gp_kernel k{GP_KERNEL_RBF, 0, &ls, 1.0f, 0.05f};
    for (int b = 0; b <= max_bucket; ++b) {
      const int64_t n = (int64_t)llround((double)bucket_rows(b) * 1.41421356);
      const int stages = (int)(round_up(n, f16::kStageCols) / f16::kStageCols);
      const int cands[] = {8, 16, 24, 32, 48, 64};
      Table probe = t;
      double best = 1e30, base = 0.0;
      int best_s = 0;
      for (int ci = -1; ci < (int)(sizeof cands / sizeof cands[0]); ++ci) {
        const int sp = ci < 0 ? 0 : cands[ci];
        if (sp > stages) continue;
        probe.f16_splits[b] = sp;
        t_override = &probe;
        double ms = 0.0;
        const gp_status st = time_calls(
            [&]() { return gp_kmvm(&k, X, n, X, n, d, V, r, O, 1, GP_PREC_FP16, 0, s); }, 5, s, &ms);
        t_override = nullptr;
        if (st != GP_OK) return st;
        if (ci < 0) base = ms;
        if (ms < best) {
          best = ms;
          best_s = sp;
        }
      }
      if (best_s != 0 && base < kMinGain * best) {   // not clearly better than the rule
        best_s = 0;
        best = base;
      }
      t.f16_splits[b] = best_s;
      t.f16_gain[b] = best > 0.0 ? base / best : 1.0;
    }
  }

  // ---- batched product: split rule and launch form on 48 uneven problems
  {
    const int np = 48, r = 8;
    std::vector<int64_t> ns(np);
    std::vector<int> ds(np);
    for (int p = 0; p < np; ++p) {
      // log-uniform n in [500, 20000] on a fixed grid; d in {4, 8, 12}
      ns[p] = (int64_t)llround(500.0 * pow(40.0, (p + 0.5) / np));
      ds[p] = 4 + 4 * (p % 3);
    }
    DevBlock mem;
    size_t bytes = 0;
    for (int p = 0; p < np; ++p) bytes += sizeof(float) * (size_t)ns[p] * (ds[p] + 2 * r) + 256;
    GP_HIP(hipMalloc(&mem.p, bytes));
    std::vector<gp_problem> probs(np);
    float ls = 1.0f;
    char* cur = static_cast<char*>(mem.p);
    for (int p = 0; p < np; ++p) {
      float* X = reinterpret_cast<float*>(cur);
      float* B = X + (size_t)ns[p] * ds[p];
      float* U = B + (size_t)ns[p] * r;
      cur += ((sizeof(float) * (size_t)ns[p] * (ds[p] + 2 * r)) + 255) & ~size_t(255);
      GP_TRY(hash_fill(X, ns[p] * ds[p], 101u + p, -2.0f, 2.0f, s));
      GP_TRY(hash_fill(B, ns[p] * r, 701u + p, -1.0f, 1.0f, s));
      probs[p] = gp_problem{gp_kernel{GP_KERNEL_RBF, 0, &ls, 1.0f, 0.05f}, X, ns[p], ds[p], B, r, U, 0};
    }
    gp_cg_opts o;
    gp_cg_default_opts(&o);
    o.tol = 0.0;
    o.max_iter = 8;
    o.min_iter = 8;
    o.true_res_every = -1;
    o.poll_every = 8;
    const int divs[] = {8, 16, 32};
    double best = 1e30, base = 0.0;
    int best_div = t.bt_split_div, best_pers = t.bt_persistent;
    Table probe = t;
    for (int pers = 0; pers < 2; ++pers)
      for (int div : divs) {
        probe.bt_split_div = div;
        probe.bt_persistent = pers;
        t_override = &probe;
        double ms = 0.0;
        const gp_status st = time_calls(
            [&]() {
              const gp_status e = gp_cg_solve_batched(np, probs.data(), &o, nullptr, s);
              return e == GP_ERR_BREAKDOWN ? GP_OK : e;
            },
            3, s, &ms);
        t_override = nullptr;
        if (st != GP_OK) return st;
        if (div == 16 && pers == 0) base = ms;
        if (ms < best) {
          best = ms;
          best_div = div;
          best_pers = pers;
        }
      }
    if (base < kMinGain * best) {   // not clearly better than the built-in rule
      best_div = 16;
      best_pers = 0;
      best = base;
    }
    t.bt_split_div = best_div;
    t.bt_persistent = best_pers;
    t.bt_gain = best > 0.0 ? base / best : 1.0;
  }

  t.tuned = 1;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_loaded = true;
    g_table = t;
    save_locked();
  }
  fill_info(t, out);
  return GP_OK;
}
