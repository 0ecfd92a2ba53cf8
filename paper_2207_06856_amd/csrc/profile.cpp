// Opt-in timing of the fused kernel-matrix product: when enabled, every
// launch is bracketed by HIP events on the launch's own stream; the host reads
// the per-launch durations after synchronising.

#include <mutex>
#include <vector>

#include "internal.h"

namespace gpmi {
namespace prof {

namespace {
struct Rec {
  hipEvent_t a, b;
  double entries;
  int kind;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool enabled() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_on;
}

void* begin(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return nullptr;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return nullptr;   // launches inside a captured graph are not timed
  hipEvent_t e = take();
  if (e && hipEventRecord(e, s) != hipSuccess) return nullptr;
  return e;
}

void end(void* token, hipStream_t s, double entries, int kind) {
  if (!token) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t e = take();
  if (!e || hipEventRecord(e, s) != hipSuccess) return;
  g_recs.push_back(Rec{static_cast<hipEvent_t>(token), e, entries, kind});
}

}  // namespace prof
}  // namespace gpmi

using namespace gpmi::prof;

extern "C" gp_status gp_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  return GP_OK;
}

extern "C" gp_status gp_profile_read(int64_t max_records, float* ms, double* entries,
                                     int32_t* kinds, int64_t* count) {
  gpmi::clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  if (count) *count = (int64_t)g_recs.size();
  const int64_t m = std::min<int64_t>(max_records, (int64_t)g_recs.size());
  for (int64_t i = 0; i < m; ++i) {
    const Rec& r = g_recs[i];
    float t = 0.0f;
    GP_HIP(hipEventSynchronize(r.b));
    GP_HIP(hipEventElapsedTime(&t, r.a, r.b));
    if (ms) ms[i] = t;
    if (entries) entries[i] = r.entries;
    if (kinds) kinds[i] = r.kind;
  }
  return GP_OK;
}

extern "C" gp_status gp_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (Rec& r : g_recs) {
    (void)hipEventSynchronize(r.b);
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return GP_OK;
}
