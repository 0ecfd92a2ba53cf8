// Error state, workspace cache and argument checks shared by the C ABI.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <map>
#include <mutex>
#include <utility>

#include "internal.h"

namespace gpmi {

static thread_local std::string t_error;

gp_status set_error(gp_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_error = buf;
  return st;
}

void clear_error() { t_error.clear(); }

namespace {
struct Block {
  void* ptr = nullptr;
  size_t cap = 0;
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Block> g_ws;
}  // namespace

namespace {
std::mutex g_bc_mu;
std::multimap<std::pair<int, size_t>, void*> g_bc;
size_t g_bc_total = 0;
}  // namespace

gp_status block_cache_get(size_t bytes, void** out) {
  *out = nullptr;
  int dev = 0;
  GP_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_bc_mu);
    auto it = g_bc.find({dev, bytes});
    if (it != g_bc.end()) {
      *out = it->second;
      g_bc.erase(it);
      g_bc_total -= bytes;
      return GP_OK;
    }
  }
  if (hipMalloc(out, bytes) != hipSuccess) {
    // the cached blocks of other sizes may be what is missing: release them
    // and try once more
    (void)hipGetLastError();
    *out = nullptr;
    if (block_cache_release() == 0) return set_error(GP_ERR_NOMEM, "cannot allocate %zu bytes", bytes);
    if (hipMalloc(out, bytes) != hipSuccess) {
      (void)hipGetLastError();
      *out = nullptr;
      return set_error(GP_ERR_NOMEM, "cannot allocate %zu bytes", bytes);
    }
  }
  return GP_OK;
}

size_t block_cache_release() {
  std::multimap<std::pair<int, size_t>, void*> drop;
  {
    std::lock_guard<std::mutex> lk(g_bc_mu);
    drop.swap(g_bc);
    g_bc_total = 0;
  }
  size_t freed = 0;
  for (auto& e : drop) {
    (void)hipFree(e.second);
    freed += e.first.second;
  }
  return freed;
}

void block_cache_put(int device, void* p, size_t bytes) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(g_bc_mu);
    if (g_bc_total + bytes <= kBlockCacheBytes) {
      g_bc.insert({{device, bytes}, p});
      g_bc_total += bytes;
      return;
    }
  }
  (void)hipFree(p);
}

size_t workspace_release() {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) cur = -1;
  size_t freed = 0;
  for (auto& e : g_ws) {
    if (!e.second.ptr) continue;
    // the stream may already be destroyed: wait for the whole device instead
    if (hipSetDevice(e.first.first) == hipSuccess && hipDeviceSynchronize() == hipSuccess) {
      (void)hipFree(e.second.ptr);
      freed += e.second.cap;
    }
    (void)hipGetLastError();
  }
  g_ws.clear();
  if (cur >= 0) (void)hipSetDevice(cur);
  return freed;
}

gp_status workspace_get(hipStream_t s, size_t bytes, Arena* out) {
  int dev = 0;
  GP_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ws_mu);
  Block& b = g_ws[{dev, s}];
  // a block far larger than what is asked for (left by a very large problem)
  // is given back rather than held for the rest of the process
  const bool oversized = b.cap > (size_t(16) << 30) && bytes < b.cap / 4;
  if (b.cap < bytes || oversized) {
    if (b.ptr) {
      GP_HIP(hipStreamSynchronize(s));
      GP_HIP(hipFree(b.ptr));
      b.ptr = nullptr;
      b.cap = 0;
    }
    // a quarter of slack lets a slightly larger next request reuse the block;
    // when that does not fit, the exact size is tried before giving up
    size_t want = bytes + bytes / 4 + (1u << 20);
    void* p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      want = bytes;
      if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(GP_ERR_NOMEM, "cannot allocate %zu bytes of workspace", want);
      }
    }
    b.ptr = p;
    b.cap = want;
  }
  out->base = static_cast<char*>(b.ptr);
  out->cap = b.cap;
  out->off = 0;
  return GP_OK;
}

gp_status check_kernel(const gp_kernel* k, int32_t d, bool need_noise, KParams* kp) {
  if (!k) return set_error(GP_ERR_ARG, "kernel parameters are NULL");
  if (d < 1 || d > kMaxDim) return set_error(GP_ERR_ARG, "d=%d outside [1, %d]", d, kMaxDim);
  if (k->kind < GP_KERNEL_RBF || k->kind > GP_KERNEL_MATERN32)
    return set_error(GP_ERR_ARG, "unknown kernel kind %d", k->kind);
  if (!k->lengthscale) return set_error(GP_ERR_ARG, "lengthscale is NULL");
  if (!(isfinite(k->outputscale) && k->outputscale > 0.0f))
    return set_error(GP_ERR_ARG, "outputscale must be finite and > 0");
  if (!(isfinite(k->noise) && k->noise >= 0.0f))
    return set_error(GP_ERR_ARG, "noise must be finite and >= 0");
  if (need_noise && !(k->noise > 0.0f))
    return set_error(GP_ERR_ARG, "noise must be > 0 for a solve or preconditioner");
  kp->kind = k->kind;
  kp->d = d;
  kp->a2 = k->outputscale;
  kp->s2 = k->noise;
  for (int m = 0; m < kMaxDim; ++m) kp->ls[m] = 1.0f;
  for (int m = 0; m < d; ++m) {
    const float l = k->ard ? k->lengthscale[m] : k->lengthscale[0];
    if (!(isfinite(l) && l > 0.0f))
      return set_error(GP_ERR_ARG, "lengthscale[%d] must be finite and > 0", k->ard ? m : 0);
    kp->ls[m] = l;
  }
  return GP_OK;
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  if (!a || !b || abytes == 0 || bbytes == 0) return false;
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + bbytes && pb < pa + abytes;
}

}  // namespace gpmi

extern "C" const char* gp_last_error(void) { return gpmi::t_error.c_str(); }

extern "C" const char* gp_version(void) { return "gpmi 0.1.0 gfx950"; }

extern "C" gp_status gp_release_cached_memory(uint64_t* bytes_freed) {
  gpmi::clear_error();
  const size_t a = gpmi::block_cache_release();
  const size_t b = gpmi::workspace_release();
  if (bytes_freed) *bytes_freed = (uint64_t)(a + b);
  return GP_OK;
}
