// gp_kmvm: the kernel matrix x multi-vector product behind the C ABI.

#include <math.h>

#include <algorithm>
#include <mutex>

#include "internal.h"

namespace gpmi {

namespace {
__global__ void fill_f32_kernel(float* p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
}  // namespace

gp_status fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n == 0) return GP_OK;
  fill_f32_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(p, n, v);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// Where a product's scratch comes from: the per-stream workspace (allocated
// and grown on demand), or a fixed caller-side block that nothing may grow.
struct ScratchSource {
  char* fixed = nullptr;     // nullptr: the stream workspace
  size_t fixed_cap = 0;
};

// Scratch bytes of the 16-bit product for a split count.
static size_t f16_bytes(int64_t n1_pad, int64_t n2_pad, int w, int rp_max, int nsplit) {
  return 2 * (size_t)n1_pad * w + 2 * (size_t)n2_pad * w + 2 * (size_t)rp_max * n2_pad +
         4 * (size_t)nsplit * n1_pad * rp_max + 12 * (size_t)rp_max + 8 * 256;
}

// The split count of the rule, or with a fixed block the largest count up to
// it whose scratch fits (fewer splits change only the order of float32 sums).
static gp_status pick_splits(const ScratchSource& src, int rule,
                             size_t (*bytes_of)(int64_t, int64_t, int, int, int), int64_t a,
                             int64_t b, int c, int e, int* nsplit, size_t* bytes) {
  int ns = rule;
  if (src.fixed)
    while (ns > 1 && bytes_of(a, b, c, e, ns) > src.fixed_cap) --ns;
  *nsplit = ns;
  *bytes = bytes_of(a, b, c, e, ns);
  if (src.fixed && *bytes > src.fixed_cap)
    return set_error(GP_ERR_TOO_LARGE,
                     "the product needs %zu bytes of scratch even with one column split; the "
                     "allocation-free entry point has %zu",
                     *bytes, src.fixed_cap);
  return GP_OK;
}

static gp_status scratch_arena(const ScratchSource& src, hipStream_t s, size_t bytes, Arena* ar) {
  if (!src.fixed) return workspace_get(s, bytes, ar);
  ar->base = src.fixed;
  ar->cap = src.fixed_cap;
  ar->off = 0;
  return GP_OK;
}

// The binary16 product of one point set in its symmetric form (r <= 16,
// operand width 32).  Its partial sums take n^2 R 4 / (2 panel) bytes; when
// that workspace cannot be allocated, *no_room is set (nothing is enqueued)
// and the caller runs the one-sided product, whose workspace is O(n).
static gp_status kmvm_f16_sym(const KParams& kp, const float* X, int64_t n, const float* V, int r,
                              float* out, bool add_noise, int scale_mode, hipStream_t s,
                              bool* no_room) {
  const int w = f16::aug_width(kp.d);
  const int64_t n_pad = f16::sym_pad(n);
  f16::SymPlan pl = f16::sym_plan(n_pad);
  const size_t bytes = 2 * 2 * (size_t)n_pad * w + 2 * 16 * (size_t)n_pad + f16::sym_bytes(pl) +
                       12 * 16 + 8 * 256;
  Arena ar;
  *no_room = false;
  if (workspace_get(s, bytes, &ar) == GP_ERR_NOMEM) {
    clear_error();
    *no_room = true;
    return GP_OK;
  }
  _Float16* Xr = ar.take<_Float16>((size_t)n_pad * w);
  _Float16* Xc = ar.take<_Float16>((size_t)n_pad * w);
  _Float16* Vt = ar.take<_Float16>((size_t)16 * n_pad);
  uint32_t* colmax = ar.take<uint32_t>(16);
  float* scale = ar.take<float>(16);
  float* inv_scale = ar.take<float>(16);
  if (!inv_scale) return set_error(GP_ERR_NOMEM, "internal: workspace sizing");
  GP_TRY(f16::sym_carve(pl, ar));
  GP_TRY(f16::sym_prepare(pl, s));
  GP_TRY(f16::prep_points(X, n, n_pad, kp, 0, Xr, s));
  GP_TRY(f16::prep_points(X, n, n_pad, kp, 1, Xc, s));
  const float fs = (float)(1.0 / sqrt((double)n));
  const float fi = (float)sqrt((double)n);
  GP_TRY(f16::quant_rhs(V, n, r, r, 16, n_pad, scale_mode, fs, fi, colmax, Vt, scale, inv_scale,
                        s));
  GP_TRY(f16::sym_launch(kp.kind, pl, Xr, Xc, Vt, nullptr, (double)n * (double)n, s));
  return f16::sym_reduce(pl, n, r, inv_scale, kp.a2, kp.s2, add_noise ? V : nullptr, r, out, r,
                         nullptr, s);
}

// FP16 product over already-validated arguments; columns in chunks of 64.
static gp_status kmvm_f16(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                          int64_t n2, const float* V, int r, float* out, bool add_noise,
                          int scale_mode, hipStream_t s, const ScratchSource& src) {
  const int w = f16::aug_width(kp.d);
  const int kc = w / 32;
  const int64_t n1_pad = round_up(n1, f16::kRowsPerBlock);
  const int64_t n2_pad = round_up(std::max<int64_t>(n2, 1), f16::kStageCols);
  const int rchunk = std::min(r, 64);
  const int rp_max = (int)round_up(rchunk, 16);
  if (!src.fixed && X1 == X2 && n1 == n2 && n1 >= f16::kSymMinN && f16::sym_supported(kp.d, r)) {
    bool no_room = false;
    GP_TRY(kmvm_f16_sym(kp, X1, n1, V, r, out, add_noise, scale_mode, s, &no_room));
    if (!no_room) return GP_OK;
  }
  int nsplit;
  size_t bytes;
  GP_TRY(pick_splits(src, f16::choose_splits(n1_pad, n2_pad), f16_bytes, n1_pad, n2_pad, w,
                     rp_max, &nsplit, &bytes));
  Arena ar;
  GP_TRY(scratch_arena(src, s, bytes, &ar));
  _Float16* Xr = ar.take<_Float16>((size_t)n1_pad * w);
  _Float16* Xc = ar.take<_Float16>((size_t)n2_pad * w);
  _Float16* Vt = ar.take<_Float16>((size_t)rp_max * n2_pad);
  float* part = ar.take<float>((size_t)nsplit * n1_pad * rp_max);
  uint32_t* colmax = ar.take<uint32_t>(rp_max);
  float* scale = ar.take<float>(rp_max);
  float* inv_scale = ar.take<float>(rp_max);
  if (!inv_scale) return set_error(GP_ERR_NOMEM, "internal: workspace sizing");

  GP_TRY(f16::prep_points(X1, n1, n1_pad, kp, 0, Xr, s));
  GP_TRY(f16::prep_points(X2, n2, n2_pad, kp, 1, Xc, s));
  const float fs = (float)(1.0 / sqrt((double)std::max<int64_t>(n2, 1)));
  const float fi = (float)sqrt((double)std::max<int64_t>(n2, 1));
  for (int c0 = 0; c0 < r; c0 += 64) {
    const int rc = std::min(64, r - c0);
    const int rb = (int)ceil_div(rc, 16);
    const int rp = 16 * rb;
    GP_TRY(f16::quant_rhs(V + c0, n2, rc, r, rp, n2_pad, scale_mode, fs, fi, colmax, Vt, scale,
                          inv_scale, s));
    GP_TRY(f16::launch_main(kp.kind, kc, rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, nullptr,
                             (double)n1 * (double)n2, s));
    GP_TRY(f16::launch_reduce(part, nsplit, n1, n1_pad, rc, rp, inv_scale, kp.a2, kp.s2,
                              add_noise ? V + c0 : nullptr, r, out + c0, r, nullptr, s));
  }
  return GP_OK;
}

// bfloat16 product over already-validated arguments; columns in chunks of 64.
static gp_status kmvm_bf16(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                           int64_t n2, const float* V, int r, float* out, bool add_noise,
                           int scale_mode, hipStream_t s, const ScratchSource& src) {
  const int w = f16::aug_width_bf16(kp.d);
  const int kc = w / 32;
  const int64_t n1_pad = round_up(n1, f16::kRowsPerBlock);
  const int64_t n2_pad = round_up(std::max<int64_t>(n2, 1), f16::kStageCols);
  const int rchunk = std::min(r, 64);
  const int rp_max = (int)round_up(rchunk, 16);
  int nsplit;
  size_t bytes;
  GP_TRY(pick_splits(src, f16::choose_splits(n1_pad, n2_pad), f16_bytes, n1_pad, n2_pad, w,
                     rp_max, &nsplit, &bytes));
  Arena ar;
  GP_TRY(scratch_arena(src, s, bytes, &ar));
  __bf16* Xr = ar.take<__bf16>((size_t)n1_pad * w);
  __bf16* Xc = ar.take<__bf16>((size_t)n2_pad * w);
  __bf16* Vt = ar.take<__bf16>((size_t)rp_max * n2_pad);
  float* part = ar.take<float>((size_t)nsplit * n1_pad * rp_max);
  uint32_t* colmax = ar.take<uint32_t>(rp_max);
  float* scale = ar.take<float>(rp_max);
  float* inv_scale = ar.take<float>(rp_max);
  if (!inv_scale) return set_error(GP_ERR_NOMEM, "internal: workspace sizing");

  GP_TRY(f16::prep_points_bf16(X1, n1, n1_pad, kp, 0, Xr, s));
  GP_TRY(f16::prep_points_bf16(X2, n2, n2_pad, kp, 1, Xc, s));
  const float fs = (float)(1.0 / sqrt((double)std::max<int64_t>(n2, 1)));
  const float fi = (float)sqrt((double)std::max<int64_t>(n2, 1));
  for (int c0 = 0; c0 < r; c0 += 64) {
    const int rc = std::min(64, r - c0);
    const int rb = (int)ceil_div(rc, 16);
    const int rp = 16 * rb;
    GP_TRY(f16::quant_rhs(V + c0, n2, rc, r, rp, n2_pad, scale_mode, fs, fi, colmax, Vt, scale,
                          inv_scale, s));
    GP_TRY(f16::launch_main_bf16(kp.kind, kc, rb, Xr, Xc, Vt, part, n1_pad, n2_pad, nsplit, nullptr,
                                 (double)n1 * (double)n2, s));
    GP_TRY(f16::launch_reduce(part, nsplit, n1, n1_pad, rc, rp, inv_scale, kp.a2, kp.s2,
                              add_noise ? V + c0 : nullptr, r, out + c0, r, nullptr, s));
  }
  return GP_OK;
}

static size_t f32_bytes(int64_t n1, int64_t, int r, int, int nsplit) {
  return 4 * (size_t)nsplit * n1 * r + 256;
}

static gp_status kmvm_f32(const KParams& kp, const float* X1, int64_t n1, const float* X2,
                          int64_t n2, const float* V, int r, float* out, bool add_noise,
                          hipStream_t s, const ScratchSource& src) {
  int nsplit;
  size_t bytes;
  GP_TRY(pick_splits(src, valu::choose_splits(n1, n2, kp.d), f32_bytes, n1, n2, r, 0, &nsplit,
                     &bytes));
  Arena ar;
  GP_TRY(scratch_arena(src, s, bytes, &ar));
  float* part = ar.take<float>((size_t)nsplit * n1 * r);
  if (!part) return set_error(GP_ERR_NOMEM, "internal: workspace sizing");
  GP_TRY(valu::launch_partial(kp, X1, n1, X2, n2, V, r, part, false, nsplit, nullptr, s));
  return valu::launch_reduce32(part, nsplit, n1, r, kp.a2, kp.s2, add_noise ? V : nullptr, out,
                               nullptr, s);
}

}  // namespace gpmi

using namespace gpmi;

// ---- allocation-free variant ----------------------------------------------
// One fixed scratch block per device, for callers that cannot allocate.  In
// host code `scratch` names a host-side stand-in, not device memory: kernels
// only ever receive the device address that hipGetSymbolAddress returns for
// the current device (each device holds its own copy of the array).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch block (looked up once per device).
gp_status noalloc_scratch(char** out) {
  int dev = 0;
  GP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(GP_ERR_ARG, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(GP_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                       hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return GP_OK;
}
}  // namespace

static gp_status kmvm_common(const gp_kernel* k, const float* X1, int64_t n1, const float* X2,
                             int64_t n2, int32_t d, const float* V, int32_t r, float* out,
                             int32_t add_noise, int32_t precision, int32_t scale_mode,
                             void* stream, bool no_alloc) {
  clear_error();
  KParams kp;
  GP_TRY(check_kernel(k, d, false, &kp));
  if (n1 < 0 || n2 < 0) return set_error(GP_ERR_ARG, "negative point count");
  if (r < 1) return set_error(GP_ERR_ARG, "r=%d must be >= 1", r);
  if (precision != GP_PREC_FP32 && precision != GP_PREC_FP16 && precision != GP_PREC_BF16)
    return set_error(GP_ERR_ARG, "precision must be GP_PREC_FP32, GP_PREC_FP16 or GP_PREC_BF16");
  if (scale_mode != 0 && scale_mode != 1) return set_error(GP_ERR_ARG, "scale_mode must be 0 or 1");
  if (n1 > 0 && (!X1 || !out)) return set_error(GP_ERR_ARG, "X1/out is NULL");
  if (n2 > 0 && (!X2 || !V)) return set_error(GP_ERR_ARG, "X2/V is NULL");
  if (add_noise && (X1 != X2 || n1 != n2))
    return set_error(GP_ERR_ARG, "add_noise needs X1 == X2 and n1 == n2");
  const size_t ob = (size_t)n1 * r * 4;
  if (overlaps(out, ob, V, (size_t)n2 * r * 4) || overlaps(out, ob, X1, (size_t)n1 * d * 4) ||
      overlaps(out, ob, X2, (size_t)n2 * d * 4))
    return set_error(GP_ERR_ARG, "out overlaps an input");
  if (n1 == 0) return GP_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n2 == 0) return fill_f32(out, n1 * r, 0.0f, s);
  ScratchSource src;
  if (no_alloc) {
    GP_TRY(noalloc_scratch(&src.fixed));
    src.fixed_cap = kNoAllocScratchBytes;
  }
  if (precision == GP_PREC_FP16)
    return kmvm_f16(kp, X1, n1, X2, n2, V, r, out, add_noise != 0, scale_mode, s, src);
  if (precision == GP_PREC_BF16)
    return kmvm_bf16(kp, X1, n1, X2, n2, V, r, out, add_noise != 0, scale_mode, s, src);
  return kmvm_f32(kp, X1, n1, X2, n2, V, r, out, add_noise != 0, s, src);
}

extern "C" gp_status gp_kmvm(const gp_kernel* k, const float* X1, int64_t n1, const float* X2,
                             int64_t n2, int32_t d, const float* V, int32_t r, float* out,
                             int32_t add_noise, int32_t precision, int32_t scale_mode,
                             void* stream) {
  return kmvm_common(k, X1, n1, X2, n2, d, V, r, out, add_noise, precision, scale_mode, stream,
                     false);
}

extern "C" gp_status gp_kmvm_noalloc(const gp_kernel* k, const float* X1, int64_t n1,
                                     const float* X2, int64_t n2, int32_t d, const float* V,
                                     int32_t r, float* out, int32_t add_noise, int32_t precision,
                                     int32_t scale_mode, void* stream) {
  return kmvm_common(k, X1, n1, X2, n2, d, V, r, out, add_noise, precision, scale_mode, stream,
                     true);
}

extern "C" uint64_t gp_kmvm_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }
