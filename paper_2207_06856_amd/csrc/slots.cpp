// Slot regions and launch-set tables shared by the batched solve and the
// serving loop.

#include <algorithm>

#include "batched.h"
#include "valu_tile.h"

namespace gpmi {
namespace bt {
namespace {

int splits_for(int64_t n_pad_c) {
  const int64_t stages = n_pad_c / f16::kStageCols;
  return (int)std::max<int64_t>(1, std::min<int64_t>(8, stages / tune::bt_split_div()));
}

int splits64_for(int64_t n) {
  const int64_t stages = ceil_div(n, (int64_t)valu::JT64);
  return (int)std::max<int64_t>(1, std::min<int64_t>(8, stages / 16));
}

// Sub-allocator over a region; with base == nullptr it only measures.
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(int64_t count) {
    const size_t bytes = ((size_t)std::max<int64_t>(count, 0) * sizeof(T) + 255) & ~size_t(255);
    T* p = (base && count > 0) ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

size_t layout(const SlotSpec& q, void* base, Seg* g) {
  Seg s{};
  s.n = q.n;
  s.d = q.d;
  s.r = q.r;
  s.rb = (int)ceil_div(q.r, 16);
  s.rp = 16 * s.rb;
  s.w = f16::aug_width(q.d);
  s.kc = s.w / 32;
  s.kind = q.kp.kind;
  s.a2 = q.kp.a2;
  s.s2 = q.kp.s2;
  for (int m = 0; m < kMaxDim; ++m) s.ls[m] = q.kp.ls[m];
  s.rank = q.rank;
  s.n_pad_r = round_up(q.n, f16::kRowsPerBlock);
  s.n_pad_c = round_up(q.n, f16::kStageCols);
  s.nsplit = splits_for(s.n_pad_c);
  s.nsplit64 = splits64_for(q.n);
  s.nchunk = (int)ceil_div(q.n, kChunkRows);
  s.max_iter = q.max_iter;
  s.min_iter = q.min_iter;
  s.tol = q.tol;
  const int64_t nr = q.n * q.r;
  const int64_t mb = (int64_t)q.max_iter + 1;
  const int64_t k = q.rank;
  Carver c{static_cast<char*>(base)};
  if (q.own_io) {
    s.X = c.take<float>(q.n * q.d);
    s.v[VB] = c.take<float>(nr);
    s.v[VX] = c.take<float>(nr);
  }
  s.v[VR] = c.take<float>(nr);
  s.v[VZ] = c.take<float>(nr);
  s.v[VD] = c.take<float>(nr);
  s.v[VQ] = c.take<float>(nr);
  if (q.reorth) {
    s.Ub = c.take<float>(mb * nr);
    if (k > 0) s.Wb = c.take<float>(mb * nr);
    s.coef = c.take<float>(mb * q.r);
    s.pcoef = c.take<float>(s.nchunk * mb * q.r);
    s.pgram = c.take<float>(s.nchunk * mb * q.r);
    s.c1 = c.take<float>(mb * q.r);
    s.gram = c.take<float>(mb * mb * q.r);
  }
  s.Xr = c.take<_Float16>(s.n_pad_r * s.w);
  s.Xc = c.take<_Float16>(s.n_pad_c * s.w);
  s.Vt = c.take<_Float16>((int64_t)s.rp * s.n_pad_c);
  s.part = c.take<float>((int64_t)s.nsplit * s.n_pad_r * s.rp);
  s.part64 = c.take<double>((int64_t)s.nsplit64 * nr);
  s.pm = c.take<float>((int64_t)s.nchunk * q.r);
  s.ps = c.take<float>((int64_t)s.nchunk * q.r);
  s.pq = c.take<double>((int64_t)s.nchunk * q.r);
  if (k > 0) {
    s.L64 = c.take<double>(k * q.n);
    s.L32 = c.take<float>(k * q.n);
    s.C = c.take<double>(k * k);
    s.Cinv = c.take<double>(k * k);
    s.diag = c.take<double>(q.n);
    s.piv = c.take<int64_t>(k);
    s.T64 = c.take<double>(k * q.r);
    s.Y32 = c.take<float>(k * q.r);
    s.ltpart = c.take<float>(s.nchunk * k * q.r);
    s.pv = c.take<double>(s.nchunk);
    s.psum = c.take<double>(s.nchunk);
    s.pi = c.take<int64_t>(s.nchunk);
  }
  if (g) *g = s;
  return c.off;
}

}  // namespace

size_t slot_bytes(const SlotSpec& q) { return layout(q, nullptr, nullptr); }

void slot_carve(const SlotSpec& q, void* base, Seg* g) { layout(q, base, g); }

void build_tab(const std::vector<Seg>& segs, const std::vector<int>& plist, HostTab* t) {
  *t = HostTab{};
  t->plist = plist;
  for (int p : plist) {
    const Seg& g = segs[p];
    for (int k = 0; k < g.nchunk; ++k)
      t->chunks.push_back(Chunk{p, k, (int64_t)k * kChunkRows,
                                std::min<int64_t>(g.n, (int64_t)(k + 1) * kChunkRows)});
    for (int64_t rb = 0; rb < g.n_pad_r / f16::kRowsPerBlock; ++rb)
      for (int sp = 0; sp < g.nsplit; ++sp) t->items.push_back(Item{p, sp, rb});
    for (int64_t rb = 0; rb < ceil_div(g.n, (int64_t)valu::aug_rows(trueres_slices_of(g.d))); ++rb)
      for (int sp = 0; sp < g.nsplit64; ++sp) t->items64.push_back(Item{p, sp, rb});
    const int tk = (g.rank + 15) / 16;
    for (int a = 0; a < tk; ++a)
      for (int b = a; b < tk; ++b) t->tiles.push_back(make_int4(p, a, b, 0));
    t->rb = std::max(t->rb, g.rb);
    t->max_rank = std::max(t->max_rank, g.rank);
    t->max_r = std::max(t->max_r, g.r);
    t->max_basis = std::max(t->max_basis, g.max_iter + 1);
    t->entries += (double)g.n * (double)g.n;
  }
  // longest work first (stages per item); ties keep the slot-list order
  auto cost = [&](const Item& it) {
    const Seg& g = segs[it.p];
    const int64_t st = g.n_pad_c / f16::kStageCols;
    return (it.split + 1) * st / g.nsplit - it.split * st / g.nsplit;
  };
  std::stable_sort(t->items.begin(), t->items.end(),
                   [&](const Item& a, const Item& b) { return cost(a) > cost(b); });
  auto cost64 = [&](const Item& it) {
    const Seg& g = segs[it.p];
    const int64_t st = ceil_div(g.n, (int64_t)valu::JT64);
    return ((it.split + 1) * st / g.nsplit64 - it.split * st / g.nsplit64) *
           (int64_t)valu::aug_rows(trueres_slices_of(g.d)) * (trueres_slices_of(g.d) + 4) *
           ceil_div(g.r, 16);
  };
  std::stable_sort(t->items64.begin(), t->items64.end(),
                   [&](const Item& a, const Item& b) { return cost64(a) > cost64(b); });
}

static size_t al(size_t b) { return (b + 255) & ~size_t(255); }

size_t tab_bytes(const HostTab& t) {
  return al(sizeof(int) * std::max<size_t>(1, t.plist.size())) +
         al(sizeof(Chunk) * std::max<size_t>(1, t.chunks.size())) +
         al(sizeof(Item) * std::max<size_t>(1, t.items.size())) +
         al(sizeof(Item) * std::max<size_t>(1, t.items64.size())) +
         al(sizeof(int4) * std::max<size_t>(1, t.tiles.size()));
}

gp_status tab_upload(const HostTab& t, void* dev, Tab* out, hipStream_t s) {
  char* b = static_cast<char*>(dev);
  size_t off = 0;
  auto put = [&](const void* src, size_t bytes, size_t cap) -> gp_status {
    if (bytes) GP_HIP(hipMemcpyAsync(b + off, src, bytes, hipMemcpyHostToDevice, s));
    off += al(cap);
    return GP_OK;
  };
  Tab T;
  T.nsel = (int)t.plist.size();
  T.plist = reinterpret_cast<const int*>(b + off);
  GP_TRY(put(t.plist.data(), sizeof(int) * t.plist.size(), sizeof(int) * std::max<size_t>(1, t.plist.size())));
  T.nchunks = (int)t.chunks.size();
  T.chunks = reinterpret_cast<const Chunk*>(b + off);
  GP_TRY(put(t.chunks.data(), sizeof(Chunk) * t.chunks.size(), sizeof(Chunk) * std::max<size_t>(1, t.chunks.size())));
  T.nitems = (int)t.items.size();
  T.items = reinterpret_cast<const Item*>(b + off);
  GP_TRY(put(t.items.data(), sizeof(Item) * t.items.size(), sizeof(Item) * std::max<size_t>(1, t.items.size())));
  T.nitems64 = (int)t.items64.size();
  T.items64 = reinterpret_cast<const Item*>(b + off);
  GP_TRY(put(t.items64.data(), sizeof(Item) * t.items64.size(), sizeof(Item) * std::max<size_t>(1, t.items64.size())));
  T.ntiles = (int)t.tiles.size();
  T.tiles = reinterpret_cast<const int4*>(b + off);
  GP_TRY(put(t.tiles.data(), sizeof(int4) * t.tiles.size(), sizeof(int4) * std::max<size_t>(1, t.tiles.size())));
  T.rb = t.rb;
  T.max_rank = t.max_rank;
  T.max_r = t.max_r;
  T.max_basis = t.max_basis;
  T.entries = t.entries;
  *out = T;
  return GP_OK;
}

}  // namespace bt
}  // namespace gpmi
