// Context, allocator, errors, structure map (A1) and plain interval lookup (A3).
#include <algorithm>
#include <limits>
#include <map>
#include <queue>

#include "hpa_internal.h"

namespace hpa {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

void fail(hpa_status s, const std::string& msg) { throw Error{s, msg}; }

namespace {

// Release every cached block to HIP (blocks may still be in use by work in
// flight, so the device is drained first).
void drop_cache(hpa_ctx* ctx) {
  if (ctx->cache.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : ctx->cache) (void)hipFreeAsync(kv.second.p, nullptr);
  (void)hipDeviceSynchronize();
  ctx->cache.clear();
}

}  // namespace

thread_local Arena t_arena;

void* dalloc(hpa_ctx* ctx, size_t bytes, hipStream_t s, size_t* cap) {
  void* p = nullptr;
  if (t_arena.base) {
    const size_t at = (t_arena.off + 255) & ~(size_t)255;
    if (at + bytes > t_arena.size)
      fail(HPA_E_BUDGET, "the call needs more than the " + std::to_string(t_arena.size) +
                             " bytes of scratch available without allocation");
    t_arena.off = at + bytes;
    t_arena.peak = std::max(t_arena.peak, t_arena.off);
    *cap = bytes;
    return t_arena.base + at;
  }
  if (ctx->custom) {
    p = ctx->alloc.alloc(bytes, s, ctx->alloc.user);
    if (!p) fail(HPA_E_NOMEM, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
    *cap = bytes;
    return p;
  }
  // a cached block released on this stream, at most twice the request (plus
  // 1 MiB) so that small requests do not pin large blocks
  std::lock_guard<std::mutex> lk(ctx->cache_mu);
  const size_t limit = bytes * 2 + (1u << 20);
  for (auto it = ctx->cache.lower_bound(bytes); it != ctx->cache.end() && it->first <= limit; ++it) {
    if (it->second.stream != s) continue;
    p = it->second.p;
    *cap = it->first;
    ctx->cache.erase(it);
    return p;
  }
  // new blocks are rounded up to 1 MiB so that similar sizes share them
  const size_t want = bytes > (1u << 20) ? (bytes + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1) : bytes;
  hipError_t e = hipMallocAsync(&p, want, s);
  if (e == hipErrorOutOfMemory && !ctx->cache.empty()) {
    (void)hipGetLastError();
    drop_cache(ctx);
    e = hipMallocAsync(&p, want, s);
  }
  if (e == hipErrorOutOfMemory || (e == hipSuccess && !p))
    fail(HPA_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  if (e != hipSuccess) fail(HPA_E_DEVICE, std::string("hipMallocAsync: ") + hipGetErrorString(e));
  *cap = want;
  return p;
}

void dfree(hpa_ctx* ctx, void* p, size_t cap, hipStream_t s) {
  if (!p) return;
  const uint8_t* q = static_cast<const uint8_t*>(p);
  if (t_arena.base && q >= t_arena.base && q < t_arena.base + t_arena.size) return;
  if (ctx->custom) {
    ctx->alloc.free(p, s, ctx->alloc.user);
    return;
  }
  std::lock_guard<std::mutex> lk(ctx->cache_mu);
  ctx->cache.emplace(cap, hpa_ctx::Cached{p, s});
}

}  // namespace hpa

using namespace hpa;

extern "C" const char* hpa_last_error(void) { return g_last_error.c_str(); }

extern "C" hpa_status hpa_ctx_create(int device, const hpa_allocator* alloc, hpa_ctx** out) {
  return guard([&] {
    if (!out) fail(HPA_E_INVAL, "out is NULL");
    int n = 0;
    HPA_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) fail(HPA_E_INVAL, "no such device");
    if (alloc && (!alloc->alloc || !alloc->free)) fail(HPA_E_INVAL, "allocator needs alloc and free");
    DeviceGuard g(device);
    auto* c = new hpa_ctx();
    c->device = device;
    if (alloc) { c->alloc = *alloc; c->custom = true; }
    hipDeviceProp_t prop;
    HPA_HIP(hipGetDeviceProperties(&prop, device));
    c->n_cu = prop.multiProcessorCount;
    if (!alloc) {
      hipMemPool_t pool;
      HPA_HIP(hipDeviceGetDefaultMemPool(&pool, device));
      uint64_t thr = std::numeric_limits<uint64_t>::max();
      HPA_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
    }
    *out = c;
  });
}

hpa_ctx::~hpa_ctx() {
  if (custom) return;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) prev = device;
  (void)hipSetDevice(device);
  std::lock_guard<std::mutex> lk(cache_mu);
  drop_cache(this);
  (void)hipSetDevice(prev);
}

extern "C" void hpa_ctx_destroy(hpa_ctx* ctx) { delete ctx; }

extern "C" hpa_status hpa_ctx_get_sync_count(const hpa_ctx* ctx, uint64_t* out) {
  return guard([&] {
    if (!ctx || !out) fail(HPA_E_INVAL, "NULL argument");
    *out = ctx->n_syncs.load(std::memory_order_relaxed);
  });
}

extern "C" hpa_status hpa_ctx_set_timing(hpa_ctx* ctx, int enable) {
  return guard([&] {
    if (!ctx) fail(HPA_E_INVAL, "ctx is NULL");
    ctx->timing = enable != 0;
    ctx->stages.clear();
  });
}

extern "C" hpa_status hpa_ctx_get_timing(const hpa_ctx* ctx, hpa_stage_time* out, uint32_t cap, uint32_t* n_stages) {
  return guard([&] {
    if (!ctx || !n_stages || (cap && !out)) fail(HPA_E_INVAL, "NULL argument");
    const uint32_t n = (uint32_t)ctx->stages.size();
    for (uint32_t i = 0; i < n && i < cap; ++i) out[i] = ctx->stages[i];
    *n_stages = n;
  });
}

namespace hpa {

StageTimer::~StageTimer() {
  for (auto& sp : spans_) {
    (void)hipEventDestroy(sp.a);
    if (sp.b) (void)hipEventDestroy(sp.b);
  }
}

void StageTimer::begin(const char* name) {
  if (!on_) return;
  Span sp{name, nullptr, nullptr, 0, 0};
  HPA_HIP(hipEventCreate(&sp.a));
  spans_.push_back(sp);
  HPA_HIP(hipEventRecord(spans_.back().a, s_));
}

void StageTimer::end(uint64_t items_in, uint64_t items_out) {
  if (!on_ || spans_.empty()) return;
  Span& sp = spans_.back();
  HPA_HIP(hipEventCreate(&sp.b));
  HPA_HIP(hipEventRecord(sp.b, s_));
  sp.in = items_in;
  sp.out = items_out;
}

void StageTimer::items(const char* name, uint64_t items_in, uint64_t items_out) {
  for (auto& sp : spans_)
    if (!strcmp(sp.name, name)) { sp.in = items_in; sp.out = items_out; }
}

void StageTimer::collect() {
  if (!on_) return;
  for (auto& sp : spans_) {
    if (!sp.b) continue;
    float ms = 0.f;
    HPA_HIP(hipEventElapsedTime(&ms, sp.a, sp.b));
    hpa_stage_time* row = nullptr;
    for (auto& r : ctx_->stages)
      if (!strcmp(r.name, sp.name)) row = &r;
    if (!row) {
      ctx_->stages.push_back(hpa_stage_time{sp.name, 0.0, 0, 0, 0});
      row = &ctx_->stages.back();
    }
    row->ms += ms;
    row->calls += 1;
    row->items_in += sp.in;
    row->items_out += sp.out;
  }
}

}  // namespace hpa

// ---------------------------------------------------------------------------
// A1: structure map (Section 5 function relocation/splitting, line map and
// inlined code; Section 6.1 calling-context expansion).  Host sweep over the
// sorted boundaries of every range.
// ---------------------------------------------------------------------------
namespace {

struct R {
  uint64_t s, e;
  uint32_t id, kind;
};

struct Built {
  std::vector<uint64_t> start, end;
  std::vector<uint32_t> scope, file, line;
  std::vector<uint32_t> parent, func;
  std::vector<uint8_t> kind;
  uint32_t n_ids = 0;
};

void sweep(const hpa_structure_desc& d, Built& out) {
  std::vector<R> fn, nest;
  std::vector<uint8_t> kind_of;
  for (uint64_t i = 0; i < d.n_scopes; ++i) {
    const hpa_scope& s = d.scopes[i];
    if (s.start >= s.end) fail(HPA_E_INVAL, "scope " + std::to_string(i) + " has start >= end");
    if (s.kind > HPA_LOOP) fail(HPA_E_INVAL, "scope " + std::to_string(i) + " has an unknown kind");
    if (s.id >= 0x7FFFFFFFu) fail(HPA_E_INVAL, "scope id too large");
    if (s.id >= kind_of.size()) kind_of.resize((size_t)s.id + 1, 0xFF);
    if (kind_of[s.id] != 0xFF && kind_of[s.id] != s.kind)
      fail(HPA_E_INVAL, "scope id " + std::to_string(s.id) + " used with two kinds");
    kind_of[s.id] = (uint8_t)s.kind;
    (s.kind == HPA_FUNC ? fn : nest).push_back(R{s.start, s.end, s.id, s.kind});
  }
  const uint32_t n_ids = (uint32_t)kind_of.size();
  std::vector<uint32_t> lo(d.n_lines);
  for (uint64_t i = 0; i < d.n_lines; ++i) {
    if (d.lines[i].start >= d.lines[i].end) fail(HPA_E_INVAL, "line range has start >= end");
    lo[i] = (uint32_t)i;
  }
  std::sort(lo.begin(), lo.end(), [&](uint32_t a, uint32_t b) { return d.lines[a].start < d.lines[b].start; });
  for (size_t i = 1; i < lo.size(); ++i)
    if (d.lines[lo[i]].start < d.lines[lo[i - 1]].end) fail(HPA_E_OVERLAP, "line ranges overlap");

  // boundaries
  std::vector<uint64_t> B;
  B.reserve(2 * (fn.size() + nest.size() + lo.size()));
  for (auto& r : fn) { B.push_back(r.s); B.push_back(r.e); }
  for (auto& r : nest) { B.push_back(r.s); B.push_back(r.e); }
  for (uint32_t i : lo) { B.push_back(d.lines[i].start); B.push_back(d.lines[i].end); }
  std::sort(B.begin(), B.end());
  B.erase(std::unique(B.begin(), B.end()), B.end());

  // functions by start; nested ranges by (start asc, end desc, kind asc, id asc): outer first
  std::sort(fn.begin(), fn.end(), [](const R& a, const R& b) { return a.s < b.s; });
  std::sort(nest.begin(), nest.end(), [](const R& a, const R& b) {
    if (a.s != b.s) return a.s < b.s;
    if (a.e != b.e) return a.e > b.e;
    if (a.kind != b.kind) return a.kind < b.kind;
    return a.id < b.id;
  });
  // owner priority: larger start, then smaller end, then smaller id
  auto worse = [](const R& a, const R& b) {
    if (a.s != b.s) return a.s < b.s;
    if (a.e != b.e) return a.e > b.e;
    return a.id > b.id;
  };
  std::priority_queue<R, std::vector<R>, decltype(worse)> heap(worse);

  out.parent.assign(n_ids, NONE32);
  out.func.assign(n_ids, NONE32);
  out.kind = kind_of;
  out.n_ids = n_ids;
  std::vector<uint8_t> placed(n_ids, 0);
  for (auto& r : fn) out.func[r.id] = r.id;

  struct Open {
    R r;
    uint32_t owner;
  };
  std::vector<Open> chain;  // open nested ranges, outermost first
  size_t fi = 0, ni = 0, li = 0;
  for (size_t b = 0; b + 1 < B.size(); ++b) {
    const uint64_t x = B[b], y = B[b + 1];
    while (fi < fn.size() && fn[fi].s == x) heap.push(fn[fi++]);
    while (!heap.empty() && heap.top().e <= x) heap.pop();
    const uint32_t owner = heap.empty() ? NONE32 : heap.top().id;
    while (!chain.empty() && chain.back().r.e <= x) chain.pop_back();
    // every open nested range must keep one owning function over all its addresses
    if (!chain.empty() && chain.back().owner != owner)
      fail(HPA_E_NOT_LAMINAR, "scope " + std::to_string(chain.back().r.id) + " spans addresses of another function");
    while (ni < nest.size() && nest[ni].s == x) {
      const R& r = nest[ni++];
      if (!chain.empty() && (r.e > chain.back().r.e || chain.back().r.id == r.id))
        fail(HPA_E_NOT_LAMINAR, "scope " + std::to_string(r.id) + " crosses scope " + std::to_string(chain.back().r.id));
      if (owner == NONE32) fail(HPA_E_NOT_LAMINAR, "scope " + std::to_string(r.id) + " starts outside every function");
      uint32_t par = chain.empty() ? owner : chain.back().r.id;
      if (placed[r.id] && (out.parent[r.id] != par || out.func[r.id] != owner))
        fail(HPA_E_NOT_LAMINAR, "ranges of scope " + std::to_string(r.id) + " have different parents");
      placed[r.id] = 1;
      out.parent[r.id] = par;
      out.func[r.id] = owner;
      chain.push_back(Open{r, owner});
    }
    if (owner == NONE32) continue;
    while (li < lo.size() && d.lines[lo[li]].end <= x) ++li;
    uint32_t f = 0, l = 0;
    if (li < lo.size() && d.lines[lo[li]].start <= x) { f = d.lines[lo[li]].file; l = d.lines[lo[li]].line; }
    const uint32_t sc = chain.empty() ? owner : chain.back().r.id;
    if (!out.start.empty() && out.end.back() == x && out.scope.back() == sc && out.file.back() == f &&
        out.line.back() == l) {
      out.end.back() = y;
    } else {
      out.start.push_back(x); out.end.push_back(y);
      out.scope.push_back(sc); out.file.push_back(f); out.line.push_back(l);
    }
  }
  if (ni < nest.size()) fail(HPA_E_NOT_LAMINAR, "scope outside every function");
}

void from_intervals(const hpa_structure_desc& d, Built& out) {
  for (uint64_t i = 0; i < d.n_iv; ++i) {
    if (d.iv_start[i] >= d.iv_end[i]) fail(HPA_E_INVAL, "interval has start >= end");
    if (i && d.iv_start[i] <= d.iv_start[i - 1]) fail(HPA_E_UNSORTED, "intervals not sorted by start");
    if (i && d.iv_start[i] < d.iv_end[i - 1]) fail(HPA_E_OVERLAP, "intervals overlap");
  }
  out.start.assign(d.iv_start, d.iv_start + d.n_iv);
  out.end.assign(d.iv_end, d.iv_end + d.n_iv);
  out.scope.resize(d.n_iv);
  for (uint64_t i = 0; i < d.n_iv; ++i) out.scope[i] = (uint32_t)i;
  out.file.assign(d.n_iv, 0);
  out.line.assign(d.n_iv, 0);
}

}  // namespace

namespace hpa {
void learned_train(hpa_structure_map* m, hipStream_t s);
}

hpa_structure_map::~hpa_structure_map() {
  if (learned) hpa::learned_free(learned);
}

namespace {

// Dense coordinates for a map (see hpa_structure_map): intervals closer than
// `gap` form one cluster; each cluster widened by 1 MiB on both sides (so
// nearby addresses outside every function stay on the grid) and rounded to
// 4 KiB pages is a window; overlapping windows merge.  The gap grows until at
// most DENSE_MAX_WIN windows remain.  The grid step 2^tz is the largest power
// of two (at most 4 KiB) dividing every interval boundary.
void build_dense(hpa_structure_map* m, const std::vector<uint64_t>& start, const std::vector<uint64_t>& end,
                 const std::vector<uint32_t>& scope, hipStream_t stream) {
  const size_t n = start.size();
  if (n == 0) return;
  uint64_t orv = 0;
  for (size_t i = 0; i < n; ++i) orv |= start[i] | end[i];
  const uint32_t tz = orv ? std::min<uint32_t>((uint32_t)__builtin_ctzll(orv), 12) : 12;
  const uint64_t MARGIN = 1ull << 20, PAGE = 4096, TOP = ~0ull & ~(PAGE - 1);
  std::vector<std::pair<uint64_t, uint64_t>> win;
  for (uint64_t gap = 1ull << 21;; gap = gap > (1ull << 60) ? ~0ull : gap * 4) {
    std::vector<std::pair<uint64_t, uint64_t>> cl;
    uint64_t lo = start[0], hi = end[0];
    for (size_t i = 1; i < n; ++i) {
      if (start[i] - hi <= gap) {
        hi = std::max(hi, end[i]);
      } else {
        cl.push_back({lo, hi});
        lo = start[i];
        hi = end[i];
      }
    }
    cl.push_back({lo, hi});
    win.clear();
    for (auto [l, h] : cl) {
      uint64_t l2 = (l >= MARGIN ? l - MARGIN : 0) & ~(PAGE - 1);
      uint64_t h2 = h >= TOP - MARGIN ? TOP : ((h + MARGIN + PAGE - 1) & ~(PAGE - 1));
      if (!win.empty() && l2 <= win.back().second) win.back().second = std::max(win.back().second, h2);
      else win.push_back({l2, h2});
    }
    if (win.size() <= DENSE_MAX_WIN || gap == ~0ull) break;
  }
  if (win.size() > DENSE_MAX_WIN) return;
  std::vector<uint64_t> lo(win.size()), hi(win.size()), d(win.size() + 1);
  uint64_t total = 0;
  for (size_t w = 0; w < win.size(); ++w) {
    lo[w] = win[w].first;
    hi[w] = win[w].second;
    d[w] = total;
    total += (hi[w] - lo[w]) >> tz;
    if (total > (1ull << 26)) return;
  }
  d[win.size()] = total;
  std::vector<uint32_t> tab(total, NONE32);
  size_t w = 0;
  for (size_t i = 0; i < n; ++i) {
    while (start[i] >= hi[w]) ++w;
    const uint64_t a = d[w] + ((start[i] - lo[w]) >> tz), b = d[w] + ((end[i] - lo[w]) >> tz);
    std::fill(tab.begin() + a, tab.begin() + b, scope[i]);
  }
  m->dense = true;
  m->dense_tz = tz;
  m->n_win = (uint32_t)win.size();
  m->n_dense = total;
  m->win_lo = upload(m->ctx, lo, stream);
  m->win_hi = upload(m->ctx, hi, stream);
  m->win_d = upload(m->ctx, d, stream);
  m->scope_of = upload(m->ctx, tab, stream);
}

}  // namespace

extern "C" hpa_status hpa_build_structure_map(hpa_ctx* ctx, const hpa_structure_desc* desc, hipStream_t stream,
                                              hpa_structure_map** out) {
  return guard([&] {
    if (!ctx || !desc || !out) fail(HPA_E_INVAL, "NULL argument");
    if (desc->n_iv && (desc->n_scopes || desc->n_lines))
      fail(HPA_E_INVAL, "give either scopes/lines or prebuilt intervals");
    if ((desc->n_scopes && !desc->scopes) || (desc->n_lines && !desc->lines) ||
        (desc->n_iv && (!desc->iv_start || !desc->iv_end)))
      fail(HPA_E_INVAL, "NULL array with nonzero count");
    if (desc->n_iv >= NONE32 || desc->n_scopes >= NONE32 / 4) fail(HPA_E_INVAL, "too many intervals");
    DeviceGuard g(ctx->device);
    Built b;
    if (desc->n_iv) from_intervals(*desc, b);
    else sweep(*desc, b);
    auto* m = new hpa_structure_map();
    try {
      m->ctx = ctx;
      m->stream = stream;
      m->n_iv = b.start.size();
      m->n_ids = b.n_ids;
      m->prebuilt = desc->n_iv != 0;
      m->start = upload(ctx, b.start, stream);
      m->end = upload(ctx, b.end, stream);
      m->scope = upload(ctx, b.scope, stream);
      m->file = upload(ctx, b.file, stream);
      m->line = upload(ctx, b.line, stream);
      m->parent = upload(ctx, b.parent, stream);
      m->kind = upload(ctx, b.kind, stream);
      m->func = upload(ctx, b.func, stream);
      // first search level: every 2^k-th start, small enough for a cache-resident table
      uint32_t shift = 0;
      while ((m->n_iv >> shift) > 4096) ++shift;
      std::vector<uint64_t> top;
      for (uint64_t i = 0; i < m->n_iv; i += (1ull << shift)) top.push_back(b.start[i]);
      m->top_n = (uint32_t)top.size();
      m->top_shift = shift;
      m->top = upload(ctx, top, stream);
      build_dense(m, b.start, b.end, b.scope, stream);
      m->h_parent = b.parent;
      m->h_func = b.func;
      m->h_kind = b.kind;
      m->h_start = std::move(b.start);
      m->h_end = std::move(b.end);
      m->h_scope = std::move(b.scope);
      if (desc->learned) learned_train(m, stream);
      sync_stream(ctx, stream);
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
  });
}

extern "C" hpa_status hpa_structure_map_view_get(const hpa_structure_map* m, hpa_structure_map_view* v) {
  return guard([&] {
    if (!m || !v) fail(HPA_E_INVAL, "NULL argument");
    v->n_intervals = m->n_iv;
    v->n_scope_ids = m->n_ids;
    v->start = m->start.as<uint64_t>();
    v->end = m->end.as<uint64_t>();
    v->scope = m->scope.as<uint32_t>();
    v->file = m->file.as<uint32_t>();
    v->line = m->line.as<uint32_t>();
    v->parent = m->parent.as<uint32_t>();
    v->kind = m->kind.as<uint8_t>();
    v->func = m->func.as<uint32_t>();
  });
}

extern "C" void hpa_structure_map_free(hpa_structure_map* m) { delete m; }

// ---------------------------------------------------------------------------
// A3 plain lookup: a two-level binary search.  The first level searches a
// table of every 2^k-th start (<= 4096 entries, 32 KB) staged in LDS; the
// second level finishes inside one block of 2^k starts in global memory.
// ---------------------------------------------------------------------------
namespace {

constexpr int LOOKUP_BLOCK = 256;

template <bool LABEL>
__global__ void __launch_bounds__(LOOKUP_BLOCK)
k_lookup_plain(const uint64_t* __restrict__ start, const uint64_t* __restrict__ end, uint64_t n_iv,
               const uint64_t* __restrict__ top, uint32_t top_n, uint32_t shift,
               const uint64_t* __restrict__ pc, uint64_t n, const unsigned long long* __restrict__ n_dev,
               const uint32_t* __restrict__ label, uint32_t* __restrict__ out) {
  __shared__ uint64_t s_top[4096];
  for (uint32_t i = threadIdx.x; i < top_n; i += LOOKUP_BLOCK) s_top[i] = top[i];
  __syncthreads();
  if (n_dev) n = min(n, (uint64_t)*n_dev);
  const uint64_t stride = (uint64_t)gridDim.x * LOOKUP_BLOCK;
  for (uint64_t i = (uint64_t)blockIdx.x * LOOKUP_BLOCK + threadIdx.x; i < n; i += stride) {
    const uint64_t q = pc[i];
    // number of top entries <= q
    uint32_t lo = 0, hi = top_n;
    while (lo < hi) {
      uint32_t mid = (lo + hi) >> 1;
      if (s_top[mid] <= q) lo = mid + 1;
      else hi = mid;
    }
    uint32_t r;
    if (lo == 0) {
      r = NONE32;
    } else {
      uint64_t b = (uint64_t)(lo - 1) << shift;
      uint64_t e = b + (1ull << shift);
      if (e > n_iv) e = n_iv;
      r = find_interval(start, end, n_iv, q, b + 1, e);
    }
    if constexpr (LABEL) r = r == NONE32 ? NONE32 : label[r];
    out[i] = r;
  }
}

}  // namespace

namespace hpa {

void launch_lookup_plain(const hpa_structure_map* m, const uint64_t* pc, uint64_t n, uint32_t* out, hipStream_t s) {
  if (n == 0) return;
  if (m->n_iv == 0) {
    HPA_HIP(hipMemsetAsync(out, 0xFF, n * sizeof(uint32_t), s));
    return;
  }
  unsigned grid = grid_for(n, LOOKUP_BLOCK, (unsigned)m->ctx->n_cu * 16);
  k_lookup_plain<false><<<grid, LOOKUP_BLOCK, 0, s>>>(m->start.as<uint64_t>(), m->end.as<uint64_t>(), m->n_iv,
                                                      m->top.as<uint64_t>(), m->top_n, m->top_shift, pc, n,
                                                      nullptr, nullptr, out);
  HPA_HIP(hipGetLastError());
}

void launch_scope_labels(const hpa_structure_map* m, const uint64_t* pc, uint64_t cap, const unsigned long long* n_dev,
                         uint32_t* scope, hipStream_t s) {
  if (cap == 0) return;
  if (m->n_iv == 0) {
    HPA_HIP(hipMemsetAsync(scope, 0xFF, cap * sizeof(uint32_t), s));
    return;
  }
  unsigned grid = grid_for(cap, LOOKUP_BLOCK, (unsigned)m->ctx->n_cu * 16);
  k_lookup_plain<true><<<grid, LOOKUP_BLOCK, 0, s>>>(m->start.as<uint64_t>(), m->end.as<uint64_t>(), m->n_iv,
                                                     m->top.as<uint64_t>(), m->top_n, m->top_shift, pc, cap, n_dev,
                                                     m->scope.as<uint32_t>(), scope);
  HPA_HIP(hipGetLastError());
}

}  // namespace hpa

extern "C" hpa_status hpa_lookup_intervals(hpa_ctx* ctx, const hpa_structure_map* map, const uint64_t* d_pc,
                                           uint64_t n, uint32_t* d_out, int mode, hipStream_t stream) {
  return guard([&] {
    if (!ctx || !map) fail(HPA_E_INVAL, "NULL argument");
    if (n && (!d_pc || !d_out)) fail(HPA_E_INVAL, "NULL array with n > 0");
    if (map->ctx != ctx) fail(HPA_E_INVAL, "map belongs to another context");
    DeviceGuard g(ctx->device);
    if (mode == HPA_LOOKUP_PLAIN) {
      launch_lookup_plain(map, d_pc, n, d_out, stream);
    } else if (mode == HPA_LOOKUP_LEARNED) {
      if (!map->learned) fail(HPA_E_UNSUPPORTED, "map was built without the learned index");
      launch_lookup_learned(map, d_pc, n, d_out, stream);
    } else {
      fail(HPA_E_INVAL, "unknown lookup mode");
    }
  });
}
