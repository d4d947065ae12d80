// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "hpa.h"

namespace hpa {

constexpr uint32_t NONE32 = 0xFFFFFFFFu;
constexpr uint64_t NONE64 = 0xFFFFFFFFFFFFFFFFull;
constexpr int NS = 16;

struct Error {
  hpa_status status;
  std::string msg;
};

[[noreturn]] void fail(hpa_status s, const std::string& msg);
void set_last_error(const std::string& msg);

#define HPA_HIP(call)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      ::hpa::fail(HPA_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

// Run `body` and translate exceptions into a status + thread-local message.
template <class F>
hpa_status guard(F&& body) {
  try {
    body();
    return HPA_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return HPA_E_NOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return HPA_E_DEVICE;
  }
}

}  // namespace hpa

struct hpa_ctx {
  int device = 0;
  hpa_allocator alloc{};
  bool custom = false;
  int n_cu = 256;
  std::atomic<uint64_t> n_syncs{0};  // host synchronisations made by the library's calls
  bool timing = false;
  std::vector<hpa_stage_time> stages;  // accumulated stage timings
  // Device blocks released by the library's buffers, by size, with the
  // stream they were released on.  A later allocation on the same stream
  // reuses one (stream order makes that safe); the blocks go back to HIP when
  // the context is destroyed, or when an allocation would otherwise fail.
  struct Cached {
    void* p;
    hipStream_t stream;
  };
  std::mutex cache_mu;
  std::multimap<size_t, Cached> cache;
  // run-time pipeline parameters chosen by the batch autotuner, kept for later calls
  bool tuned = false;
  uint32_t tuned_merge_rounds = 2, tuned_scan_wg = 4;
  ~hpa_ctx();
};

namespace hpa {

// Bump arena over a caller-provided device region: while base is set, every
// library allocation made on this thread comes from it (none is returned).
// Thread-local, so that other threads using the same context keep allocating
// normally.
struct Arena {
  uint8_t* base = nullptr;
  size_t size = 0, off = 0, peak = 0;
};
extern thread_local Arena t_arena;

// Wait for the stream on the host, counted on the context (the count is
// reported by hpa_ctx_get_sync_count).
inline void sync_stream(hpa_ctx* ctx, hipStream_t s) {
  ctx->n_syncs.fetch_add(1, std::memory_order_relaxed);
  HPA_HIP(hipStreamSynchronize(s));
}

// dalloc returns a block of at least `bytes` and its capacity in *cap; dfree
// takes the block back with that capacity.
void* dalloc(hpa_ctx* ctx, size_t bytes, hipStream_t s, size_t* cap);
void dfree(hpa_ctx* ctx, void* p, size_t cap, hipStream_t s);

// Stream-ordered device buffer owned by a scope or a handle.
struct DBuf {
  hpa_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  void* p = nullptr;
  size_t bytes = 0;  // requested size
  size_t cap = 0;    // size of the block
  DBuf() = default;
  DBuf(hpa_ctx* c, size_t n, hipStream_t s) : ctx(c), stream(s), bytes(n) { p = n ? dalloc(c, n, s, &cap) : nullptr; }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    release();
    ctx = o.ctx; stream = o.stream; p = o.p; bytes = o.bytes; cap = o.cap;
    o.p = nullptr; o.bytes = 0; o.cap = 0;
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p && ctx) dfree(ctx, p, cap, stream);  // a view of caller memory has no ctx
    p = nullptr;
    bytes = 0;
    cap = 0;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Copy a host vector into a new device buffer (at least one element, so that
// empty arrays still have a valid address).  The source is pageable memory, so
// the copy completes before returning; use on set-up paths only.
template <class T>
DBuf upload(hpa_ctx* ctx, const std::vector<T>& v, hipStream_t s) {
  DBuf b(ctx, std::max<size_t>(v.size(), 1) * sizeof(T), s);
  if (!v.empty()) {
    HPA_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    sync_stream(ctx, s);
  }
  return b;
}

struct DeviceGuard {
  int prev = 0;
  explicit DeviceGuard(int dev) {
    HPA_HIP(hipGetDevice(&prev));
    if (prev != dev) HPA_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

// hipEvent pairs around the stages of one call, on one stream; inert unless
// the context has timing on.  collect() runs after the stream is synchronised.
class StageTimer {
 public:
  StageTimer(hpa_ctx* ctx, hipStream_t s) : ctx_(ctx), s_(s), on_(ctx->timing) {}
  ~StageTimer();
  void begin(const char* name);
  void end(uint64_t items_in = 0, uint64_t items_out = 0);
  // set the item counts of an earlier span by name (known only after a sync)
  void items(const char* name, uint64_t items_in, uint64_t items_out);
  void collect();
  bool on() const { return on_; }

 private:
  struct Span {
    const char* name;
    hipEvent_t a, b;
    uint64_t in, out;
  };
  hpa_ctx* ctx_;
  hipStream_t s_;
  bool on_;
  std::vector<Span> spans_;
};

inline unsigned grid_for(uint64_t n, unsigned block, unsigned cap = 1u << 20) {
  uint64_t g = (n + block - 1) / block;
  if (g == 0) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

// Learned interval index (device side), see learned.hip.
struct LearnedModel;

}  // namespace hpa

struct hpa_structure_map {
  hpa_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  uint64_t n_iv = 0;
  uint32_t n_ids = 0;
  bool prebuilt = false;
  hpa::DBuf start, end, scope, file, line;  // intervals
  hpa::DBuf parent, kind, func;             // scope table
  hpa::DBuf top;                            // sampled starts for the first search level
  uint32_t top_n = 0, top_shift = 0;
  hpa::LearnedModel* learned = nullptr;
  std::vector<uint32_t> h_parent, h_func;   // host copies of the scope table
  std::vector<uint8_t> h_kind;
  std::vector<uint64_t> h_start, h_end;     // host copies of the intervals
  std::vector<uint32_t> h_scope;
  // Dense instruction coordinates.  The code lies in a few windows
  // [win_lo, win_hi); an address inside window w that is a multiple of
  // 2^dense_tz away from win_lo[w] has the coordinate
  // win_d[w] + ((pc - win_lo[w]) >> dense_tz), and scope_of[coordinate] is its
  // innermost scope.  dense is false when there is no code or the coordinates
  // would need more than 2^26 entries.
  bool dense = false;
  uint32_t dense_tz = 0, n_win = 0;
  uint64_t n_dense = 0;
  hpa::DBuf win_lo, win_hi, win_d, scope_of;
  ~hpa_structure_map();
};

struct hpa_attribution {
  hpa_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  const hpa_structure_map* map = nullptr;
  uint64_t n_keys = 0;
  uint32_t n_ctx = 0;
  hpa::DBuf ctx_id, pc, stall, count, scope, ctx_offsets;
};

namespace hpa {

constexpr uint32_t DENSE_MAX_WIN = 64;  // windows are staged in LDS by the kernels

// Device view of the dense coordinates (tables may be staged in LDS).
struct DenseDev {
  const uint64_t* lo;
  const uint64_t* hi;
  const uint64_t* d;         // n_win + 1 entries: first coordinate of each window, then the total
  const uint32_t* scope_of;  // n_dense entries (global memory)
  uint32_t n_win;
  uint32_t tz;
};

__device__ inline uint32_t last_le(const uint64_t* a, uint32_t n, uint64_t v) {
  // last i < n with a[i] <= v, or n when there is none (a ascending)
  if (n == 0 || a[0] > v) return n;
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Coordinate of pc, or false when pc lies outside every window or off the grid.
__device__ inline bool to_dense(const DenseDev& t, uint64_t pc, uint64_t& D) {
  if (t.n_win == 0) return false;
  const uint32_t w = last_le(t.lo, t.n_win, pc);
  if (w == t.n_win || pc >= t.hi[w]) return false;
  const uint64_t off = pc - t.lo[w];
  if (off & ((1ull << t.tz) - 1)) return false;
  D = t.d[w] + (off >> t.tz);
  return true;
}

__device__ inline uint64_t from_dense(const DenseDev& t, uint64_t D) {
  const uint32_t w = last_le(t.d, t.n_win, D);
  return t.lo[w] + ((D - t.d[w]) << t.tz);
}

// Plain lookup used by several kernels: interval index of pc or NONE32.
__device__ inline uint32_t find_interval(const uint64_t* __restrict__ start, const uint64_t* __restrict__ end,
                                         uint64_t n, uint64_t pc, uint64_t lo, uint64_t hi) {
  // invariant: answer (last start <= pc) lies in [lo - 1, hi - 1]
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (start[mid] <= pc) lo = mid + 1;
    else hi = mid;
  }
  if (lo == 0) return NONE32;
  uint64_t i = lo - 1;
  return pc < end[i] ? (uint32_t)i : NONE32;
}

void launch_lookup_plain(const hpa_structure_map* m, const uint64_t* pc, uint64_t n, uint32_t* out, hipStream_t s);
// scope[i] = innermost scope of pc[i] for i < min(cap, *n_dev) (n_dev: device counter, may be NULL)
void launch_scope_labels(const hpa_structure_map* m, const uint64_t* pc, uint64_t cap, const unsigned long long* n_dev,
                         uint32_t* scope, hipStream_t s);
void launch_lookup_learned(const hpa_structure_map* m, const uint64_t* pc, uint64_t n, uint32_t* out,
                           hipStream_t s);
void learned_free(LearnedModel* lm);
void learned_train(hpa_structure_map* m, const hpa_learned_opts* opts, hipStream_t s);
// Attribution over dense instruction coordinates, driven from the device with
// one synchronisation (attribute_dense.hip).  dense_path_fits tells whether
// the map and input sizes allow it; attribute_dense returns false, with no
// error, when some sample's pc has no dense coordinate (the caller then runs
// the general pipeline into the same handle).
bool dense_path_fits(const hpa_structure_map* map, const hpa_samples* smp);
bool attribute_dense(hpa_ctx* ctx, const hpa_structure_map* map, const hpa_samples* smp, hipStream_t s,
                     hpa_attribution* A);

// in-place exclusive scan of n u64 values; *d_total (device) receives the sum
void exscan_u64(hpa_ctx* ctx, unsigned long long* v, uint64_t n, unsigned long long* d_total, hipStream_t s);

}  // namespace hpa
