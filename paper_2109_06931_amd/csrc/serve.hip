// A9: serving ingest.  Sample buffers arrive as the measurement side fills
// them (Section 4.1: buffers are delivered when complete) and are folded, as
// they arrive, into device-resident per-profile state; the aggregation itself
// is the raw-metric sum of Section 4.5, so a profile's state after any set of
// buffers is the same whatever the order or company they arrived in.
//
// State.  One table of distinct PCs shared by the profiles (open addressing,
// 64-bit keys, a PC's slot index is its id) and, per profile, a key table:
// key = ctx << 36 | pc_id << 4 | stall, value = u64 count.  Both are filled
// lock-free: a slot is claimed by one compare-and-swap from empty and never
// changes afterwards, so a probe either finds its key, claims an empty slot,
// or moves on; no thread ever waits for another.
//
// Scheduling.  submit() queues a host buffer; a worker thread forms batches
// of queued buffers while a staging slot is free (slots are the in-flight
// memory the budget allows), copies small buffers into pinned staging and
// sends them with the batch's descriptors in one host-to-device copy, large
// ones directly, and launches one ingest kernel per batch on the slot's
// stream.  Batches on different slots overlap on the device.  A ticket
// completes when its batch's kernel has finished; latency is measured from
// submit() to the moment the worker sees that completion.
//
// Snapshot.  The table entries of one profile become weighted sample records
// (pc, ctx, stall, count) that go through the attribution path, which sorts,
// sums and labels them: the result has the layout of hpa_attribute's.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>

#include "block_prims.h"
#include "hpa_internal.h"

namespace hpa {
namespace {

constexpr int IB = 256;            // ingest threads per block
constexpr uint64_t CHUNK = 4096;   // samples per ingest block
constexpr uint64_t EMPTY = ~0ull;  // empty table slot
constexpr uint32_t MAX_PROBE = 4096;
constexpr unsigned int E_CTX = 1, E_STALL = 2, E_PCFULL = 4, E_TBLFULL = 8;

struct BatchDesc {
  uint64_t off;      // byte offset of the buffer in the device staging
  uint64_t n;        // samples
  uint32_t profile;
  uint32_t block0;   // first ingest block of the buffer
};

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Slot of pc in the shared PC table (the last slot is reserved for ~0), or
// NONE32 when the probe limit is reached.
__device__ __forceinline__ uint32_t pc_slot(unsigned long long* keys, uint64_t mask, uint64_t pc) {
  if (pc == EMPTY) return (uint32_t)(mask + 1);
  uint64_t h = mix64(pc) & mask;
  for (uint32_t p = 0; p < MAX_PROBE; ++p) {
    unsigned long long k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (k == pc) return (uint32_t)h;
    if (k == EMPTY) {
      k = atomicCAS(&keys[h], EMPTY, (unsigned long long)pc);
      if (k == EMPTY || k == pc) return (uint32_t)h;
    }
    h = (h + 1) & mask;
  }
  return NONE32;
}

__global__ void __launch_bounds__(IB)
k_ingest(const uint8_t* __restrict__ stage, const BatchDesc* __restrict__ desc, uint32_t n_desc, uint32_t n_ctx,
         unsigned long long* __restrict__ pc_keys, uint64_t pc_mask, unsigned long long* __restrict__ tkeys,
         unsigned long long* __restrict__ tcnt, uint64_t t_slots, unsigned int* __restrict__ err) {
  __shared__ uint32_t s_d;
  if (threadIdx.x == 0) {
    // the buffer this block belongs to: last descriptor with block0 <= blockIdx.x
    uint32_t lo = 0, hi = n_desc;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (desc[mid].block0 <= blockIdx.x) lo = mid;
      else hi = mid;
    }
    s_d = lo;
  }
  __syncthreads();
  const BatchDesc d = desc[s_d];
  const uint64_t b0 = (uint64_t)(blockIdx.x - d.block0) * CHUNK;
  const uint64_t b1 = min(d.n, b0 + CHUNK);
  const uint64_t* pc = reinterpret_cast<const uint64_t*>(stage + d.off);
  const uint32_t* cx = reinterpret_cast<const uint32_t*>(stage + d.off + 8 * d.n);
  const uint8_t* st = stage + d.off + 12 * d.n;
  unsigned long long* keys = tkeys + (uint64_t)d.profile * t_slots;
  unsigned long long* cnts = tcnt + (uint64_t)d.profile * t_slots;
  const uint64_t tmask = t_slots - 1;
  unsigned int e = 0;
  for (uint64_t i = b0 + threadIdx.x; i < b1; i += IB) {
    const uint64_t p = pc[i];
    const uint32_t c = cx[i];
    const uint32_t s = st[i];
    if (c >= n_ctx) { e |= E_CTX; continue; }
    if (s >= NS) { e |= E_STALL; continue; }
    const uint32_t id = pc_slot(pc_keys, pc_mask, p);
    if (id == NONE32) { e |= E_PCFULL; continue; }
    const uint64_t key = ((uint64_t)c << 36) | ((uint64_t)id << 4) | s;
    uint64_t h = mix64(key) & tmask;
    bool done = false;
    for (uint32_t q = 0; q < MAX_PROBE && !done; ++q) {
      unsigned long long k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (k == EMPTY) {
        const unsigned long long prev = atomicCAS(&keys[h], EMPTY, (unsigned long long)key);
        k = prev == EMPTY ? key : prev;
      }
      if (k == key) {
        atomicAdd(&cnts[h], 1ull);
        done = true;
      } else {
        h = (h + 1) & tmask;
      }
    }
    if (!done) e |= E_TBLFULL;
  }
  if (e) atomicOr(err, e);
}

// Snapshot: per block of table slots, count the used ones (pass 0) or write
// them as weighted records at the scanned offsets (pass 1).  A count above
// 2^32 - 1 is written as several records.
constexpr int SB = 256;

__device__ __forceinline__ uint32_t n_records(unsigned long long c) {
  return c == 0 ? 0u : (uint32_t)((c + 0xFFFFFFFEull) / 0xFFFFFFFFull);
}

__global__ void __launch_bounds__(SB)
k_snap(const unsigned long long* __restrict__ keys, const unsigned long long* __restrict__ cnts, uint64_t t_slots,
       const unsigned long long* __restrict__ pc_keys, uint64_t pc_mask, int pass,
       unsigned long long* __restrict__ blk, uint64_t* __restrict__ o_pc, uint32_t* __restrict__ o_ctx,
       uint8_t* __restrict__ o_stall, uint32_t* __restrict__ o_w) {
  __shared__ unsigned long long s_tmp[SB / WAVE + 1];
  const uint64_t i = (uint64_t)blockIdx.x * SB + threadIdx.x;
  const unsigned long long k = i < t_slots ? keys[i] : EMPTY;
  const unsigned long long c = (k != EMPTY) ? cnts[i] : 0ull;
  const unsigned long long r = n_records(c);
  unsigned long long tot;
  const unsigned long long ex = block_excl_scan<SB>(r, s_tmp, &tot);
  if (pass == 0) {
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
    return;
  }
  if (!r) return;
  const uint64_t base = blk[blockIdx.x] + ex;
  const uint32_t id = (uint32_t)((k >> 4) & 0xFFFFFFFFull);
  const uint64_t pcv = id == (uint32_t)(pc_mask + 1) ? EMPTY : (uint64_t)pc_keys[id];
  unsigned long long left = c;
  for (uint32_t j = 0; j < r; ++j) {
    const uint32_t w = (uint32_t)(left > 0xFFFFFFFFull ? 0xFFFFFFFFull : left);
    left -= w;
    o_pc[base + j] = pcv;
    o_ctx[base + j] = (uint32_t)(k >> 36);
    o_stall[base + j] = (uint8_t)(k & 15u);
    o_w[base + j] = w;
  }
}

__global__ void __launch_bounds__(1024) k_snap_scan(unsigned long long* blk, uint32_t n, unsigned long long* total) {
  __shared__ unsigned long long tmp[1024 / WAVE + 1];
  unsigned long long carry = 0;
  for (uint32_t b0 = 0; b0 < n; b0 += 1024) {
    const uint32_t b = b0 + threadIdx.x;
    const unsigned long long v = b < n ? blk[b] : 0;
    unsigned long long t;
    const unsigned long long e = block_excl_scan<1024>(v, tmp, &t);
    if (b < n) blk[b] = carry + e;
    carry += t;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

using Clock = std::chrono::steady_clock;

}  // namespace
}  // namespace hpa

using namespace hpa;

struct hpa_server {
  hpa_ctx* ctx = nullptr;
  const hpa_structure_map* map = nullptr;
  hpa_server_opts o{};
  hipStream_t init_stream = nullptr;
  DBuf pc_keys, tkeys, tcnt;
  uint64_t pc_mask = 0;

  struct Item {
    uint64_t ticket;
    uint32_t profile;
    const uint8_t* buf;
    uint64_t n;
    Clock::time_point t0;
  };
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    void* d_stage = nullptr;
    size_t d_cap = 0;
    uint8_t* h_stage = nullptr;  // pinned: descriptors, small buffers, error word
    unsigned int* h_err = nullptr;
    unsigned int* d_err = nullptr;
    std::vector<Item> items;
    bool busy = false;
    uint64_t bytes = 0;
  };
  std::vector<Slot> slots;
  size_t h_stage_bytes = 0;

  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::deque<Item> queue;
  uint64_t next_ticket = 1;
  uint64_t n_pending = 0;  // submitted and not complete
  bool stop = false, paused = false;
  int busy_slots = 0;
  std::thread worker;
  // completion records: latency (us) and status of finished tickets
  std::map<uint64_t, std::pair<double, int>> done;
  std::vector<double> lat;
  hpa_server_stats st{};
  Clock::time_point t_first{}, t_last{};
  std::string fail_msg;

  void run();
  void launch(Slot& s, std::vector<Item>& batch);
  void retire(Slot& s, Clock::time_point now);
};

namespace {
uint64_t stage_bytes(uint64_t n) { return (13 * n + 255) & ~255ull; }
constexpr uint64_t SMALL = 256 << 10;  // buffers up to this size travel through the pinned staging
}  // namespace

void hpa_server::launch(Slot& s, std::vector<Item>& batch) {
  // layout of the device staging: [descriptors][buffers ...]; the pinned
  // staging mirrors the descriptor part and the small buffers
  const uint64_t n_desc = batch.size();
  const uint64_t d_bytes = (n_desc * sizeof(BatchDesc) + 255) & ~255ull;
  std::vector<BatchDesc> desc(n_desc);
  uint64_t off = d_bytes, blocks = 0, samples = 0;
  for (size_t i = 0; i < n_desc; ++i) {
    desc[i] = BatchDesc{off, batch[i].n, batch[i].profile, (uint32_t)blocks};
    off += stage_bytes(batch[i].n);
    blocks += (batch[i].n + CHUNK - 1) / CHUNK;
    samples += batch[i].n;
  }
  std::memcpy(s.h_stage, desc.data(), n_desc * sizeof(BatchDesc));
  // contiguous prefix of small buffers goes with the descriptors in one copy
  uint64_t h_end = d_bytes;
  size_t i = 0;
  for (; i < n_desc && 13 * batch[i].n <= SMALL && desc[i].off + 13 * batch[i].n <= h_stage_bytes; ++i) {
    std::memcpy(s.h_stage + desc[i].off, batch[i].buf, 13 * batch[i].n);
    h_end = desc[i].off + 13 * batch[i].n;
  }
  HPA_HIP(hipMemcpyAsync(s.d_stage, s.h_stage, h_end, hipMemcpyHostToDevice, s.stream));
  for (; i < n_desc; ++i)
    HPA_HIP(hipMemcpyAsync(static_cast<uint8_t*>(s.d_stage) + desc[i].off, batch[i].buf, 13 * batch[i].n,
                           hipMemcpyHostToDevice, s.stream));
  HPA_HIP(hipMemsetAsync(s.d_err, 0, sizeof(unsigned int), s.stream));
  if (blocks) {
    k_ingest<<<(unsigned)blocks, IB, 0, s.stream>>>(static_cast<const uint8_t*>(s.d_stage),
                                                    static_cast<const BatchDesc*>(s.d_stage), (uint32_t)n_desc,
                                                    o.n_ctx, pc_keys.as<unsigned long long>(), pc_mask,
                                                    tkeys.as<unsigned long long>(), tcnt.as<unsigned long long>(),
                                                    o.table_slots, s.d_err);
    HPA_HIP(hipGetLastError());
  }
  HPA_HIP(hipMemcpyAsync(s.h_err, s.d_err, sizeof(unsigned int), hipMemcpyDeviceToHost, s.stream));
  HPA_HIP(hipEventRecord(s.ev, s.stream));
  s.items = std::move(batch);
  s.bytes = off;
  s.busy = true;
  st.batches += 1;
  st.samples += samples;
  st.max_inflight_bytes = std::max<uint64_t>(st.max_inflight_bytes, off);
}

void hpa_server::retire(Slot& s, Clock::time_point now) {
  const unsigned int e = *s.h_err;
  int status = HPA_OK;
  if (e & (E_CTX | E_STALL)) status = HPA_E_INVAL;
  else if (e & (E_PCFULL | E_TBLFULL)) status = HPA_E_BUDGET;
  if (status != HPA_OK) st.errors += s.items.size();
  for (const Item& it : s.items) {
    const double us = std::chrono::duration<double, std::micro>(now - it.t0).count();
    done[it.ticket] = {us, status};
    lat.push_back(us);
    st.buffers += 1;
    st.bytes += 13 * it.n;
  }
  t_last = now;
  s.items.clear();
  s.busy = false;
}

void hpa_server::run() {
  (void)hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    // retire finished batches
    bool progressed = false;
    for (Slot& s : slots) {
      if (!s.busy) continue;
      if (hipEventQuery(s.ev) == hipSuccess) {
        const size_t k = s.items.size();
        retire(s, Clock::now());
        n_pending -= k;
        --busy_slots;
        progressed = true;
      }
    }
    if (progressed) done_cv.notify_all();
    // admit queued buffers into free slots
    if (!paused) {
      for (Slot& s : slots) {
        if (s.busy || queue.empty()) continue;
        std::vector<Item> batch;
        uint64_t bytes = 0;
        while (!queue.empty() && batch.size() < o.max_batch_buffers) {
          const Item& it = queue.front();
          const uint64_t add = stage_bytes(it.n) + sizeof(BatchDesc);
          if (!batch.empty() && bytes + add + 256 > s.d_cap) break;
          batch.push_back(it);
          bytes += add;
          queue.pop_front();
        }
        if (st.batches == 0) t_first = batch.front().t0;
        try {
          launch(s, batch);
          ++busy_slots;
        } catch (const Error& e) {
          // the batch never reached the device: its tickets fail, and so does the server
          for (const Item& it : batch) done[it.ticket] = {0.0, HPA_E_DEVICE};
          n_pending -= batch.size();
          fail_msg = e.msg;
          stop = true;
          done_cv.notify_all();
        }
      }
    }
    if (stop && (queue.empty() || !fail_msg.empty()) && busy_slots == 0) break;
    if (busy_slots > 0) {
      // poll the in-flight batches
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      cv.wait(lk, [&] { return stop || (!queue.empty() && !paused); });
    }
  }
  // tickets left in the queue after a failure
  for (const Item& it : queue) done[it.ticket] = {0.0, HPA_E_DEVICE};
  n_pending -= queue.size();
  queue.clear();
  done_cv.notify_all();
}

extern "C" hpa_status hpa_server_create(hpa_ctx* ctx, const hpa_structure_map* map, const hpa_server_opts* opts,
                                        hpa_server** out) {
  return guard([&] {
    if (!ctx || !map || !opts || !out) fail(HPA_E_INVAL, "NULL argument");
    if (map->ctx != ctx) fail(HPA_E_INVAL, "map belongs to another context");
    hpa_server_opts o = *opts;
    if (o.n_profiles == 0 || o.n_ctx == 0) fail(HPA_E_INVAL, "need at least one profile and one context");
    if (o.n_ctx > (1u << 28)) fail(HPA_E_UNSUPPORTED, "more than 2^28 contexts per profile");
    if (!o.table_slots) o.table_slots = 1ull << 22;
    if (!o.pc_slots) o.pc_slots = 1ull << 20;
    if (!o.max_batch_bytes) o.max_batch_bytes = 64ull << 20;
    if (!o.n_slots) o.n_slots = 4;
    if (!o.max_batch_buffers) o.max_batch_buffers = 512;
    if (!o.hbm_budget) o.hbm_budget = 200ull * 1000 * 1000 * 1000;
    o.table_slots = pow2_at_least(o.table_slots);
    o.pc_slots = pow2_at_least(o.pc_slots);
    if (o.pc_slots > (1ull << 31)) fail(HPA_E_UNSUPPORTED, "more than 2^31 PC slots");
    const uint64_t state = (uint64_t)o.n_profiles * o.table_slots * 16 + (o.pc_slots + 1) * 8;
    const uint64_t staging = (uint64_t)o.n_slots * (o.max_batch_bytes + 4096);
    if (state + staging > o.hbm_budget)
      fail(HPA_E_BUDGET, "server state and staging need " + std::to_string(state + staging) +
                             " bytes, over the budget of " + std::to_string(o.hbm_budget));
    DeviceGuard g(ctx->device);
    auto* S = new hpa_server();
    std::unique_ptr<hpa_server> hold(S);
    S->ctx = ctx;
    S->map = map;
    S->o = o;
    S->pc_mask = o.pc_slots - 1;
    HPA_HIP(hipStreamCreateWithFlags(&S->init_stream, hipStreamNonBlocking));
    hipStream_t s = S->init_stream;
    S->pc_keys = DBuf(ctx, (o.pc_slots + 1) * 8, s);
    S->tkeys = DBuf(ctx, (uint64_t)o.n_profiles * o.table_slots * 8, s);
    S->tcnt = DBuf(ctx, (uint64_t)o.n_profiles * o.table_slots * 8, s);
    const uint64_t nk = (uint64_t)o.n_profiles * o.table_slots;
    k_fill_u64<<<4096, 256, 0, s>>>(S->pc_keys.as<unsigned long long>(), o.pc_slots + 1, EMPTY);
    k_fill_u64<<<4096, 256, 0, s>>>(S->tkeys.as<unsigned long long>(), nk, EMPTY);
    k_fill_u64<<<4096, 256, 0, s>>>(S->tcnt.as<unsigned long long>(), nk, 0ull);
    HPA_HIP(hipGetLastError());
    S->h_stage_bytes = std::min<uint64_t>(o.max_batch_bytes, 4ull << 20) + 4096;
    S->slots.resize(o.n_slots);
    for (auto& sl : S->slots) {
      HPA_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
      HPA_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
      sl.d_cap = o.max_batch_bytes + 4096;
      HPA_HIP(hipMalloc(&sl.d_stage, sl.d_cap));
      HPA_HIP(hipMalloc((void**)&sl.d_err, 256));
      HPA_HIP(hipHostMalloc((void**)&sl.h_stage, S->h_stage_bytes + 256, hipHostMallocDefault));
      sl.h_err = reinterpret_cast<unsigned int*>(sl.h_stage + S->h_stage_bytes);
      *sl.h_err = 0;
    }
    sync_stream(ctx, s);
    S->worker = std::thread([S] { S->run(); });
    *out = hold.release();
  });
}

extern "C" hpa_status hpa_server_submit(hpa_server* S, uint32_t profile, const void* buffer, uint64_t n_samples,
                                        uint64_t* ticket) {
  return guard([&] {
    if (!S || !ticket || (n_samples && !buffer)) fail(HPA_E_INVAL, "NULL argument");
    if (profile >= S->o.n_profiles) fail(HPA_E_INVAL, "profile out of range");
    if (reinterpret_cast<uintptr_t>(buffer) % 8) fail(HPA_E_INVAL, "buffer must be 8-byte aligned");
    if (stage_bytes(n_samples) + 512 > S->o.max_batch_bytes)
      fail(HPA_E_BUDGET, "buffer larger than the server's batch staging");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) fail(HPA_E_DEVICE, "server stopped: " + S->fail_msg);
    const uint64_t t = S->next_ticket++;
    S->queue.push_back(hpa_server::Item{t, profile, static_cast<const uint8_t*>(buffer), n_samples, Clock::now()});
    ++S->n_pending;
    *ticket = t;
    S->cv.notify_one();
  });
}

extern "C" hpa_status hpa_server_wait(hpa_server* S, uint64_t ticket, double* latency_us) {
  return guard([&] {
    if (!S) fail(HPA_E_INVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    if (ticket == 0 || ticket >= S->next_ticket) fail(HPA_E_INVAL, "unknown ticket");
    S->done_cv.wait(lk, [&] { return S->done.count(ticket) != 0; });
    auto it = S->done.find(ticket);
    if (latency_us) *latency_us = it->second.first;
    const int status = it->second.second;
    if (status != HPA_OK) fail((hpa_status)status, "the batch holding this buffer failed (invalid record or full table)");
  });
}

extern "C" hpa_status hpa_server_drain(hpa_server* S) {
  return guard([&] {
    if (!S) fail(HPA_E_INVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    S->done_cv.wait(lk, [&] { return S->n_pending == 0; });
    if (!S->fail_msg.empty()) fail(HPA_E_DEVICE, S->fail_msg);
  });
}

extern "C" hpa_status hpa_server_stats_get(hpa_server* S, int reset, hpa_server_stats* out) {
  return guard([&] {
    if (!S || !out) fail(HPA_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    hpa_server_stats r = S->st;
    std::vector<double> v = S->lat;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
      if (v.empty()) return 0.0;
      const size_t i = (size_t)std::min<double>((double)v.size() - 1, std::ceil(q * (double)v.size()) - 1);
      return v[i];
    };
    r.p50_us = pct(0.50);
    r.p99_us = pct(0.99);
    r.max_us = v.empty() ? 0.0 : v.back();
    double sum = 0.0;
    for (double x : v) sum += x;
    r.mean_us = v.empty() ? 0.0 : sum / (double)v.size();
    r.span_s = std::chrono::duration<double>(S->t_last - S->t_first).count();
    *out = r;
    if (reset) {
      S->st = hpa_server_stats{};
      S->lat.clear();
    }
  });
}

extern "C" hpa_status hpa_server_snapshot(hpa_server* S, uint32_t profile, hipStream_t stream,
                                          hpa_attribution** out) {
  return guard([&] {
    if (!S || !out) fail(HPA_E_INVAL, "NULL argument");
    if (profile >= S->o.n_profiles) fail(HPA_E_INVAL, "profile out of range");
    hpa_ctx* ctx = S->ctx;
    DeviceGuard g(ctx->device);
    // quiesce: no batch in flight and none launched until the table is read
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->paused = true;
      S->done_cv.wait(lk, [&] { return S->busy_slots == 0; });
    }
    struct Resume {
      hpa_server* S;
      ~Resume() {
        std::lock_guard<std::mutex> lk(S->mu);
        S->paused = false;
        S->cv.notify_one();
      }
    } resume{S};
    const uint64_t T = S->o.table_slots;
    const unsigned nb = (unsigned)((T + SB - 1) / SB);
    const unsigned long long* keys = S->tkeys.as<unsigned long long>() + (uint64_t)profile * T;
    const unsigned long long* cnts = S->tcnt.as<unsigned long long>() + (uint64_t)profile * T;
    DBuf blk(ctx, (uint64_t)nb * 8, stream), tot(ctx, 8, stream);
    k_snap<<<nb, SB, 0, stream>>>(keys, cnts, T, S->pc_keys.as<unsigned long long>(), S->pc_mask, 0,
                                  blk.as<unsigned long long>(), nullptr, nullptr, nullptr, nullptr);
    k_snap_scan<<<1, 1024, 0, stream>>>(blk.as<unsigned long long>(), nb, tot.as<unsigned long long>());
    HPA_HIP(hipGetLastError());
    unsigned long long n = 0;
    HPA_HIP(hipMemcpyAsync(&n, tot.p, 8, hipMemcpyDeviceToHost, stream));
    sync_stream(ctx, stream);
    const uint64_t n1 = std::max<uint64_t>(n, 1);
    DBuf r_pc(ctx, n1 * 8, stream), r_ctx(ctx, n1 * 4, stream), r_st(ctx, n1, stream), r_w(ctx, n1 * 4, stream);
    k_snap<<<nb, SB, 0, stream>>>(keys, cnts, T, S->pc_keys.as<unsigned long long>(), S->pc_mask, 1,
                                  blk.as<unsigned long long>(), r_pc.as<uint64_t>(), r_ctx.as<uint32_t>(),
                                  r_st.as<uint8_t>(), r_w.as<uint32_t>());
    HPA_HIP(hipGetLastError());
    hpa_samples smp{r_pc.as<uint64_t>(), r_ctx.as<uint32_t>(), r_st.as<uint8_t>(), r_w.as<uint32_t>(), n,
                    S->o.n_ctx};
    const hpa_status rc = hpa_attribute(ctx, S->map, &smp, stream, out);
    if (rc != HPA_OK) fail(rc, hpa_last_error());
  });
}

extern "C" void hpa_server_destroy(hpa_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->paused = false;
    S->cv.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  (void)hipSetDevice(S->ctx->device);
  for (auto& sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.d_stage) (void)hipFree(sl.d_stage);
    if (sl.d_err) (void)hipFree(sl.d_err);
    if (sl.h_stage) (void)hipHostFree(sl.h_stage);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  S->pc_keys.release();
  S->tkeys.release();
  S->tcnt.release();
  if (S->init_stream) {
    (void)hipStreamSynchronize(S->init_stream);
    (void)hipStreamDestroy(S->init_stream);
  }
  delete S;
}
