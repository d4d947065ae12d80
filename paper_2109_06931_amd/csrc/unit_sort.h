// Pieces shared by the attribution pipelines: unit sizes, the run record,
// the LDS layout of a sort workgroup, and the device functions that gather a
// unit's samples, find its key statistics, sort its keys, mark the unique keys
// and add up weighted counts.
#pragma once

#include "block_prims.h"
#include "hpa_internal.h"

namespace hpa {
namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;  // samples per scan tile

constexpr int UBLOCK = 1024;
constexpr int UITEMS = 16;
constexpr int UT = UBLOCK * UITEMS;  // unit capacity (samples)
constexpr int UHALF = UT / 2;        // contexts up to this size are packed together
constexpr int MAXC = 64;             // contexts per unit
constexpr int RUN_CAP = 1024;        // runs a sort workgroup copies to LDS for its gather
using Sorter = BlockRadix<UBLOCK, UITEMS>;

constexpr uint64_t M40 = (1ull << 40) - 1;
constexpr int ERR_CTX = 1, ERR_STALL = 2, ERR_WIDE = 4, ERR_SPLIT = 8;
constexpr uint64_t WIDE_CHUNK = ~0ull;  // chunk list length: left for the general chunk kernel

struct Run {
  uint64_t start;  // first sample index in the input
  uint64_t flat;   // position in context-grouped order (set by group_runs)
  uint32_t len;
  uint32_t ctx;
};

struct PlanInfo {
  unsigned long long n_runs;
  unsigned long long n_chunks;
  unsigned long long big_samples;
  unsigned long long total_keys;
  uint32_t n_units;
  uint32_t n_big;
  uint32_t max_chunks;
  uint32_t err;
  uint32_t n_bigall;   // contexts over T samples
  uint32_t n_split;    // of those, split into parts by coordinate range
  uint32_t n_virtual;  // contexts after the split (each part counts as one)
  uint32_t n_parts;    // parts of the split contexts
  unsigned long long split_samples;
  uint32_t n_merged;   // units after merging adjacent pairs
  uint32_t pad_;
};

__device__ inline int bits_for(uint64_t v) { return v ? 64 - __clzll(v) : 0; }

struct MapDev {
  const uint64_t* start;
  const uint64_t* end;
  const uint32_t* scope;
  uint64_t n_iv;
};

// A batch of profiles: every profile has its own structure map, and its
// contexts are numbered globally from ctx_base.  Kernels that handle one
// context (or a unit of contexts of one profile) look its profile up.
struct ProfMap {
  DenseDev dd;
  MapDev md;
  uint32_t ctx_base;
  int dense;
};

// ----------------------------------------------------------------------------
// Shared pieces of the sort workgroups (units and big-context chunks)
// ----------------------------------------------------------------------------
// LDS of a sort workgroup of BLOCK threads sorting up to BLOCK * ITEMS keys;
// RUNS reserves room for the run list a general-pipeline unit gathers through.
template <int BLOCK_, int ITEMS_, bool RUNS>
struct SortSmemT {
  static constexpr int BLOCK = BLOCK_;
  using S = BlockRadix<BLOCK_, ITEMS_>;
  // exchange plane of the sort; afterwards the unit's unique keys (keys of at
  // most 32 bits)
  uint32_t buf[S::BUF_WORDS];
  union {
    uint32_t cnt[S::CNT_WORDS];            // radix counter columns during the sort
    uint16_t upos[BLOCK_ * ITEMS_ + 2];    // then: sorted position of every unique key, closed by n_u
    Run runs[RUNS ? RUN_CAP : 1];          // before the sort: the runs the workgroup gathers through
  };
  uint32_t doff[S::DOFF_WORDS];
  unsigned long long pcmin[RUNS ? MAXC : 1];  // (general units only)
  uint32_t ucnt[MAXC + 1];
  unsigned long long red_or, red_max, red_min, red_ref;
  unsigned long long scan_tmp[BLOCK_ / WAVE + 1];
  uint32_t scan_tmp32[BLOCK_ / WAVE + 1];
  uint32_t last_hi[RUNS ? BLOCK_ : 1], last_lo[BLOCK_];  // high words for 64-bit keys (general units only)
  unsigned long long prefix;
  uint32_t unit, nU;
  uint64_t wlo[DENSE_MAX_WIN], whi[DENSE_MAX_WIN], wd[DENSE_MAX_WIN + 1];  // dense windows
  uint32_t far;  // a sample of the workgroup has no dense coordinate
};
using SortSmem = SortSmemT<UBLOCK, UITEMS, true>;
static_assert(UT < 65536, "16-bit sorted positions");

// One workgroup's samples in registers: pc, (stall | local context << 4), weight.
template <bool WEIGHTED>
struct Gathered {
  uint64_t pc[UITEMS];
  uint32_t meta[UITEMS];
  uint32_t w[WEIGHTED ? UITEMS : 1];
  __device__ uint32_t st(int i) const { return meta[i] & 15u; }
  __device__ uint32_t lc(int i) const { return meta[i] >> 4; }
  __device__ uint32_t wt(int i) const {
    if constexpr (WEIGHTED) return w[i];
    else return 1u;
  }
};

// Find the run of each of a thread's items and load the items.  A thread's
// items ascend, so the run of its first item comes from a binary search over
// the runs and the later ones from walking forward with the current run in
// registers.  `runs` is either the LDS copy of the runs or the global list.
template <bool WEIGHTED, class Load>
__device__ __forceinline__ void gather_runs(const Run* runs, uint64_t r_lo, uint64_t r_hi, uint64_t s0, uint64_t n_u,
                                            uint32_t cb, Load&& load) {
  uint64_t r = r_lo;
  if (n_u > threadIdx.x) {
    const uint64_t f0 = s0 + threadIdx.x;
    uint64_t hi = r_hi;
    while (hi - r > 1) {
      uint64_t mid = (r + hi) >> 1;
      if (runs[mid].flat <= f0) r = mid;
      else hi = mid;
    }
  }
  Run cur = n_u > threadIdx.x ? runs[r] : Run{0, 0, 0, cb};
#pragma unroll
  for (int i = 0; i < UITEMS; ++i) {
    if ((uint64_t)i * UBLOCK >= n_u) continue;
    const uint64_t j = (uint64_t)i * UBLOCK + threadIdx.x;
    const uint64_t flat = s0 + j;
    if (j < n_u) {
      while (flat >= cur.flat + cur.len) cur = runs[++r];
      load(i, cur.start + (flat - cur.flat), cur.ctx - cb);
    }
  }
}

// Load the unit's samples: item i of thread t is sample j = i * UBLOCK + t
// (flat position s0 + j in context-grouped order).  Run mode reads through
// the runs [r_lo, r_hi) that cover the unit, copied to LDS first when at most
// RUN_CAP of them (s_runs; the workgroup's barrier is taken inside, so every
// thread calls this); scattered mode reads flat positions, finding each item's
// context in the LDS copy of the unit's context offsets.
template <bool SCATTERED, bool WEIGHTED>
__device__ inline void gather(Gathered<WEIGHTED>& g, uint64_t s0, uint64_t n_u, uint32_t cb, const Run* __restrict__ grp,
                              uint64_t r_lo, uint64_t r_hi, const uint64_t* __restrict__ sb_lds,
                              uint32_t n_cu, const uint64_t* __restrict__ pc, const uint8_t* __restrict__ stall,
                              const uint32_t* __restrict__ weight, uint32_t* err, Run* s_runs,
                              bool runs_staged = false) {
  // every load is issued before any loaded value is used (the stall test
  // and the packing come after the loop), so a thread's loads overlap
  uint32_t st[UITEMS], lcs[UITEMS];
  auto load = [&](int i, uint64_t src, uint32_t lc) {
    g.pc[i] = pc[src];
    st[i] = stall[src];
    lcs[i] = lc;
    if constexpr (WEIGHTED) g.w[i] = weight[src];
  };
#pragma unroll
  for (int i = 0; i < UITEMS; ++i) {
    g.pc[i] = 0;
    st[i] = 0;
    lcs[i] = 0;
    if constexpr (WEIGHTED) g.w[i] = 0;
  }
  if constexpr (SCATTERED) {
    uint32_t lo = 0;
#pragma unroll
    for (int i = 0; i < UITEMS; ++i) {
      if ((uint64_t)i * UBLOCK >= n_u) continue;
      const uint64_t j = (uint64_t)i * UBLOCK + threadIdx.x;
      const uint64_t flat = s0 + j;
      if (j < n_u) {
        uint32_t hi = n_cu;  // last l with sb[l] <= flat, searching up from the previous item's context
        while (hi - lo > 1) {
          uint32_t mid = (lo + hi) >> 1;
          if (sb_lds[mid] <= flat) lo = mid;
          else hi = mid;
        }
        load(i, flat, lo);
      }
    }
  } else {
    const uint64_t nr = r_hi - r_lo;
    if (nr <= (uint64_t)RUN_CAP) {
      // the walk reads every run several times from dependent addresses: LDS
      // (runs_staged: the caller copied them and synchronised already)
      if (!runs_staged) {
        for (uint32_t k = threadIdx.x; k < nr; k += UBLOCK) s_runs[k] = grp[r_lo + k];
        __syncthreads();
      }
      gather_runs<WEIGHTED>(s_runs, 0, nr, s0, n_u, cb, load);
    } else {
      gather_runs<WEIGHTED>(grp, r_lo, r_hi, s0, n_u, cb, load);
    }
  }
  bool bad = false;
#pragma unroll
  for (int i = 0; i < UITEMS; ++i) {
    bad |= st[i] >= NS;
    g.meta[i] = (st[i] < NS ? st[i] : 0u) | (lcs[i] << 4);
  }
  if (bad) atomicOr(err, (uint32_t)ERR_STALL);
}

// Stage the dense window tables in LDS (the caller synchronises before use)
// and clear the far flag.
template <class SM>
__device__ inline DenseDev stage_dense(SM& sm, const DenseDev& t) {
  if (threadIdx.x == 0) sm.far = 0;
  for (uint32_t i = threadIdx.x; i < t.n_win; i += SM::BLOCK) {
    sm.wlo[i] = t.lo[i];
    sm.whi[i] = t.hi[i];
  }
  // a map without dense coordinates has no tables (n_win == 0, null pointers)
  if (t.n_win)
    for (uint32_t i = threadIdx.x; i <= t.n_win; i += SM::BLOCK) sm.wd[i] = t.d[i];
  return DenseDev{sm.wlo, sm.whi, sm.wd, t.scope_of, t.n_win, t.tz};
}

// Replace every gathered pc by its dense coordinate; a pc without one sets
// sm.far (the workgroup then gathers again and keeps raw pcs).
template <bool WEIGHTED>
__device__ inline void densify(SortSmem& sm, Gathered<WEIGHTED>& g, uint64_t n_u, const DenseDev& t) {
  bool bad = false;
#pragma unroll
  for (int i = 0; i < UITEMS; ++i) {
    if ((uint64_t)i * UBLOCK >= n_u) continue;
    if ((uint64_t)i * UBLOCK + threadIdx.x < n_u) {
      uint64_t D;
      if (to_dense(t, g.pc[i], D)) g.pc[i] = D;
      else bad = true;
    }
  }
  if (bad) atomicOr(&sm.far, 1u);
}

// Innermost scope of a pc: the dense table when the pc has a coordinate,
// else a binary search over the intervals.
__device__ inline uint32_t scope_of_pc(const DenseDev& t, bool dense, const uint64_t* start, const uint64_t* end,
                                       const uint32_t* scope, uint64_t n_iv, uint64_t pc) {
  uint64_t D;
  if (dense && to_dense(t, pc, D)) return t.scope_of[D];
  const uint32_t i = find_interval(start, end, n_iv, pc, 0, n_iv);
  return i == NONE32 ? NONE32 : scope[i];
}

// Build the unit's keys (local context, coordinate relative to the context's
// smallest, stall) and sort them.  Keys of at most 32 bits take one 32-bit
// sort; wider keys take two chained 32-bit sorts (low word first, the high
// word carried along, then the high word), which is the same LSD order.
template <bool WEIGHTED, class K, int IT = UITEMS>
__device__ inline void sort_reduce(SortSmem& sm, Gathered<WEIGHTED>& g, uint64_t n_u, uint32_t n_cu, K (&key)[IT],
                                   uint32_t (&val)[IT], int kbits, int pcb, uint32_t tz) {
  using S = BlockRadix<UBLOCK, IT>;
  uint32_t lo[IT], hi[IT];
  // 32-bit keys (kbits <= 31): an empty slot holds 1 << kbits, above every
  // real key, so sorting kbits + 1 bits leaves the real keys first and the
  // sort needs no per-slot test
  const uint64_t empty = sizeof(K) == 4 ? (1ull << kbits) : 0ull;
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const uint64_t j = (uint64_t)i * UBLOCK + threadIdx.x;
    uint64_t k = empty;
    if (j < n_u) {
      const uint64_t rel = (g.pc[i] - sm.pcmin[g.lc(i)]) >> tz;
      k = ((uint64_t)g.lc(i) << (pcb + 4)) | (rel << 4) | g.st(i);
    }
    lo[i] = (uint32_t)k;
    hi[i] = (uint32_t)(k >> 32);
    val[i] = g.wt(i);
  }
  if constexpr (sizeof(K) == 4) {
    if constexpr (WEIGHTED)
      S::template sort<1, true>(lo, val, hi, kbits + 1, (int)n_u, true, sm.buf, sm.cnt, sm.doff);
    else S::template sort<0, true>(lo, val, hi, kbits + 1, (int)n_u, true, sm.buf, sm.cnt, sm.doff);
#pragma unroll
    for (int i = 0; i < IT; ++i) key[i] = (K)lo[i];
  } else {
    if constexpr (WEIGHTED) {
      S::template sort<2>(lo, hi, val, 32, (int)n_u, true, sm.buf, sm.cnt, sm.doff);
      S::template sort<2>(hi, lo, val, kbits - 32, (int)n_u, false, sm.buf, sm.cnt, sm.doff);
    } else {
      S::template sort<1>(lo, hi, val, 32, (int)n_u, true, sm.buf, sm.cnt, sm.doff);
      S::template sort<1>(hi, lo, val, kbits - 32, (int)n_u, false, sm.buf, sm.cnt, sm.doff);
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) key[i] = (K)(((uint64_t)hi[i] << 32) | lo[i]);
  }
}

struct OutDev {
  uint32_t* ctx;
  uint64_t* pc;
  uint8_t* stall;
  unsigned long long* count;
  uint32_t* scope;
  uint64_t* ctx_off;
};

// Per-unit key statistics: the unit's smallest coordinate (every context's key
// is taken relative to it), the common trailing zeros of all differences, and
// the span in bits.  The lowest set bit of a - b is the lowest bit where a and
// b differ, so the common trailing zeros of all differences are those of the
// OR of every value XOR one reference value.
template <bool WEIGHTED>
__device__ inline void key_stats(SortSmem& sm, const Gathered<WEIGHTED>& g, uint64_t n_u, uint32_t n_cu, uint32_t* err,
                                 int& kbits, int& pcb, uint32_t& tz) {
  if (threadIdx.x == 0) { sm.red_or = 0; sm.red_max = 0; sm.red_min = ~0ull; }
  const uint64_t ref = n_u ? g.pc[0] : 0;  // thread 0's first item; broadcast below
  if (threadIdx.x == 0) sm.red_ref = ref;
  __syncthreads();
  const uint64_t r = sm.red_ref;
  unsigned long long mn = ~0ull, mx = 0, ox = 0;
#pragma unroll
  for (int i = 0; i < UITEMS; ++i) {
    if ((uint64_t)i * UBLOCK >= n_u) continue;
    if ((uint64_t)i * UBLOCK + threadIdx.x < n_u) {
      const unsigned long long v = g.pc[i];
      mn = v < mn ? v : mn;
      mx = v > mx ? v : mx;
      ox |= v ^ r;
    }
  }
  mn = wave_min(mn);
  mx = wave_max(mx);
  ox = wave_or(ox);
  if (lane_id() == 0) {
    atomicMin(&sm.red_min, mn);
    atomicMax(&sm.red_max, mx);
    atomicOr(&sm.red_or, ox);
  }
  __syncthreads();
  const unsigned long long lo = sm.red_min;
  tz = sm.red_or ? (uint32_t)__ffsll((long long)sm.red_or) - 1 : 0;
  pcb = bits_for((sm.red_max - lo) >> tz);
  for (uint32_t l = threadIdx.x; l < n_cu; l += UBLOCK) sm.pcmin[l] = lo;
  int cbits = bits_for(n_cu > 0 ? n_cu - 1 : 0);
  kbits = cbits + pcb + 4;
  if (kbits > 63 && threadIdx.x == 0) atomicOr(err, (uint32_t)ERR_WIDE);
  __syncthreads();
}

// After the sort (keys blocked in registers): head flags, the unique count,
// the sorted position of every unique key (sm.upos, closed by n_u), the keys
// themselves compacted into sm.buf when they fit 32 bits, and the number of
// unique keys per local context.
template <class K, class SM>
__device__ inline K prev_last(const SM& sm, int tid) {
  if constexpr (sizeof(K) == 4) return tid == 0 ? (K)0 : (K)sm.last_lo[tid - 1];
  else return tid == 0 ? (K)0 : (K)(((uint64_t)sm.last_hi[tid - 1] << 32) | sm.last_lo[tid - 1]);
}

template <class K, int IT = UITEMS, class SM>
__device__ inline uint32_t find_heads(SM& sm, const K (&key)[IT], uint64_t n_u, uint32_t n_cu, int pcb,
                                      uint32_t& first_uidx, uint32_t& nU) {
  constexpr int BLOCK = SM::BLOCK;
  const int tid = threadIdx.x;
  sm.last_lo[tid] = (uint32_t)key[IT - 1];
  if constexpr (sizeof(K) == 8) sm.last_hi[tid] = (uint32_t)((uint64_t)key[IT - 1] >> 32);
  // sm.ucnt first holds each context's first unique index (NONE32: no keys)
  for (uint32_t l = tid; l <= n_cu; l += BLOCK) sm.ucnt[l] = NONE32;
  __syncthreads();
  K prev = prev_last<K>(sm, tid);
  uint32_t heads = 0;
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    uint32_t p = (uint32_t)tid * IT + i;
    bool h = p < n_u && (p == 0 || key[i] != prev);
    heads += h;
    prev = key[i];
  }
  uint32_t tot;
  const uint32_t ex = block_excl_scan<BLOCK>(heads, sm.scan_tmp32, &tot);
  first_uidx = ex;
  nU = tot;
  prev = prev_last<K>(sm, tid);
  uint32_t u = first_uidx;
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    uint32_t p = (uint32_t)tid * IT + i;
    bool h = p < n_u && (p == 0 || key[i] != prev);
    if (h) {
      sm.upos[u] = (uint16_t)p;
      if constexpr (sizeof(K) == 4) sm.buf[u] = (uint32_t)key[i];
      // unique keys are ordered by local context: a head whose context
      // differs from the previous key's starts that context's keys
      const uint32_t lc = (uint32_t)((uint64_t)key[i] >> (pcb + 4));
      if (p == 0 || lc != (uint32_t)((uint64_t)prev >> (pcb + 4))) sm.ucnt[lc] = u;
      ++u;
    }
    prev = key[i];
  }
  if (tid == 0) sm.upos[nU] = (uint16_t)n_u;
  __syncthreads();
  // keys per context: the next non-empty context's first index (a suffix
  // minimum over the lanes of wave 0, n_cu <= 64) minus this one's; thread l
  // converts entry l, and only thread l reads it afterwards
  static_assert(MAXC <= WAVE, "one lane per local context");
  if (tid < WAVE) {
    // (the lane index is hidden from the optimiser so that the shuffle
    // sources are computed here, not hoisted out of a caller's loop)
    uint32_t l = (uint32_t)tid;
    asm volatile("" : "+v"(l));
    const uint32_t st = l < n_cu ? sm.ucnt[l] : NONE32;
    uint32_t suf = st;
    for (uint32_t d = 1; d < (uint32_t)WAVE; d <<= 1) {
      const uint32_t o = __shfl(suf, (int)min(l + d, (uint32_t)WAVE - 1), WAVE);
      if (l + d < (uint32_t)WAVE) suf = min(suf, o);
    }
    uint32_t next = __shfl(suf, (int)min(l + 1, (uint32_t)WAVE - 1), WAVE);
    if (l + 1 >= (uint32_t)WAVE) next = NONE32;
    next = min(next, nU);
    if (l < n_cu) sm.ucnt[l] = st == NONE32 ? 0u : next - st;
  }
  return heads;
}

// Weighted counts: every head writes the weight of its run inside its thread;
// runs continuing from the previous thread are added with one atomic each.
template <class K, int IT = UITEMS, class SM>
__device__ inline void weighted_counts(const SM& sm, const K (&key)[IT], const uint32_t (&val)[IT],
                                       uint64_t n_u, uint32_t first_uidx, unsigned long long* count) {
  const int tid = threadIdx.x;
  K prev = prev_last<K>(sm, tid);
  unsigned long long lead = 0, run = 0;
  bool seen = false;
  uint32_t u = first_uidx;
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    uint32_t p = (uint32_t)tid * IT + i;
    if (p < n_u) {
      bool h = p == 0 || key[i] != prev;
      if (h) {
        if (seen) count[u++] = run;
        seen = true;
        run = 0;
      }
      if (seen) run += val[i];
      else lead += val[i];
    }
    prev = key[i];
  }
  if (seen) count[u] = run;
  __threadfence();
  __syncthreads();
  if (lead) atomicAdd(&count[first_uidx - 1], lead);
}

}  // namespace
}  // namespace hpa
