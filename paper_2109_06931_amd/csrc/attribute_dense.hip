// A2-A4 for maps with dense instruction coordinates: a pipeline driven from
// the device end to end, with one host synchronisation per call (Section 4.2
// sample record; Section 4.5: a raw metric is the sum of measured values;
// Section 6.1 calling-context expansion for the scope labels).
//
//   hist      read ctx[] once (16 B per lane): per-context sample counts, one
//             atomic per run of equal contexts inside a wave's 256 samples.
//   bases     tile scans over the contexts: each context's first position in
//             context order, the list of contexts over DUT samples ("big").
//   scatter   read pc, ctx, stall (and weight) once; replace the pc by its
//             dense coordinate D and write the 4-byte record D << 4 | stall
//             at the sample's position in context order (one atomic per run).
//   split     one workgroup per big context: a histogram of its records over
//             coordinate buckets, the buckets packed greedily into parts of at
//             most DUT samples (a bucket over DUT samples is a part of its own,
//             counted instead of sorted), the records copied into bucket order.
//             Parts cover increasing coordinate ranges, so their sorted keys,
//             one after the other, are the context's keys in order.
//   plan      per tile of 1,024 contexts, consecutive contexts packed greedily
//             into units of at most DUT samples and 64 non-empty contexts; a big
//             context contributes its parts.  Units are numbered in context
//             order.
//   units     persistent workgroups take units in ticket order: load the
//             records (contiguous), sort the keys (local context, D, stall) in
//             LDS, mark unique keys, publish the unit's key count, look back
//             over the units before it for its output offset, and write the
//             final keys (ctx, pc, stall, count, scope) and its contexts'
//             offsets directly.
//
// A record whose pc has no dense coordinate (far from every window, or off
// the instruction grid) is counted; the caller then runs the general path.
#include <algorithm>
#include <memory>
#include <type_traits>

#include "block_prims.h"
#include "hpa_internal.h"
#include "unit_sort.h"

namespace hpa {
namespace {

constexpr int DB = 256;                 // hist / scatter / plan workgroup
constexpr int DI = 4;                   // samples per lane per step
constexpr int DCH = WAVE * DI;          // samples per wave step
constexpr uint32_t FAR_REC = 0xFFFFFFFFu;
constexpr int DUB = 512;                // unit workgroup (two fit one compute unit's LDS)
constexpr int DUI = 16;                 // most items per thread of a unit
constexpr int DUT = DUB * DUI;          // unit capacity (records); contexts over it are "big"
using DSmem = SortSmemT<DUB, DUI, false>;
constexpr int DNB = 4096;               // coordinate buckets of a big context
constexpr int DTILE = 1024;             // contexts per plan tile
constexpr uint32_t DU_SMALL = 0, DU_PART = 1, DU_HOT = 2;
constexpr unsigned int DERR_CTX = 1, DERR_STALL = 2, DERR_WIDE = 4, DERR_INTERNAL = 8, DERR_LOOKBACK = 16,
                       DERR_OVERFLOW = 32;
constexpr unsigned long long LB_AGG = 1ull << 62, LB_INC = 2ull << 62, LB_VAL = (1ull << 62) - 1;
constexpr uint32_t LB_SPIN_LIMIT = 1u << 25;

struct DInfo {
  unsigned long long total_keys;
  unsigned int err;
  unsigned int n_far;
  unsigned int n_big;
  unsigned int n_units;
  unsigned int ticket;
  unsigned int big_slots;
};

// One unit of work.  SMALL: records [s0, s1) of the context-ordered array,
// contexts [cb, ce) (empty ones included).  PART / HOT: records [s0, s1) of
// the bucket-ordered copy, all of context cb; a HOT part is one coordinate
// bucket starting at coordinate d0.
struct DUnit {
  uint32_t s0, s1, cb, ce, kind, d0, pad0, pad1;
};

// ---------------------------------------------------------------------------
// run structure of a wave's 256 consecutive samples
// ---------------------------------------------------------------------------
// Lane l holds positions 4l .. 4l+3.  For every position: the position of the
// head of its run (a maximal stretch of equal values inside the step), and
// whether it is the run's last position.  Invalid positions hold NONE32 and
// form runs of their own that the callers skip.
struct WaveRuns {
  uint32_t v[DI];
  int head[DI];
  bool tail[DI];
};

// Exclusive max-scan over the 64 lanes with DPP moves only (identity -1):
// row shifts by 1, 2, 4 and 8 scan each row of 16 lanes, row broadcasts of
// lanes 15 and 31 carry the row maxima, and a whole-wave shift by one lane
// makes the scan exclusive.  Every lane must be active.
__device__ inline int wave_excl_max_i(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x111, 0xF, 0xF, false));  // row_shr:1
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x112, 0xF, 0xF, false));  // row_shr:2
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x114, 0xF, 0xF, false));  // row_shr:4
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x118, 0xF, 0xF, false));  // row_shr:8
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x142, 0xA, 0xF, false));  // row_bcast:15
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return __builtin_amdgcn_update_dpp(-1, x, 0x138, 0xF, 0xF, false);        // wave_shr:1
}

// Runs of equal contexts in a wave's DI * 64 consecutive samples (lane l
// holds samples DI * l .. DI * l + DI - 1): each sample's run head and
// whether it ends its run.  The neighbours' values come by whole-wave DPP
// shifts (lane 0 and lane 63 see none).
__device__ inline void wave_runs(WaveRuns& w) {
  const int lane = lane_id();
  const uint32_t prev = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w.v[DI - 1], 0x138, 0xF, 0xF, false);  // wave_shr:1
  const uint32_t next = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w.v[0], 0x130, 0xF, 0xF, false);       // wave_shl:1
  int hp = -1;
#pragma unroll
  for (int j = 0; j < DI; ++j) {
    const bool h = j == 0 ? (lane == 0 || w.v[0] != prev) : w.v[j] != w.v[j - 1];
    if (h) hp = lane * DI + j;
    w.head[j] = hp;  // -1: the run started in an earlier lane
  }
  const int carry = wave_excl_max_i(hp);
#pragma unroll
  for (int j = 0; j < DI; ++j) {
    if (w.head[j] < 0) w.head[j] = carry;
    w.tail[j] = j + 1 < DI ? w.v[j] != w.v[j + 1] : (lane == WAVE - 1 || w.v[DI - 1] != next);
  }
}

template <bool VEC>
__device__ inline void load_ctx4(const uint32_t* __restrict__ ctx, uint64_t n, uint64_t p0, uint32_t (&v)[DI]) {
  if (VEC && p0 + DI <= n) {
    const uint4 q = *reinterpret_cast<const uint4*>(ctx + p0);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  } else {
#pragma unroll
    for (int j = 0; j < DI; ++j) v[j] = p0 + j < n ? ctx[p0 + j] : NONE32;
  }
}

// ---------------------------------------------------------------------------
// hist
// ---------------------------------------------------------------------------
template <bool VEC>
__global__ void __launch_bounds__(DB) k_d_hist(const uint32_t* __restrict__ ctx, uint64_t n, uint32_t C,
                                               uint32_t* __restrict__ hist, DInfo* __restrict__ info) {
  const uint64_t nw = (uint64_t)gridDim.x * (DB / WAVE);
  const uint64_t steps = (n + DCH - 1) / DCH;
  bool bad = false;
  for (uint64_t k = (uint64_t)blockIdx.x * (DB / WAVE) + wave_id(); k < steps; k += nw) {
    const uint64_t p0 = k * DCH + (uint64_t)lane_id() * DI;
    WaveRuns w;
    load_ctx4<VEC>(ctx, n, p0, w.v);
    wave_runs(w);
#pragma unroll
    for (int j = 0; j < DI; ++j) {
      if (p0 + j >= n) continue;
      const uint32_t c = w.v[j];
      if (c >= C) { bad = true; continue; }
      if (w.tail[j]) atomicAdd(&hist[c], (uint32_t)(lane_id() * DI + j - w.head[j] + 1));
    }
  }
  if (__any(bad) && lane_id() == 0) atomicOr(&info->err, DERR_CTX);
}

// ---------------------------------------------------------------------------
// bases: three launches of tile scans over the contexts
// ---------------------------------------------------------------------------
// Per tile: samples, big contexts, and the unit slots the big contexts may
// need (2 * ceil(n / DUT) + 1 each: greedy packing leaves no two neighbouring
// parts that would fit together).
struct DTileSums {
  unsigned long long n;
  uint32_t big, slots;
};

__device__ inline uint32_t big_slots(uint32_t n) { return 2u * ((n + DUT - 1) / DUT) + 1u; }

__global__ void __launch_bounds__(DTILE) k_d_tile_sums(const uint32_t* __restrict__ hist, uint32_t C,
                                                       DTileSums* __restrict__ ts) {
  __shared__ unsigned long long s_a[DTILE / WAVE + 1];
  __shared__ uint32_t s_b[DTILE / WAVE + 1];
  const uint32_t c = blockIdx.x * DTILE + threadIdx.x;
  const uint32_t h = c < C ? hist[c] : 0u;
  const bool big = h > (uint32_t)DUT;
  unsigned long long tn;
  uint32_t tb, tsl;
  block_excl_scan<DTILE>((unsigned long long)h, s_a, &tn);
  block_excl_scan<DTILE>((uint32_t)big, s_b, &tb);
  block_excl_scan<DTILE>(big ? big_slots(h) : 0u, s_b, &tsl);
  if (threadIdx.x == 0) ts[blockIdx.x] = DTileSums{tn, tb, tsl};
}

// Exclusive scan of the tile sums in place (one workgroup); the totals go to
// the info record.
__global__ void __launch_bounds__(1024) k_d_tile_scan(DTileSums* __restrict__ ts, uint32_t n_tiles,
                                                      DInfo* __restrict__ info) {
  __shared__ unsigned long long s_a[1024 / WAVE + 1];
  __shared__ uint32_t s_b[1024 / WAVE + 1];
  unsigned long long cn = 0;
  uint32_t cb = 0, cs = 0;
  for (uint32_t b0 = 0; b0 < n_tiles; b0 += 1024) {
    const uint32_t t = b0 + threadIdx.x;
    const DTileSums v = t < n_tiles ? ts[t] : DTileSums{0, 0, 0};
    unsigned long long tn;
    uint32_t tb, tsl;
    const unsigned long long en = block_excl_scan<1024>(v.n, s_a, &tn);
    const uint32_t eb = block_excl_scan<1024>(v.big, s_b, &tb);
    const uint32_t es = block_excl_scan<1024>(v.slots, s_b, &tsl);
    if (t < n_tiles) ts[t] = DTileSums{cn + en, cb + eb, cs + es};
    cn += tn;
    cb += tb;
    cs += tsl;
  }
  if (threadIdx.x == 0) {
    info->n_big = cb;
    info->big_slots = cs;
  }
}

// Per context: its base in context order (cbase, C + 1 entries), and for a big
// context its index among the big ones, its entry in the big list and its
// first unit slot.
__global__ void __launch_bounds__(DTILE) k_d_bases(const uint32_t* __restrict__ hist, uint32_t C,
                                                   const DTileSums* __restrict__ ts, uint32_t* __restrict__ cbase,
                                                   uint32_t* __restrict__ bidx, uint32_t* __restrict__ big_ctx,
                                                   uint32_t* __restrict__ big_slot0) {
  __shared__ unsigned long long s_a[DTILE / WAVE + 1];
  __shared__ uint32_t s_b[DTILE / WAVE + 1];
  const uint32_t c = blockIdx.x * DTILE + threadIdx.x;
  const uint32_t h = c < C ? hist[c] : 0u;
  const bool big = h > (uint32_t)DUT;
  const DTileSums base = ts[blockIdx.x];
  unsigned long long tn;
  uint32_t tb, tsl;
  const unsigned long long en = block_excl_scan<DTILE>((unsigned long long)h, s_a, &tn);
  const uint32_t eb = block_excl_scan<DTILE>((uint32_t)big, s_b, &tb);
  const uint32_t es = block_excl_scan<DTILE>(big ? big_slots(h) : 0u, s_b, &tsl);
  if (c < C) {
    cbase[c] = (uint32_t)(base.n + en);
    if (big) {
      const uint32_t b = base.big + eb;
      bidx[c] = b;
      big_ctx[b] = c;
      big_slot0[b] = base.slots + es;
    }
  }
  if (c == C - 1) cbase[C] = (uint32_t)(base.n + en + h);
}

// ---------------------------------------------------------------------------
// scatter
// ---------------------------------------------------------------------------
template <bool VEC, bool WEIGHTED>
__global__ void __launch_bounds__(DB)
k_d_scatter(const uint64_t* __restrict__ pc, const uint32_t* __restrict__ ctx, const uint8_t* __restrict__ stall,
            const uint32_t* __restrict__ weight, uint64_t n, uint32_t C, const uint32_t* __restrict__ cbase,
            uint32_t* __restrict__ cursor, DenseDev dd, uint32_t* __restrict__ rec, uint32_t* __restrict__ rw,
            DInfo* __restrict__ info) {
  __shared__ uint64_t s_lo[DENSE_MAX_WIN], s_hi[DENSE_MAX_WIN], s_d[DENSE_MAX_WIN + 1];
  __shared__ uint32_t s_base[DB / WAVE][DCH];
  for (uint32_t i = threadIdx.x; i < dd.n_win; i += DB) {
    s_lo[i] = dd.lo[i];
    s_hi[i] = dd.hi[i];
  }
  for (uint32_t i = threadIdx.x; i <= dd.n_win; i += DB) s_d[i] = dd.d[i];
  __syncthreads();
  const DenseDev t{s_lo, s_hi, s_d, dd.scope_of, dd.n_win, dd.tz};
  uint32_t* const sb = s_base[wave_id()];
  const uint64_t nw = (uint64_t)gridDim.x * (DB / WAVE);
  const uint64_t steps = (n + DCH - 1) / DCH;
  unsigned int far = 0;
  bool bad_stall = false, bad_pos = false;
  // a wave step's fields; the next step's loads are issued before this
  // step's reservations, so their latencies overlap
  struct StepIn {
    uint32_t v[DI];
    uint64_t q[DI];
    uint32_t s4;
    uint32_t wt[WEIGHTED ? DI : 1];
  };
  auto load_step = [&](uint64_t k, StepIn& in) {
    const uint64_t p0 = k * DCH + (uint64_t)lane_id() * DI;
    load_ctx4<VEC>(ctx, n, p0, in.v);
    if (VEC && p0 + DI <= n) {
      const ulonglong2 a = *reinterpret_cast<const ulonglong2*>(pc + p0);
      const ulonglong2 b = *reinterpret_cast<const ulonglong2*>(pc + p0 + 2);
      in.q[0] = a.x; in.q[1] = a.y; in.q[2] = b.x; in.q[3] = b.y;
      in.s4 = *reinterpret_cast<const uint32_t*>(stall + p0);
      if constexpr (WEIGHTED) {
        const uint4 ww = *reinterpret_cast<const uint4*>(weight + p0);
        in.wt[0] = ww.x; in.wt[1] = ww.y; in.wt[2] = ww.z; in.wt[3] = ww.w;
      }
    } else {
      in.s4 = 0;
#pragma unroll
      for (int j = 0; j < DI; ++j) {
        const bool ok = p0 + j < n;
        in.q[j] = ok ? pc[p0 + j] : 0ull;
        in.s4 |= (ok ? (uint32_t)stall[p0 + j] : 0u) << (8 * j);
        if constexpr (WEIGHTED) in.wt[j] = ok ? weight[p0 + j] : 0u;
      }
    }
  };
  uint64_t k = (uint64_t)blockIdx.x * (DB / WAVE) + wave_id();
  StepIn cur;
  if (k < steps) load_step(k, cur);
  for (; k < steps; k += nw) {
    StepIn nxt;
    if (k + nw < steps) load_step(k + nw, nxt);
    const uint64_t p0 = k * DCH + (uint64_t)lane_id() * DI;
    WaveRuns w;
#pragma unroll
    for (int j = 0; j < DI; ++j) w.v[j] = cur.v[j];
    wave_runs(w);
    // one reservation per run, by its last position; its base is left in LDS
    // at the run's head for the other positions of the run
#pragma unroll
    for (int j = 0; j < DI; ++j) {
      const uint32_t c = w.v[j];
      if (p0 + j >= n || c >= C || !w.tail[j]) continue;
      const uint32_t len = (uint32_t)(lane_id() * DI + j - w.head[j] + 1);
      uint32_t b = cbase[c] + atomicAdd(&cursor[c], len);
      if (b + len > cbase[c + 1]) {  // more samples than the histogram counted: never expected
        bad_pos = true;
        b = NONE32;
      }
      sb[w.head[j]] = b;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int j = 0; j < DI; ++j) {
      const uint32_t c = w.v[j];
      if (p0 + j >= n || c >= C) continue;
      const uint32_t b = sb[w.head[j]];
      if (b == NONE32) continue;
      const uint32_t pos = b + (uint32_t)(lane_id() * DI + j - w.head[j]);
      const uint32_t stj = (cur.s4 >> (8 * j)) & 0xFFu;
      uint32_t r;
      uint64_t D;
      if (stj >= NS) {
        bad_stall = true;
        r = 0;
      } else if (to_dense(t, cur.q[j], D)) {
        r = ((uint32_t)D << 4) | stj;
      } else {
        r = FAR_REC;
        ++far;
      }
      rec[pos] = r;
      if constexpr (WEIGHTED) rw[pos] = cur.wt[j];
    }
    // the LDS bases of this step are read before the next step writes them
    __builtin_amdgcn_wave_barrier();
    cur = nxt;
  }
  far = wave_sum(far);
  if (lane_id() == 0) {
    if (far) atomicAdd(&info->n_far, far);
  }
  if (__any(bad_stall) && lane_id() == 0) atomicOr(&info->err, DERR_STALL);
  if (__any(bad_pos) && lane_id() == 0) atomicOr(&info->err, DERR_INTERNAL);
}

// ---------------------------------------------------------------------------
// split of big contexts (one workgroup each)
// ---------------------------------------------------------------------------
constexpr int SB = 512;
constexpr int SB_PER = DNB / SB;  // buckets per thread
constexpr int SU_H = 16;          // records per thread in flight while counting
constexpr int SU_C = 8;           // ... while copying

// The end of the greedy part that starts at bucket k: the last bucket end e
// in [k + 1, DNB] with base[e] <= base[k] + DUT, and at least k + 1 (a single
// bucket over DUT samples).  base is non-decreasing, so the test holds on a
// prefix of the range: wave 0 probes it 64-ary in two rounds (every lane
// gets the answer).
__device__ inline uint32_t part_end(const uint32_t* s_base, uint32_t k) {
  static_assert(DNB <= WAVE * WAVE, "two 64-ary rounds cover the buckets");
  const int lane = lane_id();
  const uint32_t lim = s_base[k] + (uint32_t)DUT;
  const uint32_t lo = k + 1, n = (uint32_t)DNB - lo + 1;  // candidates lo .. DNB
  const uint32_t st = (n + WAVE - 1) / WAVE;                  // <= WAVE
  uint32_t idx = lo + (uint32_t)lane * st;
  unsigned long long m = __ballot(idx <= (uint32_t)DNB && s_base[idx <= (uint32_t)DNB ? idx : DNB] <= lim);
  if (m == 0) return lo;  // bucket k alone is over DUT
  const uint32_t j0 = lo + (uint32_t)(63 - __clzll((long long)m)) * st;  // last probe that holds
  idx = j0 + (uint32_t)lane;
  m = __ballot((uint32_t)lane < st && idx <= (uint32_t)DNB && s_base[idx <= (uint32_t)DNB ? idx : DNB] <= lim);
  return j0 + (uint32_t)(63 - __clzll((long long)m));
}

template <bool WEIGHTED>
__global__ void __launch_bounds__(SB)
k_d_split(const uint32_t* __restrict__ big_ctx, const uint32_t* __restrict__ big_slot0,
          const uint32_t* __restrict__ cbase, const uint32_t* __restrict__ rec, const uint32_t* __restrict__ rw,
          uint32_t bshift, uint32_t* __restrict__ rec2, uint32_t* __restrict__ rw2, DUnit* __restrict__ bunits,
          uint32_t* __restrict__ n_bunits, DInfo* __restrict__ info) {
  __shared__ uint32_t s_cnt[DNB];   // bucket counts, then cursors
  __shared__ uint32_t s_base[DNB + 1];
  __shared__ uint32_t s_tmp[SB / WAVE + 1];
  const uint32_t b = blockIdx.x;
  if (b >= info->n_big) return;
  const uint32_t c = big_ctx[b];
  const uint32_t s0 = cbase[c], nc = cbase[c + 1] - s0;
  for (int i = threadIdx.x; i < DNB; i += SB) s_cnt[i] = 0;
  __syncthreads();
  // SU_H records per thread are loaded before any is counted, so the loads
  // overlap
  for (uint32_t i0 = 0; i0 < nc; i0 += SU_H * SB) {
    uint32_t r[SU_H];
#pragma unroll
    for (int u = 0; u < SU_H; ++u) {
      const uint32_t i = i0 + (uint32_t)u * SB + threadIdx.x;
      r[u] = i < nc ? rec[s0 + i] : FAR_REC;
    }
#pragma unroll
    for (int u = 0; u < SU_H; ++u) {
      if (r[u] == FAR_REC) continue;
      const uint32_t k = (r[u] >> 4) >> bshift;
      atomicAdd(&s_cnt[k < (uint32_t)DNB ? k : DNB - 1], 1u);
    }
  }
  __syncthreads();
  // bucket bases: each thread scans its SB_PER consecutive buckets
  {
    uint32_t loc[SB_PER], sum = 0;
#pragma unroll
    for (int j = 0; j < SB_PER; ++j) {
      loc[j] = sum;
      sum += s_cnt[threadIdx.x * SB_PER + j];
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan<SB>(sum, s_tmp, &tot);
#pragma unroll
    for (int j = 0; j < SB_PER; ++j) s_base[threadIdx.x * SB_PER + j] = ex + loc[j];
    if (threadIdx.x == 0) s_base[DNB] = tot;
  }
  __syncthreads();
  // greedy packing along the chain of part ends (wave 0); parts start at
  // non-empty buckets, and empty buckets before a part's first records join
  // it.  The other waves clear the cursors meanwhile.
  const uint32_t total = s_base[DNB];
  if (threadIdx.x < WAVE) {
    const uint32_t slot0 = big_slot0[b], cap = big_slots(nc);
    uint32_t k = 0, m = 0;
    while (k < (uint32_t)DNB && s_base[k] < total) {
      const uint32_t e = part_end(s_base, k);
      const uint32_t len = s_base[e] - s_base[k];
      // a single bucket over DUT samples is counted, not sorted
      const bool hot = len > (uint32_t)DUT;
      if (threadIdx.x == 0) {
        if (m < cap) {
          bunits[slot0 + m] = DUnit{s0 + s_base[k], s0 + s_base[e], c, c + 1, hot ? DU_HOT : DU_PART, k << bshift, 0, 0};
        } else {
          atomicOr(&info->err, DERR_INTERNAL);
        }
      }
      ++m;
      k = e;
    }
    if (threadIdx.x == 0) n_bunits[b] = m < cap ? m : cap;
  } else {
    for (int i = threadIdx.x - WAVE; i < DNB; i += SB - WAVE) s_cnt[i] = 0;
  }
  __syncthreads();
  // records into bucket order
  for (uint32_t i0 = 0; i0 < nc; i0 += SU_C * SB) {
    uint32_t r[SU_C], wv[SU_C];
#pragma unroll
    for (int u = 0; u < SU_C; ++u) {
      const uint32_t i = i0 + (uint32_t)u * SB + threadIdx.x;
      r[u] = i < nc ? rec[s0 + i] : FAR_REC;
      if constexpr (WEIGHTED) wv[u] = i < nc ? rw[s0 + i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < SU_C; ++u) {
      if (r[u] == FAR_REC) continue;
      uint32_t k = (r[u] >> 4) >> bshift;
      k = k < (uint32_t)DNB ? k : DNB - 1;
      const uint32_t p = s_base[k] + atomicAdd(&s_cnt[k], 1u);
      rec2[s0 + p] = r[u];
      if constexpr (WEIGHTED) rw2[s0 + p] = wv[u];
    }
  }
}

// ---------------------------------------------------------------------------
// plan: greedy packing per tile of contexts
// ---------------------------------------------------------------------------
// A unit of small contexts starting at context i takes the longest run of
// contexts [i, j) with at most DUT records, at most maxc non-empty contexts
// and at most DUB contexts (the greedy rule, so every constraint is monotone in
// j); a big context is a segment of its own, with its parts as units.  Every
// thread finds next[i] for its contexts by binary search over the tile's
// prefix sums (a big context counts DUT + 1 records, so no unit reaches over
// it); thread 0 follows the chain from the tile's first context, which visits
// exactly the segment starts; a scan over the segments gives their first
// units, and every thread writes the descriptors of its segments.  The count
// launch (tile_off null) only records the tile's unit count.
constexpr uint32_t SEG_BIG = 0x80000000u;
constexpr int PL_PER = DTILE / DB;  // contexts per thread

__global__ void __launch_bounds__(DB)
k_d_plan(const uint32_t* __restrict__ hist, uint32_t C, uint32_t maxc, const uint32_t* __restrict__ bidx,
         const DUnit* __restrict__ bunits, const uint32_t* __restrict__ big_slot0, const uint32_t* __restrict__ n_bunits,
         const uint32_t* __restrict__ cbase, uint32_t* __restrict__ tile_units, const uint32_t* __restrict__ tile_off,
         DUnit* __restrict__ units) {
  __shared__ uint32_t s_ps[DTILE + 1];   // records before each context (big ones count DUT + 1)
  __shared__ uint32_t s_pn[DTILE + 1];   // non-empty contexts before each context
  __shared__ uint32_t s_next[DTILE];     // end of the segment that would start at each context
  __shared__ uint32_t s_seg[DTILE + 1];  // segment starts in order (| SEG_BIG), closed by the tile end
  __shared__ uint32_t s_useg[DTILE + 1]; // first unit of each segment (tile-relative), closed by the count
  __shared__ uint32_t s_tmp[DB / WAVE + 1];
  __shared__ uint32_t s_nseg;
  const uint32_t c0 = blockIdx.x * DTILE;
  const uint32_t nt = min((uint32_t)DTILE, C - c0);
  const int tid = threadIdx.x;
  // prefix sums: each thread owns PL_PER consecutive contexts
  uint32_t h[PL_PER], ls = 0, ln = 0;
#pragma unroll
  for (int q = 0; q < PL_PER; ++q) {
    const uint32_t i = tid * PL_PER + q;
    h[q] = i < nt ? hist[c0 + i] : 0u;
    ls += h[q] > (uint32_t)DUT ? (uint32_t)DUT + 1 : h[q];
    ln += h[q] > 0;
  }
  uint32_t ts, tn;
  uint32_t es = block_excl_scan<DB>(ls, s_tmp, &ts);
  uint32_t en = block_excl_scan<DB>(ln, s_tmp, &tn);
#pragma unroll
  for (int q = 0; q < PL_PER; ++q) {
    const uint32_t i = tid * PL_PER + q;
    s_ps[i] = es;
    s_pn[i] = en;
    es += h[q] > (uint32_t)DUT ? (uint32_t)DUT + 1 : h[q];
    en += h[q] > 0;
  }
  if (tid == 0) {
    s_ps[DTILE] = ts;
    s_pn[DTILE] = tn;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PL_PER; ++q) {
    const uint32_t i = tid * PL_PER + q;
    if (i >= nt) continue;
    uint32_t j;
    if (h[q] > (uint32_t)DUT) {
      j = i + 1;
    } else {
      // largest j <= min(nt, i + DUB) with ps[j] - ps[i] <= DUT and pn[j] - pn[i] <= maxc
      const uint32_t ls_lim = s_ps[i] + (uint32_t)DUT, ln_lim = s_pn[i] + maxc;
      uint32_t lo = i + 1, hi = min(nt, i + (uint32_t)DUB);
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (s_ps[mid] <= ls_lim && s_pn[mid] <= ln_lim) lo = mid;
        else hi = mid - 1;
      }
      j = lo;
    }
    s_next[i] = j;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t k = 0;
    for (uint32_t i = 0; i < nt; i = s_next[i]) {
      const bool big = s_ps[i + 1] - s_ps[i] > (uint32_t)DUT;
      s_seg[k++] = i | (big ? SEG_BIG : 0u);
    }
    s_seg[k] = nt;
    s_nseg = k;
  }
  __syncthreads();
  // first unit of each segment: a small segment is one unit, a big context
  // one per part
  const uint32_t nseg = s_nseg;
  {
    uint32_t cnt[PL_PER], loc = 0;
#pragma unroll
    for (int q = 0; q < PL_PER; ++q) {
      const uint32_t k = tid * PL_PER + q;
      cnt[q] = 0;
      if (k < nseg) {
        const uint32_t sg = s_seg[k];
        cnt[q] = (sg & SEG_BIG) ? n_bunits[bidx[c0 + (sg & ~SEG_BIG)]] : 1u;
      }
      loc += cnt[q];
    }
    uint32_t tot;
    uint32_t e = block_excl_scan<DB>(loc, s_tmp, &tot);
#pragma unroll
    for (int q = 0; q < PL_PER; ++q) {
      const uint32_t k = tid * PL_PER + q;
      if (k < nseg) s_useg[k] = e;
      e += cnt[q];
    }
    if (tid == 0) {
      s_useg[nseg] = tot;
      if (!tile_off) tile_units[blockIdx.x] = tot;
    }
  }
  if (!tile_off) return;
  __syncthreads();
  DUnit* out = units + tile_off[blockIdx.x];
  for (uint32_t k = tid; k < nseg; k += DB) {
    const uint32_t sg = s_seg[k], u0 = s_useg[k];
    const uint32_t i = sg & ~SEG_BIG, c = c0 + i;
    if (sg & SEG_BIG) {
      const uint32_t b = bidx[c], o = big_slot0[b], nb = s_useg[k + 1] - u0;
      for (uint32_t q = 0; q < nb; ++q) out[u0 + q] = bunits[o + q];
    } else {
      const uint32_t ce = c0 + (s_seg[k + 1] & ~SEG_BIG);
      out[u0] = DUnit{cbase[c], cbase[ce], c, ce, DU_SMALL, 0, 0, 0};
    }
  }
}

// exclusive scan of the tiles' unit counts (one workgroup)
__global__ void __launch_bounds__(1024) k_d_unit_scan(const uint32_t* __restrict__ tile_units, uint32_t n_tiles,
                                                      uint32_t* __restrict__ tile_off, DInfo* __restrict__ info) {
  __shared__ uint32_t s_t[1024 / WAVE + 1];
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < n_tiles; b0 += 1024) {
    const uint32_t t = b0 + threadIdx.x;
    const uint32_t v = t < n_tiles ? tile_units[t] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<1024>(v, s_t, &tot);
    if (t < n_tiles) tile_off[t] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) info->n_units = carry;
}

// ---------------------------------------------------------------------------
// units
// ---------------------------------------------------------------------------
struct DUnitArgs {
  const DUnit* units;
  const uint32_t* rec;
  const uint32_t* rw;
  const uint32_t* rec2;
  const uint32_t* rw2;
  const uint32_t* hist;
  const uint32_t* cbase;
  uint32_t C;
  uint32_t bshift;
  DenseDev dd;
  DInfo* info;
  unsigned long long* status;  // per unit: look-back word
  // per workgroup, two slots of DUT keys (one for the unit being sorted, one
  // for the unit waiting to be written): the keys as u32, with their counts
  // as u16 (a unit's count is at most DUT) or, with weights, as u64
  uint32_t* stage_key;
  uint16_t* stage_c16;
  unsigned long long* stage_cnt;
  OutDev out;
};

// A sorted unit whose keys wait in a staging slot for their offset.
struct DPend {
  DUnit d;
  uint32_t t, nU, dmin, dmax, nl, slot;
  bool valid;
};

struct DUnitSmem {
  DPend pend[2];                 // per slot: the unit staged there (kept in LDS, not registers)
  // the unit claimed next and its descriptor (its context bases and records
  // are fetched into LDS while the previous unit is written out)
  DUnit d;
  uint32_t cbpf[DUB + 1];        // context bases of the unit's contexts (small units), closed by the next
  uint32_t lstart[MAXC + 1];     // record offset of each non-empty local context, closed by n_u
  uint32_t lctx[2][MAXC];        // per slot: context id of each local context
  uint8_t lrank[2][DUB];         // per slot and context of the unit: non-empty contexts before it
  unsigned long long loff[2][MAXC + 1];  // per slot: keys of the local contexts before each
  unsigned long long P;
  uint32_t t, nl, red_min, red_max;
  uint32_t tmp[DUB / WAVE + 1];
};

// Decoupled look-back over the units' key counts, in two halves: a unit
// publishes its count as soon as it knows it, and finds its offset (the keys
// of all units before it) only when it is about to write, one unit later, so
// that predecessors slower than itself rarely keep it waiting.  Unit 0 is
// inclusive at once.
__device__ inline void publish_count(unsigned long long* status, uint32_t t, unsigned long long agg) {
  __hip_atomic_store(&status[t], (t == 0 ? LB_INC : LB_AGG) | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by every lane of wave 0 after publish_count(t); lane l reads the
// word of unit j - l, so one round of loads covers 64 predecessors: the words
// up to the nearest inclusive one are summed when all of them are there;
// otherwise the ready words before the first missing one are summed and the
// window moves past them.  Publishes the unit's inclusive count.  The wait is
// bounded, so a broken chain ends the kernel with an error instead of hanging
// it.
__device__ inline unsigned long long look_back(unsigned long long* status, uint32_t t, unsigned long long agg,
                                               unsigned int* err) {
  const int lane = lane_id();
  if (t == 0) return 0;
  unsigned long long excl = 0;
  long long j = (long long)t - 1;  // newest predecessor not yet summed
  uint32_t spins = 0;
  while (true) {
    const long long q = j - lane;
    // before unit 0 stands an inclusive zero (unit 0 is always inclusive, so
    // the window never needs it; it only keeps the lanes well defined)
    const unsigned long long s =
        q >= 0 ? __hip_atomic_load(&status[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : LB_INC;
    const unsigned long long f = s & ~LB_VAL;
    const unsigned long long missing = __ballot(f == 0);
    const unsigned long long inc = __ballot(f == LB_INC);
    // lanes 0 .. li hold the words up to the nearest inclusive one (li = 63
    // when there is none in the window)
    const int li = inc ? __ffsll((long long)inc) - 1 : WAVE - 1;
    const unsigned long long need = li == WAVE - 1 ? ~0ull : ((2ull << li) - 1ull);
    if (missing & need) {
      const int nr = __ffsll((long long)(missing & need)) - 1;  // first lane without a word
      if (nr == 0) {
        if (++spins > LB_SPIN_LIMIT ||
            ((spins & 1023u) == 0 &&
             (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & DERR_LOOKBACK))) {
          if (lane == 0) atomicOr(err, DERR_LOOKBACK);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += wave_sum(lane < nr ? (s & LB_VAL) : 0ull);
      j -= nr;
      continue;
    }
    excl += wave_sum(lane <= li ? (s & LB_VAL) : 0ull);
    if (inc) break;
    j -= WAVE;
  }
  if (lane == 0) __hip_atomic_store(&status[t], LB_INC | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

// A value every lane holds alike, moved to scalar registers.
__device__ inline unsigned long long uniform_u64(unsigned long long v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// Copy n words from global memory into LDS without passing through
// registers (the LDS DMA of global_load_lds): wave w moves the 64-word chunks
// w, w + 8, ...; lane l the word l of each.  The copy is complete once the
// issuing waves have waited for their vector memory counter.
__device__ inline void lds_fetch(uint32_t* lds_dst, const uint32_t* src, uint32_t n) {
  uint32_t l = (uint32_t)lane_id();
  asm volatile("" : "+v"(l));  // keep the per-lane addresses out of the caller's loop invariants
  for (uint32_t c = (uint32_t)wave_id(); c * WAVE < n; c += DUB / WAVE)
    if (c * WAVE + l < n) __builtin_amdgcn_global_load_lds(src + c * WAVE + l, lds_dst + c * WAVE, 4, 0, 0);
}

__device__ inline void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0) only

// The last unit closes the context offsets and reports the key count.
__device__ inline void close_units(const DUnitArgs& a, unsigned long long end) {
  a.out.ctx_off[a.C] = end;
  a.info->total_keys = end;
}

// A counted part: one coordinate bucket [d0, d0 + 2^bshift) of one context.
// Its keys (coordinate offset, stall) are counted in LDS, HOT_CAP counters at
// a time (a bucket may span several such chunks of its key range); the
// non-empty counters, in order, are the part's keys.  The first sweep counts
// the keys of every chunk, so that the part can publish its count; a part of
// one chunk then writes from the counters it has, a wider one counts each
// chunk again while writing.
constexpr uint32_t HOT_CAP = DUT;  // counters in the sort's exchange plane

template <bool WEIGHTED>
__device__ inline uint32_t hot_count(DSmem& sm, DUnitSmem& du, const DUnitArgs& a, const DUnit& d, uint32_t k0,
                                     uint32_t R, bool& ovf) {
  const int tid = threadIdx.x;
  uint32_t* cnt = sm.buf;
  const uint32_t kn = min(HOT_CAP, R - k0);
  for (uint32_t i = tid; i < kn; i += DUB) cnt[i] = 0;
  __syncthreads();
  constexpr int HU = 4;  // records per thread in flight
  for (uint32_t i0 = d.s0; i0 < d.s1; i0 += HU * DUB) {
    uint32_t r[HU], wv[HU];
#pragma unroll
    for (int u = 0; u < HU; ++u) {
      const uint32_t i = i0 + (uint32_t)u * DUB + tid;
      r[u] = i < d.s1 ? a.rec2[i] : FAR_REC;
      wv[u] = WEIGHTED ? (i < d.s1 ? a.rw2[i] : 0u) : 1u;
    }
#pragma unroll
    for (int u = 0; u < HU; ++u) {
      if (r[u] == FAR_REC) continue;
      const uint32_t k = (((r[u] >> 4) - d.d0) << 4) | (r[u] & 15u);
      if (k >= R) {
        ovf = true;
        continue;
      }
      if (k < k0 || k >= k0 + kn) continue;
      const uint32_t old = atomicAdd(&cnt[k - k0], wv[u]);
      ovf |= old + wv[u] < old;
    }
  }
  __syncthreads();
  // thread t owns a block of `per` consecutive counters
  const uint32_t per = (kn + DUB - 1) / DUB;
  uint32_t mine = 0;
  for (uint32_t j = 0; j < per; ++j) {
    const uint32_t i = tid * per + j;
    mine += i < kn && cnt[i] != 0;
  }
  return mine;
}

template <bool WEIGHTED>
__device__ inline void hot_emit(DSmem& sm, const DUnitArgs& a, const DUnit& d, uint32_t k0, uint32_t R,
                                uint64_t o) {
  const int tid = threadIdx.x;
  const uint32_t* cnt = sm.buf;
  const uint32_t kn = min(HOT_CAP, R - k0);
  const uint32_t per = (kn + DUB - 1) / DUB;
  for (uint32_t j = 0; j < per; ++j) {
    const uint32_t i = tid * per + j;
    if (i >= kn || cnt[i] == 0) continue;
    const uint32_t k = k0 + i;
    const uint64_t D = d.d0 + (k >> 4);
    a.out.ctx[o] = d.cb;
    a.out.pc[o] = from_dense(a.dd, D);
    a.out.stall[o] = (uint8_t)(k & 15u);
    a.out.count[o] = cnt[i];
    a.out.scope[o] = a.dd.scope_of[D];
    ++o;
  }
}

// A counted part publishes its count and waits for its offset at once (its
// keys live in the counters, not in a staging slot).
template <bool WEIGHTED>
__device__ inline void hot_unit(DSmem& sm, DUnitSmem& du, const DUnitArgs& a, const DUnit& d, uint32_t n_units) {
  const int tid = threadIdx.x;
  const uint32_t R = (1u << a.bshift) * NS;  // the bucket's key range
  const uint32_t nch = (R + HOT_CAP - 1) / HOT_CAP;
  bool ovf = false;
  uint32_t nU = 0, first = 0, mine = 0;
  for (uint32_t ch = 0; ch < nch; ++ch) {
    mine = hot_count<WEIGHTED>(sm, du, a, d, ch * HOT_CAP, R, ovf);
    uint32_t tot;
    first = block_excl_scan<DUB>(mine, du.tmp, &tot);
    nU += tot;
  }
  if (ovf) atomicOr(&a.info->err, DERR_OVERFLOW);
  if (tid < WAVE) {
    if (tid == 0) publish_count(a.status, du.t, nU);
    const unsigned long long p = look_back(a.status, du.t, nU, &a.info->err);
    if (tid == 0) du.P = p;
  }
  __syncthreads();
  const unsigned long long P = du.P;
  if (tid == 0 && d.s0 == a.cbase[d.cb]) a.out.ctx_off[d.cb] = P;
  if (tid == 0 && du.t == n_units - 1) close_units(a, P + nU);
  if (nch == 1) {  // the counters of the only chunk are still in LDS
    hot_emit<WEIGHTED>(sm, a, d, 0, R, P + first);
    return;
  }
  uint64_t base = P;
  for (uint32_t ch = 0; ch < nch; ++ch) {
    bool o2 = false;
    mine = hot_count<WEIGHTED>(sm, du, a, d, ch * HOT_CAP, R, o2);
    uint32_t tot;
    first = block_excl_scan<DUB>(mine, du.tmp, &tot);
    hot_emit<WEIGHTED>(sm, a, d, ch * HOT_CAP, R, base + first);
    base += tot;
    __syncthreads();  // the next chunk clears the counters
  }
}

__device__ inline uint64_t slot_base(uint32_t slot) { return ((uint64_t)blockIdx.x * 2 + slot) * DUT; }

// Sort and reduce one SMALL or PART unit of n_u > 0 records with IT items
// per thread (the least that holds it: a sort pass costs in proportion to the
// slots it sorts), publish its key count, and stage its unique keys and
// counts in the slot.
template <bool WEIGHTED, int IT>
__device__ __forceinline__ void sort_unit(DSmem& sm, DUnitSmem& du, const DUnitArgs& a, const DUnit& d,
                                          const uint32_t* __restrict__ rec, const uint32_t* __restrict__ rw,
                                          uint32_t n_u, uint32_t nl, uint32_t t, uint32_t slot, uint32_t& nU,
                                          uint32_t& dmin_out, uint32_t& dmax_out) {
  using S = BlockRadix<DUB, IT>;
  const int tid = threadIdx.x;
  // every record's local context, from the contexts' start offsets, in the
  // LDS of the radix counters (free until the sort)
  uint8_t* const lctx_of = reinterpret_cast<uint8_t*>(sm.cnt);
  for (uint32_t l = 0; l < nl; ++l)
    for (uint32_t p = du.lstart[l] + tid; p < du.lstart[l + 1]; p += DUB) lctx_of[p] = (uint8_t)l;
  __syncthreads();
  // gather: item i of thread t is record i * DUB + t of the unit (D << 4 |
  // stall).  Unweighted records were fetched into the exchange plane while
  // the previous unit was written; weighted ones are read from global memory
  // here (coalesced).
  uint32_t key[IT], val[IT];
  uint32_t dmin = 0xFFFFFFFFu, dmax = 0;
  // (the thread index is hidden from the optimiser here, so that the slot
  // indices are recomputed per unit instead of being hoisted out of the unit
  // loop, where they would be held, or spilled, for the whole kernel)
  uint32_t tq = (uint32_t)tid;
  asm volatile("" : "+v"(tq));
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    key[i] = 0;
    val[i] = 0;
    const uint32_t j = (uint32_t)i * DUB + tq;
    if (j < n_u) {
      uint32_t r = WEIGHTED ? rec[d.s0 + j] : sm.buf[j];
      if (r == FAR_REC) r = 0;  // the call is redone by the general path
      key[i] = r;
      if constexpr (WEIGHTED) val[i] = rw[d.s0 + j];
      const uint32_t D = r >> 4;
      dmin = min(dmin, D);
      dmax = max(dmax, D);
    }
  }
  // unit-wide coordinate range: keys are taken relative to its smallest
  dmin = wave_min_u32(dmin);
  dmax = wave_max_u32(dmax);
  if (lane_id() == 0) {
    atomicMin(&du.red_min, dmin);
    atomicMax(&du.red_max, dmax);
  }
  __syncthreads();
  dmin = du.red_min;
  dmin_out = dmin;
  dmax_out = du.red_max;
  const int pcb = bits_for(du.red_max - dmin);
  const int kbits = bits_for(nl - 1) + pcb + 4;
  // the plan keeps local contexts few enough that keys fit 31 bits
  if (kbits > 31 && tid == 0) atomicOr(&a.info->err, DERR_WIDE);
  const uint32_t empty = 1u << min(kbits, 31);
  // keys: local context, coordinate offset, stall (the local context from
  // the LDS table, still intact: the sort has not begun)
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const uint32_t j = (uint32_t)i * DUB + tq;
    const uint32_t v = key[i];
    key[i] = j < n_u ? ((uint32_t)lctx_of[j] << (pcb + 4)) | (((v >> 4) - dmin) << 4) | (v & 15u) : empty;
  }
  // empty slots sort after every key: kbits + 1 bits, no per-slot test
  if constexpr (WEIGHTED)
    S::template sort<1, true>(key, val, val, min(kbits, 31) + 1, (int)n_u, true, sm.buf, sm.cnt, sm.doff);
  else
    S::template sort<0, true>(key, val, val, min(kbits, 31) + 1, (int)n_u, true, sm.buf, sm.cnt, sm.doff);
  uint32_t first;
  find_heads<uint32_t, IT>(sm, key, n_u, nl, pcb, first, nU);
  if (tid == 0) publish_count(a.status, t, nU);
  // stage the compacted keys and their counts (consecutive threads take
  // consecutive keys)
  uint32_t* const skey = a.stage_key + slot_base(slot);
  if constexpr (WEIGHTED) {
    for (uint32_t ui = tid; ui < nU; ui += DUB) skey[ui] = sm.buf[ui];
    weighted_counts<uint32_t, IT>(sm, key, val, n_u, first, a.stage_cnt + slot_base(slot));
  } else if (tid >= WAVE) {
    // waves 1.. stage; wave 0 goes on to the look-back and the claim, whose
    // loads would otherwise wait behind these stores (a wave's memory
    // operations complete in order)
    uint16_t* const sc16 = a.stage_c16 + slot_base(slot);
    for (uint32_t ui = tid - WAVE; ui < nU; ui += DUB - WAVE) {
      skey[ui] = sm.buf[ui];
      sc16[ui] = (uint16_t)(sm.upos[ui + 1] - sm.upos[ui]);
    }
  }
}

// Find the waiting unit's offset (the only wait on other workgroups) ...
__device__ inline void flush_offset(DUnitSmem& du, const DUnitArgs& a, uint32_t slot) {
  const int tid = threadIdx.x;
  const DPend pd = du.pend[slot];
  if (!pd.valid) return;
  if (tid < WAVE) {
    const unsigned long long p = look_back(a.status, pd.t, pd.nU, &a.info->err);
    if (tid == 0) du.P = p;
  }
  __syncthreads();
}

// ... then write its keys from the staging slot (flush_offset has set
// du.P), then the offsets of its contexts.  The output bases are made
// uniform so that every store addresses with a 32-bit offset, and the
// outputs, not read again here, bypass the caches.
template <bool WEIGHTED>
__device__ inline void flush_write(DUnitSmem& du, const DUnitArgs& a, uint32_t slot, uint32_t n_units) {
  const int tid = threadIdx.x;
  const DPend pd = du.pend[slot];
  if (!pd.valid) return;
  const unsigned long long P = uniform_u64(du.P);
  const uint32_t nU = pd.nU, dmin = pd.dmin;
  const uint32_t* const skey = a.stage_key + slot_base(pd.slot);
  const uint16_t* const sc16 = a.stage_c16 + slot_base(pd.slot);
  const unsigned long long* const scnt = a.stage_cnt + slot_base(pd.slot);
  const int pcb = bits_for(pd.dmax - dmin);
  const uint32_t pmask = (1u << pcb) - 1u;
  uint32_t* const octx = a.out.ctx + P;
  uint64_t* const opc = a.out.pc + P;
  uint8_t* const ostall = a.out.stall + P;
  unsigned long long* const ocnt = a.out.count + P;
  uint32_t* const oscope = a.out.scope + P;
  const uint32_t* const lctx = du.lctx[pd.slot];
  // the windows the unit's coordinates can fall in; up to WR of them are
  // held in registers (their first coordinates and pc bases), so a key's pc
  // needs no search
  constexpr int WR = 4;
  const uint32_t w0 = last_le(a.dd.d, a.dd.n_win, (uint64_t)dmin);
  const uint32_t w1 = last_le(a.dd.d, a.dd.n_win, (uint64_t)pd.dmax);
  const bool few = w1 - w0 < (uint32_t)WR;
  uint32_t wfirst[WR];
  uint64_t wbase[WR];  // pc of coordinate 0 if the window extended down to it
#pragma unroll
  for (int q = 0; q < WR; ++q) {
    const uint32_t w = min(w0 + (uint32_t)q, w1);
    wfirst[q] = q == 0 ? 0u : (w0 + (uint32_t)q <= w1 ? (uint32_t)a.dd.d[w] : 0xFFFFFFFFu);
    wbase[q] = a.dd.lo[w] - (a.dd.d[w] << a.dd.tz);
  }
  // OB keys per thread per sweep: their staged keys and counts, then their
  // scope labels, are all requested before the sweep's first store (a row j
  // is read only when the unit has keys there, a condition the whole
  // workgroup shares; a slot past nU reads coordinate dmin)
  constexpr int OB = 8;
  uint32_t tq = (uint32_t)tid;  // hidden from the optimiser, as in the gather
  asm volatile("" : "+v"(tq));
  for (uint32_t u0 = 0; u0 < nU; u0 += OB * DUB) {
    uint32_t sk[OB];
    uint32_t sc[OB];
    typename std::conditional<WEIGHTED, unsigned long long, uint32_t>::type wc[OB];
#pragma unroll
    for (int j = 0; j < OB; ++j) {
      sk[j] = 0;
      wc[j] = 0;
      if (u0 + (uint32_t)j * DUB < nU) {
        const uint32_t ui = u0 + (uint32_t)j * DUB + tq;
        sk[j] = skey[ui];
        if constexpr (WEIGHTED) wc[j] = scnt[ui];
        else wc[j] = sc16[ui];
      }
    }
#pragma unroll
    for (int j = 0; j < OB; ++j) {
      sc[j] = 0;
      const uint32_t ui = u0 + (uint32_t)j * DUB + tq;
      if (u0 + (uint32_t)j * DUB < nU)
        sc[j] = a.dd.scope_of[dmin + (ui < nU ? (sk[j] >> 4) & pmask : 0u)];
    }
#pragma unroll
    for (int j = 0; j < OB; ++j) {
      const uint32_t ui = u0 + (uint32_t)j * DUB + tq;
      if (ui < nU) {
        const uint32_t kk = sk[j];
        const uint32_t lc = kk >> (pcb + 4);
        const uint32_t D = dmin + ((kk >> 4) & pmask);
        uint64_t pc;
        if (few) {
          uint64_t b = wbase[0];
#pragma unroll
          for (int q = 1; q < WR; ++q) b = D >= wfirst[q] ? wbase[q] : b;
          pc = b + ((uint64_t)D << a.dd.tz);
        } else {
          pc = from_dense(a.dd, D);
        }
        __builtin_nontemporal_store(lctx[lc < pd.nl ? lc : 0], &octx[ui]);
        __builtin_nontemporal_store(pc, &opc[ui]);
        __builtin_nontemporal_store((uint8_t)(kk & 15u), &ostall[ui]);
        __builtin_nontemporal_store((unsigned long long)wc[j], &ocnt[ui]);
        __builtin_nontemporal_store(sc[j], &oscope[ui]);
      }
    }
  }
  // context offsets: every context of the unit (empty ones included) starts
  // after the keys of the non-empty contexts before it
  const DUnit& d = pd.d;
  if (d.kind == DU_PART) {
    if (tid == 0 && d.s0 == a.cbase[d.cb]) a.out.ctx_off[d.cb] = P;
  } else {
    for (uint32_t i = tid; i < d.ce - d.cb; i += DUB) {
      const uint32_t r = du.lrank[pd.slot][i];
      a.out.ctx_off[d.cb + i] = P + du.loff[pd.slot][r < pd.nl ? r : pd.nl];
    }
  }
  if (tid == 0 && pd.t == n_units - 1) close_units(a, P + nU);
  __syncthreads();  // the slot's tables are rebuilt by the next unit but one
}

// Fetch what unit `dn` (number tn) needs into LDS before its turn: the bases
// of its contexts (small units) and, unweighted, its records (into the
// exchange plane, which is free between one unit's staging and the next
// unit's sort).  A counted part reads its records itself.
template <bool WEIGHTED>
__device__ inline void prefetch_unit(DSmem& sm, DUnitSmem& du, const DUnitArgs& a, const DUnit& dn, uint32_t tn,
                                     uint32_t n_units) {
  if (tn >= n_units || dn.kind == DU_HOT) return;
  if (dn.kind != DU_PART) lds_fetch(du.cbpf, a.cbase + dn.cb, dn.ce - dn.cb + 1);
  if constexpr (!WEIGHTED) lds_fetch(sm.buf, (dn.kind == DU_PART ? a.rec2 : a.rec) + dn.s0, dn.s1 - dn.s0);
}

// Claim the next unit and read its descriptor (into du.t, du.d).  Called
// only when the workgroup has published the key count of every unit it
// holds, so that no other workgroup can be kept waiting on a unit claimed
// here while this one waits in turn.
__device__ inline void claim_unit(DUnitSmem& du, const DUnitArgs& a, uint32_t n_units) {
  if (threadIdx.x == 0) {
    const uint32_t t = atomicAdd(&a.info->ticket, 1u);
    du.t = t;
    if (t < n_units) du.d = a.units[t];
  }
  __syncthreads();
}

template <bool WEIGHTED>
__global__ void __launch_bounds__(DUB, 4) k_d_units(DUnitArgs a) {
  __shared__ DSmem sm;
  __shared__ DUnitSmem du;
  const int tid = threadIdx.x;
  // dense windows in LDS once
  a.dd = stage_dense(sm, a.dd);
  const uint32_t n_units = a.info->n_units;
  if (tid == 0) du.pend[0].valid = du.pend[1].valid = false;
  claim_unit(du, a, n_units);
  prefetch_unit<WEIGHTED>(sm, du, a, du.d, du.t, n_units);
  wait_vmem();
  __syncthreads();
  uint32_t slot = 0;
  while (true) {
    const uint32_t t = du.t;
    if (t >= n_units) break;
    const DUnit d = du.d;
    if (d.kind == DU_HOT) {
      flush_offset(du, a, slot ^ 1u);
      flush_write<WEIGHTED>(du, a, slot ^ 1u, n_units);
      if (tid == 0) du.pend[slot ^ 1u].valid = false;
      hot_unit<WEIGHTED>(sm, du, a, d, n_units);
      __syncthreads();  // the counters are free for the next unit's records
      claim_unit(du, a, n_units);
      prefetch_unit<WEIGHTED>(sm, du, a, du.d, du.t, n_units);
    } else {
      const bool part = d.kind == DU_PART;
      const uint32_t* rec = part ? a.rec2 : a.rec;
      const uint32_t* rw = part ? a.rw2 : a.rw;
      const uint64_t n_u = d.s1 - d.s0;
      // the unit's non-empty contexts and every context's rank among them
      if (part) {
        if (tid == 0) {
          du.red_min = 0xFFFFFFFFu;
          du.red_max = 0;
          du.nl = 1;
          du.lstart[0] = 0;
          du.lstart[1] = (uint32_t)n_u;
          du.lctx[slot][0] = d.cb;
        }
      } else {
        const uint32_t nc = d.ce - d.cb;  // <= DUB
        const uint32_t c = d.cb + tid;
        const uint32_t cb0 = (uint32_t)tid < nc ? du.cbpf[tid] : 0u;
        const uint32_t h = (uint32_t)tid < nc ? du.cbpf[tid + 1] - cb0 : 0u;
        uint32_t nl;
        const uint32_t r = block_excl_scan<DUB>(h > 0 ? 1u : 0u, du.tmp, &nl);
        if ((uint32_t)tid < nc) {
          du.lrank[slot][tid] = (uint8_t)min(r, (uint32_t)MAXC);
          if (h > 0 && r < (uint32_t)MAXC) {
            du.lstart[r] = cb0 - d.s0;
            du.lctx[slot][r] = c;
          }
        }
        if (tid == 0) {
          du.red_min = 0xFFFFFFFFu;
          du.red_max = 0;
          du.nl = nl;
          if (nl > (uint32_t)MAXC) atomicOr(&a.info->err, DERR_INTERNAL);
          du.lstart[nl < (uint32_t)MAXC ? nl : MAXC] = (uint32_t)n_u;
        }
      }
      __syncthreads();
      const uint32_t nl = min(du.nl, (uint32_t)MAXC);
      uint32_t nU = 0, dmin = 0, dmax = 0;
      if (n_u == 0) {  // only empty contexts
        if (tid == 0) publish_count(a.status, t, 0);
      } else if (n_u <= 4u * DUB) {
        sort_unit<WEIGHTED, 4>(sm, du, a, d, rec, rw, (uint32_t)n_u, nl, t, slot, nU, dmin, dmax);
      } else if (n_u <= 8u * DUB) {
        sort_unit<WEIGHTED, 8>(sm, du, a, d, rec, rw, (uint32_t)n_u, nl, t, slot, nU, dmin, dmax);
      } else {
        sort_unit<WEIGHTED, DUI>(sm, du, a, d, rec, rw, (uint32_t)n_u, nl, t, slot, nU, dmin, dmax);
      }
      // keys before each local context (sm.ucnt holds keys per local
      // context; wave 0 wrote it and reads it here)
      if (tid < WAVE) {
        const uint32_t l = (uint32_t)tid;
        const uint32_t v = n_u > 0 && l < nl ? sm.ucnt[l] : 0u;
        const uint32_t inc = wave_incl_scan_u32(v);
        du.loff[slot][l] = inc - v;
        if (l == WAVE - 1) du.loff[slot][MAXC] = inc;
      }
      if (tid == 0) du.pend[slot] = DPend{d, t, nU, dmin, dmax, nl, slot, true};
      // the previous unit's offset is due by now; once it is known, every
      // unit held here has published its count: claim the next unit and
      // fetch its data while the previous unit is written
      flush_offset(du, a, slot ^ 1u);
      claim_unit(du, a, n_units);
      prefetch_unit<WEIGHTED>(sm, du, a, du.d, du.t, n_units);
      flush_write<WEIGHTED>(du, a, slot ^ 1u, n_units);
      slot ^= 1u;
    }
    // the fetches have landed
    wait_vmem();
    __syncthreads();
  }
  flush_offset(du, a, slot ^ 1u);
  flush_write<WEIGHTED>(du, a, slot ^ 1u, n_units);
}

}  // namespace

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
bool dense_path_fits(const hpa_structure_map* map, const hpa_samples* smp) {
  if (!map->dense || map->n_win == 0 || map->n_win > DENSE_MAX_WIN) return false;
  if (smp->n >= (1ull << 32) - 1 || smp->n_ctx >= (1u << 31)) return false;
  // records hold a coordinate in 26 bits (a record below FAR_REC)
  return map->n_dense <= (1ull << 26);
}

// Returns false (nothing written, no error) when a sample's pc has no dense
// coordinate: the caller then runs the general pipeline.
bool attribute_dense(hpa_ctx* ctx, const hpa_structure_map* map, const hpa_samples* smp, hipStream_t s,
                     hpa_attribution* A) {
  const uint64_t n = smp->n;
  const uint32_t C = smp->n_ctx;
  const bool weighted = smp->weight != nullptr;
  StageTimer tm(ctx, s);
  uint32_t bshift = 0;
  while (((map->n_dense - 1) >> bshift) >= (uint64_t)DNB) ++bshift;
  const uint32_t n_tiles = (C + DTILE - 1) / DTILE;
  // key = (local context, coordinate offset, stall) in 31 bits: the offset
  // needs at most the bits of n_dense - 1, so a unit takes at most
  // 2^(27 - those bits) non-empty contexts (and at most MAXC)
  uint32_t dbits = 0;
  while (dbits < 64 && ((map->n_dense - 1) >> dbits)) ++dbits;
  const uint32_t maxc = dbits >= 27 ? 1u : std::min<uint32_t>((uint32_t)MAXC, 1u << (27 - dbits));
  const uint64_t max_big = n / (DUT + 1) + 1;
  // sum over big contexts of 2 * ceil(n_c / DUT) + 1 <= 2 * (N / DUT + n_big) + n_big
  const uint64_t max_bslots = 2 * (n / DUT) + 3 * max_big + 8;
  const uint64_t max_units = (uint64_t)C + max_bslots + n_tiles;
  DBuf d_info(ctx, sizeof(DInfo), s), d_hist(ctx, (uint64_t)C * 4, s), d_cbase(ctx, ((uint64_t)C + 1) * 4, s),
      d_cursor(ctx, (uint64_t)C * 4, s), d_bidx(ctx, (uint64_t)C * 4, s),
      d_ts(ctx, (uint64_t)n_tiles * sizeof(DTileSums), s), d_bctx(ctx, max_big * 4, s),
      d_bslot0(ctx, max_big * 4, s), d_nbu(ctx, max_big * 4, s), d_bunits(ctx, max_bslots * sizeof(DUnit), s),
      d_tu(ctx, (uint64_t)n_tiles * 4, s), d_toff(ctx, (uint64_t)n_tiles * 4, s),
      d_units(ctx, max_units * sizeof(DUnit), s), d_status(ctx, max_units * 8, s), d_rec(ctx, n * 4, s),
      d_rec2(ctx, n * 4, s), d_rw, d_rw2;
  if (weighted) {
    d_rw = DBuf(ctx, n * 4, s);
    d_rw2 = DBuf(ctx, n * 4, s);
  }
  HPA_HIP(hipMemsetAsync(d_info.p, 0, sizeof(DInfo), s));
  HPA_HIP(hipMemsetAsync(d_hist.p, 0, (uint64_t)C * 4, s));
  HPA_HIP(hipMemsetAsync(d_cursor.p, 0, (uint64_t)C * 4, s));
  HPA_HIP(hipMemsetAsync(d_status.p, 0, max_units * 8, s));
  DInfo* info = d_info.as<DInfo>();
  const bool vec = ((uintptr_t)smp->pc % 16 == 0) && ((uintptr_t)smp->ctx % 16 == 0) &&
                   ((uintptr_t)smp->stall % 4 == 0) && (!weighted || (uintptr_t)smp->weight % 16 == 0);
  const unsigned grid = (unsigned)std::max<uint64_t>(
      1, std::min<uint64_t>((n + DCH * (DB / WAVE) - 1) / (DCH * (DB / WAVE)), (uint64_t)ctx->n_cu * 8));
  tm.begin("d_hist");
  if (vec) k_d_hist<true><<<grid, DB, 0, s>>>(smp->ctx, n, C, d_hist.as<uint32_t>(), info);
  else k_d_hist<false><<<grid, DB, 0, s>>>(smp->ctx, n, C, d_hist.as<uint32_t>(), info);
  HPA_HIP(hipGetLastError());
  tm.end(n, 0);
  tm.begin("d_bases");
  k_d_tile_sums<<<n_tiles, DTILE, 0, s>>>(d_hist.as<uint32_t>(), C, d_ts.as<DTileSums>());
  k_d_tile_scan<<<1, 1024, 0, s>>>(d_ts.as<DTileSums>(), n_tiles, info);
  k_d_bases<<<n_tiles, DTILE, 0, s>>>(d_hist.as<uint32_t>(), C, d_ts.as<DTileSums>(), d_cbase.as<uint32_t>(),
                                      d_bidx.as<uint32_t>(), d_bctx.as<uint32_t>(), d_bslot0.as<uint32_t>());
  HPA_HIP(hipGetLastError());
  tm.end(C, 0);
  const DenseDev dd{map->win_lo.as<uint64_t>(), map->win_hi.as<uint64_t>(), map->win_d.as<uint64_t>(),
                    map->scope_of.as<uint32_t>(), map->n_win, map->dense_tz};
  tm.begin("d_scatter");
#define HPA_SCATTER(V, W)                                                                                       \
  k_d_scatter<V, W><<<grid, DB, 0, s>>>(smp->pc, smp->ctx, smp->stall, smp->weight, n, C, d_cbase.as<uint32_t>(), \
                                        d_cursor.as<uint32_t>(), dd, d_rec.as<uint32_t>(), d_rw.as<uint32_t>(), info)
  if (vec) {
    if (weighted) HPA_SCATTER(true, true);
    else HPA_SCATTER(true, false);
  } else {
    if (weighted) HPA_SCATTER(false, true);
    else HPA_SCATTER(false, false);
  }
#undef HPA_SCATTER
  HPA_HIP(hipGetLastError());
  tm.end(n, n);
  tm.begin("d_split");
  if (weighted)
    k_d_split<true><<<(unsigned)max_big, SB, 0, s>>>(d_bctx.as<uint32_t>(), d_bslot0.as<uint32_t>(),
                                                     d_cbase.as<uint32_t>(), d_rec.as<uint32_t>(),
                                                     d_rw.as<uint32_t>(), bshift, d_rec2.as<uint32_t>(),
                                                     d_rw2.as<uint32_t>(), d_bunits.as<DUnit>(),
                                                     d_nbu.as<uint32_t>(), info);
  else
    k_d_split<false><<<(unsigned)max_big, SB, 0, s>>>(d_bctx.as<uint32_t>(), d_bslot0.as<uint32_t>(),
                                                      d_cbase.as<uint32_t>(), d_rec.as<uint32_t>(), nullptr, bshift,
                                                      d_rec2.as<uint32_t>(), nullptr, d_bunits.as<DUnit>(),
                                                      d_nbu.as<uint32_t>(), info);
  HPA_HIP(hipGetLastError());
  tm.end();
  tm.begin("d_plan");
  k_d_plan<<<n_tiles, DB, 0, s>>>(d_hist.as<uint32_t>(), C, maxc, d_bidx.as<uint32_t>(), d_bunits.as<DUnit>(),
                                  d_bslot0.as<uint32_t>(), d_nbu.as<uint32_t>(), d_cbase.as<uint32_t>(),
                                  d_tu.as<uint32_t>(), nullptr, nullptr);
  k_d_unit_scan<<<1, 1024, 0, s>>>(d_tu.as<uint32_t>(), n_tiles, d_toff.as<uint32_t>(), info);
  k_d_plan<<<n_tiles, DB, 0, s>>>(d_hist.as<uint32_t>(), C, maxc, d_bidx.as<uint32_t>(), d_bunits.as<DUnit>(),
                                  d_bslot0.as<uint32_t>(), d_nbu.as<uint32_t>(), d_cbase.as<uint32_t>(),
                                  d_tu.as<uint32_t>(), d_toff.as<uint32_t>(), d_units.as<DUnit>());
  HPA_HIP(hipGetLastError());
  tm.end();
  // outputs (the key count is known only at the end: room for n keys)
  const uint64_t cap = n ? n : 1;
  if (!A->ctx_id.p) {
    A->ctx_id = DBuf(ctx, cap * 4, s);
    A->pc = DBuf(ctx, cap * 8, s);
    A->stall = DBuf(ctx, cap, s);
    A->count = DBuf(ctx, cap * 8, s);
    A->scope = DBuf(ctx, cap * 4, s);
    A->ctx_offsets = DBuf(ctx, ((uint64_t)C + 1) * 8, s);
  }
  DUnitArgs ua{};
  ua.units = d_units.as<DUnit>();
  ua.rec = d_rec.as<uint32_t>();
  ua.rw = d_rw.as<uint32_t>();
  ua.rec2 = d_rec2.as<uint32_t>();
  ua.rw2 = d_rw2.as<uint32_t>();
  ua.hist = d_hist.as<uint32_t>();
  ua.cbase = d_cbase.as<uint32_t>();
  ua.C = C;
  ua.bshift = bshift;
  ua.dd = dd;
  ua.info = info;
  ua.status = d_status.as<unsigned long long>();
  ua.out = OutDev{A->ctx_id.as<uint32_t>(), A->pc.as<uint64_t>(), A->stall.as<uint8_t>(),
                  A->count.as<unsigned long long>(), A->scope.as<uint32_t>(), A->ctx_offsets.as<uint64_t>()};
  // two resident workgroups per compute unit (each sort takes a little under
  // half of the LDS): one's memory phases overlap the other's sort.  Small
  // inputs take fewer workgroups (about one per DUT / 2 samples), which also
  // bounds the staging slots below.
  const unsigned ugrid = (unsigned)std::max<uint64_t>(
      1, std::min<uint64_t>({max_units, 2ull * ctx->n_cu, (n + DUT / 2 - 1) / (DUT / 2)}));
  // two staging slots of DUT keys per workgroup
  const uint64_t n_slots = 2ull * ugrid * DUT;
  DBuf d_skey(ctx, n_slots * 4, s), d_scnt(ctx, n_slots * (weighted ? 8 : 2), s);
  ua.stage_key = d_skey.as<uint32_t>();
  ua.stage_c16 = weighted ? nullptr : d_scnt.as<uint16_t>();
  ua.stage_cnt = weighted ? d_scnt.as<unsigned long long>() : nullptr;
  tm.begin("units_dense");
  if (weighted) k_d_units<true><<<ugrid, DUB, 0, s>>>(ua);
  else k_d_units<false><<<ugrid, DUB, 0, s>>>(ua);
  HPA_HIP(hipGetLastError());
  tm.end();
  DInfo h{};
  HPA_HIP(hipMemcpyAsync(&h, d_info.p, sizeof(h), hipMemcpyDeviceToHost, s));
  sync_stream(ctx, s);
  if (h.err & DERR_CTX) fail(HPA_E_INVAL, "a sample has ctx >= n_ctx");
  if (h.err & DERR_STALL) fail(HPA_E_INVAL, "a sample has stall >= 16");
  if (h.n_far) return false;  // the general path handles pcs without dense coordinates
  if (h.err & DERR_OVERFLOW) return false;  // a counted part's weights overflow 32 bits
  if (h.err & (DERR_INTERNAL | DERR_LOOKBACK | DERR_WIDE))
    fail(HPA_E_DEVICE, "internal error in the dense attribution pipeline (flags " + std::to_string(h.err) + ")");
  A->n_keys = h.total_keys;
  if (tm.on()) {
    tm.items("units_dense", n, h.total_keys);
    tm.items("d_split", 0, h.n_big);
    tm.items("d_plan", C, h.n_units);
    tm.collect();
  }
  return true;
}

}  // namespace hpa
