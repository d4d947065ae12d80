// A2-A4: stream PC samples once, form (context, pc, stall) keys and aggregate
// them into sorted unique keys with counts (Section 4.2 sample record; Section
// 4.5: a raw metric is the sum of measured values), then label each key's pc
// with its innermost scope (Section 6.1 calling-context expansion).
//
// Samples arrive per kernel invocation, so the context id is constant over long
// runs of the stream (Section 4.2: a buffer of PC samples belongs to one kernel
// launch and its placeholder).  The pipeline uses that:
//
//   scan_ctx    read ctx[] once (4 B/sample): run boundaries, per-context
//               sample and run counts (one 64-bit atomic per run), run list.
//   split       contexts over T samples: a histogram over coordinate buckets,
//               parts of at most T samples by coordinate range, which stand
//               in for the context as virtual contexts.
//   plan        parallel tile scans over the (virtual) contexts: bases,
//               packing into work units of <= T samples, adjacent unit pairs
//               merged when they fit, contexts that stay over T samples.
//   group_runs  order the run list by context (atomic cursors; a run learns
//               its offset inside its context from the same atomic); the
//               samples of split contexts are copied into part order.
//   units       one workgroup per unit: gather the unit's samples from its
//               runs (pc 8 B + stall 1 B, read once), map pcs to dense
//               coordinates, pack keys, LSD radix sort in LDS, run-length
//               reduce, stage the packed unique keys at the unit's first sample
//               position; then a scan gives the output offsets and a write
//               pass unpacks the keys (pc, scope label from the dense table).
//   chunk path  contexts over T samples that cannot be split: chunk sort,
//               pairwise merge rounds, duplicate combine, written where the
//               unit pass placed them.
//
// When runs are short (shuffled input) the run list would cost more than the
// samples themselves; the samples are then scattered into context order first.
#include <algorithm>
#include <chrono>
#include <mutex>
#include <memory>

#include "block_prims.h"
#include "hpa_internal.h"
#include "unit_sort.h"

namespace hpa {
namespace {


// ----------------------------------------------------------------------------
// scan_ctx: run detection over ctx[] (Section 4.2: one placeholder per buffer)
// ----------------------------------------------------------------------------
// Workgroups take tiles of SCAN_TILE samples in turn.  For each tile the
// workgroup finds the run heads, reserves that many run slots with one atomic
// per tile, then writes the runs and adds each run to its context's histogram
// word (one 64-bit atomic per run: run count << 40 | samples).  A run is cut at
// every tile start.
__device__ inline void scan_tile_heads(const uint32_t* __restrict__ ctx, uint64_t t0, int cnt, uint32_t* s_ctx,
                                       uint64_t (&mask)[SCAN_ITEMS]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const int j = i * SCAN_BLOCK + tid;
    if (j < cnt) s_ctx[j] = ctx[t0 + j];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const int j = i * SCAN_BLOCK + tid;
    mask[i] = __ballot(j < cnt && (j == 0 || s_ctx[j] != s_ctx[j - 1]));
  }
}

// One pass over the context array: every tile's run heads, one reservation
// in the run list per tile (runs are grouped by context later, so their order
// here is free), the runs and the per-context histogram.  A run never crosses
// a tile boundary.
__global__ void __launch_bounds__(SCAN_BLOCK)
k_scan_ctx(const uint32_t* __restrict__ ctx, uint64_t n, uint32_t n_ctx, unsigned long long* __restrict__ hist,
           Run* __restrict__ runs, uint64_t run_cap, PlanInfo* __restrict__ info) {
  constexpr int NWS = SCAN_BLOCK / WAVE;
  static_assert(SCAN_ITEMS * NWS == WAVE, "one lane per (item, wave) head count");
  __shared__ uint32_t s_ctx[SCAN_TILE];
  __shared__ uint32_t s_head[SCAN_TILE];
  __shared__ uint32_t s_wcnt[SCAN_ITEMS * NWS];
  __shared__ unsigned long long s_base;
  __shared__ uint32_t s_R;
  const int tid = threadIdx.x;
  const uint64_t n_tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const uint64_t t0 = tile * SCAN_TILE;
    const int cnt = (int)min((uint64_t)SCAN_TILE, n - t0);
    uint64_t mask[SCAN_ITEMS];
    scan_tile_heads(ctx, t0, cnt, s_ctx, mask);
    if (lane_id() == 0)
#pragma unroll
      for (int i = 0; i < SCAN_ITEMS; ++i) s_wcnt[i * NWS + wave_id()] = (uint32_t)__popcll(mask[i]);
    __syncthreads();
    // rank among the tile's heads = prefix over (item, wave, lane)
    if (tid < WAVE) {
      const uint32_t a = s_wcnt[tid];
      const uint32_t inc = wave_incl_scan_u32(a);
      s_wcnt[tid] = inc - a;
      if (tid == WAVE - 1) {
        s_R = inc;
        s_base = atomicAdd(&info->n_runs, (unsigned long long)inc);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
      const int j = i * SCAN_BLOCK + tid;
      const uint64_t below = mask[i] & ((1ull << lane_id()) - 1);
      if ((mask[i] >> lane_id()) & 1) s_head[s_wcnt[i * NWS + wave_id()] + (uint32_t)__popcll(below)] = (uint32_t)j;
    }
    __syncthreads();
    const uint32_t R = s_R;
    const unsigned long long base = s_base;
    for (uint32_t k = tid; k < R; k += SCAN_BLOCK) {
      const uint32_t p = s_head[k];
      const uint32_t len = (k + 1 < R ? s_head[k + 1] : (uint32_t)cnt) - p;
      const uint32_t c = s_ctx[p];
      if (c >= n_ctx) {
        atomicOr(&info->err, (uint32_t)ERR_CTX);
        continue;
      }
      atomicAdd(&hist[c], (1ull << 40) | (unsigned long long)len);
      const uint64_t g = base + k;
      if (g < run_cap) runs[g] = Run{t0 + p, 0, len, c};
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// plan: contexts are packed into units in order.  A unit is a run of
// contexts packed together; unit_big holds the big-context index of a unit of
// one context over T samples, UNIT_PLAIN for a unit read through the run
// list, and UNIT_PART for a unit of parts of a split context (grp, when
// given, names the split context a part belongs to, NONE32 for the others;
// units never mix groups).
// ----------------------------------------------------------------------------
constexpr int PLAN_BLOCK = 1024;
constexpr int PLAN_ITEMS = 8;
constexpr int32_t UNIT_PLAIN = -1, UNIT_PART = -2;

enum : uint8_t { KIND_S = 0, KIND_M = 1, KIND_B = 2 };

__device__ inline uint8_t ctx_kind(uint64_t n) { return n <= (uint64_t)UHALF ? KIND_S : (n <= (uint64_t)UT ? KIND_M : KIND_B); }

// The plan runs as five launches over tiles of PLAN_BLOCK contexts, one per
// thread: tile sums of the per-context quantities; their exclusive scan (one
// workgroup); per context the bases and the big-context lists, plus the unit
// start flags and their count per tile; the scan of those counts; the unit
// list.  A unit starts at context c when c is the first context, when c or
// c - 1 is not packable (over T/2 samples), every MAXC contexts, where the
// running count of packable samples crosses a multiple of T/2 between c - 1
// and c, where the group changes, and (a batch of profiles) where the profile
// changes.
struct PlanVals {
  unsigned long long n, r, ps, big, ch, bs;  // samples, runs, packable samples, big contexts, chunks, big samples
};

__device__ inline PlanVals plan_vals(const unsigned long long* hist, uint32_t n_ctx, uint32_t c) {
  PlanVals v{0, 0, 0, 0, 0, 0};
  if (c >= n_ctx) return v;
  const unsigned long long h = hist[c];
  v.n = h & M40;
  v.r = h >> 40;
  const uint8_t k = ctx_kind(v.n);
  if (k == KIND_S) v.ps = v.n;
  if (k == KIND_B) {
    v.big = 1;
    v.ch = (v.n + UT - 1) / UT;
    v.bs = v.n;
  }
  return v;
}

constexpr int PLAN_NV = 6;

__global__ void __launch_bounds__(PLAN_BLOCK) k_plan_sums(const unsigned long long* __restrict__ hist, uint32_t n_ctx,
                                                          unsigned long long* __restrict__ tile_sum,
                                                          PlanInfo* __restrict__ info) {
  __shared__ unsigned long long s_red[PLAN_NV][PLAN_BLOCK / WAVE];
  const uint32_t c = blockIdx.x * PLAN_BLOCK + threadIdx.x;
  const PlanVals v = plan_vals(hist, n_ctx, c);
  const unsigned long long x[PLAN_NV] = {v.n, v.r, v.ps, v.big, v.ch, v.bs};
#pragma unroll
  for (int k = 0; k < PLAN_NV; ++k) {
    const unsigned long long t = wave_sum(x[k]);
    if (lane_id() == 0) s_red[k][wave_id()] = t;
  }
  if (v.big) atomicMax(&info->max_chunks, (uint32_t)v.ch);
  __syncthreads();
  if (threadIdx.x < PLAN_NV) {
    unsigned long long t = 0;
    for (int w = 0; w < PLAN_BLOCK / WAVE; ++w) t += s_red[threadIdx.x][w];
    tile_sum[(uint64_t)blockIdx.x * PLAN_NV + threadIdx.x] = t;
  }
}

// Exclusive scan over the tiles of every quantity (in place); the totals
// close the base arrays and go to the plan summary.
__global__ void __launch_bounds__(1024) k_plan_tile_scan(unsigned long long* __restrict__ tile_sum, uint32_t n_tiles,
                                                         uint32_t n_ctx, uint64_t* __restrict__ sbase,
                                                         uint64_t* __restrict__ rbase,
                                                         uint64_t* __restrict__ big_sbase,
                                                         uint64_t* __restrict__ big_chunk,
                                                         PlanInfo* __restrict__ info) {
  __shared__ unsigned long long s_tmp[1024 / WAVE + 1];
  unsigned long long carry[PLAN_NV] = {0, 0, 0, 0, 0, 0};
  for (uint32_t b0 = 0; b0 < n_tiles; b0 += 1024) {
    const uint32_t i = b0 + threadIdx.x;
#pragma unroll
    for (int k = 0; k < PLAN_NV; ++k) {
      const unsigned long long x = i < n_tiles ? tile_sum[(uint64_t)i * PLAN_NV + k] : 0ull;
      unsigned long long tot;
      const unsigned long long ex = block_excl_scan<1024>(x, s_tmp, &tot);
      if (i < n_tiles) tile_sum[(uint64_t)i * PLAN_NV + k] = carry[k] + ex;
      carry[k] += tot;
    }
  }
  if (threadIdx.x == 0) {
    sbase[n_ctx] = carry[0];
    rbase[n_ctx] = carry[1];
    big_chunk[carry[3]] = carry[4];
    big_sbase[carry[3]] = carry[5];
    info->n_big = (uint32_t)carry[3];
    info->n_chunks = carry[4];
    info->big_samples = carry[5];
  }
}

__global__ void __launch_bounds__(PLAN_BLOCK)
k_plan_starts(const unsigned long long* __restrict__ hist, uint32_t n_ctx, const uint32_t* __restrict__ grp,
              const uint32_t* __restrict__ pgrp, const unsigned long long* __restrict__ tile_off, uint64_t* __restrict__ sbase,
              uint64_t* __restrict__ rbase, uint32_t* __restrict__ big_ctx, uint64_t* __restrict__ big_sbase,
              uint64_t* __restrict__ big_chunk, uint8_t* __restrict__ start, uint32_t* __restrict__ tile_starts) {
  __shared__ unsigned long long s_tmp[PLAN_BLOCK / WAVE + 1];
  __shared__ uint32_t s_tmp32[PLAN_BLOCK / WAVE + 1];
  const uint32_t c = blockIdx.x * PLAN_BLOCK + threadIdx.x;
  const PlanVals v = plan_vals(hist, n_ctx, c);
  const unsigned long long* off = tile_off + (uint64_t)blockIdx.x * PLAN_NV;
  unsigned long long t;
  const unsigned long long sb = off[0] + block_excl_scan<PLAN_BLOCK>(v.n, s_tmp, &t);
  const unsigned long long rb = off[1] + block_excl_scan<PLAN_BLOCK>(v.r, s_tmp, &t);
  const unsigned long long ps = off[2] + block_excl_scan<PLAN_BLOCK>(v.ps, s_tmp, &t);
  const unsigned long long bg = off[3] + block_excl_scan<PLAN_BLOCK>(v.big, s_tmp, &t);
  const unsigned long long ch = off[4] + block_excl_scan<PLAN_BLOCK>(v.ch, s_tmp, &t);
  const unsigned long long bs = off[5] + block_excl_scan<PLAN_BLOCK>(v.bs, s_tmp, &t);
  uint32_t st = 0;
  if (c < n_ctx) {
    sbase[c] = sb;
    rbase[c] = rb;
    const uint8_t k = ctx_kind(v.n);
    if (k == KIND_B) {
      big_ctx[bg] = c;
      big_sbase[bg] = bs;
      big_chunk[bg] = ch;
    }
    // the context before: its kind and the packable count before it
    const uint64_t n_prev = c > 0 ? (hist[c - 1] & M40) : 0;
    const uint8_t kp = c > 0 ? ctx_kind(n_prev) : KIND_S;
    const uint64_t ps_prev = ps - (c > 0 && kp == KIND_S ? n_prev : 0);
    st = c == 0 || k != KIND_S || kp != KIND_S || (c % MAXC) == 0 || (ps / UHALF) != (ps_prev / UHALF) ||
         (grp && grp[c] != grp[c - 1]) || (pgrp && pgrp[c] != pgrp[c - 1]);
    start[c] = (uint8_t)st;
  }
  uint32_t tot;
  block_excl_scan<PLAN_BLOCK>(st, s_tmp32, &tot);
  if (threadIdx.x == 0) tile_starts[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(PLAN_BLOCK)
k_plan_units(const unsigned long long* __restrict__ hist, uint32_t n_ctx, const uint32_t* __restrict__ grp,
             const unsigned long long* __restrict__ tile_off, const uint8_t* __restrict__ start,
             const uint32_t* __restrict__ tile_starts, uint32_t* __restrict__ unit_begin,
             int32_t* __restrict__ unit_big, PlanInfo* __restrict__ info) {
  __shared__ unsigned long long s_tmp[PLAN_BLOCK / WAVE + 1];
  __shared__ uint32_t s_tmp32[PLAN_BLOCK / WAVE + 1];
  const uint32_t c = blockIdx.x * PLAN_BLOCK + threadIdx.x;
  const PlanVals v = plan_vals(hist, n_ctx, c);
  unsigned long long t;
  const unsigned long long bg = tile_off[(uint64_t)blockIdx.x * PLAN_NV + 3] + block_excl_scan<PLAN_BLOCK>(v.big, s_tmp, &t);
  const uint32_t st = c < n_ctx ? start[c] : 0u;
  uint32_t tot;
  const uint32_t u = tile_starts[blockIdx.x] + block_excl_scan<PLAN_BLOCK>(st, s_tmp32, &tot);
  if (st) {
    unit_begin[u] = c;
    unit_big[u] = ctx_kind(v.n) == KIND_B ? (int32_t)bg : (grp && grp[c] != NONE32 ? UNIT_PART : UNIT_PLAIN);
  }
  if (c == n_ctx - 1) {
    unit_begin[u + st] = n_ctx;
    info->n_units = u + st;
  }
}

// Unit pairs (2m, 2m + 1) merge when both are read the same way (plain units,
// or parts of one split context) and together hold at most T samples and MAXC
// contexts: the band rule above leaves units about half full on average, and
// a sort costs in proportion to its slots.  Three launches over tiles of
// PLAN_BLOCK units (the count n_units comes from the plan on the device): the
// kept units per tile, their scan, and the new unit list.
// Between merge rounds: the merged count becomes the unit count.
__global__ void k_set_units(PlanInfo* __restrict__ info) { info->n_units = info->n_merged; }
// Without merge rounds the plan's units are the final ones.
__global__ void k_keep_units(PlanInfo* __restrict__ info) { info->n_merged = info->n_units; }

__device__ inline bool merge_pair(const uint32_t* unit_begin, const int32_t* unit_big, const uint64_t* sbase,
                                  const uint32_t* grp, const uint32_t* pgrp, uint32_t nu, uint32_t a) {
  if (a + 1 >= nu) return false;
  const int32_t ba = unit_big[a], bb = unit_big[a + 1];
  if (ba >= 0 || ba != bb) return false;
  const uint32_t c0 = unit_begin[a], c1 = unit_begin[a + 1], c2 = unit_begin[a + 2];
  if (grp && grp[c0] != grp[c1]) return false;
  if (pgrp && pgrp[c0] != pgrp[c1]) return false;
  return c2 - c0 <= (uint32_t)MAXC && sbase[c2] - sbase[c0] <= (uint64_t)UT;
}

__device__ inline uint32_t unit_kept(const uint32_t* unit_begin, const int32_t* unit_big, const uint64_t* sbase,
                                     const uint32_t* grp, const uint32_t* pgrp, uint32_t nu, uint32_t u) {
  if (u >= nu) return 0u;
  return (u & 1u) && merge_pair(unit_begin, unit_big, sbase, grp, pgrp, nu, u - 1) ? 0u : 1u;
}

__global__ void __launch_bounds__(PLAN_BLOCK)
k_merge_count(const uint32_t* __restrict__ unit_begin, const int32_t* __restrict__ unit_big,
              const uint64_t* __restrict__ sbase, const uint32_t* __restrict__ grp, const uint32_t* __restrict__ pgrp,
              const PlanInfo* __restrict__ info, uint32_t* __restrict__ tile_sum) {
  __shared__ uint32_t s_tmp[PLAN_BLOCK / WAVE + 1];
  const uint32_t nu = info->n_units;
  const uint32_t u = blockIdx.x * PLAN_BLOCK + threadIdx.x;
  uint32_t tot;
  block_excl_scan<PLAN_BLOCK>(unit_kept(unit_begin, unit_big, sbase, grp, pgrp, nu, u), s_tmp, &tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(PLAN_BLOCK)
k_merge_write(const uint32_t* __restrict__ unit_begin, const int32_t* __restrict__ unit_big,
              const uint64_t* __restrict__ sbase, const uint32_t* __restrict__ grp, const uint32_t* __restrict__ pgrp,
              uint32_t n_ctx,
              const uint32_t* __restrict__ tile_off, uint32_t* __restrict__ out_begin, int32_t* __restrict__ out_big,
              PlanInfo* __restrict__ info) {
  __shared__ uint32_t s_tmp[PLAN_BLOCK / WAVE + 1];
  const uint32_t nu = info->n_units;
  const uint32_t u = blockIdx.x * PLAN_BLOCK + threadIdx.x;
  const uint32_t keep = unit_kept(unit_begin, unit_big, sbase, grp, pgrp, nu, u);
  uint32_t tot;
  const uint32_t v = tile_off[blockIdx.x] + block_excl_scan<PLAN_BLOCK>(keep, s_tmp, &tot);
  if (keep) {
    out_begin[v] = unit_begin[u];
    out_big[v] = unit_big[u];
  }
  if (u == nu - 1) {
    out_begin[v + keep] = n_ctx;
    info->n_merged = v + keep;
  }
}

// ----------------------------------------------------------------------------
// group_runs: runs ordered by context; one 64-bit atomic gives both the run's
// slot and its sample offset within the context.  With split contexts, vsolo
// maps a context to its virtual id (NONE32 for a split context, whose samples
// are scattered into parts instead), and the grouped run carries that id.
// ----------------------------------------------------------------------------
__global__ void k_group_runs(const Run* __restrict__ runs, uint64_t n_runs, const uint32_t* __restrict__ vsolo,
                             const uint64_t* __restrict__ sbase, const uint64_t* __restrict__ rbase,
                             unsigned long long* __restrict__ cur, Run* __restrict__ grouped) {
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_runs; r += (uint64_t)gridDim.x * blockDim.x) {
    Run x = runs[r];
    if (vsolo) {
      const uint32_t v = vsolo[x.ctx];
      if (v == NONE32) continue;
      x.ctx = v;
    }
    unsigned long long old = atomicAdd(&cur[x.ctx], (1ull << 40) | (unsigned long long)x.len);
    uint64_t k = old >> 40, soff = old & M40;
    x.flat = sbase[x.ctx] + soff;
    grouped[rbase[x.ctx] + k] = x;
  }
}

// ----------------------------------------------------------------------------
// Split of big contexts by coordinate range
//
// A context with more than T samples is cut into parts of at most T samples
// along its dense coordinates: a histogram of its samples over NB coordinate
// buckets (bucket = D >> bshift), buckets packed in order into parts by the
// plan's packing rule, and its samples scattered into part order.  The parts
// of a context cover increasing coordinate ranges, so sorting each part on its
// own and concatenating the results gives the context's keys in order; the
// parts then pass through the unit passes as contexts of their own (virtual
// contexts).  A context with a pc outside the dense coordinates, or with one
// bucket over T samples, keeps the chunk path.
// ----------------------------------------------------------------------------
constexpr int NB = 1024;  // coordinate buckets per big context
constexpr int SPLIT_BLOCK = 256;
constexpr int SPLIT_ITEMS = 8;
constexpr int SPLIT_ROUND = SPLIT_BLOCK * SPLIT_ITEMS;  // samples per workgroup round
constexpr uint32_t SPLIT_NO = 0xFFFFFFFFu;               // no parts: the context keeps the chunk path

// Contexts over T samples get an index (in no particular order).
__global__ void k_big_index(const unsigned long long* __restrict__ hist, uint32_t n_ctx, int32_t* __restrict__ big_of,
                            PlanInfo* __restrict__ info) {
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n_ctx; c += gridDim.x * blockDim.x)
    big_of[c] = (hist[c] & M40) > (uint64_t)UT ? (int32_t)atomicAdd(&info->n_bigall, 1u) : -1;
}

__device__ inline void stage_windows(uint64_t* lo, uint64_t* hi, uint64_t* d, const DenseDev& t, int nthreads) {
  for (uint32_t i = threadIdx.x; i < t.n_win; i += nthreads) {
    lo[i] = t.lo[i];
    hi[i] = t.hi[i];
  }
  if (t.n_win)
    for (uint32_t i = threadIdx.x; i <= t.n_win; i += nthreads) d[i] = t.d[i];
}

// Bucket histogram of every big context, one run at a time per workgroup (a
// run belongs to one context); a pc without a dense coordinate flags its
// context.
__global__ void __launch_bounds__(SPLIT_BLOCK)
k_big_hist(const Run* __restrict__ runs, uint64_t n_runs, const int32_t* __restrict__ big_of,
           const uint64_t* __restrict__ pc, DenseDev dd, uint32_t bshift, uint32_t* __restrict__ bhist,
           uint32_t* __restrict__ bflag) {
  __shared__ uint32_t s_h[NB];
  __shared__ uint64_t s_lo[DENSE_MAX_WIN], s_hi[DENSE_MAX_WIN], s_d[DENSE_MAX_WIN + 1];
  stage_windows(s_lo, s_hi, s_d, dd, SPLIT_BLOCK);
  const DenseDev t{s_lo, s_hi, s_d, dd.scope_of, dd.n_win, dd.tz};
  for (uint64_t r = blockIdx.x; r < n_runs; r += gridDim.x) {
    const Run x = runs[r];
    const int32_t b = big_of[x.ctx];
    if (b < 0) continue;
    for (int k = threadIdx.x; k < NB; k += SPLIT_BLOCK) s_h[k] = 0;
    __syncthreads();
    bool far = false;
    for (uint32_t o = 0; o < x.len; o += SPLIT_ROUND) {
      uint64_t v[SPLIT_ITEMS];
#pragma unroll
      for (int i = 0; i < SPLIT_ITEMS; ++i) {
        const uint32_t j = o + i * SPLIT_BLOCK + threadIdx.x;
        v[i] = j < x.len ? pc[x.start + j] : 0;
      }
#pragma unroll
      for (int i = 0; i < SPLIT_ITEMS; ++i) {
        const uint32_t j = o + i * SPLIT_BLOCK + threadIdx.x;
        uint64_t D;
        if (j >= x.len) continue;
        if (to_dense(t, v[i], D)) atomicAdd(&s_h[(uint32_t)(D >> bshift)], 1u);
        else far = true;
      }
    }
    if (far) atomicOr(&bflag[b], 1u);
    __syncthreads();
    for (int k = threadIdx.x; k < NB; k += SPLIT_BLOCK)
      if (s_h[k]) atomicAdd(&bhist[(uint64_t)b * NB + k], s_h[k]);
    __syncthreads();
  }
}

// Parts of every big context, one wave each: bucket k starts a part when it is
// the first, when it or the bucket before holds over T/2 samples, or when the
// running count of the other (light) buckets crosses a multiple of T/2 between
// the bucket before and this one.  A part then holds one heavy bucket (at most
// T samples) or light buckets whose running counts start within one T/2 band,
// fewer than T samples.  part_of gets each bucket's part, psum (zeroed) each
// part's samples, n_parts the count (SPLIT_NO: keep the chunk path).
__global__ void __launch_bounds__(256)
k_big_parts(const uint32_t* __restrict__ bhist, const uint32_t* __restrict__ bflag, uint32_t n_big,
            uint32_t* __restrict__ part_of, uint32_t* __restrict__ psum, uint32_t* __restrict__ n_parts) {
  constexpr int PER = NB / WAVE;
  const uint32_t b = blockIdx.x * (256 / WAVE) + wave_id();
  if (b >= n_big) return;
  const uint32_t l = lane_id();
  const uint32_t* h = bhist + (uint64_t)b * NB + l * PER;
  uint32_t cnt[PER];
  uint32_t light = 0;
  bool over = false;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    cnt[i] = h[i];
    over |= cnt[i] > (uint32_t)UT;
    light += cnt[i] <= (uint32_t)UHALF ? cnt[i] : 0u;
  }
  const uint32_t light_incl = wave_incl_scan(light);
  if (wave_or((uint32_t)over) || bflag[b]) {
    if (l == 0) n_parts[b] = SPLIT_NO;
    return;
  }
  // the bucket before this lane's first: its exclusive light count and weight
  uint32_t prevL = __shfl_up(light_incl - (cnt[PER - 1] <= (uint32_t)UHALF ? cnt[PER - 1] : 0u), 1, WAVE);
  bool prevH = __shfl_up(cnt[PER - 1] > (uint32_t)UHALF ? 1 : 0, 1, WAVE) != 0;
  uint32_t L = light_incl - light;
  uint32_t starts = 0;
  uint32_t st[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const bool heavy = cnt[i] > (uint32_t)UHALF;
    const bool first = l == 0 && i == 0;
    st[i] = first || heavy || prevH || (L / UHALF) != (prevL / UHALF);
    starts += st[i];
    prevL = L;
    prevH = heavy;
    L += heavy ? 0u : cnt[i];
  }
  const uint32_t s_incl = wave_incl_scan(starts);
  uint32_t part = s_incl - starts;  // starts before this lane
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    part += st[i];
    const uint64_t k = (uint64_t)b * NB + l * PER + i;
    part_of[k] = part - 1;
    if (cnt[i]) atomicAdd(&psum[(uint64_t)b * NB + part - 1], cnt[i]);
  }
  if (l == WAVE - 1) n_parts[b] = s_incl;
}

// Virtual contexts: every context stays one, except a split context, which
// becomes its parts.  Three launches over tiles of VT contexts: the number of
// virtual contexts per tile, an exclusive scan of those (one workgroup), then
// the writes: the virtual histogram (count, and runs for contexts read through
// the run list; parts have none), the real context of every virtual one, its
// group (the split context, or NONE32), the first virtual id of every context
// (vbase, closed by the total) and vsolo (the virtual id of an unsplit
// context, NONE32 for a split one).
constexpr int VT = 1024;

__device__ inline uint32_t n_virtual_of(const int32_t* big_of, const uint32_t* n_parts, uint32_t c) {
  const int32_t b = big_of[c];
  return (b >= 0 && n_parts[b] != SPLIT_NO) ? n_parts[b] : 1u;
}

__global__ void __launch_bounds__(VT) k_virtual_count(uint32_t n_ctx, const int32_t* __restrict__ big_of,
                                                      const uint32_t* __restrict__ n_parts,
                                                      uint32_t* __restrict__ tile_sum) {
  __shared__ uint32_t s_tmp[VT / WAVE + 1];
  const uint32_t c = blockIdx.x * VT + threadIdx.x;
  const uint32_t nv = c < n_ctx ? n_virtual_of(big_of, n_parts, c) : 0u;
  uint32_t tot;
  block_excl_scan<VT>(nv, s_tmp, &tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// Exclusive scan of n per-tile values in place (one workgroup); the total goes
// to *total.
__global__ void __launch_bounds__(1024) k_tile_scan(uint32_t* __restrict__ v, uint32_t n, uint32_t* __restrict__ total) {
  __shared__ uint32_t s_tmp[1024 / WAVE + 1];
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < n; b0 += 1024) {
    const uint32_t i = b0 + threadIdx.x;
    const uint32_t x = i < n ? v[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<1024>(x, s_tmp, &tot);
    if (i < n) v[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(VT)
k_virtual_write(const unsigned long long* __restrict__ hist, uint32_t n_ctx, const int32_t* __restrict__ big_of,
                const uint32_t* __restrict__ n_parts, const uint32_t* __restrict__ psum,
                const uint32_t* __restrict__ tile_off, unsigned long long* __restrict__ vhist,
                uint32_t* __restrict__ vreal, uint32_t* __restrict__ vgrp, uint32_t* __restrict__ vbase,
                uint32_t* __restrict__ vsolo, PlanInfo* __restrict__ info) {
  __shared__ uint32_t s_tmp[VT / WAVE + 1];
  const uint32_t c = blockIdx.x * VT + threadIdx.x;
  const uint32_t nv = c < n_ctx ? n_virtual_of(big_of, n_parts, c) : 0u;
  uint32_t tot;
  const uint32_t v = tile_off[blockIdx.x] + block_excl_scan<VT>(nv, s_tmp, &tot);
  if (c >= n_ctx) return;
  vbase[c] = v;
  if (c == n_ctx - 1) {
    vbase[n_ctx] = v + nv;
    info->n_virtual = v + nv;
  }
  const int32_t b = big_of[c];
  if (b >= 0 && n_parts[b] != SPLIT_NO) {
    vsolo[c] = NONE32;
    for (uint32_t p = 0; p < nv; ++p) {
      vhist[v + p] = psum[(uint64_t)b * NB + p];
      vreal[v + p] = c;
      vgrp[v + p] = c;
    }
    atomicAdd(&info->n_split, 1u);
    atomicAdd(&info->n_parts, nv);
    atomicAdd(&info->split_samples, hist[c] & M40);
  } else {
    vsolo[c] = v;
    vhist[v] = hist[c];
    vreal[v] = c;
    vgrp[v] = NONE32;
  }
}

// Scatter the samples of split contexts into part order (flat positions of
// the virtual contexts), one run per workgroup at a time: per round, each
// item's part and its rank among the round's items of that part (LDS
// counters), one global reservation per part, then the writes.  A
// reservation past the part's end (which the histogram rules out) is
// reported and its items dropped.
__global__ void __launch_bounds__(SPLIT_BLOCK)
k_big_scatter(const Run* __restrict__ runs, uint64_t n_runs, const int32_t* __restrict__ big_of,
              const uint32_t* __restrict__ n_parts, const uint32_t* __restrict__ part_of,
              const uint32_t* __restrict__ vbase, const uint64_t* __restrict__ sbase,
              unsigned long long* __restrict__ vcur, const uint64_t* __restrict__ pc,
              const uint8_t* __restrict__ stall, const uint32_t* __restrict__ weight, DenseDev dd, uint32_t bshift,
              uint64_t* __restrict__ tpc, uint8_t* __restrict__ tst, uint32_t* __restrict__ tw,
              uint32_t* __restrict__ err) {
  __shared__ uint32_t s_cnt[NB];
  __shared__ unsigned long long s_base[NB];
  __shared__ uint64_t s_lo[DENSE_MAX_WIN], s_hi[DENSE_MAX_WIN], s_d[DENSE_MAX_WIN + 1];
  stage_windows(s_lo, s_hi, s_d, dd, SPLIT_BLOCK);
  const DenseDev t{s_lo, s_hi, s_d, dd.scope_of, dd.n_win, dd.tz};
  for (uint64_t r = blockIdx.x; r < n_runs; r += gridDim.x) {
    const Run x = runs[r];
    const int32_t b = big_of[x.ctx];
    if (b < 0) continue;
    const uint32_t np = n_parts[b];
    if (np == SPLIT_NO) continue;
    const uint32_t vb = vbase[x.ctx];
    for (uint32_t o = 0; o < x.len; o += SPLIT_ROUND) {
      for (uint32_t k = threadIdx.x; k < np; k += SPLIT_BLOCK) s_cnt[k] = 0;
      __syncthreads();
      uint64_t v[SPLIT_ITEMS];
      uint32_t part[SPLIT_ITEMS], rank[SPLIT_ITEMS];
#pragma unroll
      for (int i = 0; i < SPLIT_ITEMS; ++i) {
        const uint32_t j = o + i * SPLIT_BLOCK + threadIdx.x;
        v[i] = j < x.len ? pc[x.start + j] : 0;
      }
#pragma unroll
      for (int i = 0; i < SPLIT_ITEMS; ++i) {
        const uint32_t j = o + i * SPLIT_BLOCK + threadIdx.x;
        part[i] = NONE32;
        rank[i] = 0;
        uint64_t D;
        if (j >= x.len) continue;
        // the histogram found a coordinate for every pc of a split context,
        // in a bucket of some part
        const uint32_t p = to_dense(t, v[i], D) ? part_of[(uint64_t)b * NB + (uint32_t)(D >> bshift)] : NONE32;
        if (p < np) {
          part[i] = p;
          rank[i] = atomicAdd(&s_cnt[p], 1u);
        } else {
          atomicOr(err, (uint32_t)ERR_SPLIT);
        }
      }
      __syncthreads();
      for (uint32_t k = threadIdx.x; k < np; k += SPLIT_BLOCK) {
        const uint32_t c = s_cnt[k];
        if (!c) continue;
        const unsigned long long at = sbase[vb + k] + atomicAdd(&vcur[vb + k], (unsigned long long)c);
        if (at + c > sbase[vb + k + 1]) {
          atomicOr(err, (uint32_t)ERR_SPLIT);
          s_base[k] = ~0ull;
        } else {
          s_base[k] = at;
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < SPLIT_ITEMS; ++i) {
        if (part[i] == NONE32) continue;
        const unsigned long long at = s_base[part[i]];
        if (at == ~0ull) continue;
        const uint64_t src = x.start + o + i * SPLIT_BLOCK + threadIdx.x;
        tpc[at + rank[i]] = v[i];
        tst[at + rank[i]] = stall[src];
        if (tw) tw[at + rank[i]] = weight[src];
      }
      __syncthreads();
    }
  }
}

// scatter: samples into context order (used when runs are short)
__global__ void k_scatter(const uint64_t* __restrict__ pc, const uint32_t* __restrict__ ctx,
                          const uint8_t* __restrict__ stall, const uint32_t* __restrict__ weight, uint64_t n,
                          const uint64_t* __restrict__ sbase, unsigned long long* __restrict__ cur,
                          uint64_t* __restrict__ opc, uint8_t* __restrict__ ostall, uint32_t* __restrict__ ow,
                          uint32_t n_ctx) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t c = ctx[i];
    if (c >= n_ctx) continue;
    uint64_t pos = sbase[c] + atomicAdd(&cur[c], 1ull);
    opc[pos] = pc[i];
    ostall[pos] = stall[i];
    if (ow) ow[pos] = weight[i];
  }
}


// ----------------------------------------------------------------------------
// units: sort pass, offsets, write pass
//
// The sort pass treats every unit on its own: the unit's unique keys, still
// packed and in order, go to a staging area at the unit's first sample
// position (a unit never has more unique keys than samples) together with
// their counts and the unit's decoding parameters.  A scan over the units'
// key counts then gives every unit its output offset and every context its
// key range, and the write pass unpacks the keys (coordinate -> pc, scope
// label) into the outputs.  No unit waits for another.
// ----------------------------------------------------------------------------
struct UnitMeta {
  unsigned long long lo;  // smallest coordinate of the unit (keys are relative to it)
  uint32_t nU;            // unique keys
  uint16_t pcb, tz;       // coordinate field width, common trailing zeros
  uint32_t flags;         // UM_* bits
  uint32_t pad;
};
constexpr uint32_t UM_DONE = 1, UM_WIDE = 2, UM_DENSE = 4;

// Everything a unit's workgroup needs first, in one record, so that its
// start is one load rather than a chain of dependent ones.
struct UnitDesc {
  uint64_t s0, s1;  // flat sample range
  uint64_t r0, r1;  // grouped run range
  uint32_t cb, ce;  // (virtual) context range
  int32_t big;      // unit_big
  uint32_t pad;
};

__global__ void k_unit_desc(const uint32_t* __restrict__ unit_begin, const int32_t* __restrict__ unit_big,
                            const uint64_t* __restrict__ sbase, const uint64_t* __restrict__ rbase, uint32_t n_units,
                            UnitDesc* __restrict__ desc) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n_units; u += gridDim.x * blockDim.x) {
    const uint32_t cb = unit_begin[u], ce = unit_begin[u + 1];
    desc[u] = UnitDesc{sbase[cb], sbase[ce], rbase[cb], rbase[ce], cb, ce, unit_big[u], 0u};
  }
}

struct UnitArgs {
  const uint64_t* pc;
  const uint8_t* stall;
  const uint32_t* weight;
  const uint64_t* sbase;
  const uint64_t* rbase;
  const Run* grouped;
  const uint32_t* unit_begin;
  const int32_t* unit_big;
  PlanInfo* info;
  uint32_t n_units;
  uint32_t n_ctx;
  DenseDev dd;
  int dense;                   // the map has dense coordinates
  UnitMeta* meta;              // per unit
  uint32_t* ucnt;              // per unit, MAXC entries: unique keys per local context
  uint32_t* skey;              // staging, by sample position: packed key (low word)
  uint32_t* shi;               // high word (units with keys wider than 32 bits)
  uint32_t* scnt;              // count (unweighted)
  unsigned long long* scnt64;  // count (weighted)
  int32_t kind;                // the unit class a sort launch handles (UNIT_PLAIN or UNIT_PART)
  const uint32_t* vreal;       // real context of every virtual one (null: no split contexts)
  const UnitDesc* desc;        // per unit
  const ProfMap* pm;           // batch of profiles: per profile maps (null: one profile, dd / dense above)
  const uint32_t* cprof;       // batch: profile of every (real) context
};

// Stage the unit's unique keys, counts and decoding parameters.
template <bool WEIGHTED, class K, int IT = UITEMS>
__device__ __forceinline__ void unit_body(SortSmem& sm, const UnitArgs& a, uint32_t u, uint32_t cb, uint32_t ce,
                                          uint64_t n_u, Gathered<WEIGHTED>& g, int kbits, int pcb, uint32_t tz,
                                          bool dense) {
  const uint32_t n_cu = ce - cb;
  K key[IT];
  uint32_t val[IT];
  sort_reduce<WEIGHTED, K, IT>(sm, g, n_u, n_cu, key, val, kbits, pcb, tz);
  uint32_t first, nU;
  find_heads<K, IT>(sm, key, n_u, n_cu, pcb, first, nU);
  const uint64_t s0 = a.sbase[cb];
  for (uint32_t l = threadIdx.x; l < n_cu; l += UBLOCK) a.ucnt[(uint64_t)u * MAXC + l] = sm.ucnt[l];
  if (threadIdx.x == 0)
    a.meta[u] = UnitMeta{sm.pcmin[0], nU, (uint16_t)pcb, (uint16_t)tz,
                         UM_DONE | (sizeof(K) == 8 ? UM_WIDE : 0u) | (dense ? UM_DENSE : 0u), 0u};
  uint32_t* const skey = a.skey + s0;
  uint32_t* const scnt = a.scnt + s0;
  if constexpr (sizeof(K) == 4) {
    // consecutive lanes take consecutive keys from the compacted copy in LDS
    for (uint32_t ui = threadIdx.x; ui < nU; ui += UBLOCK) {
      skey[ui] = sm.buf[ui];
      if constexpr (!WEIGHTED) scnt[ui] = (uint32_t)sm.upos[ui + 1] - (uint32_t)sm.upos[ui];
    }
  } else {
    uint32_t* const shi = a.shi + s0;
    K prev = prev_last<K>(sm, threadIdx.x);
    uint32_t ui = first;
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const uint32_t p = threadIdx.x * IT + i;
      const bool h = p < n_u && (p == 0 || key[i] != prev);
      prev = key[i];
      if (!h) continue;
      skey[ui] = (uint32_t)(uint64_t)key[i];
      shi[ui] = (uint32_t)((uint64_t)key[i] >> 32);
      if constexpr (!WEIGHTED) scnt[ui] = (uint32_t)sm.upos[ui + 1] - p;
      ++ui;
    }
  }
  if constexpr (WEIGHTED) weighted_counts<K, IT>(sm, key, val, n_u, first, a.scnt64 + s0);
}

// Sort pass.  GENERAL = false handles keys of at most 32 bits (registers sized
// for them) and marks the other units UM_WIDE; GENERAL = true, launched next,
// handles only those.
template <bool WEIGHTED, bool SCATTERED, bool GENERAL>
__global__ void __launch_bounds__(UBLOCK) k_units32(UnitArgs a) {
  __shared__ SortSmem sm;
  __shared__ uint64_t s_sb[MAXC + 1];
  const uint32_t u = blockIdx.x;
  const UnitDesc d = a.desc[u];
  // units of the other class, or a big context (its keys come from the chunk path)
  if (d.big != a.kind) return;
  if (GENERAL && a.meta[u].flags != UM_WIDE) return;
  const uint32_t cb = d.cb, ce = d.ce;
  const uint64_t s0 = d.s0;
  const uint64_t n_u = d.s1 - s0;
  // context bases, window tables and (when they fit) the runs, behind one barrier
  for (uint32_t l = threadIdx.x; l <= ce - cb; l += UBLOCK) s_sb[l] = a.sbase[cb + l];
  DenseDev src = a.dd;
  int map_dense = a.dense;
  if (a.pm) {  // a unit holds contexts of one profile
    const ProfMap& pmp = a.pm[a.cprof[a.vreal ? a.vreal[cb] : cb]];
    src = pmp.dd;
    map_dense = pmp.dense;
  }
  const DenseDev t = stage_dense(sm, src);  // LDS view (empty when the map has no dense coordinates)
  const uint64_t r0 = SCATTERED ? 0 : d.r0, r1 = SCATTERED ? 0 : d.r1;
  const bool staged = !SCATTERED && r1 - r0 <= (uint64_t)RUN_CAP;
  if (staged)
    for (uint32_t k = threadIdx.x; k < r1 - r0; k += UBLOCK) sm.runs[k] = a.grouped[r0 + k];
  __syncthreads();
  Gathered<WEIGHTED> g;
  gather<SCATTERED, WEIGHTED>(g, s0, n_u, cb, a.grouped, r0, r1, s_sb, ce - cb, a.pc, a.stall, a.weight,
                              &a.info->err, sm.runs, staged);
  bool dense = false;
  if (map_dense) {
    densify(sm, g, n_u, t);
    __syncthreads();
    dense = sm.far == 0;
    if (!dense)  // the runs are still in LDS: the sort has not touched them
      gather<SCATTERED, WEIGHTED>(g, s0, n_u, cb, a.grouped, r0, r1, s_sb, ce - cb, a.pc, a.stall, a.weight,
                                  &a.info->err, sm.runs, staged);
  }
  // key width decides the register type of the sort
  int kbits, pcb;
  uint32_t tz;
  key_stats(sm, g, n_u, ce - cb, &a.info->err, kbits, pcb, tz);
  if (kbits > 63) {  // reported as an error after the call; the unit contributes nothing
    for (uint32_t l = threadIdx.x; l < ce - cb; l += UBLOCK) a.ucnt[(uint64_t)u * MAXC + l] = 0;
    if (threadIdx.x == 0) a.meta[u] = UnitMeta{0, 0, 0, 0, UM_DONE, 0};
    return;
  }
  if (!GENERAL && kbits > 31) {
    if (threadIdx.x == 0) a.meta[u] = UnitMeta{0, 0, 0, 0, UM_WIDE, 0};
    return;
  }
  __syncthreads();
  if constexpr (GENERAL) {
    if (kbits > 31) {
      unit_body<WEIGHTED, uint64_t>(sm, a, u, cb, ce, n_u, g, kbits, pcb, tz, dense);
      return;
    }
  }
  // items per thread sized to the unit: a sort pass costs in proportion to
  // the slots it sorts, padding included
  if (n_u <= 4u * UBLOCK) unit_body<WEIGHTED, uint32_t, 4>(sm, a, u, cb, ce, n_u, g, kbits, pcb, tz, dense);
  else if (n_u <= 8u * UBLOCK) unit_body<WEIGHTED, uint32_t, 8>(sm, a, u, cb, ce, n_u, g, kbits, pcb, tz, dense);
  else unit_body<WEIGHTED, uint32_t, UITEMS>(sm, a, u, cb, ce, n_u, g, kbits, pcb, tz, dense);
}

// Output offsets: exclusive scan of the units' key counts (a big context's
// count comes from the chunk path), one workgroup.
__global__ void __launch_bounds__(1024) k_unit_offsets(const UnitMeta* __restrict__ meta,
                                                       const int32_t* __restrict__ unit_big,
                                                       const uint64_t* __restrict__ big_U, uint32_t n_units,
                                                       uint32_t n_ctx, uint64_t* __restrict__ unit_off,
                                                       uint64_t* __restrict__ ctx_off, PlanInfo* __restrict__ info) {
  __shared__ unsigned long long s_tmp[1024 / WAVE + 1];
  unsigned long long carry = 0;
  for (uint32_t b0 = 0; b0 < n_units; b0 += 1024) {
    const uint32_t u = b0 + threadIdx.x;
    unsigned long long v = 0;
    if (u < n_units) {
      const int32_t big = unit_big[u];
      v = big >= 0 ? big_U[big] : meta[u].nU;
    }
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan<1024>(v, s_tmp, &tot);
    if (u < n_units) unit_off[u] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    unit_off[n_units] = carry;
    ctx_off[n_ctx] = carry;
    info->total_keys = carry;
  }
}

// Context offsets: one wave per unit scans its per-context key counts.  With
// split contexts the unit's contexts are virtual: a real context's offset is
// that of its first virtual context.
__global__ void __launch_bounds__(256) k_ctx_offsets(const uint32_t* __restrict__ unit_begin,
                                                     const int32_t* __restrict__ unit_big,
                                                     const uint32_t* __restrict__ ucnt,
                                                     const uint64_t* __restrict__ unit_off, uint32_t n_units,
                                                     const uint32_t* __restrict__ vreal,
                                                     const uint32_t* __restrict__ vbase,
                                                     uint64_t* __restrict__ ctx_off, uint64_t* __restrict__ big_out) {
  const uint32_t u = blockIdx.x * (256 / WAVE) + wave_id();
  if (u >= n_units) return;
  const uint32_t cb = unit_begin[u], ce = unit_begin[u + 1];
  const uint64_t off = unit_off[u];
  const int32_t big = unit_big[u];
  if (big >= 0) {  // one context
    if (lane_id() == 0) {
      ctx_off[vreal ? vreal[cb] : cb] = off;
      big_out[big] = off;
    }
    return;
  }
  const uint32_t l = lane_id();
  const uint32_t v = l < ce - cb ? ucnt[(uint64_t)u * MAXC + l] : 0u;
  const uint32_t inc = wave_incl_scan(v);
  if (l < ce - cb) {
    const uint32_t vc = cb + l;
    const uint32_t c = vreal ? vreal[vc] : vc;
    if (!vreal || vbase[c] == vc) ctx_off[c] = off + inc - v;
  }
}

// Write pass: unpack every unit's staged keys into the outputs.
constexpr int WBLOCK = 512;
constexpr int WBATCH = 4;
__global__ void __launch_bounds__(WBLOCK) k_units_write(UnitArgs a, const uint64_t* __restrict__ unit_off,
                                                       MapDev map, OutDev out, int weighted) {
  __shared__ uint64_t s_lo[DENSE_MAX_WIN], s_hi[DENSE_MAX_WIN], s_d[DENSE_MAX_WIN + 1];
  const uint32_t u = blockIdx.x;
  const UnitDesc du = a.desc[u];
  if (du.big >= 0) return;
  const UnitMeta m = a.meta[u];
  if (m.nU == 0) return;
  const bool dense = (m.flags & UM_DENSE) != 0, wide = (m.flags & UM_WIDE) != 0;
  DenseDev t = a.dd;
  int map_dense = a.dense;
  uint32_t cbase = 0;
  if (a.pm) {
    const ProfMap& pmp = a.pm[a.cprof[a.vreal ? a.vreal[du.cb] : du.cb]];
    t = pmp.dd;
    map_dense = pmp.dense;
    map = pmp.md;
    cbase = pmp.ctx_base;
  }
  if (map_dense) {
    for (uint32_t i = threadIdx.x; i < t.n_win; i += WBLOCK) {
      s_lo[i] = t.lo[i];
      s_hi[i] = t.hi[i];
    }
    for (uint32_t i = threadIdx.x; i <= t.n_win; i += WBLOCK) s_d[i] = t.d[i];
    t.lo = s_lo;
    t.hi = s_hi;
    t.d = s_d;
  }
  __syncthreads();
  const uint32_t cb = du.cb;
  const uint64_t s0 = du.s0, o0 = unit_off[u];
  const uint64_t pmask = m.pcb >= 64 ? ~0ull : ((1ull << m.pcb) - 1);
  const uint32_t* __restrict__ skey = a.skey + s0;
  // the staging arrays a call does not use are null
  const uint32_t* __restrict__ shi = a.shi ? a.shi + s0 : nullptr;
  const uint32_t* __restrict__ scnt = a.scnt ? a.scnt + s0 : nullptr;
  const unsigned long long* __restrict__ scnt64 = a.scnt64 ? a.scnt64 + s0 : nullptr;
  // WBATCH keys per thread per step: all loads are issued before the
  // dependent table lookups and the stores
  for (uint32_t b0 = 0; b0 < m.nU; b0 += WBLOCK * WBATCH) {
    uint64_t k[WBATCH];
    unsigned long long c[WBATCH];
#pragma unroll
    for (int q = 0; q < WBATCH; ++q) {
      const uint32_t ui = b0 + q * WBLOCK + threadIdx.x;
      k[q] = 0;
      c[q] = 0;
      if (ui < m.nU) {
        k[q] = skey[ui];
        if (wide) k[q] |= (uint64_t)shi[ui] << 32;
        c[q] = weighted ? scnt64[ui] : (unsigned long long)scnt[ui];
      }
    }
#pragma unroll
    for (int q = 0; q < WBATCH; ++q) {
      const uint32_t ui = b0 + q * WBLOCK + threadIdx.x;
      if (ui >= m.nU) continue;
      const uint32_t lc = (uint32_t)(k[q] >> (m.pcb + 4));
      const uint64_t v = m.lo + (((k[q] >> 4) & pmask) << m.tz);
      const uint64_t o = o0 + ui;
      out.ctx[o] = (a.vreal ? a.vreal[cb + lc] : cb + lc) - cbase;
      out.stall[o] = (uint8_t)(k[q] & 15);
      out.count[o] = c[q];
      if (dense) {
        out.pc[o] = from_dense(t, v);
        out.scope[o] = t.scope_of[v];
      } else {
        out.pc[o] = v;
        // a unit with a pc off the dense grid, or a batch profile without
        // dense coordinates: binary search (a single map without them is
        // labelled by its own pass afterwards)
        if (map_dense || a.pm) {
          const uint32_t iv = find_interval(map.start, map.end, map.n_iv, v, 0, map.n_iv);
          out.scope[o] = iv == NONE32 ? NONE32 : map.scope[iv];
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// big contexts: chunk sort -> merge rounds -> heads -> write
// ----------------------------------------------------------------------------
struct BigArgs {
  const uint64_t* pc;
  const uint8_t* stall;
  const uint32_t* weight;
  const uint64_t* sbase;
  const uint64_t* rbase;
  const Run* grouped;
  const uint32_t* big_ctx;
  const uint64_t* big_sbase;
  const uint64_t* big_chunk;
  uint32_t n_big;
  uint64_t n_chunks;
  PlanInfo* info;
  DenseDev dd;
  int dense;
  const uint32_t* vreal;  // real context of every virtual one (null: no split contexts)
  const ProfMap* pm;      // batch of profiles (null: one profile)
  const uint32_t* cprof;
};

struct ListBuf {
  uint64_t* pc;
  uint8_t* stall;
  unsigned long long* cnt;
  uint64_t* len;  // per chunk: length of the list that starts at this chunk
};

__device__ inline uint32_t chunk_owner(const uint64_t* big_chunk, uint32_t n_big, uint64_t ch) {
  uint32_t lo = 0, hi = n_big;  // last b with big_chunk[b] <= ch
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (big_chunk[mid] <= ch) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Hand the sorted unique keys to `emit(ui, local ctx, coordinate, stall,
// count)` in unique-key order.  32-bit keys come from their compacted copy in
// LDS, so consecutive lanes take consecutive keys (coalesced output); wider
// keys are emitted by the thread that holds them.  The coordinate is the
// dense coordinate or the pc, whichever the keys were built from.
template <class K, class Emit>
__device__ inline void emit_keys(const SortSmem& sm, const K (&key)[UITEMS], uint64_t n_u, uint32_t first,
                                 uint32_t nU, int pcb, uint32_t tz, Emit&& emit) {
  const uint64_t pmask = pcb >= 64 ? ~0ull : ((1ull << pcb) - 1);
  if constexpr (sizeof(K) == 4) {
    for (uint32_t ui = threadIdx.x; ui < nU; ui += UBLOCK) {
      const uint64_t kk = sm.buf[ui];
      const uint32_t cnt = (uint32_t)sm.upos[ui + 1] - (uint32_t)sm.upos[ui];
      const uint32_t lc = (uint32_t)(kk >> (pcb + 4));
      emit(ui, lc, sm.pcmin[lc] + (((kk >> 4) & pmask) << tz), (uint8_t)(kk & 15), cnt);
    }
  } else {
    K prev = prev_last<K>(sm, threadIdx.x);
    uint32_t ui = first;
#pragma unroll
    for (int i = 0; i < UITEMS; ++i) {
      uint32_t p = threadIdx.x * UITEMS + i;
      bool h = p < n_u && (p == 0 || key[i] != prev);
      prev = key[i];
      if (!h) continue;
      const uint64_t kk = (uint64_t)key[i];
      const uint32_t lc = (uint32_t)(kk >> (pcb + 4));
      emit(ui, lc, sm.pcmin[lc] + (((kk >> 4) & pmask) << tz), (uint8_t)(kk & 15), (uint32_t)sm.upos[ui + 1] - p);
      ++ui;
    }
  }
}

// Sort one chunk of a big context and write its unique keys (real pcs) as a
// sorted list.
template <bool WEIGHTED, class K>
__device__ __forceinline__ void chunk_body(SortSmem& sm, const ListBuf& o, uint64_t ch, uint64_t obase, Gathered<WEIGHTED>& g,
                           uint64_t n_u, int kbits, int pcb, uint32_t tz, bool dense, const DenseDev& t) {
  K key[UITEMS];
  uint32_t val[UITEMS];
  sort_reduce<WEIGHTED, K>(sm, g, n_u, 1, key, val, kbits, pcb, tz);
  uint32_t first, nU;
  find_heads<K>(sm, key, n_u, 1, pcb, first, nU);
  if (threadIdx.x == 0) o.len[ch] = nU;
  uint64_t* const t_pc = o.pc + obase;
  uint8_t* const t_st = o.stall + obase;
  unsigned long long* const t_cnt = o.cnt + obase;
  emit_keys<K>(sm, key, n_u, first, nU, pcb, tz, [=](uint32_t ui, uint32_t, uint64_t v, uint8_t st, uint32_t cnt) {
    t_pc[ui] = dense ? from_dense(t, v) : v;
    t_st[ui] = st;
    if constexpr (!WEIGHTED) t_cnt[ui] = cnt;
  });
  if constexpr (WEIGHTED) weighted_counts<K>(sm, key, val, n_u, first, t_cnt);
}

// GENERAL = false sorts the chunks whose keys fit 32 bits and marks the others
// (list length WIDE_CHUNK); GENERAL = true, launched next, sorts only those.
template <bool WEIGHTED, bool SCATTERED, bool GENERAL>
__global__ void __launch_bounds__(UBLOCK) k_big_chunks(BigArgs a, ListBuf o) {
  __shared__ SortSmem sm;
  __shared__ uint64_t s_sb[2];
  const uint64_t ch = blockIdx.x;
  if (GENERAL && o.len[ch] != WIDE_CHUNK) return;
  const uint32_t b = chunk_owner(a.big_chunk, a.n_big, ch);
  const uint32_t c = a.big_ctx[b];
  const uint64_t j = ch - a.big_chunk[b];
  const uint64_t nc = a.sbase[c + 1] - a.sbase[c];
  const uint64_t s0 = a.sbase[c] + j * UT;
  const uint64_t n_u = min((uint64_t)UT, nc - j * UT);
  if (threadIdx.x == 0) { s_sb[0] = a.sbase[c]; s_sb[1] = a.sbase[c + 1]; }
  DenseDev src = a.dd;
  int map_dense = a.dense;
  if (a.pm) {
    const ProfMap& pmp = a.pm[a.cprof[a.vreal ? a.vreal[c] : c]];
    src = pmp.dd;
    map_dense = pmp.dense;
  }
  const DenseDev t = stage_dense(sm, src);  // LDS view (empty when the map has no dense coordinates)
  __syncthreads();
  Gathered<WEIGHTED> g;
  gather<SCATTERED, WEIGHTED>(g, s0, n_u, c, a.grouped, SCATTERED ? 0 : a.rbase[c], SCATTERED ? 0 : a.rbase[c + 1],
                              s_sb, 1, a.pc, a.stall, a.weight, &a.info->err, sm.runs);
  bool dense = false;
  if (map_dense) {
    densify(sm, g, n_u, t);
    __syncthreads();
    dense = sm.far == 0;
    if (!dense)
      gather<SCATTERED, WEIGHTED>(g, s0, n_u, c, a.grouped, SCATTERED ? 0 : a.rbase[c], SCATTERED ? 0 : a.rbase[c + 1],
                                  s_sb, 1, a.pc, a.stall, a.weight, &a.info->err, sm.runs);
  }
  int kbits, pcb;
  uint32_t tz;
  key_stats(sm, g, n_u, 1, &a.info->err, kbits, pcb, tz);
  const uint64_t obase = a.big_sbase[b] + j * UT;
  if (kbits > 63) {
    if (threadIdx.x == 0) o.len[ch] = 0;
    return;
  }
  if (!GENERAL && kbits > 31) {
    if (threadIdx.x == 0) o.len[ch] = WIDE_CHUNK;
    return;
  }
  __syncthreads();
  if constexpr (GENERAL) chunk_body<WEIGHTED, uint64_t>(sm, o, ch, obase, g, n_u, kbits, pcb, tz, dense, t);
  else chunk_body<WEIGHTED, uint32_t>(sm, o, ch, obase, g, n_u, kbits, pcb, tz, dense, t);
}

__device__ inline bool key_less(uint64_t pa, uint8_t sa, uint64_t pb, uint8_t sb) {
  return pa < pb || (pa == pb && sa < sb);
}

// One merge round: lists of 2^r chunks pair up into lists of 2^(r+1) chunks.
__global__ void __launch_bounds__(256) k_big_merge(BigArgs a, ListBuf in, ListBuf out, int r) {
  const uint64_t ch = blockIdx.x;
  const uint32_t b = chunk_owner(a.big_chunk, a.n_big, ch);
  const uint64_t c0 = a.big_chunk[b], nch = a.big_chunk[b + 1] - c0;
  const uint64_t j = ch - c0;
  const uint64_t L = j >> r;               // my list
  const uint64_t first_mine = L << r;      // first chunk of my list
  const uint64_t other = L ^ 1ull;
  const uint64_t first_other = other << r;
  const uint64_t first_merged = (L >> 1) << (r + 1);
  const bool is_b = (L & 1) != 0;
  const uint64_t len_mine = in.len[c0 + first_mine];
  const uint64_t len_other = first_other < nch ? in.len[c0 + first_other] : 0;
  const uint64_t base = a.big_sbase[b];
  const uint64_t mine_off = base + first_mine * UT, other_off = base + first_other * UT;
  const uint64_t out_off = base + first_merged * UT;
  const uint64_t e0 = (j - first_mine) * UT;
  if (threadIdx.x == 0 && j == first_merged) {
    uint64_t la = is_b ? len_other : len_mine, lb = is_b ? len_mine : len_other;
    out.len[c0 + first_merged] = la + lb;
  }
  for (uint64_t e = e0 + threadIdx.x; e < e0 + UT && e < len_mine; e += blockDim.x) {
    uint64_t p = in.pc[mine_off + e];
    uint8_t s = in.stall[mine_off + e];
    unsigned long long cnt = in.cnt[mine_off + e];
    // rank in the other list: A elements go before equal B elements
    uint64_t lo = 0, hi = len_other;
    while (lo < hi) {
      uint64_t mid = (lo + hi) >> 1;
      uint64_t q = in.pc[other_off + mid];
      uint8_t qs = in.stall[other_off + mid];
      bool go_right = is_b ? !key_less(p, s, q, qs) : key_less(q, qs, p, s);
      if (go_right) lo = mid + 1;
      else hi = mid;
    }
    uint64_t pos = out_off + e + lo;
    out.pc[pos] = p;
    out.stall[pos] = s;
    out.cnt[pos] = cnt;
  }
}

// heads per chunk-sized slot of each big context's final list
__global__ void __launch_bounds__(256) k_big_heads(BigArgs a, ListBuf fin, unsigned long long* slot_heads) {
  __shared__ unsigned long long s_tmp[256 / WAVE + 1];
  const uint64_t ch = blockIdx.x;
  const uint32_t b = chunk_owner(a.big_chunk, a.n_big, ch);
  const uint64_t c0 = a.big_chunk[b];
  const uint64_t len = fin.len[c0];
  const uint64_t base = a.big_sbase[b];
  const uint64_t e0 = (ch - c0) * UT;
  unsigned long long h = 0;
  for (uint64_t e = e0 + threadIdx.x; e < e0 + UT && e < len; e += blockDim.x)
    h += e == 0 || fin.pc[base + e] != fin.pc[base + e - 1] || fin.stall[base + e] != fin.stall[base + e - 1];
  unsigned long long tot;
  block_excl_scan<256>(h, s_tmp, &tot);
  if (threadIdx.x == 0) slot_heads[ch] = tot;
}

// exclusive scan of slot head counts (one workgroup), per-context totals
__global__ void __launch_bounds__(1024) k_big_scan(BigArgs a, unsigned long long* slot_heads, uint64_t* big_U) {
  __shared__ unsigned long long s_tmp[1024 / WAVE + 1];
  unsigned long long carry = 0;
  for (uint64_t b0 = 0; b0 < a.n_chunks; b0 += 1024) {
    uint64_t i = b0 + threadIdx.x;
    unsigned long long v = i < a.n_chunks ? slot_heads[i] : 0;
    unsigned long long tot;
    unsigned long long ex = block_excl_scan<1024>(v, s_tmp, &tot);
    if (i < a.n_chunks) slot_heads[i] = carry + ex;
    carry += tot;
    __syncthreads();
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < a.n_big; b += 1024) {
    uint64_t c0 = a.big_chunk[b], c1 = a.big_chunk[b + 1];
    unsigned long long end = c1 < a.n_chunks ? slot_heads[c1] : carry;
    big_U[b] = end - slot_heads[c0];
  }
}

__global__ void __launch_bounds__(256) k_big_write(BigArgs a, ListBuf fin, const unsigned long long* slot_prefix,
                                                   const uint64_t* big_out, MapDev map, OutDev out) {
  __shared__ unsigned long long s_tmp[256 / WAVE + 1];
  const uint64_t ch = blockIdx.x;
  const uint32_t b = chunk_owner(a.big_chunk, a.n_big, ch);
  const uint64_t c0 = a.big_chunk[b];
  const uint32_t c = a.big_ctx[b];
  const uint64_t len = fin.len[c0];
  const uint64_t base = a.big_sbase[b];
  const uint64_t e0 = (ch - c0) * UT;
  const unsigned long long slot0 = slot_prefix[ch] - slot_prefix[c0];
  unsigned long long done = 0;
  for (uint64_t eb = e0; eb < e0 + UT && eb < len; eb += blockDim.x) {
    uint64_t e = eb + threadIdx.x;
    bool h = e < len && e < e0 + UT &&
             (e == 0 || fin.pc[base + e] != fin.pc[base + e - 1] || fin.stall[base + e] != fin.stall[base + e - 1]);
    unsigned long long tot;
    unsigned long long ex = block_excl_scan<256>((unsigned long long)h, s_tmp, &tot);
    if (h) {
      uint64_t p = fin.pc[base + e];
      uint8_t s = fin.stall[base + e];
      unsigned long long cnt = fin.cnt[base + e];
      for (uint64_t f = e + 1; f < len && fin.pc[base + f] == p && fin.stall[base + f] == s; ++f) cnt += fin.cnt[base + f];
      uint64_t o = big_out[b] + slot0 + done + ex;
      const uint32_t rc = a.vreal ? a.vreal[c] : c;
      if (a.pm) {
        const ProfMap& pmp = a.pm[a.cprof[rc]];
        out.ctx[o] = rc - pmp.ctx_base;
        out.scope[o] = scope_of_pc(pmp.dd, pmp.dense != 0, pmp.md.start, pmp.md.end, pmp.md.scope, pmp.md.n_iv, p);
      } else {
        out.ctx[o] = rc;
        if (a.dense) out.scope[o] = scope_of_pc(a.dd, true, map.start, map.end, map.scope, map.n_iv, p);
      }
      out.pc[o] = p;
      out.stall[o] = s;
      out.count[o] = cnt;
    }
    done += tot;
  }
}

}  // namespace
}  // namespace hpa

using namespace hpa;

namespace hpa {

// Run-time parameters of the pipeline (chosen by the batch autotuner).
struct Knobs {
  uint32_t merge_rounds = 2;    // rounds of adjacent unit-pair merges
  uint32_t scan_wg_per_cu = 4;  // workgroups per CU of the context scan
};

// A batch of profiles for one pipeline run: per profile maps and the profile
// of every global context (device), and the profiles' maps (host).
struct BatchRun {
  const ProfMap* pm = nullptr;
  const uint32_t* cprof = nullptr;
};

// The attribution pipeline.  With `batch`, the samples' contexts are global
// ids over the batch's profiles (units never mix profiles, each unit and big
// context uses its profile's map, output contexts are local to their profile)
// and big contexts always take the chunk path.
// With `into`, the result goes into that caller-owned object (and its output
// arrays are the caller's when `into` already holds non-owning views).
hpa_attribution* attribute_impl(hpa_ctx* ctx, const hpa_structure_map* map, const BatchRun* batch,
                                const hpa_samples* smp, hipStream_t stream, const Knobs& kn,
                                hpa_attribution* into) {
  {
    hipStream_t s = stream;
    const uint64_t n = smp->n;
    const uint32_t C = smp->n_ctx;
    auto* A = into ? into : new hpa_attribution();
    std::unique_ptr<hpa_attribution> hold(into ? nullptr : A);
    A->ctx = ctx;
    A->stream = s;
    A->map = map;
    A->n_ctx = C;
    const uint64_t cap = n ? n : 1;
    if (!A->ctx_id.p) {
      A->ctx_id = DBuf(ctx, cap * 4, s);
      A->pc = DBuf(ctx, cap * 8, s);
      A->stall = DBuf(ctx, cap, s);
      A->count = DBuf(ctx, cap * 8, s);
      A->scope = DBuf(ctx, cap * 4, s);
      A->ctx_offsets = DBuf(ctx, ((uint64_t)C + 1) * 8, s);
    }
    if (n == 0) {
      HPA_HIP(hipMemsetAsync(A->ctx_offsets.p, 0, ((uint64_t)C + 1) * 8, s));
      sync_stream(ctx, s);
      A->n_keys = 0;
      hold.release();
      return A;
    }
    StageTimer tm(ctx, s);
    // --- scan ctx, plan ---
    tm.begin("scan_ctx");
    const uint64_t run_cap = std::min<uint64_t>(std::max<uint64_t>(n / 8, 1024), 1ull << 24);
    DBuf d_info(ctx, sizeof(PlanInfo), s);
    DBuf d_hist(ctx, (uint64_t)C * 8, s);
    DBuf d_runs(ctx, run_cap * sizeof(Run), s);
    HPA_HIP(hipMemsetAsync(d_info.p, 0, sizeof(PlanInfo), s));
    HPA_HIP(hipMemsetAsync(d_hist.p, 0, (uint64_t)C * 8, s));
    {
      uint64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
      // as many workgroups as are resident at once (four per CU at its
      // 33 KB of LDS), each looping over tiles
      unsigned grid = (unsigned)std::min<uint64_t>(tiles, (uint64_t)ctx->n_cu * kn.scan_wg_per_cu);
      k_scan_ctx<<<grid, SCAN_BLOCK, 0, s>>>(smp->ctx, n, C, d_hist.as<unsigned long long>(), d_runs.as<Run>(),
                                             run_cap, d_info.as<PlanInfo>());
      HPA_HIP(hipGetLastError());
    }
    // the run/scatter decision needs the run count, the split the number of
    // contexts over T samples
    DBuf d_bigof(ctx, (uint64_t)C * 4, s);
    k_big_index<<<grid_for(C, 256, ctx->n_cu * 8), 256, 0, s>>>(d_hist.as<unsigned long long>(), C,
                                                                  d_bigof.as<int32_t>(), d_info.as<PlanInfo>());
    HPA_HIP(hipGetLastError());
    PlanInfo info;
    HPA_HIP(hipMemcpyAsync(&info, d_info.p, sizeof(info), hipMemcpyDeviceToHost, s));
    sync_stream(ctx, s);
    if (info.err & ERR_CTX) fail(HPA_E_INVAL, "a sample has ctx >= n_ctx");
    const bool scattered = info.n_runs > run_cap;
    tm.end(n, 0);
    const bool weighted = smp->weight != nullptr;
    // --- split of big contexts by coordinate range (run list and dense map only) ---
    const bool split = !batch && !scattered && map->dense && info.n_bigall > 0;
    uint32_t CV = C;  // contexts after the split
    DBuf d_vhist, d_vreal, d_vgrp, d_vbase, d_vsolo, d_bhist, d_bflag, d_partof, d_psum, d_nparts;
    uint32_t bshift = 0;
    const DenseDev dd{map->win_lo.as<uint64_t>(), map->win_hi.as<uint64_t>(), map->win_d.as<uint64_t>(),
                      map->scope_of.as<uint32_t>(), map->n_win, map->dense_tz};
    if (split) {
      tm.begin("split_plan");
      const uint32_t NBIG = info.n_bigall;
      // every coordinate D < n_dense has its bucket D >> bshift below NB
      while (((map->n_dense - 1) >> bshift) >= (uint64_t)NB) ++bshift;
      d_bhist = DBuf(ctx, (uint64_t)NBIG * NB * 4, s);
      d_bflag = DBuf(ctx, (uint64_t)NBIG * 4, s);
      d_partof = DBuf(ctx, (uint64_t)NBIG * NB * 4, s);
      d_psum = DBuf(ctx, (uint64_t)NBIG * NB * 4, s);
      d_nparts = DBuf(ctx, (uint64_t)NBIG * 4, s);
      HPA_HIP(hipMemsetAsync(d_bhist.p, 0, d_bhist.bytes, s));
      HPA_HIP(hipMemsetAsync(d_bflag.p, 0, d_bflag.bytes, s));
      HPA_HIP(hipMemsetAsync(d_psum.p, 0, d_psum.bytes, s));
      k_big_hist<<<(unsigned)std::min<uint64_t>(std::max<uint64_t>(info.n_runs, 1), (uint64_t)ctx->n_cu * 8),
                   SPLIT_BLOCK, 0, s>>>(d_runs.as<Run>(), info.n_runs, d_bigof.as<int32_t>(), smp->pc, dd, bshift,
                                        d_bhist.as<uint32_t>(), d_bflag.as<uint32_t>());
      k_big_parts<<<(NBIG + 3) / 4, 256, 0, s>>>(d_bhist.as<uint32_t>(), d_bflag.as<uint32_t>(), NBIG,
                                                d_partof.as<uint32_t>(), d_psum.as<uint32_t>(),
                                                d_nparts.as<uint32_t>());
      // at most NB parts per big context
      const uint64_t cv_cap = (uint64_t)C + (uint64_t)NBIG * (NB - 1);
      d_vhist = DBuf(ctx, cv_cap * 8, s);
      d_vreal = DBuf(ctx, cv_cap * 4, s);
      d_vgrp = DBuf(ctx, cv_cap * 4, s);
      d_vbase = DBuf(ctx, ((uint64_t)C + 1) * 4, s);
      d_vsolo = DBuf(ctx, (uint64_t)C * 4, s);
      const uint32_t vtiles = (C + VT - 1) / VT;
      DBuf d_vtile(ctx, ((uint64_t)vtiles + 1) * 4, s);
      k_virtual_count<<<vtiles, VT, 0, s>>>(C, d_bigof.as<int32_t>(), d_nparts.as<uint32_t>(),
                                           d_vtile.as<uint32_t>());
      k_tile_scan<<<1, 1024, 0, s>>>(d_vtile.as<uint32_t>(), vtiles, d_vtile.as<uint32_t>() + vtiles);
      k_virtual_write<<<vtiles, VT, 0, s>>>(d_hist.as<unsigned long long>(), C, d_bigof.as<int32_t>(),
                                           d_nparts.as<uint32_t>(), d_psum.as<uint32_t>(), d_vtile.as<uint32_t>(),
                                           d_vhist.as<unsigned long long>(), d_vreal.as<uint32_t>(),
                                           d_vgrp.as<uint32_t>(), d_vbase.as<uint32_t>(), d_vsolo.as<uint32_t>(),
                                           d_info.as<PlanInfo>());
      HPA_HIP(hipGetLastError());
      HPA_HIP(hipMemcpyAsync(&info, d_info.p, sizeof(info), hipMemcpyDeviceToHost, s));
      sync_stream(ctx, s);
      CV = info.n_virtual;
      tm.end(info.split_samples, info.n_parts);
    }
    // --- plan over the (virtual) contexts ---
    tm.begin("plan");
    DBuf d_sbase(ctx, ((uint64_t)CV + 1) * 8, s);
    DBuf d_rbase(ctx, ((uint64_t)CV + 1) * 8, s);
    DBuf d_ubeg(ctx, ((uint64_t)CV + 1) * 4, s);
    DBuf d_ubig(ctx, ((uint64_t)CV + 1) * 4, s);
    DBuf d_bctx(ctx, ((uint64_t)CV + 1) * 4, s);
    DBuf d_bsb(ctx, ((uint64_t)CV + 1) * 8, s);
    DBuf d_bch(ctx, ((uint64_t)CV + 1) * 8, s);
    {
      const unsigned long long* vh = split ? d_vhist.as<unsigned long long>() : d_hist.as<unsigned long long>();
      const uint32_t* vg = split ? d_vgrp.as<uint32_t>() : nullptr;
      const uint32_t ptiles = (CV + PLAN_BLOCK - 1) / PLAN_BLOCK;
      DBuf d_psums(ctx, (uint64_t)ptiles * PLAN_NV * 8, s);
      DBuf d_pstart(ctx, (uint64_t)CV, s);
      DBuf d_pts(ctx, ((uint64_t)ptiles + 1) * 4, s);
      k_plan_sums<<<ptiles, PLAN_BLOCK, 0, s>>>(vh, CV, d_psums.as<unsigned long long>(), d_info.as<PlanInfo>());
      k_plan_tile_scan<<<1, 1024, 0, s>>>(d_psums.as<unsigned long long>(), ptiles, CV, d_sbase.as<uint64_t>(),
                                          d_rbase.as<uint64_t>(), d_bsb.as<uint64_t>(), d_bch.as<uint64_t>(),
                                          d_info.as<PlanInfo>());
      const uint32_t* pg = batch ? batch->cprof : nullptr;
      k_plan_starts<<<ptiles, PLAN_BLOCK, 0, s>>>(vh, CV, vg, pg, d_psums.as<unsigned long long>(), d_sbase.as<uint64_t>(),
                                                 d_rbase.as<uint64_t>(), d_bctx.as<uint32_t>(), d_bsb.as<uint64_t>(),
                                                 d_bch.as<uint64_t>(), d_pstart.as<uint8_t>(), d_pts.as<uint32_t>());
      k_tile_scan<<<1, 1024, 0, s>>>(d_pts.as<uint32_t>(), ptiles, d_pts.as<uint32_t>() + ptiles);
      k_plan_units<<<ptiles, PLAN_BLOCK, 0, s>>>(vh, CV, vg, d_psums.as<unsigned long long>(), d_pstart.as<uint8_t>(),
                                                d_pts.as<uint32_t>(), d_ubeg.as<uint32_t>(), d_ubig.as<int32_t>(),
                                                d_info.as<PlanInfo>());
      // merge adjacent unit pairs, twice (at most CV units: tiles over CV);
      // each round reads the unit count the previous one left in n_units
      DBuf d_ubeg2(ctx, ((uint64_t)CV + 1) * 4, s);
      DBuf d_ubig2(ctx, ((uint64_t)CV + 1) * 4, s);
      if (kn.merge_rounds == 0) k_keep_units<<<1, 1, 0, s>>>(d_info.as<PlanInfo>());
      for (uint32_t round = 0; round < kn.merge_rounds; ++round) {
        if (round) {
          k_set_units<<<1, 1, 0, s>>>(d_info.as<PlanInfo>());
        }
        const uint32_t* pgm = pg;
        k_merge_count<<<ptiles, PLAN_BLOCK, 0, s>>>(d_ubeg.as<uint32_t>(), d_ubig.as<int32_t>(), d_sbase.as<uint64_t>(),
                                                   vg, pgm, d_info.as<PlanInfo>(), d_pts.as<uint32_t>());
        k_tile_scan<<<1, 1024, 0, s>>>(d_pts.as<uint32_t>(), ptiles, d_pts.as<uint32_t>() + ptiles);
        k_merge_write<<<ptiles, PLAN_BLOCK, 0, s>>>(d_ubeg.as<uint32_t>(), d_ubig.as<int32_t>(), d_sbase.as<uint64_t>(),
                                                   vg, pgm, CV, d_pts.as<uint32_t>(), d_ubeg2.as<uint32_t>(),
                                                   d_ubig2.as<int32_t>(), d_info.as<PlanInfo>());
        HPA_HIP(hipGetLastError());
        std::swap(d_ubeg, d_ubeg2);
        std::swap(d_ubig, d_ubig2);
      }
      HPA_HIP(hipGetLastError());
    }
    HPA_HIP(hipMemcpyAsync(&info, d_info.p, sizeof(info), hipMemcpyDeviceToHost, s));
    sync_stream(ctx, s);
    tm.end(CV, info.n_units);
    const uint32_t* vreal = split ? d_vreal.as<uint32_t>() : nullptr;
    // --- order samples by context ---
    DBuf d_cur(ctx, (uint64_t)CV * 8, s);
    HPA_HIP(hipMemsetAsync(d_cur.p, 0, (uint64_t)CV * 8, s));
    DBuf d_grp, d_spc, d_sst, d_sw, d_tpc, d_tst, d_tw;
    const uint64_t* src_pc = smp->pc;
    const uint8_t* src_st = smp->stall;
    const uint32_t* src_w = smp->weight;
    tm.begin(scattered ? "scatter" : "group_runs");
    if (!scattered) {
      d_grp = DBuf(ctx, std::max<uint64_t>(info.n_runs, 1) * sizeof(Run), s);
      k_group_runs<<<grid_for(info.n_runs, 256, ctx->n_cu * 8), 256, 0, s>>>(
          d_runs.as<Run>(), info.n_runs, split ? d_vsolo.as<uint32_t>() : nullptr, d_sbase.as<uint64_t>(),
          d_rbase.as<uint64_t>(), d_cur.as<unsigned long long>(), d_grp.as<Run>());
      HPA_HIP(hipGetLastError());
      if (split) {
        // the samples of split contexts into part order, at the parts' flat positions
        d_tpc = DBuf(ctx, n * 8, s);
        d_tst = DBuf(ctx, n, s);
        if (weighted) d_tw = DBuf(ctx, n * 4, s);
        k_big_scatter<<<(unsigned)std::min<uint64_t>(std::max<uint64_t>(info.n_runs, 1), (uint64_t)ctx->n_cu * 8),
                        SPLIT_BLOCK, 0, s>>>(
            d_runs.as<Run>(), info.n_runs, d_bigof.as<int32_t>(), d_nparts.as<uint32_t>(), d_partof.as<uint32_t>(),
            d_vbase.as<uint32_t>(), d_sbase.as<uint64_t>(), d_cur.as<unsigned long long>(), smp->pc, smp->stall,
            smp->weight, dd, bshift, d_tpc.as<uint64_t>(), d_tst.as<uint8_t>(),
            weighted ? d_tw.as<uint32_t>() : nullptr, &d_info.as<PlanInfo>()->err);
        HPA_HIP(hipGetLastError());
      }
    } else {
      d_spc = DBuf(ctx, n * 8, s);
      d_sst = DBuf(ctx, n, s);
      if (weighted) d_sw = DBuf(ctx, n * 4, s);
      k_scatter<<<grid_for(n, 256, ctx->n_cu * 16), 256, 0, s>>>(
          smp->pc, smp->ctx, smp->stall, smp->weight, n, d_sbase.as<uint64_t>(), d_cur.as<unsigned long long>(),
          d_spc.as<uint64_t>(), d_sst.as<uint8_t>(), weighted ? d_sw.as<uint32_t>() : nullptr, C);
      HPA_HIP(hipGetLastError());
      src_pc = d_spc.as<uint64_t>();
      src_st = d_sst.as<uint8_t>();
      src_w = weighted ? d_sw.as<uint32_t>() : nullptr;
    }
    tm.end(scattered ? n : info.n_runs, 0);
    d_runs.release();
    // --- big contexts ---
    DBuf d_bigU(ctx, ((uint64_t)info.n_big + 1) * 8, s);
    DBuf d_bigout(ctx, ((uint64_t)info.n_big + 1) * 8, s);
    DBuf d_slot;
    ListBuf L[2] = {};
    DBuf lbuf[2][4];
    int fin = 0;
    BigArgs ba{src_pc, src_st, src_w, d_sbase.as<uint64_t>(), d_rbase.as<uint64_t>(), d_grp.as<Run>(),
               d_bctx.as<uint32_t>(), d_bsb.as<uint64_t>(), d_bch.as<uint64_t>(), info.n_big, info.n_chunks,
               d_info.as<PlanInfo>()};
    ba.dd = dd;
    ba.dense = map->dense ? 1 : 0;
    ba.vreal = vreal;
    ba.pm = batch ? batch->pm : nullptr;
    ba.cprof = batch ? batch->cprof : nullptr;
    if (info.n_big) {
      tm.begin("big_sort");
      const uint64_t bs = info.big_samples;
      for (int k = 0; k < 2; ++k) {
        lbuf[k][0] = DBuf(ctx, bs * 8, s);
        lbuf[k][1] = DBuf(ctx, bs, s);
        lbuf[k][2] = DBuf(ctx, bs * 8, s);
        lbuf[k][3] = DBuf(ctx, info.n_chunks * 8, s);
        L[k] = ListBuf{lbuf[k][0].as<uint64_t>(), lbuf[k][1].as<uint8_t>(),
                       lbuf[k][2].as<unsigned long long>(), lbuf[k][3].as<uint64_t>()};
      }
      unsigned g = (unsigned)info.n_chunks;
      // the narrow kernel first; the general one then takes the chunks it left
      if (weighted) {
        if (scattered) {
          k_big_chunks<true, true, false><<<g, UBLOCK, 0, s>>>(ba, L[0]);
          k_big_chunks<true, true, true><<<g, UBLOCK, 0, s>>>(ba, L[0]);
        } else {
          k_big_chunks<true, false, false><<<g, UBLOCK, 0, s>>>(ba, L[0]);
          k_big_chunks<true, false, true><<<g, UBLOCK, 0, s>>>(ba, L[0]);
        }
      } else {
        if (scattered) {
          k_big_chunks<false, true, false><<<g, UBLOCK, 0, s>>>(ba, L[0]);
          k_big_chunks<false, true, true><<<g, UBLOCK, 0, s>>>(ba, L[0]);
        } else {
          k_big_chunks<false, false, false><<<g, UBLOCK, 0, s>>>(ba, L[0]);
          k_big_chunks<false, false, true><<<g, UBLOCK, 0, s>>>(ba, L[0]);
        }
      }
      HPA_HIP(hipGetLastError());
      int r = 0;
      while ((1ull << r) < info.max_chunks) {
        k_big_merge<<<g, 256, 0, s>>>(ba, L[fin], L[fin ^ 1], r);
        HPA_HIP(hipGetLastError());
        fin ^= 1;
        ++r;
      }
      d_slot = DBuf(ctx, info.n_chunks * 8, s);
      k_big_heads<<<g, 256, 0, s>>>(ba, L[fin], d_slot.as<unsigned long long>());
      k_big_scan<<<1, 1024, 0, s>>>(ba, d_slot.as<unsigned long long>(), d_bigU.as<uint64_t>());
      HPA_HIP(hipGetLastError());
      tm.end(info.big_samples, 0);
    }
    // --- unit passes: sort (narrow, then the wide units), offsets, write ---
    const uint32_t NU = info.n_merged;
    DBuf d_udesc(ctx, std::max<uint64_t>(NU, 1) * sizeof(UnitDesc), s);
    k_unit_desc<<<grid_for(NU, 256, ctx->n_cu * 8), 256, 0, s>>>(d_ubeg.as<uint32_t>(), d_ubig.as<int32_t>(),
                                                                  d_sbase.as<uint64_t>(), d_rbase.as<uint64_t>(), NU,
                                                                  d_udesc.as<UnitDesc>());
    DBuf d_meta(ctx, std::max<uint64_t>(NU, 1) * sizeof(UnitMeta), s);
    DBuf d_ucnt(ctx, std::max<uint64_t>(NU, 1) * MAXC * 4, s);
    DBuf d_uoff(ctx, ((uint64_t)NU + 1) * 8, s);
    DBuf d_skey(ctx, n * 4, s), d_shi(ctx, n * 4, s), d_scnt;
    if (weighted) d_scnt = DBuf(ctx, n * 8, s);
    else d_scnt = DBuf(ctx, n * 4, s);
    MapDev md{map->start.as<uint64_t>(), map->end.as<uint64_t>(), map->scope.as<uint32_t>(), map->n_iv};
    OutDev od{A->ctx_id.as<uint32_t>(), A->pc.as<uint64_t>(), A->stall.as<uint8_t>(),
              A->count.as<unsigned long long>(), A->scope.as<uint32_t>(), A->ctx_offsets.as<uint64_t>()};
    UnitArgs ua{src_pc, src_st, src_w, d_sbase.as<uint64_t>(), d_rbase.as<uint64_t>(), d_grp.as<Run>(),
                d_ubeg.as<uint32_t>(), d_ubig.as<int32_t>(), d_info.as<PlanInfo>(), NU, C, dd,
                map->dense ? 1 : 0, d_meta.as<UnitMeta>(), d_ucnt.as<uint32_t>(), d_skey.as<uint32_t>(),
                d_shi.as<uint32_t>(), weighted ? nullptr : d_scnt.as<uint32_t>(),
                weighted ? d_scnt.as<unsigned long long>() : nullptr, UNIT_PLAIN, vreal, d_udesc.as<UnitDesc>(),
                batch ? batch->pm : nullptr, batch ? batch->cprof : nullptr};
    // the narrow launch over plain units is timed on its own: it is the
    // dominant kernel; the launches for wide keys and for parts follow
#define HPA_UNITS(W, S, A, NAME)                          \
  do {                                                    \
    if (NAME) tm.begin(NAME);                             \
    k_units32<W, S, false><<<NU, UBLOCK, 0, s>>>(A);      \
    if (NAME) tm.end();                                   \
    if (NAME) tm.begin("units_other");                    \
    k_units32<W, S, true><<<NU, UBLOCK, 0, s>>>(A);       \
  } while (0)
    if (weighted) {
      if (scattered) HPA_UNITS(true, true, ua, "units_plain");
      else HPA_UNITS(true, false, ua, "units_plain");
    } else {
      if (scattered) HPA_UNITS(false, true, ua, "units_plain");
      else HPA_UNITS(false, false, ua, "units_plain");
    }
    if (split) {
      // units of parts read the scattered copies at their flat positions
      UnitArgs pa = ua;
      pa.pc = d_tpc.as<uint64_t>();
      pa.stall = d_tst.as<uint8_t>();
      pa.weight = weighted ? d_tw.as<uint32_t>() : nullptr;
      pa.kind = UNIT_PART;
      if (weighted) HPA_UNITS(true, true, pa, (const char*)nullptr);
      else HPA_UNITS(false, true, pa, (const char*)nullptr);
    }
#undef HPA_UNITS
    HPA_HIP(hipGetLastError());
    tm.end();
    tm.begin("unit_write");
    k_unit_offsets<<<1, 1024, 0, s>>>(d_meta.as<UnitMeta>(), d_ubig.as<int32_t>(), d_bigU.as<uint64_t>(), NU, C,
                                      d_uoff.as<uint64_t>(), A->ctx_offsets.as<uint64_t>(), d_info.as<PlanInfo>());
    k_ctx_offsets<<<(NU + 3) / 4, 256, 0, s>>>(d_ubeg.as<uint32_t>(), d_ubig.as<int32_t>(), d_ucnt.as<uint32_t>(),
                                              d_uoff.as<uint64_t>(), NU, vreal,
                                              split ? d_vbase.as<uint32_t>() : nullptr,
                                              A->ctx_offsets.as<uint64_t>(), d_bigout.as<uint64_t>());
    k_units_write<<<NU, WBLOCK, 0, s>>>(ua, d_uoff.as<uint64_t>(), md, od, weighted ? 1 : 0);
    HPA_HIP(hipGetLastError());
    tm.end();
    if (info.n_big) {
      tm.begin("big_write");
      k_big_write<<<(unsigned)info.n_chunks, 256, 0, s>>>(ba, L[fin], d_slot.as<unsigned long long>(),
                                                        d_bigout.as<uint64_t>(), md, od);
      HPA_HIP(hipGetLastError());
      tm.end();
    }
    if (!batch && !map->dense) {
      // no dense coordinates: label every key with a binary search
      tm.begin("scope_labels");
      launch_scope_labels(map, A->pc.as<uint64_t>(), n, &d_info.as<PlanInfo>()->total_keys, A->scope.as<uint32_t>(),
                          s);
      tm.end();
    }
    HPA_HIP(hipMemcpyAsync(&info, d_info.p, sizeof(info), hipMemcpyDeviceToHost, s));
    sync_stream(ctx, s);
    if (info.err & ERR_STALL) fail(HPA_E_INVAL, "a sample has stall >= 16");
    if (info.err & ERR_SPLIT) fail(HPA_E_DEVICE, "internal error: a split context's samples missed their parts");
    if (info.err & ERR_WIDE) fail(HPA_E_UNSUPPORTED, "the PCs of one context span more than 2^56 bytes");
    A->n_keys = info.total_keys;
    if (tm.on()) {
      std::vector<uint64_t> bu(info.n_big);
      if (info.n_big) {
        HPA_HIP(hipMemcpyAsync(bu.data(), d_bigU.p, info.n_big * 8, hipMemcpyDeviceToHost, s));
        sync_stream(ctx, s);
      }
      uint64_t big_keys = 0;
      for (uint64_t v : bu) big_keys += v;
      tm.items("units_plain", n - info.big_samples - info.split_samples, 0);
      tm.items("units_other", info.split_samples, 0);
      tm.items("unit_write", info.total_keys - big_keys, info.total_keys - big_keys);
      tm.items("big_write", 0, big_keys);
      if (!map->dense) tm.items("scope_labels", info.total_keys, info.total_keys);
      tm.collect();
    }
    hold.release();
    return A;
  }
}

// One attribution: the dense pipeline when the map and sizes allow it, else
// (or when a sample's pc turns out to have no dense coordinate) the general
// pipeline, into the same handle.
hpa_attribution* attribute_any(hpa_ctx* ctx, const hpa_structure_map* map, const hpa_samples* smp, hipStream_t s,
                               hpa_attribution* into) {
  if (smp->n > 0 && dense_path_fits(map, smp)) {
    auto* A = into ? into : new hpa_attribution();
    std::unique_ptr<hpa_attribution> hold(into ? nullptr : A);
    A->ctx = ctx;
    A->stream = s;
    A->map = map;
    A->n_ctx = smp->n_ctx;
    const size_t arena_off = t_arena.off;
    if (attribute_dense(ctx, map, smp, s, A)) {
      hold.release();
      return A;
    }
    // the dense pipeline's working buffers are no longer in use (it has
    // synchronised): an arena may hand their space out again
    if (t_arena.base) t_arena.off = arena_off;
    attribute_impl(ctx, map, nullptr, smp, s, Knobs{}, A);
    hold.release();
    return A;
  }
  return attribute_impl(ctx, map, nullptr, smp, s, Knobs{}, into);
}

}  // namespace hpa

extern "C" hpa_status hpa_attribute(hpa_ctx* ctx, const hpa_structure_map* map, const hpa_samples* smp,
                                    hipStream_t stream, hpa_attribution** out) {
  return guard([&] {
    if (!ctx || !map || !smp || !out) fail(HPA_E_INVAL, "NULL argument");
    if (map->ctx != ctx) fail(HPA_E_INVAL, "map belongs to another context");
    if (smp->n && (!smp->pc || !smp->ctx || !smp->stall)) fail(HPA_E_INVAL, "NULL sample array");
    if (smp->n_ctx == 0 || smp->n_ctx >= 0x7FFFFFFFu) fail(HPA_E_INVAL, "n_ctx out of range");
    if (smp->n >= (1ull << 40)) fail(HPA_E_INVAL, "too many samples for one call");
    DeviceGuard dg(ctx->device);
    *out = attribute_any(ctx, map, smp, stream, nullptr);
  });
}

extern "C" hpa_status hpa_attribution_view_get(const hpa_attribution* a, hpa_attribution_view* v) {
  return guard([&] {
    if (!a || !v) fail(HPA_E_INVAL, "NULL argument");
    v->n_keys = a->n_keys;
    v->n_ctx = a->n_ctx;
    v->ctx = a->ctx_id.as<uint32_t>();
    v->pc = a->pc.as<uint64_t>();
    v->stall = a->stall.as<uint8_t>();
    v->count = a->count.as<uint64_t>();
    v->scope = a->scope.as<uint32_t>();
    v->ctx_offsets = a->ctx_offsets.as<uint64_t>();
  });
}

extern "C" void hpa_attribution_free(hpa_attribution* a) { delete a; }

// ============================================================================
// A batch of profiles (Section 6.1: profiles processed as concurrent tasks):
// the profiles' contexts are numbered globally, so one run of the pipeline
// attributes every profile of a round at once -- each stage is one launch
// over the whole round, and the hardware spreads the round's units over the
// chip however uneven the profiles are.  Rounds keep the working set under a
// preset sample count (the out-of-core rounds of Section 6.2).
// ============================================================================
namespace hpa {
namespace {

// global context of every record of a round: local ctx + its profile's base
__global__ void __launch_bounds__(256)
k_global_ctx(const uint32_t* __restrict__ ctx, uint64_t n, const uint64_t* __restrict__ soff,
             const uint32_t* __restrict__ cbase, uint32_t P, uint32_t* __restrict__ g, PlanInfo* __restrict__ info) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    uint32_t lo = 0, hi = P;  // last profile with soff <= i
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (soff[mid] <= i) lo = mid;
      else hi = mid;
    }
    const uint32_t c = ctx[i];
    if (c >= cbase[lo + 1] - cbase[lo]) {
      atomicOr(&info->err, (uint32_t)ERR_CTX);
      g[i] = 0;
    } else {
      g[i] = cbase[lo] + c;
    }
  }
}

__global__ void __launch_bounds__(256)
k_fill_cprof(const uint32_t* __restrict__ cbase, uint32_t P, uint32_t G, uint32_t* __restrict__ cprof) {
  for (uint32_t c = blockIdx.x * 256 + threadIdx.x; c < G; c += gridDim.x * 256) {
    uint32_t lo = 0, hi = P;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (cbase[mid] <= c) lo = mid;
      else hi = mid;
    }
    cprof[c] = lo;
  }
}

// Per profile of a round: first key, and its context offsets rebased to it.
__global__ void __launch_bounds__(256)
k_rebase(const uint64_t* __restrict__ ctx_off, const uint32_t* __restrict__ cbase, uint32_t P,
         uint64_t* __restrict__ first_key, uint64_t* __restrict__ rebased) {
  const uint32_t total = cbase[P] + P;  // C_p + 1 entries per profile
  for (uint32_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
    uint32_t lo = 0, hi = P;  // last profile whose entries start at or before e
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (cbase[mid] + mid <= e) lo = mid;
      else hi = mid;
    }
    const uint32_t j = e - (cbase[lo] + lo);
    const uint64_t k0 = ctx_off[cbase[lo]];
    rebased[e] = ctx_off[cbase[lo] + j] - k0;
    if (j == 0) first_key[lo] = k0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) first_key[P] = ctx_off[cbase[P]];
}

// A round of profiles that share one map, gathered: the round's records are
// cut into chunks of at most GATHER_CHUNK records of one profile each (chunk
// k: profile chunk_prof[k], round records [chunk_start[k], chunk_start[k+1])),
// and record i of profile p is record src[p] + (i - doff[p]) of the batch
// arrays.  Its global context, and (when the profiles are not adjacent in the
// batch arrays, pc_out set) its pc, stall and weight, go to contiguous round
// arrays.  One workgroup per chunk at a time, so no record searches for its
// profile.
constexpr uint32_t GATHER_CHUNK = 1u << 16;

__global__ void __launch_bounds__(256)
k_gather_round(const uint64_t* __restrict__ pc, const uint32_t* __restrict__ ctx, const uint8_t* __restrict__ stall,
               const uint32_t* __restrict__ weight, const uint64_t* __restrict__ chunk_start,
               const uint32_t* __restrict__ chunk_prof, uint32_t n_chunks, const uint64_t* __restrict__ doff,
               const uint64_t* __restrict__ src, const uint32_t* __restrict__ cbase, uint32_t* __restrict__ g,
               uint64_t* __restrict__ pc_out, uint8_t* __restrict__ st_out, uint32_t* __restrict__ wt_out,
               PlanInfo* __restrict__ info) {
  bool bad = false;
  for (uint32_t k = blockIdx.x; k < n_chunks; k += gridDim.x) {
    const uint32_t p = chunk_prof[k];
    const uint64_t i0 = chunk_start[k], i1 = chunk_start[k + 1];
    const uint64_t shift = src[p] - doff[p];  // batch index = round index + shift
    const uint32_t base = cbase[p], nc = cbase[p + 1] - base;
    for (uint64_t i = i0 + threadIdx.x; i < i1; i += 256) {
      const uint64_t j = i + shift;
      const uint32_t c = ctx[j];
      bad |= c >= nc;
      g[i] = c < nc ? base + c : 0u;
      if (pc_out) {
        pc_out[i] = pc[j];
        st_out[i] = stall[j];
        if (wt_out) wt_out[i] = weight[j];
      }
    }
  }
  if (__any(bad) && (threadIdx.x & (WAVE - 1)) == 0) atomicOr(&info->err, (uint32_t)ERR_CTX);
}

// Keys of the dense pipeline name global contexts: make them local to their
// profile (the general pipeline writes them local already).
__global__ void __launch_bounds__(256)
k_localize_ctx(uint32_t* __restrict__ key_ctx, uint64_t n_keys, const uint32_t* __restrict__ cprof,
               const uint32_t* __restrict__ cbase) {
  for (uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x; k < n_keys; k += (uint64_t)gridDim.x * 256) {
    const uint32_t c = key_ctx[k];
    key_ctx[k] = c - cbase[cprof[c]];
  }
}

}  // namespace
}  // namespace hpa

struct hpa_batch {
  hpa_ctx* ctx = nullptr;
  struct Round {
    hpa_attribution* a = nullptr;
    DBuf rebased;
  };
  std::vector<Round> rounds;
  struct Prof {
    uint32_t round, n_ctx;
    uint64_t key0, n_keys, reb0;  // first key in the round, keys, first rebased entry
  };
  std::vector<Prof> prof;
  hpa_batch_info info{};
  ~hpa_batch() {
    for (auto& r : rounds)
      if (r.a) hpa_attribution_free(r.a);
  }
};

namespace {

struct RoundPlan {
  uint32_t p0, p1;  // profiles [p0, p1)
  uint64_t s0, s1;  // samples
};

// One round: device tables, global contexts, the pipeline, per-profile offsets.
void run_round(hpa_ctx* ctx, const hpa_profile_desc* pd, const hpa_samples* smp, const RoundPlan& r,
               const std::vector<uint64_t>& soff_all, hipStream_t s, const Knobs& kn, hpa_batch* B, bool keep) {
  const uint32_t P = r.p1 - r.p0;
  std::vector<ProfMap> pm(P);
  std::vector<uint32_t> cbase(P + 1);
  std::vector<uint64_t> soff(P + 1);
  uint64_t G = 0;
  for (uint32_t i = 0; i < P; ++i) {
    const hpa_structure_map* m = pd[r.p0 + i].map;
    cbase[i] = (uint32_t)G;
    soff[i] = soff_all[r.p0 + i] - r.s0;
    pm[i].dd = DenseDev{m->win_lo.as<uint64_t>(), m->win_hi.as<uint64_t>(), m->win_d.as<uint64_t>(),
                        m->scope_of.as<uint32_t>(), m->n_win, m->dense_tz};
    pm[i].md = MapDev{m->start.as<uint64_t>(), m->end.as<uint64_t>(), m->scope.as<uint32_t>(), m->n_iv};
    pm[i].ctx_base = (uint32_t)G;
    pm[i].dense = m->dense ? 1 : 0;
    G += pd[r.p0 + i].n_ctx;
  }
  cbase[P] = (uint32_t)G;
  soff[P] = r.s1 - r.s0;
  DBuf d_pm = upload(ctx, pm, s), d_cbase = upload(ctx, cbase, s), d_soff = upload(ctx, soff, s);
  DBuf d_cprof(ctx, std::max<uint64_t>(G, 1) * 4, s);
  k_fill_cprof<<<grid_for(G, 256, ctx->n_cu * 8), 256, 0, s>>>(d_cbase.as<uint32_t>(), P, (uint32_t)G,
                                                               d_cprof.as<uint32_t>());
  const uint64_t n = r.s1 - r.s0;
  DBuf d_g(ctx, std::max<uint64_t>(n, 1) * 4, s), d_info(ctx, sizeof(PlanInfo), s);
  HPA_HIP(hipMemsetAsync(d_info.p, 0, sizeof(PlanInfo), s));
  if (n)
    k_global_ctx<<<grid_for(n, 256, ctx->n_cu * 16), 256, 0, s>>>(smp->ctx + r.s0, n, d_soff.as<uint64_t>(),
                                                                  d_cbase.as<uint32_t>(), P, d_g.as<uint32_t>(),
                                                                  d_info.as<PlanInfo>());
  HPA_HIP(hipGetLastError());
  PlanInfo info{};
  HPA_HIP(hipMemcpyAsync(&info, d_info.p, sizeof(info), hipMemcpyDeviceToHost, s));
  sync_stream(ctx, s);
  if (info.err & ERR_CTX) fail(HPA_E_INVAL, "a sample's ctx is not below its profile's n_ctx");
  hpa_samples rs{smp->pc + r.s0, d_g.as<uint32_t>(), smp->stall + r.s0, smp->weight ? smp->weight + r.s0 : nullptr,
                 n, (uint32_t)G};
  BatchRun br{d_pm.as<ProfMap>(), d_cprof.as<uint32_t>()};
  hpa_attribution* a = attribute_impl(ctx, pd[r.p0].map, &br, &rs, s, kn, nullptr);
  if (!keep) {
    hpa_attribution_free(a);
    return;
  }
  hpa_batch::Round R;
  R.a = a;
  R.rebased = DBuf(ctx, ((uint64_t)G + P) * 8, s);
  DBuf d_k0(ctx, ((uint64_t)P + 1) * 8, s);
  k_rebase<<<grid_for(G + P, 256, ctx->n_cu * 8), 256, 0, s>>>(a->ctx_offsets.as<uint64_t>(), d_cbase.as<uint32_t>(),
                                                               P, d_k0.as<uint64_t>(), R.rebased.as<uint64_t>());
  HPA_HIP(hipGetLastError());
  std::vector<uint64_t> k0(P + 1);
  HPA_HIP(hipMemcpyAsync(k0.data(), d_k0.p, (P + 1) * 8, hipMemcpyDeviceToHost, s));
  sync_stream(ctx, s);
  const uint32_t ri = (uint32_t)B->rounds.size();
  for (uint32_t i = 0; i < P; ++i)
    B->prof[r.p0 + i] = hpa_batch::Prof{ri, pd[r.p0 + i].n_ctx, k0[i], k0[i + 1] - k0[i], (uint64_t)cbase[i] + i};
  B->rounds.push_back(std::move(R));
  B->info.total_keys += k0[P];
}

// Batches whose profiles share a few maps are taken map by map: the profiles
// of one map (in batch order) form rounds of their own, and a round whose map
// has dense coordinates runs the dense pipeline over the profiles' global
// contexts (falling back to the general pipeline, as a single call does, when
// a pc has no dense coordinate); other rounds run the general pipeline.
// Returns false, and leaves the batch to rounds of consecutive profiles, when
// the maps are too many for grouping to pay (more than 64, or fewer than two
// profiles per map).
bool group_by_map(const hpa_profile_desc* pd, uint32_t n_profiles, std::vector<uint32_t>& order) {
  std::vector<const hpa_structure_map*> maps;
  for (uint32_t p = 0; p < n_profiles; ++p) {
    const hpa_structure_map* m = pd[p].map;
    if (std::find(maps.begin(), maps.end(), m) == maps.end()) {
      if (maps.size() == 64) return false;
      maps.push_back(m);
    }
  }
  if (2 * maps.size() > n_profiles) return false;
  order.clear();
  for (const hpa_structure_map* m : maps)
    for (uint32_t p = 0; p < n_profiles; ++p)
      if (pd[p].map == m) order.push_back(p);
  return true;
}

// A table inside a shared device buffer.
struct TabView {
  const DBuf* b;
  size_t off;
  template <class T>
  T* as() const { return reinterpret_cast<T*>(static_cast<unsigned char*>(b->p) + off); }
};

// One round of profiles `ids` (one map, batch order within it).
void run_round_grouped(hpa_ctx* ctx, const hpa_profile_desc* pd, const hpa_samples* smp,
                       const std::vector<uint32_t>& ids, const std::vector<uint64_t>& soff_all, hipStream_t s,
                       const Knobs& kn, hpa_batch* B) {
  const uint32_t P = (uint32_t)ids.size();
  const hpa_structure_map* map = pd[ids[0]].map;
  std::vector<ProfMap> pm(P);
  std::vector<uint32_t> cbase(P + 1);
  std::vector<uint64_t> doff(P + 1), src(P);
  uint64_t G = 0, n = 0;
  bool adjacent = true;
  for (uint32_t i = 0; i < P; ++i) {
    const uint32_t p = ids[i];
    cbase[i] = (uint32_t)G;
    doff[i] = n;
    src[i] = soff_all[p];
    if (i > 0 && soff_all[ids[i - 1] + 1] != soff_all[p]) adjacent = false;
    pm[i].dd = DenseDev{map->win_lo.as<uint64_t>(), map->win_hi.as<uint64_t>(), map->win_d.as<uint64_t>(),
                        map->scope_of.as<uint32_t>(), map->n_win, map->dense_tz};
    pm[i].md = MapDev{map->start.as<uint64_t>(), map->end.as<uint64_t>(), map->scope.as<uint32_t>(), map->n_iv};
    pm[i].ctx_base = (uint32_t)G;
    pm[i].dense = map->dense ? 1 : 0;
    G += pd[p].n_ctx;
    n += pd[p].n_samples;
  }
  cbase[P] = (uint32_t)G;
  doff[P] = n;
  const uint64_t s0 = soff_all[ids[0]];
  // chunks of one profile each for the gather
  std::vector<uint64_t> chunk_start;
  std::vector<uint32_t> chunk_prof;
  for (uint32_t i = 0; i < P; ++i)
    for (uint64_t a = doff[i]; a < doff[i + 1]; a += GATHER_CHUNK) {
      chunk_start.push_back(a);
      chunk_prof.push_back(i);
    }
  const uint32_t n_chunks = (uint32_t)chunk_prof.size();
  chunk_start.push_back(n);
  if (chunk_prof.empty()) chunk_prof.push_back(0);
  // the round's tables in one upload (one synchronisation), each at a
  // 256-byte aligned offset
  std::vector<unsigned char> tab;
  auto place = [&](const void* p, size_t bytes) {
    const size_t off = (tab.size() + 255) & ~(size_t)255;
    tab.resize(off + bytes);
    if (bytes) std::memcpy(tab.data() + off, p, bytes);
    return off;
  };
  const size_t o_pm = place(pm.data(), pm.size() * sizeof(ProfMap));
  const size_t o_cbase = place(cbase.data(), cbase.size() * 4);
  const size_t o_doff = place(doff.data(), doff.size() * 8);
  const size_t o_src = place(src.data(), src.size() * 8);
  const size_t o_cstart = place(chunk_start.data(), chunk_start.size() * 8);
  const size_t o_cprof = place(chunk_prof.data(), chunk_prof.size() * 4);
  DBuf d_tab = upload(ctx, tab, s);
  const TabView d_pm{&d_tab, o_pm}, d_cbase{&d_tab, o_cbase}, d_doff{&d_tab, o_doff}, d_src{&d_tab, o_src},
      d_cstart{&d_tab, o_cstart}, d_cprof_of{&d_tab, o_cprof};
  DBuf d_cprof(ctx, std::max<uint64_t>(G, 1) * 4, s);
  k_fill_cprof<<<grid_for(G, 256, ctx->n_cu * 8), 256, 0, s>>>(d_cbase.as<uint32_t>(), P, (uint32_t)G,
                                                               d_cprof.as<uint32_t>());
  const bool weighted = smp->weight != nullptr;
  DBuf d_g(ctx, std::max<uint64_t>(n, 1) * 4, s), d_info(ctx, sizeof(PlanInfo), s);
  DBuf d_pc, d_st, d_wt;
  if (!adjacent) {
    d_pc = DBuf(ctx, std::max<uint64_t>(n, 1) * 8, s);
    d_st = DBuf(ctx, std::max<uint64_t>(n, 1), s);
    if (weighted) d_wt = DBuf(ctx, std::max<uint64_t>(n, 1) * 4, s);
  }
  HPA_HIP(hipMemsetAsync(d_info.p, 0, sizeof(PlanInfo), s));
  if (n_chunks)
    k_gather_round<<<std::min<uint32_t>(n_chunks, ctx->n_cu * 8), 256, 0, s>>>(
        smp->pc, smp->ctx, smp->stall, smp->weight, d_cstart.as<uint64_t>(), d_cprof_of.as<uint32_t>(), n_chunks,
        d_doff.as<uint64_t>(), d_src.as<uint64_t>(), d_cbase.as<uint32_t>(), d_g.as<uint32_t>(),
        adjacent ? nullptr : d_pc.as<uint64_t>(), adjacent ? nullptr : d_st.as<uint8_t>(),
        adjacent || !weighted ? nullptr : d_wt.as<uint32_t>(), d_info.as<PlanInfo>());
  HPA_HIP(hipGetLastError());
  PlanInfo info{};
  HPA_HIP(hipMemcpyAsync(&info, d_info.p, sizeof(info), hipMemcpyDeviceToHost, s));
  sync_stream(ctx, s);
  if (info.err & ERR_CTX) fail(HPA_E_INVAL, "a sample's ctx is not below its profile's n_ctx");
  hpa_samples rs{adjacent ? smp->pc + s0 : d_pc.as<uint64_t>(), d_g.as<uint32_t>(),
                 adjacent ? smp->stall + s0 : d_st.as<uint8_t>(),
                 !weighted ? nullptr : (adjacent ? smp->weight + s0 : d_wt.as<uint32_t>()), n, (uint32_t)G};
  auto* A = new hpa_attribution();
  std::unique_ptr<hpa_attribution> hold(A);
  A->ctx = ctx;
  A->stream = s;
  A->map = map;
  A->n_ctx = (uint32_t)G;
  if (n > 0 && dense_path_fits(map, &rs) && attribute_dense(ctx, map, &rs, s, A)) {
    if (A->n_keys)
      k_localize_ctx<<<grid_for(A->n_keys, 256, ctx->n_cu * 16), 256, 0, s>>>(
          A->ctx_id.as<uint32_t>(), A->n_keys, d_cprof.as<uint32_t>(), d_cbase.as<uint32_t>());
    HPA_HIP(hipGetLastError());
  } else {
    BatchRun br{d_pm.as<ProfMap>(), d_cprof.as<uint32_t>()};
    attribute_impl(ctx, map, &br, &rs, s, kn, A);
  }
  hpa_batch::Round R;
  R.a = hold.release();
  R.rebased = DBuf(ctx, ((uint64_t)G + P) * 8, s);
  DBuf d_k0(ctx, ((uint64_t)P + 1) * 8, s);
  k_rebase<<<grid_for(G + P, 256, ctx->n_cu * 8), 256, 0, s>>>(R.a->ctx_offsets.as<uint64_t>(),
                                                               d_cbase.as<uint32_t>(), P, d_k0.as<uint64_t>(),
                                                               R.rebased.as<uint64_t>());
  HPA_HIP(hipGetLastError());
  std::vector<uint64_t> k0(P + 1);
  HPA_HIP(hipMemcpyAsync(k0.data(), d_k0.p, (P + 1) * 8, hipMemcpyDeviceToHost, s));
  sync_stream(ctx, s);
  const uint32_t ri = (uint32_t)B->rounds.size();
  for (uint32_t i = 0; i < P; ++i)
    B->prof[ids[i]] = hpa_batch::Prof{ri, pd[ids[i]].n_ctx, k0[i], k0[i + 1] - k0[i], (uint64_t)cbase[i] + i};
  B->rounds.push_back(std::move(R));
  B->info.total_keys += k0[P];
}

}  // namespace

extern "C" hpa_status hpa_attribute_batched(hpa_ctx* ctx, uint32_t n_profiles, const hpa_profile_desc* pd,
                                            const hpa_samples* smp, const hpa_batch_opts* opts, hipStream_t stream,
                                            hpa_batch** out) {
  return guard([&] {
    if (!ctx || !pd || !smp || !out || n_profiles == 0) fail(HPA_E_INVAL, "NULL argument or no profiles");
    if (smp->n && (!smp->pc || !smp->ctx || !smp->stall)) fail(HPA_E_INVAL, "NULL sample array");
    std::vector<uint64_t> soff(n_profiles + 1, 0);
    for (uint32_t p = 0; p < n_profiles; ++p) {
      if (!pd[p].map || pd[p].map->ctx != ctx) fail(HPA_E_INVAL, "profile map missing or of another context");
      if (pd[p].n_ctx == 0 || pd[p].n_ctx >= 0x7FFFFFFFu) fail(HPA_E_INVAL, "profile n_ctx out of range");
      soff[p + 1] = soff[p] + pd[p].n_samples;
    }
    if (soff[n_profiles] != smp->n) fail(HPA_E_INVAL, "samples->n differs from the profiles' total");
    hpa_batch_opts o{};
    if (opts) o = *opts;
    const uint64_t cap = o.max_round_samples ? o.max_round_samples : (1ull << 31);
    // rounds: consecutive profiles up to `cap` samples and 2^31 contexts
    std::vector<RoundPlan> plan;
    {
      uint32_t p0 = 0;
      while (p0 < n_profiles) {
        uint32_t p1 = p0 + 1;
        uint64_t ns = pd[p0].n_samples, nc = pd[p0].n_ctx;
        while (p1 < n_profiles && ns + pd[p1].n_samples <= cap && nc + pd[p1].n_ctx < 0x7FFFFFFFull) {
          ns += pd[p1].n_samples;
          nc += pd[p1].n_ctx;
          ++p1;
        }
        if (ns >= (1ull << 40)) fail(HPA_E_INVAL, "a profile has too many samples");
        plan.push_back(RoundPlan{p0, p1, soff[p0], soff[p1]});
        p0 = p1;
      }
    }
    DeviceGuard dg(ctx->device);
    hipStream_t s = stream;
    auto* B = new hpa_batch();
    std::unique_ptr<hpa_batch> hold(B);
    B->ctx = ctx;
    B->prof.resize(n_profiles);
    Knobs kn;
    if (o.merge_rounds <= 3 && opts) kn.merge_rounds = o.merge_rounds;
    if (o.scan_wg_per_cu) kn.scan_wg_per_cu = o.scan_wg_per_cu;
    if (o.autotune) {
      if (ctx->tuned) {
        kn.merge_rounds = ctx->tuned_merge_rounds;
        kn.scan_wg_per_cu = ctx->tuned_scan_wg;
      } else {
        // pilot: the first round's leading profiles, up to 2^26 samples
        RoundPlan pilot = plan[0];
        while (pilot.p1 > pilot.p0 + 1 && soff[pilot.p1] - soff[pilot.p0] > (1ull << 26)) --pilot.p1;
        pilot.s1 = soff[pilot.p1];
        hipEvent_t e0, e1;
        HPA_HIP(hipEventCreate(&e0));
        HPA_HIP(hipEventCreate(&e1));
        float best = 3.4e38f;
        Knobs bk = kn;
        const auto t0 = std::chrono::steady_clock::now();
        run_round(ctx, pd, smp, pilot, soff, s, kn, B, false);  // warm-up
        for (uint32_t mr = 0; mr <= 3; ++mr)
          for (uint32_t wg : {2u, 4u, 8u}) {
            Knobs k{mr, wg};
            HPA_HIP(hipEventRecord(e0, s));
            run_round(ctx, pd, smp, pilot, soff, s, k, B, false);
            HPA_HIP(hipEventRecord(e1, s));
            HPA_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            HPA_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) { best = ms; bk = k; }
          }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        B->info.tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        kn = bk;
        ctx->tuned = true;
        ctx->tuned_merge_rounds = kn.merge_rounds;
        ctx->tuned_scan_wg = kn.scan_wg_per_cu;
      }
    }
    std::vector<uint32_t> order;
    if (group_by_map(pd, n_profiles, order)) {
      // rounds of one map each, up to `cap` samples and 2^31 contexts
      std::vector<uint32_t> ids;
      uint64_t ns = 0, nc = 0;
      for (uint32_t k = 0; k <= n_profiles; ++k) {
        const uint32_t p = k < n_profiles ? order[k] : 0u;
        if (!ids.empty() && (k == n_profiles || pd[p].map != pd[ids[0]].map || ns + pd[p].n_samples > cap ||
                             nc + pd[p].n_ctx >= 0x7FFFFFFFull)) {
          run_round_grouped(ctx, pd, smp, ids, soff, s, kn, B);
          ids.clear();
          ns = nc = 0;
        }
        if (k == n_profiles) break;
        ids.push_back(p);
        ns += pd[p].n_samples;
        nc += pd[p].n_ctx;
      }
    } else {
      for (const RoundPlan& r : plan) run_round(ctx, pd, smp, r, soff, s, kn, B, true);
    }
    B->info.n_rounds = (uint32_t)B->rounds.size();
    B->info.merge_rounds = kn.merge_rounds;
    B->info.scan_wg_per_cu = kn.scan_wg_per_cu;
    B->info.autotuned = o.autotune ? 1 : 0;
    *out = hold.release();
  });
}

extern "C" hpa_status hpa_batch_profile_view(const hpa_batch* b, uint32_t profile, hpa_attribution_view* v) {
  return guard([&] {
    if (!b || !v) fail(HPA_E_INVAL, "NULL argument");
    if (profile >= b->prof.size()) fail(HPA_E_INVAL, "profile out of range");
    const hpa_batch::Prof& p = b->prof[profile];
    const hpa_attribution* a = b->rounds[p.round].a;
    v->n_keys = p.n_keys;
    v->n_ctx = p.n_ctx;
    v->ctx = a->ctx_id.as<uint32_t>() + p.key0;
    v->pc = a->pc.as<uint64_t>() + p.key0;
    v->stall = a->stall.as<uint8_t>() + p.key0;
    v->count = a->count.as<uint64_t>() + p.key0;
    v->scope = a->scope.as<uint32_t>() + p.key0;
    v->ctx_offsets = b->rounds[p.round].rebased.as<uint64_t>() + p.reb0;
  });
}

extern "C" hpa_status hpa_batch_info_get(const hpa_batch* b, hpa_batch_info* out) {
  return guard([&] {
    if (!b || !out) fail(HPA_E_INVAL, "NULL argument");
    *out = b->info;
  });
}

extern "C" void hpa_batch_free(hpa_batch* b) { delete b; }

// ============================================================================
// Attribution without allocation, for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// it).  Every working buffer of the pipeline comes from one file-scope device
// array, `scratch`, through a bump arena (this thread's allocations only); the outputs are the
// caller's arrays.  The array's device address is looked up once per device
// (its host-side name is not a device address).  Calls that overlap on one
// GPU share the array and race.
// ============================================================================
namespace {

constexpr size_t SCRATCH_BYTES = (size_t)HPA_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// Device address of this device's copy of `scratch` (the device is current).
void* scratch_ptr(int device) {
  if (device < 0 || device >= 64) fail(HPA_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      fail(HPA_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

// Routes this thread's library allocations to the arena for the guard's
// lifetime.
struct ArenaGuard {
  ArenaGuard(void* base, size_t size) {
    t_arena.base = static_cast<uint8_t*>(base);
    t_arena.size = size;
    t_arena.off = 0;
    t_arena.peak = 0;
  }
  ~ArenaGuard() { t_arena.base = nullptr; }
};

}  // namespace

extern "C" hpa_status hpa_attribute_noalloc(hpa_ctx* ctx, const hpa_structure_map* map, const hpa_samples* smp,
                                            uint32_t* out_ctx, uint64_t* out_pc, uint8_t* out_stall,
                                            uint64_t* out_count, uint32_t* out_scope, uint64_t* out_ctx_offsets,
                                            uint64_t* n_keys, uint64_t* scratch_used, hipStream_t stream) {
  return guard([&] {
    if (!ctx || !map || !smp || !n_keys) fail(HPA_E_INVAL, "NULL argument");
    if (map->ctx != ctx) fail(HPA_E_INVAL, "map belongs to another context");
    if (smp->n && (!smp->pc || !smp->ctx || !smp->stall)) fail(HPA_E_INVAL, "NULL sample array");
    if (!out_ctx || !out_pc || !out_stall || !out_count || !out_scope || !out_ctx_offsets)
      fail(HPA_E_INVAL, "NULL output array");
    if (smp->n_ctx == 0 || smp->n_ctx > HPA_NOALLOC_MAX_CTX)
      fail(HPA_E_INVAL, "n_ctx must be in [1, " + std::to_string(HPA_NOALLOC_MAX_CTX) + "] without allocation");
    if (smp->n > HPA_NOALLOC_MAX_SAMPLES)
      fail(HPA_E_INVAL, "at most " + std::to_string(HPA_NOALLOC_MAX_SAMPLES) + " samples without allocation");
    if (ctx->custom) fail(HPA_E_UNSUPPORTED, "a context with a caller allocator: use hpa_attribute");
    if (ctx->timing) fail(HPA_E_UNSUPPORTED, "stage timing creates events: turn it off for this call");
    DeviceGuard dg(ctx->device);
    void* base = scratch_ptr(ctx->device);
    ArenaGuard ag(base, SCRATCH_BYTES);
    hpa_attribution A;
    // the outputs are the caller's (non-owning views)
    A.ctx_id.p = out_ctx;
    A.pc.p = out_pc;
    A.stall.p = out_stall;
    A.count.p = out_count;
    A.scope.p = out_scope;
    A.ctx_offsets.p = out_ctx_offsets;
    attribute_any(ctx, map, smp, stream, &A);
    *n_keys = A.n_keys;
    if (scratch_used) *scratch_used = t_arena.peak;
    for (DBuf* b : {&A.ctx_id, &A.pc, &A.stall, &A.count, &A.scope, &A.ctx_offsets}) b->p = nullptr;
  });
}
