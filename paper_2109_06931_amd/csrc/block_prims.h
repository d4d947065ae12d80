// Wavefront and workgroup primitives for gfx950 (wave64): scans, reductions,
// and an LDS-staged LSD radix sort over keys held in registers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hpa {

constexpr int WAVE = 64;

__device__ inline int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }
__device__ inline int wave_id() { return (int)(threadIdx.x / WAVE); }

// Inclusive scan over the 64 lanes of a wave for 32-bit values with DPP moves
// (no LDS traffic): row shifts by 1, 2, 4 and 8 scan each row of 16 lanes, then
// row broadcasts of lane 15 (into rows 1 and 3) and lane 31 (into rows 2 and 3)
// carry the row totals.  Every lane must be active.
__device__ inline uint32_t wave_incl_scan_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false); // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false); // row_bcast:31
  return v;
}

// The same scan over N independent values, one DPP step for all of them
// before the next, so that no step waits on the one just before it.
template <int N>
__device__ inline void wave_incl_scan_u32_n(uint32_t (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[k], 0x111, 0xF, 0xF, true);
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[k], 0x112, 0xF, 0xF, true);
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[k], 0x114, 0xF, 0xF, true);
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[k], 0x118, 0xF, 0xF, true);
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[k], 0x142, 0xA, 0xF, false);
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[k], 0x143, 0xC, 0xF, false);
}

// Minimum and maximum over the 64 lanes of a wave for 32-bit values, with the
// DPP steps of wave_incl_scan_u32: a lane whose source is out of its row, and a
// row the mask leaves out, keep their own value, which leaves a minimum or
// maximum unchanged.  Lane 63 ends with the wave's result; every lane gets it.
// Every lane must be active.
__device__ inline uint32_t wave_min_u32(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x111, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x112, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x114, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x118, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, WAVE - 1);
}

__device__ inline uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x111, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x112, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x114, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x118, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, WAVE - 1);
}

__device__ inline uint32_t wave_last_u32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, WAVE - 1); }

template <class T>
__device__ inline T wave_incl_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    T t = __shfl_up(v, d, WAVE);
    if (lane >= d) v += t;
  }
  return v;
}

template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
  return v;
}

template <class T>
__device__ inline T wave_max(T v) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) {
    T o = __shfl_xor(v, d, WAVE);
    v = o > v ? o : v;
  }
  return v;
}

template <class T>
__device__ inline T wave_min(T v) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) {
    T o = __shfl_xor(v, d, WAVE);
    v = o < v ? o : v;
  }
  return v;
}

template <class T>
__device__ inline T wave_or(T v) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) v |= __shfl_xor(v, d, WAVE);
  return v;
}

// Exclusive scan over the workgroup; returns the thread's exclusive prefix and
// writes the total to *total.  Each wave scans its lanes and publishes its
// total in s_tmp (BLOCK / WAVE entries); after one barrier every thread adds
// the totals of the waves before its own (no serial pass by one thread); a
// second barrier lets the next call reuse s_tmp.  Contains barriers: every
// thread of the block must call it.
template <int BLOCK, class T>
__device__ inline T block_excl_scan(T v, T* s_tmp, T* total) {
  constexpr int NW = BLOCK / WAVE;
  T inc;
  if constexpr (sizeof(T) == 4) inc = (T)wave_incl_scan_u32((uint32_t)v);
  else inc = wave_incl_scan(v);
  if (lane_id() == WAVE - 1) s_tmp[wave_id()] = inc;
  __syncthreads();
  const int w = wave_id();
  T before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const T t = s_tmp[i];
    all += t;
    before += i < w ? t : (T)0;
  }
  *total = all;
  __syncthreads();
  return before + inc - v;
}

// LSD radix sort of up to BLOCK * ITEMS keys held in registers, 4-bit digits.
//
// Order: item i of thread t stands at position t * ITEMS + i ("blocked"), and
// every pass is stable in that order.  The starting order is whatever the
// caller gathered (for an aggregation the order of equal keys is irrelevant);
// only the validity test differs: in the starting arrangement item i of
// thread t is valid when i * BLOCK + t < n ("striped"), afterwards when
// t * ITEMS + i < n.
//
// A pass: each thread counts its digits in registers (16 four-bit counters in
// one 64-bit register; the thread's last item is kept aside, so a counter
// never exceeds ITEMS - 1 <= 15); the 16 counts, widened to 16-bit pairs in 8
// columns, are scanned over each wave's lanes in registers; the wave
// totals, scanned over the waves and offset by the scanned digit totals, give
// each thread its own table in LDS of where its keys of each digit start (one
// word per digit, at digit * BLOCK + thread, so a wave's accesses fall in
// distinct banks); each item takes its new position from its digit's word
// with an LDS fetch-and-add, in item order, so equal digits keep their order
// without any count in registers, and the key is written there in the
// exchange plane and read back blocked.
template <int BLOCK, int ITEMS>
struct BlockRadix {
  static constexpr int T = BLOCK * ITEMS;
  static constexpr int NW = BLOCK / WAVE;
  static constexpr int BUF_WORDS = T + T / 32;  // exchange plane, padded every 32 words
  static constexpr int CNT_WORDS = 16 * BLOCK;  // per digit, one position word per thread
  static constexpr int DOFF_WORDS = 8 * NW;     // per wave: the 8 column totals
  static_assert(T < 65536, "16-bit counters");
  static_assert(ITEMS >= 2 && ITEMS <= 16, "4-bit per-thread counters hold ITEMS - 1");

  __device__ static inline int pad(int i) { return i + (i >> 5); }
  // pad(t * ITEMS + i) for the ITEMS slots of thread t: one base plus i, since
  // a thread's slots never straddle a multiple of 32 (ITEMS divides 32)
  static_assert(32 % ITEMS == 0, "a thread's slots must not straddle a padding boundary");
  __device__ static inline int row_base(int t) { return t * ITEMS + ((t * ITEMS) >> 5); }

  // Sort the first n 32-bit keys on bits [0, bits); the NV payload arrays
  // (v0, then v1) move with their keys.  Afterwards position p is item
  // p % ITEMS of thread p / ITEMS; positions >= n hold no key.  `striped`
  // gives the validity test of the starting arrangement.  s_buf: BUF_WORDS,
  // s_cnt: CNT_WORDS, s_doff: DOFF_WORDS (separate regions).
  //
  // FULL: every item of every thread holds a key (the caller pads empty slots
  // with keys that sort last), so no slot needs a validity test.
  template <int NV, bool FULL = false>
  __device__ static __forceinline__ void sort(uint32_t (&key)[ITEMS], uint32_t (&v0)[ITEMS], uint32_t (&v1)[ITEMS],
                                              int bits, int n, bool striped, uint32_t* s_buf, uint32_t* s_cnt,
                                              uint32_t* s_doff) {
    const int tid = (int)threadIdx.x;
    if (FULL) n = T;
#define HPA_VALID(i) (FULL || (striped ? (i) * BLOCK + tid : tid * ITEMS + (i)) < n)
    for (int shift = 0; shift < bits; shift += 4) {
      // 1. per-thread digit counts of items 0 .. ITEMS - 2; the last item's
      //    digit (16: none) is added when the columns are formed
      uint64_t h = 0;
#pragma unroll
      for (int i = 0; i < ITEMS - 1; ++i)
        if (HPA_VALID(i)) h += 1ull << (__builtin_amdgcn_ubfe(key[i], (uint32_t)shift, 4u) * 4);
      const uint32_t dl = HPA_VALID(ITEMS - 1) ? __builtin_amdgcn_ubfe(key[ITEMS - 1], (uint32_t)shift, 4u) : 16u;
      // 2. widen to 16-bit pairs (column k holds digits 2k low and 2k+1
      //    high) and scan every column over the wave's lanes in registers;
      //    the wave totals go to LDS
      uint32_t ex[8], inc[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t w = (uint32_t)(h >> (8 * k));
        ex[k] = (w & 0xFu) | ((w & 0xF0u) << 12);
        if ((dl >> 1) == (uint32_t)k) ex[k] += 1u << ((dl & 1u) * 16);
        inc[k] = ex[k];
      }
      wave_incl_scan_u32_n(inc);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        ex[k] = inc[k] - ex[k];
        if (lane_id() == WAVE - 1) s_doff[wave_id() * 8 + k] = inc[k];
      }
      __syncthreads();
      // 3. every wave derives its own column offsets from all the wave
      //    totals (no second barrier): lane k < 8 sums column k over all
      //    waves and over the waves before its own; the exclusive scan of
      //    the 16 digit totals, as pairs over lanes 0..7, gives the digit
      //    offsets; lane k's packed offsets reach every lane by readlane.
      //    Halves never carry: every count is below T < 65536.
      uint32_t dof[8];
      {
        const int k = lane_id();
        uint32_t tot = 0, below = 0;
        if (k < 8) {
#pragma unroll
          for (int w = 0; w < NW; ++w) {
            const uint32_t t = s_doff[w * 8 + k];
            tot += t;
            below += w < wave_id() ? t : 0u;
          }
        }
        const uint32_t pair = k < 8 ? (tot & 0xFFFFu) + (tot >> 16) : 0u;
        const uint32_t lo = wave_incl_scan_u32(pair) - pair;
        const uint32_t mine = (lo | ((lo + (tot & 0xFFFFu)) << 16)) + below;
#pragma unroll
        for (int j = 0; j < 8; ++j) dof[j] = (uint32_t)__builtin_amdgcn_readlane((int)mine, j);
      }
      // every thread's own table: digit offset + wave prefix + lane prefix,
      // one word per digit (used only by the same thread)
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t v = dof[k] + ex[k];
        s_cnt[(2 * k) * BLOCK + tid] = v & 0xFFFFu;
        s_cnt[(2 * k + 1) * BLOCK + tid] = v >> 16;
      }
      // 4. positions: each item fetches its digit's word and advances it.
      // The digits are extracted again rather than kept from step 1: holding
      // 2 x ITEMS values across the scans costs more registers than the
      // shifts.
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) asm volatile("" : "+v"(key[i]));
      auto position = [&](int i) -> uint32_t {
        const uint32_t d = __builtin_amdgcn_ubfe(key[i], (uint32_t)shift, 4u);
        return atomicAdd(&s_cnt[d * BLOCK + tid], 1u);
      };
      if constexpr (NV == 0) {
        // one plane: write each key as soon as its position is known
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
          if (HPA_VALID(i)) s_buf[pad((int)position(i))] = key[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) key[i] = (FULL || tid * ITEMS + i < n) ? s_buf[row_base(tid) + i] : 0u;
        __syncthreads();
      } else {
        uint32_t pos[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) pos[i] = HPA_VALID(i) ? position(i) : 0u;
        exchange_u32(v0, pos, s_buf, n, striped);
        if constexpr (NV == 2) exchange_u32(v1, pos, s_buf, n, striped);
        exchange_u32(key, pos, s_buf, n, striped);
      }
      striped = false;
    }
#undef HPA_VALID
  }

  // Move valid v[i] to position pos[i] and read the plane back blocked.
  __device__ static inline void exchange_u32(uint32_t (&v)[ITEMS], const uint32_t (&pos)[ITEMS], uint32_t* s_buf,
                                             int n, bool striped) {
    const int tid = (int)threadIdx.x;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
      if ((striped ? i * BLOCK + tid : tid * ITEMS + i) < n) s_buf[pad((int)pos[i])] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) v[i] = tid * ITEMS + i < n ? s_buf[row_base(tid) + i] : 0u;
    __syncthreads();
  }
};

}  // namespace hpa
