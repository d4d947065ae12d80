// Wavefront and workgroup primitives for gfx950 (wave64): scans, reductions,
// and an LDS-staged LSD radix sort over keys held in registers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hpa {

constexpr int WAVE = 64;

__device__ inline int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }
__device__ inline int wave_id() { return (int)(threadIdx.x / WAVE); }

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
// writes the total to *total.  s_tmp needs BLOCK / WAVE + 1 entries.  Contains
// barriers: every thread of the block must call it.
template <int BLOCK, class T>
__device__ inline T block_excl_scan(T v, T* s_tmp, T* total) {
  constexpr int NW = BLOCK / WAVE;
  T inc = wave_incl_scan(v);
  if (lane_id() == WAVE - 1) s_tmp[wave_id()] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      T t = s_tmp[w];
      s_tmp[w] = run;
      run += t;
    }
    s_tmp[NW] = run;
  }
  __syncthreads();
  T r = s_tmp[wave_id()] + inc - v;
  *total = s_tmp[NW];
  __syncthreads();
  return r;
}

// LSD radix sort of BLOCK * ITEMS keys held in registers (blocked arrangement
// after every pass: thread t holds sequence positions t*ITEMS .. t*ITEMS+ITEMS-1).
// Digit ranks come from per-thread counters in LDS, one column per thread, so
// counting is conflict-free and stable.  Two 16-bit counters share a word
// (digits 2k and 2k+1); a column scan over threads scans both halves at once
// because no half can exceed BLOCK * ITEMS < 65536.  Keys and values travel
// through one padded 32-bit LDS plane at a time.
template <int BLOCK, int ITEMS, int RBITS>
struct BlockRadix {
  static constexpr int T = BLOCK * ITEMS;
  static constexpr int D = 1 << RBITS;
  static constexpr int NW = BLOCK / WAVE;
  static constexpr int BUF_WORDS = T + T / 32;    // exchange plane, padded every 32 words
  static constexpr int CNT_WORDS = (D / 2) * BLOCK;
  static constexpr int DOFF_WORDS = D;
  static_assert(T < 65536, "16-bit counters");
  static_assert(RBITS >= 1, "digit pairs");

  __device__ static inline int pad(int i) { return i + (i >> 5); }

  // `wide` == false: the high words of 64-bit values are all zero and stay so.
  // Move valid values to their ranks and read them back blocked.
  template <class V>
  __device__ static inline void exchange(V (&v)[ITEMS], const uint32_t (&rank)[ITEMS], uint32_t* s_buf, bool wide,
                                         int n, bool striped) {
    const int tid = (int)threadIdx.x;
    const int nplanes = (sizeof(V) == 8 && wide) ? 2 : 1;
    // a wave whose first blocked position is past n holds nothing after the exchange
    const bool wave_has = (int)(threadIdx.x & ~(WAVE - 1)) * ITEMS < n;
    uint32_t lo[ITEMS];
    for (int plane = 0; plane < nplanes; ++plane) {
      if (striped) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          if (i * BLOCK >= n) continue;
          if (i * BLOCK + tid < n) s_buf[pad((int)rank[i])] = (uint32_t)((uint64_t)v[i] >> (32 * plane));
        }
      } else if (wave_has) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
          if (tid * ITEMS + i < n) s_buf[pad((int)rank[i])] = (uint32_t)((uint64_t)v[i] >> (32 * plane));
      }
      __syncthreads();
      if (wave_has) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          uint32_t x = tid * ITEMS + i < n ? s_buf[pad(tid * ITEMS + i)] : 0u;
          if (plane == 0) lo[i] = x;
          else v[i] = (V)(((uint64_t)x << 32) | lo[i]);
        }
      }
      __syncthreads();
    }
    if (nplanes == 1) {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) v[i] = (V)lo[i];
    }
  }

  // Sort the first n keys (in the starting arrangement: item i of thread t is
  // element i * BLOCK + t) on bits [0, bits); `val` moves with its key when
  // HAS_VAL.  Afterwards the sorted keys are blocked: position p is item
  // p % ITEMS of thread p / ITEMS, and positions >= n hold no key.  When
  // bits <= 32 (and bits > 0), s_buf[pad(p)] still holds the key at position p.
  template <class K, bool HAS_VAL>
  __device__ static void sort(K (&key)[ITEMS], uint32_t (&val)[ITEMS], int bits, int n, uint32_t* s_buf,
                              uint32_t* s_cnt, uint32_t* s_doff) {
    const int tid = (int)threadIdx.x;
    bool striped = true;
    for (int shift = 0; shift < bits; shift += RBITS) {
      for (int i = tid; i < CNT_WORDS / 4; i += BLOCK) reinterpret_cast<uint4*>(s_cnt)[i] = make_uint4(0, 0, 0, 0);
      __syncthreads();
      uint32_t rank[ITEMS];
      const bool wave_has = striped || (int)(threadIdx.x & ~(WAVE - 1)) * ITEMS < n;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) rank[i] = 0;
      if (wave_has) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          if (striped && i * BLOCK >= n) continue;
          const bool ok = (striped ? i * BLOCK + tid : tid * ITEMS + i) < n;
          if (ok) {
            uint32_t d = (uint32_t)(key[i] >> shift) & (D - 1);
            uint32_t* c = &s_cnt[(d >> 1) * BLOCK + tid];
            uint32_t sh = (d & 1) * 16;
            uint32_t w = *c;
            rank[i] = (w >> sh) & 0xFFFFu;
            *c = w + (1u << sh);
          }
        }
      }
      __syncthreads();
      // exclusive scan of every counter column over threads; digit totals to s_doff
      for (int k = wave_id(); k < D / 2; k += NW) {
        uint32_t run = 0;
#pragma unroll
        for (int c0 = 0; c0 < BLOCK; c0 += WAVE) {
          uint32_t a = s_cnt[k * BLOCK + c0 + lane_id()];
          uint32_t inc = wave_incl_scan(a);
          s_cnt[k * BLOCK + c0 + lane_id()] = run + inc - a;
          run += __shfl(inc, WAVE - 1, WAVE);
        }
        if (lane_id() == 0) {
          s_doff[2 * k] = run & 0xFFFFu;
          s_doff[2 * k + 1] = run >> 16;
        }
      }
      __syncthreads();
      if (tid < WAVE) {
        uint32_t acc = 0;
        for (int d0 = 0; d0 < D; d0 += WAVE) {
          int d = d0 + lane_id();
          uint32_t a = d < D ? s_doff[d] : 0;
          uint32_t inc = wave_incl_scan(a);
          if (d < D) s_doff[d] = acc + inc - a;
          acc += __shfl(inc, WAVE - 1, WAVE);
        }
      }
      __syncthreads();
      if (wave_has) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          if (striped && i * BLOCK >= n) continue;
          const bool ok = (striped ? i * BLOCK + tid : tid * ITEMS + i) < n;
          if (ok) {
            uint32_t d = (uint32_t)(key[i] >> shift) & (D - 1);
            uint32_t w = s_cnt[(d >> 1) * BLOCK + tid];
            rank[i] += ((w >> ((d & 1) * 16)) & 0xFFFFu) + s_doff[d];
          }
        }
      }
      __syncthreads();
      // values first, so that the plane left in s_buf holds the keys' low words
      if constexpr (HAS_VAL) exchange(val, rank, s_buf, true, n, striped);
      exchange(key, rank, s_buf, bits > 32, n, striped);
      striped = false;
    }
  }
};

}  // namespace hpa
