// CPU stand-in for the HIP runtime and the device intrinsics the library uses,
// for running the library's kernel sources on the host (tests only; the
// library never includes it).  Every workgroup runs as real threads, one per
// lane; the workgroups of a launch run one after another; every cross-lane
// operation (shuffle, ballot, DPP move, readlane, wave barrier) waits for all
// 64 lanes of its wave, so a kernel that reaches one from divergent code, or
// relies on lanes waiting for each other without one, stops there.  "Device"
// memory is host memory, filled with garbage when allocated.  A check of the
// kernels' logic and indexing (with AddressSanitizer on the host build), not a
// model of the GPU's caches or of concurrent workgroups.
#pragma once
#include <algorithm>
#include <atomic>
#include <barrier>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) (&(x))

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
inline thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;

struct uint4 { uint32_t x, y, z, w; };
struct ulonglong2 { unsigned long long x, y; };

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2 };
typedef void* hipStream_t;
typedef void* hipMemPool_t;
struct EmuEvent { std::chrono::steady_clock::time_point t; };
typedef EmuEvent* hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum { hipMemPoolAttrReleaseThreshold = 0, hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipHostMallocDefault = 0 };
struct hipDeviceProp_t { int multiProcessorCount; char name[256]; };

// ---- per-launch lane machinery -------------------------------------------
struct EmuWave {
  std::barrier<> bar{64};
  uint64_t slot[64];
};
struct EmuBlock {
  std::unique_ptr<std::barrier<>> bar;
  std::vector<std::unique_ptr<EmuWave>> waves;
};
inline thread_local EmuBlock* emu_blk = nullptr;

inline void __syncthreads() { emu_blk->bar->arrive_and_wait(); }
inline unsigned emu_lane() { return threadIdx.x & 63u; }
inline EmuWave& emu_wave() { return *emu_blk->waves[threadIdx.x / 64]; }

template <class T>
inline uint64_t emu_bits(T v) {
  uint64_t u = 0;
  std::memcpy(&u, &v, sizeof(T));
  return u;
}
template <class T>
inline T emu_from(uint64_t u) {
  T v;
  std::memcpy(&v, &u, sizeof(T));
  return v;
}
template <class T, class F>
inline T emu_xlane(T v, F pick) {
  EmuWave& w = emu_wave();
  w.slot[emu_lane()] = emu_bits(v);
  w.bar.arrive_and_wait();
  const uint64_t r = pick(w.slot, (int)emu_lane());
  w.bar.arrive_and_wait();
  return emu_from<T>(r);
}
template <class T>
inline T __shfl(T v, int src, int = 64) {
  return emu_xlane(v, [&](const uint64_t* s, int) { return s[src & 63]; });
}
template <class T>
inline T __shfl_up(T v, unsigned d, int = 64) {
  const uint64_t own = emu_bits(v);
  return emu_xlane(v, [&](const uint64_t* s, int l) { return l >= (int)d ? s[l - d] : own; });
}
template <class T>
inline T __shfl_down(T v, unsigned d, int = 64) {
  const uint64_t own = emu_bits(v);
  return emu_xlane(v, [&](const uint64_t* s, int l) { return l + (int)d < 64 ? s[l + d] : own; });
}
template <class T>
inline T __shfl_xor(T v, int m, int = 64) {
  return emu_xlane(v, [&](const uint64_t* s, int l) { return s[(l ^ m) & 63]; });
}
inline unsigned long long __ballot(int p) {
  return emu_xlane<unsigned long long>(p ? 1ull : 0ull, [&](const uint64_t* s, int) {
    uint64_t m = 0;
    for (int i = 0; i < 64; ++i) m |= (s[i] & 1ull) << i;
    return m;
  });
}
inline int __any(int p) { return __ballot(p) != 0; }
// LDS DMA: lane l writes `size` bytes at dst + off + l * size
inline void __builtin_amdgcn_global_load_lds(const void* src, void* dst, unsigned size, int off, int) {
  std::memcpy(static_cast<char*>(dst) + off + (threadIdx.x & 63u) * size, src, size);
}
inline void __builtin_amdgcn_s_waitcnt(int) {}
inline int __builtin_amdgcn_readfirstlane(int v) {
  return emu_xlane(v, [&](const uint64_t* s, int) { return s[0]; });
}
inline int __builtin_amdgcn_readlane(int v, int l) {
  return emu_xlane(v, [&](const uint64_t* s, int) { return s[l & 63]; });
}
// DPP moves used by the wave scans: row_shr:1..15, row_bcast:15, row_bcast:31
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  (void)bank_mask;
  const int own_old = old;
  return emu_xlane(src, [&](const uint64_t* s, int l) -> uint64_t {
    const int row = l / 16, in = l % 16;
    if (!((row_mask >> row) & 1)) return emu_bits(own_old);
    if (ctrl >= 0x111 && ctrl <= 0x11F) {
      const int n = ctrl & 0xF;
      if (in >= n) return s[l - n];
      return bound_ctrl ? 0ull : emu_bits(own_old);
    }
    if (ctrl == 0x138) return l >= 1 ? s[l - 1] : (bound_ctrl ? 0ull : emu_bits(own_old));   // wave_shr:1
    if (ctrl == 0x130) return l <= 62 ? s[l + 1] : (bound_ctrl ? 0ull : emu_bits(own_old));  // wave_shl:1
    if (ctrl == 0x142) return row >= 1 ? s[row * 16 - 1] : emu_bits(own_old);
    if (ctrl == 0x143) return row >= 2 ? s[31] : emu_bits(own_old);
    std::fprintf(stderr, "emu: dpp control %#x not modelled\n", ctrl);
    std::abort();
  }) & 0xFFFFFFFFull;
}
inline void __builtin_amdgcn_wave_barrier() { emu_wave().bar.arrive_and_wait(); }
#define __builtin_amdgcn_fence(order, scope) std::atomic_thread_fence(std::memory_order_seq_cst)
inline void __builtin_amdgcn_s_sleep(int) { std::this_thread::yield(); }
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __threadfence_block() { std::atomic_thread_fence(std::memory_order_seq_cst); }

inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __clzll(long long v) { return v ? __builtin_clzll((unsigned long long)v) : 64; }
inline int __ffsll(long long v) { return __builtin_ffsll(v); }
template <class T>
inline void __builtin_nontemporal_store(T v, T* p) { *p = v; }
inline uint32_t __builtin_amdgcn_ubfe(uint32_t v, uint32_t off, uint32_t w) {
  off &= 31; w &= 31;
  return w ? (v >> off) & ((1u << w) - 1u) : 0u;
}
using std::max;
using std::min;
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
inline unsigned max(unsigned a, unsigned b) { return a > b ? a : b; }
inline uint64_t min(uint64_t a, uint64_t b) { return a < b ? a : b; }
inline uint64_t max(uint64_t a, uint64_t b) { return a > b ? a : b; }
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }

// ---- atomics ----------------------------------------------------------------
template <class T, class U>
inline T atomicAdd(T* p, U v) { return __atomic_fetch_add(p, (T)v, __ATOMIC_SEQ_CST); }
template <class T, class U>
inline T atomicOr(T* p, U v) { return __atomic_fetch_or(p, (T)v, __ATOMIC_SEQ_CST); }
template <class T, class U>
inline T atomicMin(T* p, U v) {
  T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while ((T)v < cur && !__atomic_compare_exchange_n(p, &cur, (T)v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {}
  return cur;
}
template <class T, class U>
inline T atomicMax(T* p, U v) {
  T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while ((T)v > cur && !__atomic_compare_exchange_n(p, &cur, (T)v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {}
  return cur;
}
template <class T, class U, class V>
inline T atomicCAS(T* p, U cmp, V v) {
  T c = (T)cmp;
  __atomic_compare_exchange_n(p, &c, (T)v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
  return c;
}
#define __HIP_MEMORY_SCOPE_AGENT 0
#define __HIP_MEMORY_SCOPE_WORKGROUP 0
template <class T>
inline T __hip_atomic_load(const T* p, int, int) { return __atomic_load_n(p, __ATOMIC_SEQ_CST); }
template <class T, class U>
inline void __hip_atomic_store(T* p, U v, int, int) { __atomic_store_n(p, (T)v, __ATOMIC_SEQ_CST); }

// ---- runtime ---------------------------------------------------------------
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "emu"; }
inline hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  p->multiProcessorCount = 4;
  std::strcpy(p->name, "emu");
  return hipSuccess;
}
inline hipError_t hipDeviceGetDefaultMemPool(hipMemPool_t* p, int) { *p = nullptr; return hipSuccess; }
inline hipError_t hipMemPoolSetAttribute(hipMemPool_t, int, void*) { return hipSuccess; }
inline hipError_t hipMallocAsync(void** p, size_t n, hipStream_t) {
  *p = std::aligned_alloc(256, (n + 255) & ~(size_t)255);
  if (*p) std::memset(*p, 0xA5, n);  // garbage, as fresh device memory may hold
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipMalloc(void** p, size_t n) { return hipMallocAsync(p, n, nullptr); }
inline hipError_t hipFreeAsync(void* p, hipStream_t) { std::free(p); return hipSuccess; }
inline hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t = nullptr) { std::memset(p, v, n); return hipSuccess; }
inline hipError_t hipMemset(void* p, int v, size_t n) { std::memset(p, v, n); return hipSuccess; }
inline hipError_t hipMemset2DAsync(void* p, size_t pitch, int v, size_t w, size_t h, hipStream_t) {
  for (size_t i = 0; i < h; ++i) std::memset((char*)p + i * pitch, v, w);
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t = nullptr) {
  std::memmove(d, s, n);
  return hipSuccess;
}
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k) { return hipMemcpyAsync(d, s, n, k); }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = new EmuEvent{}; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, int) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { e->t = std::chrono::steady_clock::now(); return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
  return hipSuccess;
}
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }

// kernel launch: `k<<<g, b, sh, s>>>(args)` is rewritten to
// emu_launch(g, b, [&] { k(args); })
inline void emu_launch(dim3 g, dim3 b, std::function<void()> f) {
  EmuBlock blk;
  blk.bar = std::make_unique<std::barrier<>>((std::ptrdiff_t)b.x);
  for (unsigned w = 0; w < (b.x + 63) / 64; ++w) blk.waves.push_back(std::make_unique<EmuWave>());
  std::vector<std::thread> th;
  th.reserve(b.x);
  for (unsigned t = 0; t < b.x; ++t)
    th.emplace_back([&, t] {
      threadIdx = dim3(t);
      blockDim = b;
      gridDim = g;
      emu_blk = &blk;
      for (unsigned bi = 0; bi < g.x; ++bi) {
        blockIdx = dim3(bi);
        f();
        blk.bar->arrive_and_wait();
      }
    });
  for (auto& x : th) x.join();
}
template <class G, class B>
inline void emu_launch(G g, B b, size_t, hipStream_t, std::function<void()> f) {
  emu_launch(dim3((unsigned)g), dim3((unsigned)b), f);
}
