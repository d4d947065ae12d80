// A7: learned interval index.
//
// A two-stage model over the sorted interval starts s[0..M) predicts where a
// query address q falls, and a bounded search around the prediction finds
// the answer; a verification step and the plain binary search keep every
// answer exact, so the model only ever changes the speed of a lookup.
//
//   root   a multilayer perceptron, 2 inputs -> 64 -> 64 -> 1 with ReLU,
//          FP32, trained on the device by the forward/backward kernels below
//          (Adam, mean squared error) to map a start to its rank fraction
//          i / M; its output, times the number of leaves, picks a leaf;
//   leaf   a linear model rank ~ slope * (q - base) + intercept in FP32,
//          fitted by least squares to the starts the root sends to it;
//   window per leaf, the largest amounts by which the rounded prediction
//          undershoots and overshoots the true rank, taken over every start
//          routed to the leaf and over every start - 1 routed to it (the last
//          address before that start), evaluated with the same FP32
//          expression the lookup uses.  The leaf prediction is monotone in
//          q, so a query whose bracketing starts s[i] and s[i+1] - 1 both
//          route to its leaf has its answer inside the window;
//   search binary search for the last start <= q inside the window, then the
//          check s[i] <= q < s[i+1]; a query that fails it (the root is not
//          monotone, or a window was capped) takes the plain two-level binary
//          search.  Finally q < end[i] decides between i and "unmapped".
//
// Features of q (t = q - s[0], which fits 64 bits): the high part
// (t >> sh) / ((span >> sh) + 1), exact in FP32 because sh leaves at most 24
// bits, and the low part (t mod 2^sh) / 2^sh.
#include <cmath>
#include <cstring>
#include <memory>

#include "block_prims.h"
#include "hpa_internal.h"

namespace hpa {

namespace {

constexpr int NH = 64;  // hidden width
// parameter layout (floats): W1[64][2], b1[64], W2[64][64], b2[64], w3[64], b3
constexpr int P_W1 = 0, P_B1 = P_W1 + NH * 2, P_W2 = P_B1 + NH, P_B2 = P_W2 + NH * NH, P_W3 = P_B2 + NH,
              P_B3 = P_W3 + NH, NPARAM = P_B3 + 1;
static_assert(NPARAM == HPA_LEARNED_NPARAM, "parameter count in the header");

struct Norm {
  uint64_t s0;   // first start
  uint32_t sh;   // shift of the high feature
  float inv_hi;  // 1 / ((span >> sh) + 1)
  float inv_lo;  // 1 / 2^sh
};

__device__ __forceinline__ void features(const Norm& nm, uint64_t q, float& x0, float& x1) {
  const uint64_t t = q - nm.s0;
  x0 = (float)(t >> nm.sh) * nm.inv_hi;
  x1 = (float)(t & ((1ull << nm.sh) - 1ull)) * nm.inv_lo;
}

// The root's parameters, staged in LDS by every kernel that routes keys: the
// first layer as (w_x0, w_x1, bias, 0) per hidden unit, the second layer
// transposed (k-major, so that the 32 lanes reading one input k for 32
// outputs hit 32 banks), then its biases, the output weights and bias.
struct RootLds {
  float4 w1b1[NH];
  float w2t[NH * NH];  // w2t[k * NH + j] = W2[j][k]
  float b2[NH], w3[NH];
  float b3;
};

__device__ inline void stage_root(RootLds& R, const float* __restrict__ P) {
  for (int k = threadIdx.x; k < NH; k += blockDim.x)
    R.w1b1[k] = make_float4(P[P_W1 + 2 * k], P[P_W1 + 2 * k + 1], P[P_B1 + k], 0.f);
  for (int i = threadIdx.x; i < NH * NH; i += blockDim.x) R.w2t[(i % NH) * NH + i / NH] = P[P_W2 + i];
  for (int k = threadIdx.x; k < NH; k += blockDim.x) {
    R.b2[k] = P[P_B2 + k];
    R.w3[k] = P[P_W3 + k];
  }
  if (threadIdx.x == 0) R.b3 = P[P_B3];
}

typedef float mfma_acc16 __attribute__((ext_vector_type(16)));

// The root's output for the 64 keys of a wave (one per lane), on the matrix
// cores: the 64 x 64 hidden layer is a product of W2 with the first layer's
// outputs for 32 keys at a time (v_mfma_f32_32x32x2f32, two 32-row tiles, K
// in steps of 2).  In a step lane l supplies W2[row l % 32][k] and the first
// layer's unit k for key l % 32, with k = 2s + l / 32; after the last step
// its register r holds hidden row 8 (r / 4) + 4 (l / 32) + r % 4 of that key.
// The output layer then sums the lane's rows, and the two lanes of a key add
// their halves.  Every lane of the wave must call it.  Every kernel that
// routes a key calls this one function, so training-time windows and lookups
// see bit-identical values.
__device__ inline float route_wave(const RootLds& R, float x0, float x1) {
  const int l = lane_id(), h = l >> 5, n = l & 31;
  float y_own = 0.f;
#pragma unroll 1
  for (int g = 0; g < 2; ++g) {
    // the keys of lanes 32g .. 32g + 31, at both lane halves
    const float gx0 = __shfl(x0, g * 32 + n, WAVE), gx1 = __shfl(x1, g * 32 + n, WAVE);
    float part = 0.f;
#pragma unroll 1
    for (int tile = 0; tile < 2; ++tile) {
      mfma_acc16 acc = {};
#pragma unroll 2
      for (int s = 0; s < NH / 2; ++s) {
        const int k = 2 * s + h;
        const float4 wb = R.w1b1[k];
        const float b = fmaxf(fmaf(wb.y, gx1, fmaf(wb.x, gx0, wb.z)), 0.f);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(R.w2t[k * NH + 32 * tile + n], b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = 32 * tile + 8 * (r / 4) + 4 * h + (r % 4);
        part = fmaf(R.w3[m], fmaxf(acc[r] + R.b2[m], 0.f), part);
      }
    }
    const float other = __shfl_xor(part, 32, WAVE);
    // the same sum in both lanes of a key: the lower half's part first
    const float y = (h == 0 ? part + other : other + part) + R.b3;
    if (h == g) y_own = y;
  }
  return y_own;
}

__device__ __forceinline__ uint32_t leaf_of_output(float y, uint32_t n_leaf) {
  const float f = floorf(y * (float)n_leaf);
  if (!(f > 0.f)) return 0;  // also NaN
  if (f >= (float)(n_leaf - 1)) return n_leaf - 1;
  return (uint32_t)f;
}

struct Leaves {
  const uint64_t* base;
  const float* slope;
  const float* icpt;
  const uint32_t* elo;  // window below the prediction
  const uint32_t* ehi;  // window above the prediction
};

// Rounded rank prediction of leaf L for q, clamped to [0, M - 1].
__device__ __forceinline__ uint64_t leaf_predict(const uint64_t* base, const float* slope, const float* icpt,
                                                 uint32_t L, uint64_t q, uint64_t M) {
  const int64_t d = (int64_t)(q - base[L]);
  const float p = floorf(fmaf(slope[L], (float)d, icpt[L]));
  if (!(p > 0.f)) return 0;
  if (p >= (float)(M - 1)) return M - 1;
  const uint64_t r = (uint64_t)p;
  return r < M - 1 ? r : M - 1;
}

// ---------------------------------------------------------------------------
// training: forward/backward over a minibatch, per-block partial gradients
// ---------------------------------------------------------------------------
constexpr int TB = 128;     // samples (threads) per block
constexpr int LDP = NH + 1;  // padded LDS row

// Partial gradient of sum_b scale * (y_b - t_b)^2 over this block's samples;
// partial[blockIdx][NPARAM] receives the block's sum of squared errors.  With
// `hashed` the rows of the minibatch come from a multiplicative hash of
// (step, position) into [0, n_rows); otherwise row = position.
__global__ void __launch_bounds__(TB)
k_mlp_grad(const float* __restrict__ P, const float* __restrict__ X, const float* __restrict__ T, uint64_t n_rows,
           uint64_t batch, uint64_t step, int hashed, float scale, float* __restrict__ partial) {
  __shared__ float s_h1[TB * LDP];
  __shared__ float s_h2[TB * LDP];  // h2, later the layer-1 deltas
  __shared__ float s_d2[TB * LDP];
  __shared__ float s_x[TB * 2];
  __shared__ float s_dy[TB];
  const int tid = threadIdx.x;
  const uint64_t pos = (uint64_t)blockIdx.x * TB + tid;
  const bool valid = pos < batch;
  uint64_t row = 0;
  if (valid) {
    if (hashed) {
      const uint64_t h = (step * batch + pos + 1) * 0x9E3779B97F4A7C15ull;
      row = (h >> 11) % n_rows;
    } else {
      row = pos;
    }
  }
  const float x0 = valid ? X[2 * row] : 0.f, x1 = valid ? X[2 * row + 1] : 0.f;
  float h1[NH], a2[NH];
#pragma unroll
  for (int k = 0; k < NH; ++k) h1[k] = fmaxf(fmaf(P[P_W1 + 2 * k + 1], x1, fmaf(P[P_W1 + 2 * k], x0, P[P_B1 + k])), 0.f);
  float y = P[P_B3];
  for (int j = 0; j < NH; ++j) {
    float a = P[P_B2 + j];
#pragma unroll
    for (int k = 0; k < NH; ++k) a = fmaf(P[P_W2 + NH * j + k], h1[k], a);
    a2[j] = a;
    y = fmaf(P[P_W3 + j], fmaxf(a, 0.f), y);
  }
  const float err = valid ? y - T[row] : 0.f;
  const float dy = 2.f * err * scale;
  s_dy[tid] = dy;
  s_x[2 * tid] = x0;
  s_x[2 * tid + 1] = x1;
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    s_h1[tid * LDP + k] = h1[k];
    s_h2[tid * LDP + k] = fmaxf(a2[k], 0.f);
    s_d2[tid * LDP + k] = a2[k] > 0.f ? dy * P[P_W3 + k] : 0.f;
  }
  __syncthreads();
  float* out = partial + (uint64_t)blockIdx.x * (NPARAM + 1);
  // W2: thread tid owns rows j in [4 * (tid / 8), +4) and columns k in [8 * (tid % 8), +8)
  {
    const int j0 = 4 * (tid >> 3), k0 = 8 * (tid & 7);
    float acc[4][8];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 8; ++b) acc[a][b] = 0.f;
    for (int s = 0; s < TB; ++s) {
      float d[4], h[8];
#pragma unroll
      for (int a = 0; a < 4; ++a) d[a] = s_d2[s * LDP + j0 + a];
#pragma unroll
      for (int b = 0; b < 8; ++b) h[b] = s_h1[s * LDP + k0 + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = fmaf(d[a], h[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 8; ++b) out[P_W2 + NH * (j0 + a) + k0 + b] = acc[a][b];
  }
  // b2, w3 (threads 0..63), b3 and the loss (thread 64)
  if (tid < NH) {
    float gb = 0.f, gw = 0.f;
    for (int s = 0; s < TB; ++s) {
      gb += s_d2[s * LDP + tid];
      gw = fmaf(s_dy[s], s_h2[s * LDP + tid], gw);
    }
    out[P_B2 + tid] = gb;
    out[P_W3 + tid] = gw;
  } else if (tid == NH) {
    float g = 0.f;
    for (int s = 0; s < TB; ++s) g += s_dy[s];
    out[P_B3] = g;
  }
  __syncthreads();
  // layer-1 deltas: d1[k] = (h1[k] > 0) * sum_j W2[j][k] d2[j]
  {
    float d1[NH];
#pragma unroll
    for (int k = 0; k < NH; ++k) d1[k] = 0.f;
    for (int j = 0; j < NH; ++j) {
      const float dj = s_d2[tid * LDP + j];
#pragma unroll
      for (int k = 0; k < NH; ++k) d1[k] = fmaf(P[P_W2 + NH * j + k], dj, d1[k]);
    }
#pragma unroll
    for (int k = 0; k < NH; ++k) s_h2[tid * LDP + k] = h1[k] > 0.f ? d1[k] : 0.f;
  }
  s_d2[tid * LDP] = err * err;  // row 0 of d2 is no longer needed by this thread
  __syncthreads();
  if (tid < NH) {
    float g0 = 0.f, g1 = 0.f, gb = 0.f;
    for (int s = 0; s < TB; ++s) {
      const float d = s_h2[s * LDP + tid];
      g0 = fmaf(d, s_x[2 * s], g0);
      g1 = fmaf(d, s_x[2 * s + 1], g1);
      gb += d;
    }
    out[P_W1 + 2 * tid] = g0;
    out[P_W1 + 2 * tid + 1] = g1;
    out[P_B1 + tid] = gb;
  } else if (tid == NH) {
    float l = 0.f;
    for (int s = 0; s < TB; ++s) l += s_d2[s * LDP];
    out[NPARAM] = l;
  }
}

// Sum the blocks' partial gradients in block order; with adam != 0 take one
// Adam step on P (moments m, v; bias corrections b1t = 1 - beta1^t, b2t).
__global__ void __launch_bounds__(256)
k_mlp_reduce(const float* __restrict__ partial, uint32_t n_blocks, float* __restrict__ grad, float* __restrict__ P,
             float* __restrict__ m, float* __restrict__ v, int adam, float lr, float b1t, float b2t) {
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p > (uint32_t)NPARAM) return;
  float g = 0.f;
  for (uint32_t b = 0; b < n_blocks; ++b) g += partial[(uint64_t)b * (NPARAM + 1) + p];
  if (grad) grad[p] = g;
  if (adam && p < (uint32_t)NPARAM) {
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    const float mm = beta1 * m[p] + (1.f - beta1) * g;
    const float vv = beta2 * v[p] + (1.f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    P[p] = P[p] - lr * (mm / b1t) / (sqrtf(vv / b2t) + eps);
  }
}

// Training rows from evenly spaced starts: features and target i / M.
__global__ void k_make_rows(const uint64_t* __restrict__ start, uint64_t M, uint64_t n_rows, Norm nm,
                            float* __restrict__ X, float* __restrict__ T) {
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rows) return;
  const uint64_t i = n_rows == M ? r : (r * M) / n_rows;  // r < 2^32, M < 2^32
  float x0, x1;
  features(nm, start[i], x0, x1);
  X[2 * r] = x0;
  X[2 * r + 1] = x1;
  T[r] = (float)((double)i / (double)M);
}

// ---------------------------------------------------------------------------
// leaves
// ---------------------------------------------------------------------------
constexpr int RB = 256;

__global__ void __launch_bounds__(RB, 4)
k_route(const uint64_t* __restrict__ start, uint64_t M, Norm nm, const float* __restrict__ P, uint32_t n_leaf,
        uint16_t* __restrict__ leaf_of, unsigned long long* __restrict__ base) {
  __shared__ RootLds R;
  stage_root(R, P);
  __syncthreads();
  const uint64_t i = (uint64_t)blockIdx.x * RB + threadIdx.x;
  // every lane routes (the wave computes together); lanes past M route the
  // last start and write nothing
  const uint64_t q = start[i < M ? i : M - 1];
  float x0, x1;
  features(nm, q, x0, x1);
  const uint32_t L = leaf_of_output(route_wave(R, x0, x1), n_leaf);
  if (i >= M) return;
  leaf_of[i] = (uint16_t)L;
  atomicMin(&base[L], (unsigned long long)q);
}

// per leaf: count, sum x, sum y, sum xx, sum xy with x = start - base, y = rank
__global__ void __launch_bounds__(RB)
k_leaf_sums(const uint64_t* __restrict__ start, uint64_t M, const uint16_t* __restrict__ leaf_of,
            const unsigned long long* __restrict__ base, double* __restrict__ sums) {
  const uint64_t i = (uint64_t)blockIdx.x * RB + threadIdx.x;
  if (i >= M) return;
  const uint32_t L = leaf_of[i];
  const double x = (double)(start[i] - base[L]), y = (double)i;
  double* s = sums + 5ull * L;
  atomicAdd(&s[0], 1.0);
  atomicAdd(&s[1], x);
  atomicAdd(&s[2], y);
  atomicAdd(&s[3], x * x);
  atomicAdd(&s[4], x * y);
}

__global__ void k_leaf_fit(const double* __restrict__ sums, uint32_t n_leaf, float* __restrict__ slope,
                           float* __restrict__ icpt) {
  const uint32_t L = blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= n_leaf) return;
  const double* s = sums + 5ull * L;
  const double n = s[0];
  double a = 0.0, b = 0.0;
  if (n > 0.0) {
    const double mx = s[1] / n, my = s[2] / n;
    const double sxx = s[3] - n * mx * mx, sxy = s[4] - n * mx * my;
    a = sxx > 0.0 ? sxy / sxx : 0.0;
    if (!(a > 0.0)) a = 0.0;  // keep the prediction monotone in q
    b = my - a * mx;
  }
  slope[L] = (float)a;
  icpt[L] = (float)b;
}

// Windows: for every start s[i] (rank i) and every s[i] - 1 with i > 0 (rank
// i - 1): route, predict, and widen its leaf's window to cover the rank.
// Misses larger than cap are left uncovered (counted): their queries take the
// fallback search.
__global__ void __launch_bounds__(RB, 4)
k_leaf_windows(const uint64_t* __restrict__ start, uint64_t M, Norm nm, const float* __restrict__ P, uint32_t n_leaf,
               const uint16_t* __restrict__ leaf_of, const unsigned long long* __restrict__ base,
               const float* __restrict__ slope, const float* __restrict__ icpt, uint32_t cap,
               unsigned int* __restrict__ elo, unsigned int* __restrict__ ehi,
               unsigned long long* __restrict__ uncovered) {
  __shared__ RootLds R;
  stage_root(R, P);
  __syncthreads();
  const uint64_t i = (uint64_t)blockIdx.x * RB + threadIdx.x;
  unsigned long long miss = 0;
  // the key just below each start is routed by the whole wave (lanes without
  // one route a stand-in and ignore it)
  uint32_t L1;
  {
    const uint64_t iq = i < M ? i : M - 1;
    const uint64_t q1 = start[iq] - (iq > 0 ? 1 : 0);
    float x0, x1;
    features(nm, q1, x0, x1);
    L1 = leaf_of_output(route_wave(R, x0, x1), n_leaf);
  }
  if (i < M) {
    const uint64_t* bs = reinterpret_cast<const uint64_t*>(base);
    for (int k = 0; k < 2; ++k) {
      if (k == 1 && i == 0) break;
      const uint64_t q = k == 0 ? start[i] : start[i] - 1;
      const uint64_t rank = k == 0 ? i : i - 1;
      const uint32_t L = k == 0 ? (uint32_t)leaf_of[i] : L1;
      const uint64_t pred = leaf_predict(bs, slope, icpt, L, q, M);
      if (pred >= rank) {
        const uint64_t d = pred - rank;
        if (d <= cap) atomicMax(&elo[L], (unsigned int)d);
        else ++miss;
      } else {
        const uint64_t d = rank - pred;
        if (d <= cap) atomicMax(&ehi[L], (unsigned int)d);
        else ++miss;
      }
    }
  }
  miss = wave_sum(miss);
  if (lane_id() == 0 && miss) atomicAdd(uncovered, miss);
}

// ---------------------------------------------------------------------------
// lookup
// ---------------------------------------------------------------------------
constexpr int LB = 512;

template <bool STATS>
__global__ void __launch_bounds__(LB, 3)
k_lookup_learned(const uint64_t* __restrict__ start, const uint64_t* __restrict__ end, uint64_t M, Norm nm,
                 const float* __restrict__ P, uint32_t n_leaf, const uint64_t* __restrict__ lbase,
                 const float* __restrict__ slope, const float* __restrict__ icpt, const uint32_t* __restrict__ elo,
                 const uint32_t* __restrict__ ehi, const uint64_t* __restrict__ top, uint32_t top_n, uint32_t shift,
                 const uint64_t* __restrict__ pc, uint64_t n, uint32_t* __restrict__ out,
                 unsigned long long* __restrict__ stats) {
  __shared__ uint64_t s_top[4096];
  __shared__ RootLds R;
  for (uint32_t i = threadIdx.x; i < top_n; i += LB) s_top[i] = top[i];
  stage_root(R, P);
  __syncthreads();
  const uint64_t s_last = start[M - 1];
  unsigned long long probes = 0, fallbacks = 0;
  const uint64_t stride = (uint64_t)gridDim.x * LB;
  // whole waves go round the loop together, since every lane routes
  const uint64_t t0 = (uint64_t)blockIdx.x * LB + threadIdx.x - (uint64_t)lane_id();
  for (uint64_t tw = t0; tw < n; tw += stride) {
    const uint64_t t = tw + (uint64_t)lane_id();
    const bool live = t < n;
    const uint64_t q = pc[live ? t : n - 1];
    float x0, x1;
    features(nm, q < nm.s0 ? nm.s0 : q, x0, x1);
    const float y = route_wave(R, x0, x1);
    if (!live) continue;
    uint64_t ans;  // last i with start[i] <= q, or M when q < start[0]
    if (q < nm.s0) {
      ans = M;
    } else if (q >= s_last) {
      ans = M - 1;
    } else {
      const uint32_t L = leaf_of_output(y, n_leaf);
      const uint64_t pred = leaf_predict(lbase, slope, icpt, L, q, M);
      const uint64_t lo0 = pred > elo[L] ? pred - elo[L] : 0;
      uint64_t hi0 = pred + ehi[L];
      if (hi0 > M - 1) hi0 = M - 1;
      // last i in [lo0, hi0] with start[i] <= q (lo0 - 1 marks "none")
      uint64_t lo = lo0, hi = hi0 + 1;
      while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (STATS) ++probes;
        if (start[mid] <= q) lo = mid + 1;
        else hi = mid;
      }
      // verify: start[i] <= q < start[i + 1] (q < start[M-1] here, so i < M - 1)
      bool ok = lo > lo0;
      if (ok) {
        ans = lo - 1;
        if (lo > hi0) {  // the window's last start is <= q: the next start decides
          if (STATS) ++probes;
          ok = q < start[lo];
        }
      }
      if (!ok) {
        if (STATS) ++fallbacks;
        uint32_t a = 0, b = top_n;
        while (a < b) {
          const uint32_t mid = (a + b) >> 1;
          if (s_top[mid] <= q) a = mid + 1;
          else b = mid;
        }
        uint64_t bb = (uint64_t)(a - 1) << shift, ee = bb + (1ull << shift);
        if (ee > M) ee = M;
        uint64_t l2 = bb + 1, h2 = ee;
        while (l2 < h2) {
          const uint64_t mid = (l2 + h2) >> 1;
          if (STATS) ++probes;
          if (start[mid] <= q) l2 = mid + 1;
          else h2 = mid;
        }
        ans = l2 - 1;
      }
    }
    out[t] = (ans < M && q < end[ans]) ? (uint32_t)ans : NONE32;
  }
  if (STATS) {
    probes = wave_sum(probes);
    fallbacks = wave_sum(fallbacks);
    if (lane_id() == 0) {
      atomicAdd(&stats[0], probes);
      atomicAdd(&stats[1], fallbacks);
    }
  }
}

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

struct LearnedModel {
  Norm nm{};
  uint32_t n_leaf = 0;
  hpa_learned_stats st{};
  DBuf P, base, slope, icpt, elo, ehi;
};

namespace {

Norm make_norm(uint64_t s0, uint64_t s_last) {
  Norm nm{};
  nm.s0 = s0;
  const uint64_t span = s_last - s0;
  uint32_t bits = 0;
  while (bits < 64 && (span >> bits)) ++bits;
  nm.sh = bits > 24 ? bits - 24 : 0;
  nm.inv_hi = (float)(1.0 / ((double)(span >> nm.sh) + 1.0));
  nm.inv_lo = (float)(1.0 / (double)(1ull << nm.sh));
  return nm;
}

// Kaiming-style uniform initialisation from a fixed seed.
std::vector<float> init_params(uint64_t seed) {
  std::vector<float> p(NPARAM, 0.f);
  uint64_t s = seed;
  auto u = [&](float bound) { return (float)(((double)(splitmix(s) >> 11) * 0x1.0p-53 * 2.0 - 1.0) * bound); };
  for (int i = 0; i < NH * 2; ++i) p[P_W1 + i] = u(std::sqrt(6.f / 2.f));
  for (int i = 0; i < NH; ++i) p[P_B1 + i] = u(0.5f);
  for (int i = 0; i < NH * NH; ++i) p[P_W2 + i] = u(std::sqrt(6.f / NH));
  for (int i = 0; i < NH; ++i) p[P_B2 + i] = u(0.1f);
  for (int i = 0; i < NH; ++i) p[P_W3 + i] = u(std::sqrt(3.f / NH));
  p[P_B3] = 0.f;
  return p;
}

void launch_grad(const float* P, const float* X, const float* T, uint64_t n_rows, uint64_t batch, uint64_t step,
                 int hashed, float* partial, hipStream_t s) {
  const unsigned nb = (unsigned)((batch + TB - 1) / TB);
  k_mlp_grad<<<nb, TB, 0, s>>>(P, X, T, n_rows, batch, step, hashed, 1.f / (float)batch, partial);
  HPA_HIP(hipGetLastError());
}

}  // namespace

void learned_train(hpa_structure_map* m, const hpa_learned_opts* o, hipStream_t s) {
  hpa_ctx* ctx = m->ctx;
  const uint64_t M = m->n_iv;
  if (M < 2) fail(HPA_E_UNSUPPORTED, "a learned index needs at least two intervals");
  if (M > 0xFFFFFFFFull) fail(HPA_E_UNSUPPORTED, "a learned index over more than 2^32 intervals");
  hpa_learned_opts d{};
  d.n_leaves = 4096;
  d.train_steps = 2000;
  d.batch = 8192;
  d.train_rows = 1u << 20;
  d.lr = 2e-3f;
  d.window_cap = 1u << 16;
  d.seed = 2109069310ull;
  if (o) {
    if (o->n_leaves) d.n_leaves = o->n_leaves;
    d.train_steps = o->train_steps;
    if (o->batch) d.batch = o->batch;
    if (o->train_rows) d.train_rows = o->train_rows;
    if (o->lr > 0.f) d.lr = o->lr;
    if (o->window_cap) d.window_cap = o->window_cap;
    if (o->seed) d.seed = o->seed;
  }
  if (d.n_leaves < 1 || d.n_leaves > 65536) fail(HPA_E_INVAL, "n_leaves must be in [1, 65536]");
  auto* lm = new LearnedModel();
  std::unique_ptr<LearnedModel> hold(lm);
  lm->n_leaf = d.n_leaves;
  lm->nm = make_norm(m->h_start.front(), m->h_start.back());
  const std::vector<float> p0 = init_params(d.seed);
  lm->P = upload(ctx, p0, s);
  const uint64_t n_rows = std::min<uint64_t>(d.train_rows, M);
  StageTimer tm(ctx, s);
  // training rows and Adam steps (no host round trip inside the loop)
  tm.begin("learned_train");
  if (d.train_steps > 0) {
    DBuf X(ctx, n_rows * 2 * 4, s), T(ctx, n_rows * 4, s);
    k_make_rows<<<grid_for(n_rows, 256), 256, 0, s>>>(m->start.as<uint64_t>(), M, n_rows, lm->nm, X.as<float>(),
                                                      T.as<float>());
    HPA_HIP(hipGetLastError());
    const uint64_t batch = d.batch;
    const unsigned nb = (unsigned)((batch + TB - 1) / TB);
    DBuf part(ctx, (uint64_t)nb * (NPARAM + 1) * 4, s), mom(ctx, NPARAM * 4, s), vel(ctx, NPARAM * 4, s);
    HPA_HIP(hipMemsetAsync(mom.p, 0, NPARAM * 4, s));
    HPA_HIP(hipMemsetAsync(vel.p, 0, NPARAM * 4, s));
    double b1t = 1.0, b2t = 1.0;
    for (uint32_t it = 0; it < d.train_steps; ++it) {
      launch_grad(lm->P.as<float>(), X.as<float>(), T.as<float>(), n_rows, batch, it, 1, part.as<float>(), s);
      b1t *= 0.9;
      b2t *= 0.999;
      // cosine decay to 1% of the initial rate
      const double f = 0.01 + 0.99 * 0.5 * (1.0 + std::cos(M_PI * (double)it / (double)d.train_steps));
      k_mlp_reduce<<<(NPARAM + 1 + 255) / 256, 256, 0, s>>>(part.as<float>(), nb, nullptr, lm->P.as<float>(),
                                                          mom.as<float>(), vel.as<float>(), 1, (float)(d.lr * f),
                                                          (float)(1.0 - b1t), (float)(1.0 - b2t));
      HPA_HIP(hipGetLastError());
    }
    // final loss over all rows
    const unsigned nbr = (unsigned)((n_rows + TB - 1) / TB);
    DBuf part2(ctx, (uint64_t)nbr * (NPARAM + 1) * 4, s), g(ctx, (NPARAM + 1) * 4, s);
    launch_grad(lm->P.as<float>(), X.as<float>(), T.as<float>(), n_rows, n_rows, 0, 0, part2.as<float>(), s);
    k_mlp_reduce<<<(NPARAM + 1 + 255) / 256, 256, 0, s>>>(part2.as<float>(), nbr, g.as<float>(), nullptr, nullptr,
                                                        nullptr, 0, 0.f, 1.f, 1.f);
    HPA_HIP(hipGetLastError());
    float loss = 0.f;
    HPA_HIP(hipMemcpyAsync(&loss, g.as<float>() + NPARAM, 4, hipMemcpyDeviceToHost, s));
    sync_stream(ctx, s);
    lm->st.train_mse = (double)loss / (double)n_rows;
  }
  tm.end(n_rows, 0);
  // leaves: route every start, fit, windows
  tm.begin("learned_leaves");
  const uint32_t NL = d.n_leaves;
  DBuf leaf_of(ctx, M * 2, s), sums(ctx, 5ull * NL * 8, s), unc(ctx, 8, s);
  lm->base = DBuf(ctx, (uint64_t)NL * 8, s);
  lm->slope = DBuf(ctx, (uint64_t)NL * 4, s);
  lm->icpt = DBuf(ctx, (uint64_t)NL * 4, s);
  lm->elo = DBuf(ctx, (uint64_t)NL * 4, s);
  lm->ehi = DBuf(ctx, (uint64_t)NL * 4, s);
  HPA_HIP(hipMemsetAsync(lm->base.p, 0xFF, (uint64_t)NL * 8, s));
  HPA_HIP(hipMemsetAsync(sums.p, 0, 5ull * NL * 8, s));
  HPA_HIP(hipMemsetAsync(lm->elo.p, 0, (uint64_t)NL * 4, s));
  HPA_HIP(hipMemsetAsync(lm->ehi.p, 0, (uint64_t)NL * 4, s));
  HPA_HIP(hipMemsetAsync(unc.p, 0, 8, s));
  const unsigned g = grid_for(M, RB, 1u << 30);
  k_route<<<g, RB, 0, s>>>(m->start.as<uint64_t>(), M, lm->nm, lm->P.as<float>(), NL, leaf_of.as<uint16_t>(),
                           lm->base.as<unsigned long long>());
  HPA_HIP(hipGetLastError());
  k_leaf_sums<<<g, RB, 0, s>>>(m->start.as<uint64_t>(), M, leaf_of.as<uint16_t>(), lm->base.as<unsigned long long>(),
                               sums.as<double>());
  HPA_HIP(hipGetLastError());
  k_leaf_fit<<<(NL + 255) / 256, 256, 0, s>>>(sums.as<double>(), NL, lm->slope.as<float>(), lm->icpt.as<float>());
  HPA_HIP(hipGetLastError());
  k_leaf_windows<<<g, RB, 0, s>>>(m->start.as<uint64_t>(), M, lm->nm, lm->P.as<float>(), NL, leaf_of.as<uint16_t>(),
                                  lm->base.as<unsigned long long>(), lm->slope.as<float>(), lm->icpt.as<float>(),
                                  d.window_cap, lm->elo.as<unsigned int>(), lm->ehi.as<unsigned int>(),
                                  unc.as<unsigned long long>());
  HPA_HIP(hipGetLastError());
  tm.end(M, 0);
  std::vector<uint32_t> elo(NL), ehi(NL);
  std::vector<double> hs(5ull * NL);
  unsigned long long uncovered = 0;
  HPA_HIP(hipMemcpyAsync(hs.data(), sums.p, 5ull * NL * 8, hipMemcpyDeviceToHost, s));
  HPA_HIP(hipMemcpyAsync(elo.data(), lm->elo.p, (uint64_t)NL * 4, hipMemcpyDeviceToHost, s));
  HPA_HIP(hipMemcpyAsync(ehi.data(), lm->ehi.p, (uint64_t)NL * 4, hipMemcpyDeviceToHost, s));
  HPA_HIP(hipMemcpyAsync(&uncovered, unc.p, 8, hipMemcpyDeviceToHost, s));
  sync_stream(ctx, s);
  tm.collect();
  // the window a lookup searches, averaged over the starts (each start
  // weighs by the leaf it is routed to)
  double sumw = 0.0, n_routed = 0.0;
  uint32_t maxw = 0;
  for (uint32_t L = 0; L < NL; ++L) {
    const uint32_t w = elo[L] + ehi[L] + 1;
    sumw += hs[5ull * L] * w;
    n_routed += hs[5ull * L];
    if (hs[5ull * L] > 0.0) maxw = std::max(maxw, w);
  }
  lm->st.n_leaves = NL;
  lm->st.train_steps = d.train_steps;
  lm->st.mean_window = n_routed > 0.0 ? sumw / n_routed : 0.0;
  lm->st.max_window = maxw;
  lm->st.uncovered = uncovered;
  if (m->learned) learned_free(m->learned);
  m->learned = hold.release();
}

void learned_train(hpa_structure_map* m, hipStream_t s) { learned_train(m, nullptr, s); }

void launch_lookup_learned(const hpa_structure_map* m, const uint64_t* pc, uint64_t n, uint32_t* out, hipStream_t s,
                           unsigned long long* stats) {
  const LearnedModel* lm = m->learned;
  if (n == 0) return;
  const unsigned grid = grid_for(n, LB, (unsigned)m->ctx->n_cu * 16);
  auto args = [&](auto kern) {
    kern<<<grid, LB, 0, s>>>(m->start.as<uint64_t>(), m->end.as<uint64_t>(), m->n_iv, lm->nm, lm->P.as<float>(),
                             lm->n_leaf, lm->base.as<uint64_t>(), lm->slope.as<float>(), lm->icpt.as<float>(),
                             lm->elo.as<uint32_t>(), lm->ehi.as<uint32_t>(), m->top.as<uint64_t>(), m->top_n,
                             m->top_shift, pc, n, out, stats);
  };
  if (stats) args(k_lookup_learned<true>);
  else args(k_lookup_learned<false>);
  HPA_HIP(hipGetLastError());
}

void launch_lookup_learned(const hpa_structure_map* m, const uint64_t* pc, uint64_t n, uint32_t* out, hipStream_t s) {
  launch_lookup_learned(m, pc, n, out, s, nullptr);
}

void learned_free(LearnedModel* lm) { delete lm; }

}  // namespace hpa

using namespace hpa;

extern "C" hpa_status hpa_learned_train(hpa_ctx* ctx, hpa_structure_map* map, const hpa_learned_opts* opts,
                                        hipStream_t stream) {
  return guard([&] {
    if (!ctx || !map) fail(HPA_E_INVAL, "NULL argument");
    if (map->ctx != ctx) fail(HPA_E_INVAL, "map belongs to another context");
    DeviceGuard g(ctx->device);
    learned_train(map, opts, stream);
  });
}

extern "C" hpa_status hpa_learned_stats_get(const hpa_structure_map* map, hpa_learned_stats* out) {
  return guard([&] {
    if (!map || !out) fail(HPA_E_INVAL, "NULL argument");
    if (!map->learned) fail(HPA_E_UNSUPPORTED, "map has no learned index");
    *out = map->learned->st;
    out->params = map->learned->P.as<float>();
  });
}

extern "C" hpa_status hpa_lookup_learned_counted(hpa_ctx* ctx, const hpa_structure_map* map, const uint64_t* d_pc,
                                                 uint64_t n, uint32_t* d_out, unsigned long long* d_counts,
                                                 hipStream_t stream) {
  return guard([&] {
    if (!ctx || !map || !d_counts) fail(HPA_E_INVAL, "NULL argument");
    if (n && (!d_pc || !d_out)) fail(HPA_E_INVAL, "NULL array with n > 0");
    if (map->ctx != ctx) fail(HPA_E_INVAL, "map belongs to another context");
    if (!map->learned) fail(HPA_E_UNSUPPORTED, "map was built without the learned index");
    DeviceGuard g(ctx->device);
    launch_lookup_learned(map, d_pc, n, d_out, stream, d_counts);
  });
}

extern "C" hpa_status hpa_learned_grad(hpa_ctx* ctx, const float* d_params, const float* d_x, const float* d_t,
                                       uint64_t n, float* d_grad, hipStream_t stream) {
  return guard([&] {
    if (!ctx || !d_params || !d_grad) fail(HPA_E_INVAL, "NULL argument");
    if (n == 0 || !d_x || !d_t) fail(HPA_E_INVAL, "need at least one row");
    DeviceGuard g(ctx->device);
    const unsigned nb = (unsigned)((n + TB - 1) / TB);
    DBuf part(ctx, (uint64_t)nb * (NPARAM + 1) * 4, stream);
    k_mlp_grad<<<nb, TB, 0, stream>>>(d_params, d_x, d_t, n, n, 0, 0, 1.f / (float)n, part.as<float>());
    HPA_HIP(hipGetLastError());
    k_mlp_reduce<<<(NPARAM + 1 + 255) / 256, 256, 0, stream>>>(part.as<float>(), nb, d_grad, nullptr, nullptr, nullptr,
                                                               0, 0.f, 1.f, 1.f);
    HPA_HIP(hipGetLastError());
    sync_stream(ctx, stream);
  });
}
