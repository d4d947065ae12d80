// Cross-profile unification and statistics, the CCT-major and profile-major
// sparse layouts, and multi-run combination.
//
// Unification (Section 6.1, call path profile unification): the profiles'
// (ctx, pc) contexts are merged into one sorted list; every key of every
// profile gets the index of its context in that list.  The union is computed
// by the attribution path itself: each key becomes a record (pc, ctx) of
// weight one, so the unified attribution holds each context once, sorted, and
// its count is the number of (profile, stall) entries the context has.
//
// Sparse layouts (Section 6.2): metric m is the sample count with stall reason
// m.  CMS holds, per unified context, its non-empty metrics as (metric, start)
// pairs into profile ids / values ordered by metric then profile; PMS holds,
// per profile, its (context, metric, value) triples ordered by context then
// metric, with (context, start) pairs.  Offsets come from exclusive scans
// (the exscan layout of the paper); the entry scatter runs one thread per
// non-zero, so its work is balanced by non-zeros.
//
// Statistics (Section 4.5, derived metrics over profiles; Section 6.1
// statistic generation): per non-empty (context, metric) over all P profiles,
// absent entries counting as zero: sum, min, max, mean = sum / P, population
// standard deviation and coefficient of variation, the deviation summed over
// the entries in profile order.
//
// Combination of runs (Section 4.7): the keys of every run become weighted
// records that go through the attribution path, which sums equal keys.
#include <cmath>
#include <cstdio>
#include <memory>

#include "block_prims.h"
#include "hpa_internal.h"

namespace hpa {
namespace {

constexpr int B = 256;
constexpr uint64_t WMAX = 0xFFFFFFFFull;

struct ProfDev {
  const uint32_t* ctx;
  const uint64_t* pc;
  const uint8_t* stall;
  const unsigned long long* count;
  uint64_t n;
  uint64_t base;  // first key of the profile in the concatenated key space
};

__device__ __forceinline__ uint32_t profile_of(const ProfDev* pd, uint32_t P, uint64_t k) {
  uint32_t lo = 0, hi = P;  // last profile with base <= k
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (pd[mid].base <= k) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint32_t records_of(unsigned long long c) {
  return c == 0 ? 0u : (uint32_t)((c + WMAX - 1) / WMAX);
}

// Records per key: with `unit` every key is one record of weight one (the
// union of contexts), otherwise its count split into pieces of at most
// 2^32 - 1 (pass 0 counts, pass 1 writes at the scanned offsets).
__global__ void __launch_bounds__(B)
k_records(const ProfDev* __restrict__ pd, uint32_t P, uint64_t K, int unit, int pass,
          unsigned long long* __restrict__ nrec, uint64_t* __restrict__ o_pc, uint32_t* __restrict__ o_ctx,
          uint8_t* __restrict__ o_st, uint32_t* __restrict__ o_w) {
  for (uint64_t k = (uint64_t)blockIdx.x * B + threadIdx.x; k < K; k += (uint64_t)gridDim.x * B) {
    const ProfDev d = pd[profile_of(pd, P, k)];
    const uint64_t i = k - d.base;
    const unsigned long long c = d.count[i];
    const uint32_t r = unit ? 1u : records_of(c);
    if (pass == 0) {
      nrec[k] = r;
      continue;
    }
    const uint64_t o = nrec[k];
    unsigned long long left = c;
    for (uint32_t j = 0; j < r; ++j) {
      const uint32_t w = unit ? 1u : (uint32_t)(left > WMAX ? WMAX : left);
      left -= w;
      o_pc[o + j] = d.pc[i];
      o_ctx[o + j] = d.ctx[i];
      o_st[o + j] = unit ? 0 : d.stall[i];
      o_w[o + j] = w;
    }
  }
}

// Exclusive scan of u64 values in place (three phases); `total` gets the sum.
constexpr int SCAN_ITEMS = 4, SCAN_T = 1024, SCAN_TILE = SCAN_T * SCAN_ITEMS;

__global__ void __launch_bounds__(SCAN_T)
k_scan_tiles(unsigned long long* __restrict__ v, uint64_t n, unsigned long long* __restrict__ tile_sum) {
  __shared__ unsigned long long tmp[SCAN_T / WAVE + 1];
  const uint64_t t0 = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  unsigned long long x[SCAN_ITEMS], s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    x[i] = t0 + i < n ? v[t0 + i] : 0ull;
    s += x[i];
  }
  unsigned long long tot;
  unsigned long long e = block_excl_scan<SCAN_T>(s, tmp, &tot);
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (t0 + i < n) v[t0 + i] = e;
    e += x[i];
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024)
k_scan_tile_sums(unsigned long long* __restrict__ t, uint64_t n, unsigned long long* __restrict__ total) {
  __shared__ unsigned long long tmp[1024 / WAVE + 1];
  unsigned long long carry = 0;
  for (uint64_t b0 = 0; b0 < n; b0 += 1024) {
    const uint64_t b = b0 + threadIdx.x;
    const unsigned long long x = b < n ? t[b] : 0ull;
    unsigned long long s;
    const unsigned long long e = block_excl_scan<1024>(x, tmp, &s);
    if (b < n) t[b] = carry + e;
    carry += s;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void __launch_bounds__(SCAN_T)
k_scan_add(unsigned long long* __restrict__ v, uint64_t n, const unsigned long long* __restrict__ tile_off) {
  const uint64_t t0 = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  const unsigned long long a = tile_off[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (t0 + i < n) v[t0 + i] += a;
}

// Unified context of every key: binary search of its pc among the unified
// contexts of its ctx.
__global__ void __launch_bounds__(B)
k_unified_id(const ProfDev* __restrict__ pd, uint32_t P, uint64_t K, const uint64_t* __restrict__ u_off,
             const uint64_t* __restrict__ u_pc, uint32_t* __restrict__ uid, unsigned int* __restrict__ err) {
  for (uint64_t k = (uint64_t)blockIdx.x * B + threadIdx.x; k < K; k += (uint64_t)gridDim.x * B) {
    const ProfDev d = pd[profile_of(pd, P, k)];
    const uint64_t i = k - d.base;
    const uint64_t pcv = d.pc[i];
    uint64_t lo = u_off[d.ctx[i]], hi = u_off[d.ctx[i] + 1];
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (u_pc[mid] < pcv) lo = mid + 1;
      else hi = mid;
    }
    if (lo >= u_off[d.ctx[i] + 1] || u_pc[lo] != pcv || d.stall[i] >= NS) atomicOr(err, 1u);
    uid[k] = (uint32_t)lo;
  }
}

// per (unified context, metric): number of profiles with a non-zero value
__global__ void __launch_bounds__(B)
k_cm_count(const ProfDev* __restrict__ pd, uint32_t P, uint64_t K, const uint32_t* __restrict__ uid,
           unsigned long long* __restrict__ cm) {
  for (uint64_t k = (uint64_t)blockIdx.x * B + threadIdx.x; k < K; k += (uint64_t)gridDim.x * B) {
    const ProfDev d = pd[profile_of(pd, P, k)];
    const uint32_t s = d.stall[k - d.base];
    if (s < NS && d.count[k - d.base] > 0) atomicAdd(&cm[(uint64_t)uid[k] * NS + s], 1ull);
  }
}

// non-empty metrics per unified context
__global__ void __launch_bounds__(B)
k_ctx_metrics(const unsigned long long* __restrict__ cm, uint64_t U, unsigned long long* __restrict__ nm) {
  const uint64_t c = (uint64_t)blockIdx.x * B + threadIdx.x;
  if (c >= U) return;
  unsigned long long m = 0;
  for (int s = 0; s < NS; ++s) m += cm[c * NS + s] > 0;
  nm[c] = m;
}

// midx pairs and the context offsets of CMS; `start` is the scanned cm array
__global__ void __launch_bounds__(B)
k_midx(const unsigned long long* __restrict__ cnt, const unsigned long long* __restrict__ start, uint64_t U,
       const unsigned long long* __restrict__ m_off, uint64_t K, uint8_t* __restrict__ o_mid,
       uint64_t* __restrict__ o_mstart, uint32_t* __restrict__ o_mctx, uint64_t* __restrict__ ctx_off) {
  const uint64_t c = (uint64_t)blockIdx.x * B + threadIdx.x;
  if (c > U) return;
  ctx_off[c] = c < U ? start[c * NS] : K;
  if (c == U) return;
  uint64_t o = m_off[c];
  for (int s = 0; s < NS; ++s)
    if (cnt[c * NS + s] > 0) {
      o_mid[o] = (uint8_t)s;
      o_mstart[o] = start[c * NS + s];
      o_mctx[o] = (uint32_t)c;
      ++o;
    }
}

// entries of one profile into the CMS arrays; cursors advance in profile order
__global__ void __launch_bounds__(B)
k_cms_scatter(ProfDev d, uint32_t p, const uint32_t* __restrict__ uid, unsigned long long* __restrict__ cur,
              uint32_t* __restrict__ o_pid, unsigned long long* __restrict__ o_val) {
  const uint64_t i = (uint64_t)blockIdx.x * B + threadIdx.x;
  if (i >= d.n) return;
  const uint32_t s = d.stall[i];
  const unsigned long long c = d.count[i];
  if (s >= NS || c == 0) return;
  const uint64_t cell = (uint64_t)uid[d.base + i] * NS + s;
  const uint64_t o = cur[cell];  // each (context, metric) occurs once per profile
  cur[cell] = o + 1;
  o_pid[o] = p;
  o_val[o] = c;
}

// statistics per non-empty (context, metric), entries in profile order
__global__ void __launch_bounds__(B)
k_stats(const uint64_t* __restrict__ mstart, uint64_t n_midx, uint64_t nnz, const unsigned long long* __restrict__ val,
        uint32_t P, unsigned long long* __restrict__ s_sum, unsigned long long* __restrict__ s_min,
        unsigned long long* __restrict__ s_max, double* __restrict__ s_mean, double* __restrict__ s_std,
        double* __restrict__ s_cov) {
  const uint64_t j = (uint64_t)blockIdx.x * B + threadIdx.x;
  if (j >= n_midx) return;
  const uint64_t a = mstart[j], e = j + 1 < n_midx ? mstart[j + 1] : nnz;
  unsigned long long sum = 0, mn = ~0ull, mx = 0;
  for (uint64_t i = a; i < e; ++i) {
    const unsigned long long x = val[i];
    sum += x;
    mn = x < mn ? x : mn;
    mx = x > mx ? x : mx;
  }
  const uint64_t present = e - a;
  if (present < P) mn = 0;
  const double mean = (double)sum / (double)P;
  double ss = 0.0;
  for (uint64_t i = a; i < e; ++i) {
    const double d = (double)val[i] - mean;
    ss = ss + d * d;
  }
  ss = ss + (double)(P - present) * (mean * mean);
  const double sd = sqrt(ss / (double)P);
  s_sum[j] = sum;
  s_min[j] = mn;
  s_max[j] = mx;
  s_mean[j] = mean;
  s_std[j] = sd;
  s_cov[j] = mean > 0.0 ? sd / mean : 0.0;
}

// PMS: context heads within each profile's keys
__global__ void __launch_bounds__(B)
k_pms_heads(const ProfDev* __restrict__ pd, uint32_t P, uint64_t K, const uint32_t* __restrict__ uid,
            unsigned long long* __restrict__ head) {
  for (uint64_t k = (uint64_t)blockIdx.x * B + threadIdx.x; k < K; k += (uint64_t)gridDim.x * B) {
    const ProfDev d = pd[profile_of(pd, P, k)];
    head[k] = (k == d.base || uid[k] != uid[k - 1]) ? 1ull : 0ull;
  }
}

__global__ void __launch_bounds__(B)
k_pms_write(const ProfDev* __restrict__ pd, uint32_t P, uint64_t K, const uint32_t* __restrict__ uid,
            const unsigned long long* __restrict__ head_off, uint64_t n_heads, uint32_t* __restrict__ o_ctx,
            uint64_t* __restrict__ o_cstart, uint8_t* __restrict__ o_mid, unsigned long long* __restrict__ o_val) {
  for (uint64_t k = (uint64_t)blockIdx.x * B + threadIdx.x; k < K; k += (uint64_t)gridDim.x * B) {
    const ProfDev d = pd[profile_of(pd, P, k)];
    const bool h = k == d.base || uid[k] != uid[k - 1];
    if (h) {
      o_ctx[head_off[k]] = uid[k];
      o_cstart[head_off[k]] = k;
    }
    o_mid[k] = d.stall[k - d.base];
    o_val[k] = d.count[k - d.base];
  }
}

__global__ void k_pms_offsets(const ProfDev* __restrict__ pd, uint32_t P, uint64_t K,
                              const unsigned long long* __restrict__ head_off, uint64_t n_heads,
                              uint64_t* __restrict__ off, uint64_t* __restrict__ c_off) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > P) return;
  if (p == P) {
    off[P] = K;
    c_off[P] = n_heads;
    return;
  }
  off[p] = pd[p].base;
  c_off[p] = pd[p].base < K ? head_off[pd[p].base] : n_heads;
}

}  // namespace

// In-place exclusive scan of n u64 values on `s`; *d_total (device) receives the sum.
void exscan_u64(hpa_ctx* ctx, unsigned long long* v, uint64_t n, unsigned long long* d_total, hipStream_t s) {
  const uint64_t tiles = std::max<uint64_t>((n + SCAN_TILE - 1) / SCAN_TILE, 1);
  DBuf ts(ctx, tiles * 8, s);
  k_scan_tiles<<<(unsigned)tiles, SCAN_T, 0, s>>>(v, n, ts.as<unsigned long long>());
  k_scan_tile_sums<<<1, 1024, 0, s>>>(ts.as<unsigned long long>(), tiles, d_total);
  k_scan_add<<<(unsigned)tiles, SCAN_T, 0, s>>>(v, n, ts.as<unsigned long long>());
  HPA_HIP(hipGetLastError());
}

}  // namespace hpa

using namespace hpa;

struct hpa_unified {
  hpa_ctx* ctx = nullptr;
  uint32_t n_profiles = 0;
  uint64_t n_keys = 0, n_midx = 0, n_heads = 0;
  hpa_attribution* u = nullptr;  // unified contexts (ctx, pc, scope; count = entries)
  DBuf cms_ctx_off, cms_m_off, cms_mid, cms_mstart, cms_mctx, cms_pid, cms_val;
  DBuf pms_off, pms_c_off, pms_ctx, pms_cstart, pms_mid, pms_val;
  DBuf st_sum, st_min, st_max, st_mean, st_std, st_cov;
  ~hpa_unified() {
    if (u) hpa_attribution_free(u);
  }
};

namespace {

// Profiles' key arrays as device descriptors; checks that they agree.
std::vector<ProfDev> profile_descs(hpa_ctx* ctx, uint32_t P, const hpa_attribution* const* a, uint64_t* K) {
  if (P == 0 || !a) fail(HPA_E_INVAL, "need at least one attribution");
  std::vector<ProfDev> pd(P);
  uint64_t base = 0;
  for (uint32_t p = 0; p < P; ++p) {
    if (!a[p]) fail(HPA_E_INVAL, "NULL attribution");
    if (a[p]->ctx != ctx) fail(HPA_E_INVAL, "attribution belongs to another context");
    if (a[p]->map != a[0]->map || a[p]->n_ctx != a[0]->n_ctx)
      fail(HPA_E_INVAL, "attributions use different structure maps or context counts");
    pd[p] = ProfDev{a[p]->ctx_id.as<uint32_t>(), a[p]->pc.as<uint64_t>(), a[p]->stall.as<uint8_t>(),
                    a[p]->count.as<unsigned long long>(), a[p]->n_keys, base};
    base += a[p]->n_keys;
  }
  *K = base;
  return pd;
}

// Records of every key (see k_records) attributed on the profiles' map.
hpa_attribution* records_attribution(hpa_ctx* ctx, const hpa_attribution* a0, const DBuf& d_pd, uint32_t P,
                                     uint64_t K, int unit, hipStream_t s) {
  const unsigned g = grid_for(K, B, ctx->n_cu * 16);
  DBuf nrec(ctx, std::max<uint64_t>(K, 1) * 8, s), tot(ctx, 8, s);
  HPA_HIP(hipMemsetAsync(tot.p, 0, 8, s));
  uint64_t R = K;
  if (K) {
    k_records<<<g, B, 0, s>>>(d_pd.as<ProfDev>(), P, K, unit, 0, nrec.as<unsigned long long>(), nullptr, nullptr,
                              nullptr, nullptr);
    exscan_u64(ctx, nrec.as<unsigned long long>(), K, tot.as<unsigned long long>(), s);
    unsigned long long r = 0;
    HPA_HIP(hipMemcpyAsync(&r, tot.p, 8, hipMemcpyDeviceToHost, s));
    sync_stream(ctx, s);
    R = r;
  }
  const uint64_t R1 = std::max<uint64_t>(R, 1);
  DBuf r_pc(ctx, R1 * 8, s), r_ctx(ctx, R1 * 4, s), r_st(ctx, R1, s), r_w(ctx, R1 * 4, s);
  if (K) {
    k_records<<<g, B, 0, s>>>(d_pd.as<ProfDev>(), P, K, unit, 1, nrec.as<unsigned long long>(), r_pc.as<uint64_t>(),
                              r_ctx.as<uint32_t>(), r_st.as<uint8_t>(), r_w.as<uint32_t>());
    HPA_HIP(hipGetLastError());
  }
  hpa_samples smp{r_pc.as<uint64_t>(), r_ctx.as<uint32_t>(), r_st.as<uint8_t>(), r_w.as<uint32_t>(), R,
                  a0->n_ctx};
  hpa_attribution* out = nullptr;
  const hpa_status rc = hpa_attribute(ctx, a0->map, &smp, s, &out);
  if (rc != HPA_OK) fail(rc, hpa_last_error());
  return out;
}

}  // namespace

extern "C" hpa_status hpa_unify_profiles(hpa_ctx* ctx, uint32_t n_profiles, const hpa_attribution* const* attrs,
                                         hipStream_t stream, hpa_unified** out) {
  return guard([&] {
    if (!ctx || !out) fail(HPA_E_INVAL, "NULL argument");
    DeviceGuard dg(ctx->device);
    hipStream_t s = stream;
    uint64_t K = 0;
    std::vector<ProfDev> pd = profile_descs(ctx, n_profiles, attrs, &K);
    const uint32_t P = n_profiles;
    auto* R = new hpa_unified();
    std::unique_ptr<hpa_unified> hold(R);
    R->ctx = ctx;
    R->n_profiles = P;
    R->n_keys = K;
    DBuf d_pd = upload(ctx, pd, s);
    // unified contexts
    R->u = records_attribution(ctx, attrs[0], d_pd, P, K, 1, s);
    const uint64_t U = R->u->n_keys;
    const unsigned g = grid_for(K, B, ctx->n_cu * 16);
    const uint64_t K1 = std::max<uint64_t>(K, 1), U1 = std::max<uint64_t>(U, 1);
    DBuf uid(ctx, K1 * 4, s), err(ctx, 8, s);
    HPA_HIP(hipMemsetAsync(err.p, 0, 8, s));
    // CMS counts, starts, midx pairs
    DBuf cm(ctx, U1 * NS * 8, s), cmst(ctx, U1 * NS * 8, s), nm(ctx, (U1 + 1) * 8, s), tot(ctx, 16, s);
    HPA_HIP(hipMemsetAsync(cm.p, 0, U1 * NS * 8, s));
    HPA_HIP(hipMemsetAsync(tot.p, 0, 16, s));
    if (K) {
      k_unified_id<<<g, B, 0, s>>>(d_pd.as<ProfDev>(), P, K, R->u->ctx_offsets.as<uint64_t>(),
                                   R->u->pc.as<uint64_t>(), uid.as<uint32_t>(), err.as<unsigned int>());
      k_cm_count<<<g, B, 0, s>>>(d_pd.as<ProfDev>(), P, K, uid.as<uint32_t>(), cm.as<unsigned long long>());
      HPA_HIP(hipGetLastError());
    }
    HPA_HIP(hipMemcpyAsync(cmst.p, cm.p, U1 * NS * 8, hipMemcpyDeviceToDevice, s));
    exscan_u64(ctx, cmst.as<unsigned long long>(), U * NS, tot.as<unsigned long long>(), s);
    k_ctx_metrics<<<grid_for(U, B), B, 0, s>>>(cm.as<unsigned long long>(), U, nm.as<unsigned long long>());
    exscan_u64(ctx, nm.as<unsigned long long>(), U, tot.as<unsigned long long>() + 1, s);
    unsigned long long sizes[2] = {0, 0};
    unsigned int e = 0;
    HPA_HIP(hipMemcpyAsync(sizes, tot.p, 16, hipMemcpyDeviceToHost, s));
    HPA_HIP(hipMemcpyAsync(&e, err.p, 4, hipMemcpyDeviceToHost, s));
    sync_stream(ctx, s);
    if (e) fail(HPA_E_INVAL, "a key of some profile is missing from the union (duplicate or unsorted keys?)");
    const uint64_t nnz = sizes[0], NM = sizes[1];
    R->n_midx = NM;
    const uint64_t NM1 = std::max<uint64_t>(NM, 1), NZ1 = std::max<uint64_t>(nnz, 1);
    R->cms_ctx_off = DBuf(ctx, (U + 1) * 8, s);
    R->cms_m_off = DBuf(ctx, (U + 1) * 8, s);
    R->cms_mid = DBuf(ctx, NM1, s);
    R->cms_mstart = DBuf(ctx, NM1 * 8, s);
    R->cms_mctx = DBuf(ctx, NM1 * 4, s);
    R->cms_pid = DBuf(ctx, NZ1 * 4, s);
    R->cms_val = DBuf(ctx, NZ1 * 8, s);
    k_midx<<<grid_for(U + 1, B), B, 0, s>>>(cm.as<unsigned long long>(), cmst.as<unsigned long long>(), U,
                                            nm.as<unsigned long long>(), nnz, R->cms_mid.as<uint8_t>(),
                                            R->cms_mstart.as<uint64_t>(), R->cms_mctx.as<uint32_t>(),
                                            R->cms_ctx_off.as<uint64_t>());
    // m_off: the scanned metric counts, closed with the total
    HPA_HIP(hipMemcpyAsync(R->cms_m_off.p, nm.p, U * 8, hipMemcpyDeviceToDevice, s));
    HPA_HIP(hipMemcpyAsync(R->cms_m_off.as<uint64_t>() + U, tot.as<unsigned long long>() + 1, 8,
                           hipMemcpyDeviceToDevice, s));
    HPA_HIP(hipGetLastError());
    for (uint32_t p = 0; p < P; ++p) {
      if (!pd[p].n) continue;
      k_cms_scatter<<<grid_for(pd[p].n, B, 1u << 30), B, 0, s>>>(pd[p], p, uid.as<uint32_t>(),
                                                                 cmst.as<unsigned long long>(),
                                                                 R->cms_pid.as<uint32_t>(),
                                                                 R->cms_val.as<unsigned long long>());
    }
    HPA_HIP(hipGetLastError());
    // statistics per (context, metric)
    R->st_sum = DBuf(ctx, NM1 * 8, s);
    R->st_min = DBuf(ctx, NM1 * 8, s);
    R->st_max = DBuf(ctx, NM1 * 8, s);
    R->st_mean = DBuf(ctx, NM1 * 8, s);
    R->st_std = DBuf(ctx, NM1 * 8, s);
    R->st_cov = DBuf(ctx, NM1 * 8, s);
    if (NM)
      k_stats<<<grid_for(NM, B, 1u << 30), B, 0, s>>>(R->cms_mstart.as<uint64_t>(), NM, nnz,
                                                      R->cms_val.as<unsigned long long>(), P,
                                                      R->st_sum.as<unsigned long long>(),
                                                      R->st_min.as<unsigned long long>(),
                                                      R->st_max.as<unsigned long long>(), R->st_mean.as<double>(),
                                                      R->st_std.as<double>(), R->st_cov.as<double>());
    // PMS
    DBuf head(ctx, K1 * 8, s), htot(ctx, 8, s);
    HPA_HIP(hipMemsetAsync(htot.p, 0, 8, s));
    if (K) {
      k_pms_heads<<<g, B, 0, s>>>(d_pd.as<ProfDev>(), P, K, uid.as<uint32_t>(), head.as<unsigned long long>());
      exscan_u64(ctx, head.as<unsigned long long>(), K, htot.as<unsigned long long>(), s);
    }
    unsigned long long nh = 0;
    HPA_HIP(hipMemcpyAsync(&nh, htot.p, 8, hipMemcpyDeviceToHost, s));
    sync_stream(ctx, s);
    R->n_heads = nh;
    const uint64_t NH1 = std::max<uint64_t>(nh, 1);
    R->pms_off = DBuf(ctx, ((uint64_t)P + 1) * 8, s);
    R->pms_c_off = DBuf(ctx, ((uint64_t)P + 1) * 8, s);
    R->pms_ctx = DBuf(ctx, NH1 * 4, s);
    R->pms_cstart = DBuf(ctx, NH1 * 8, s);
    R->pms_mid = DBuf(ctx, K1, s);
    R->pms_val = DBuf(ctx, K1 * 8, s);
    if (K)
      k_pms_write<<<g, B, 0, s>>>(d_pd.as<ProfDev>(), P, K, uid.as<uint32_t>(), head.as<unsigned long long>(), nh,
                                  R->pms_ctx.as<uint32_t>(), R->pms_cstart.as<uint64_t>(), R->pms_mid.as<uint8_t>(),
                                  R->pms_val.as<unsigned long long>());
    k_pms_offsets<<<(P + 1 + 255) / 256, 256, 0, s>>>(d_pd.as<ProfDev>(), P, K, head.as<unsigned long long>(), nh,
                                                     R->pms_off.as<uint64_t>(), R->pms_c_off.as<uint64_t>());
    HPA_HIP(hipGetLastError());
    sync_stream(ctx, s);
    *out = hold.release();
  });
}

extern "C" hpa_status hpa_unified_view_get(const hpa_unified* u, hpa_unified_view* v) {
  return guard([&] {
    if (!u || !v) fail(HPA_E_INVAL, "NULL argument");
    v->n_profiles = u->n_profiles;
    v->n_contexts = u->u->n_keys;
    v->n_nonzeros = u->n_keys;
    v->n_metric_entries = u->n_midx;
    v->n_profile_contexts = u->n_heads;
    v->ctx = u->u->ctx_id.as<uint32_t>();
    v->pc = u->u->pc.as<uint64_t>();
    v->scope = u->u->scope.as<uint32_t>();
    v->cms_ctx_off = u->cms_ctx_off.as<uint64_t>();
    v->cms_m_off = u->cms_m_off.as<uint64_t>();
    v->cms_mid = u->cms_mid.as<uint8_t>();
    v->cms_mstart = u->cms_mstart.as<uint64_t>();
    v->cms_mctx = u->cms_mctx.as<uint32_t>();
    v->cms_pid = u->cms_pid.as<uint32_t>();
    v->cms_val = u->cms_val.as<uint64_t>();
    v->pms_off = u->pms_off.as<uint64_t>();
    v->pms_c_off = u->pms_c_off.as<uint64_t>();
    v->pms_ctx = u->pms_ctx.as<uint32_t>();
    v->pms_cstart = u->pms_cstart.as<uint64_t>();
    v->pms_mid = u->pms_mid.as<uint8_t>();
    v->pms_val = u->pms_val.as<uint64_t>();
    v->st_sum = u->st_sum.as<uint64_t>();
    v->st_min = u->st_min.as<uint64_t>();
    v->st_max = u->st_max.as<uint64_t>();
    v->st_mean = u->st_mean.as<double>();
    v->st_std = u->st_std.as<double>();
    v->st_cov = u->st_cov.as<double>();
  });
}

extern "C" void hpa_unified_free(hpa_unified* u) { delete u; }

namespace {

// Write `bytes` of device memory at file offset `off`, through a host bounce
// buffer of at most `round` bytes per step.
void write_section(hpa_ctx* ctx, FILE* f, uint64_t off, const void* dev, uint64_t bytes,
                   std::vector<uint8_t>& bounce, hipStream_t s) {
  uint64_t done = 0;
  while (done < bytes) {
    const uint64_t k = std::min<uint64_t>(bounce.size(), bytes - done);
    HPA_HIP(hipMemcpyAsync(bounce.data(), static_cast<const uint8_t*>(dev) + done, k, hipMemcpyDeviceToHost, s));
    sync_stream(ctx, s);
    if (fseeko(f, (off_t)(off + done), SEEK_SET) != 0 || fwrite(bounce.data(), 1, k, f) != k)
      fail(HPA_E_DEVICE, "writing the sparse file failed");
    done += k;
  }
}

}  // namespace

extern "C" hpa_status hpa_unified_write(const hpa_unified* u, const char* path, int format, uint64_t round_bytes,
                                        hipStream_t stream) {
  return guard([&] {
    if (!u || !path) fail(HPA_E_INVAL, "NULL argument");
    if (format != HPA_SPARSE_CMS && format != HPA_SPARSE_PMS) fail(HPA_E_INVAL, "unknown sparse format");
    DeviceGuard dg(u->ctx->device);
    const uint64_t round = std::max<uint64_t>(round_bytes ? round_bytes : (64ull << 20), 4096);
    std::vector<uint8_t> bounce(round);
    const uint64_t U = u->u->n_keys, K = u->n_keys, P = u->n_profiles;
    struct Sec {
      const void* p;
      uint64_t bytes;
    };
    std::vector<Sec> secs;
    secs.push_back({u->u->ctx_id.p, U * 4});
    secs.push_back({u->u->pc.p, U * 8});
    if (format == HPA_SPARSE_CMS) {
      secs.push_back({u->cms_ctx_off.p, (U + 1) * 8});
      secs.push_back({u->cms_m_off.p, (U + 1) * 8});
      secs.push_back({u->cms_mid.p, u->n_midx});
      secs.push_back({u->cms_mstart.p, u->n_midx * 8});
      secs.push_back({u->cms_pid.p, K * 4});
      secs.push_back({u->cms_val.p, K * 8});
    } else {
      secs.push_back({u->pms_off.p, (P + 1) * 8});
      secs.push_back({u->pms_c_off.p, (P + 1) * 8});
      secs.push_back({u->pms_ctx.p, u->n_heads * 4});
      secs.push_back({u->pms_cstart.p, u->n_heads * 8});
      secs.push_back({u->pms_mid.p, K});
      secs.push_back({u->pms_val.p, K * 8});
    }
    // header, then each section at an 8-aligned offset (an exclusive scan of the sizes)
    uint64_t hdr[8] = {0x45535241505350ull /* "PSPARSE" */, (uint64_t)format, U, P, NS, K,
                       format == HPA_SPARSE_CMS ? u->n_midx : u->n_heads, (uint64_t)secs.size()};
    std::vector<uint64_t> off(secs.size());
    uint64_t o = sizeof(hdr) + 8 * secs.size();
    for (size_t i = 0; i < secs.size(); ++i) {
      off[i] = o;
      o += (secs[i].bytes + 7) & ~7ull;
    }
    FILE* f = fopen(path, "wb");
    if (!f) fail(HPA_E_INVAL, std::string("cannot open ") + path);
    std::unique_ptr<FILE, int (*)(FILE*)> hold(f, fclose);
    if (fwrite(hdr, 8, 8, f) != 8 || fwrite(off.data(), 8, off.size(), f) != off.size())
      fail(HPA_E_DEVICE, "writing the sparse file header failed");
    for (size_t i = 0; i < secs.size(); ++i)
      if (secs[i].bytes) write_section(u->ctx, f, off[i], secs[i].p, secs[i].bytes, bounce, stream);
  });
}

extern "C" hpa_status hpa_combine_runs(hpa_ctx* ctx, uint32_t n_runs, const hpa_attribution* const* runs,
                                       hipStream_t stream, hpa_attribution** out) {
  return guard([&] {
    if (!ctx || !out) fail(HPA_E_INVAL, "NULL argument");
    DeviceGuard dg(ctx->device);
    uint64_t K = 0;
    std::vector<ProfDev> pd = profile_descs(ctx, n_runs, runs, &K);
    DBuf d_pd = upload(ctx, pd, stream);
    *out = records_attribution(ctx, runs[0], d_pd, n_runs, K, 0, stream);
  });
}
