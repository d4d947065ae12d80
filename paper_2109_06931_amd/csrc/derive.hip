// A6: derived metrics (Section 6.1 "Statistic Generation": values propagate up
// the calling context tree; Section 7.1: warp issue rate W = (S - S_stall) / S,
// S the total samples and S_stall the stalled ones; reason 0 is "not stalled").
//
//   k_cct_incl    one workgroup per context: inclusive value of every GPU CCT
//                 node, deepest level first; a node adds its children's
//                 inclusive rows in child order (children are found from the
//                 preorder layout and subtree sizes); then S and W.
//   k_host_own    per context: its own samples per stall reason.
//   k_host_up     one workgroup: host calling-context tree, deepest contexts
//                 first, integer sums into the parent; then W per context.
//   k_scope       one workgroup per context: for every scope on the ancestor
//                 chain of a sampled scope, the samples of the scope and all
//                 scopes nested in it (integer), rows by ascending scope id,
//                 unmapped PCs last; counted, scanned, then written.
#include <memory>

#include "block_prims.h"
#include "hpa_internal.h"

// accessors defined in apportion.hip
struct hpa_gpu_cct;
struct hpa_callgraph_plan;
namespace hpa {
const uint64_t* cct_node_off(const hpa_gpu_cct* t);
const uint64_t* cct_size(const hpa_gpu_cct* t);
const uint32_t* cct_depth(const hpa_gpu_cct* t);
const double* cct_excl(const hpa_gpu_cct* t);
uint64_t cct_n_nodes(const hpa_gpu_cct* t);
const hpa_callgraph_plan* cct_plan(const hpa_gpu_cct* t);
const hpa_attribution* cct_attr(const hpa_gpu_cct* t);
uint32_t plan_n_ctx(const hpa_callgraph_plan* p);
const hpa_structure_map* plan_map(const hpa_callgraph_plan* p);
const uint32_t* plan_ctx_parent(const hpa_callgraph_plan* p);
const uint32_t* plan_depth_order(const hpa_callgraph_plan* p);
const std::vector<uint32_t>& plan_h_depth(const hpa_callgraph_plan* p);
const std::vector<uint32_t>& plan_h_depth_order(const hpa_callgraph_plan* p);
const uint32_t* plan_depth_lvl(const hpa_callgraph_plan* p);
uint32_t plan_n_depth_lvl(const hpa_callgraph_plan* p);
}  // namespace hpa

namespace hpa {
namespace {

constexpr int DBLOCK = 256;
// error bits raised by the kernels (checked by the host)
constexpr unsigned int ERR_SCOPE = 1, ERR_STALL = 2, ERR_TREE = 4;

__device__ inline double issue_rate(double S, double Sst) { return S == 0.0 ? 0.0 : (S - Sst) / S; }

__global__ void __launch_bounds__(DBLOCK)
k_cct_incl(const uint64_t* __restrict__ node_off, const uint64_t* __restrict__ size, const uint32_t* __restrict__ depth,
           const double* __restrict__ excl, uint32_t n_ctx, unsigned int* ticket, double* __restrict__ incl,
           double* __restrict__ S_out, double* __restrict__ W_out, unsigned int* err) {
  __shared__ uint32_t s_c, s_maxd;
  while (true) {
    if (threadIdx.x == 0) { s_c = atomicAdd(ticket, 1u); s_maxd = 0; }
    __syncthreads();
    const uint32_t c = s_c;
    if (c >= n_ctx) break;
    const uint64_t b = node_off[c], e = node_off[c + 1];
    uint32_t md = 0;
    for (uint64_t i = b + threadIdx.x; i < e; i += DBLOCK) md = max(md, depth[i]);
    md = wave_max(md);
    if (lane_id() == 0) atomicMax(&s_maxd, md);
    __syncthreads();
    const uint32_t maxd = s_maxd;
    for (int d = (int)maxd; d >= 0 && e > b; --d) {
      for (uint64_t i = b + threadIdx.x; i < e; i += DBLOCK) {
        if (depth[i] != (uint32_t)d) continue;
        double v[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) v[s] = excl[i * NS + s];
        const uint64_t end = i + size[i];
        if (size[i] == 0 || end > e) { atomicOr(err, ERR_TREE); continue; }
        for (uint64_t ch = i + 1; ch < end; ch += size[ch]) {
          if (size[ch] == 0) { atomicOr(err, ERR_TREE); break; }
#pragma unroll
          for (int s = 0; s < NS; ++s) v[s] = v[s] + incl[ch * NS + s];
        }
        double S = 0.0, Sst = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          incl[i * NS + s] = v[s];
          S = S + v[s];
        }
#pragma unroll
        for (int s = 1; s < NS; ++s) Sst = Sst + v[s];
        S_out[i] = S;
        W_out[i] = issue_rate(S, Sst);
      }
      __threadfence_block();
      __syncthreads();
    }
    __syncthreads();
  }
}

// own samples per context and stall
__global__ void __launch_bounds__(DBLOCK)
k_host_own(const uint64_t* __restrict__ ctx_off, const uint8_t* __restrict__ stall,
           const unsigned long long* __restrict__ count, uint32_t n_ctx, unsigned long long* __restrict__ own,
           unsigned int* err) {
  __shared__ unsigned long long s_row[NS];
  for (uint32_t c = blockIdx.x; c < n_ctx; c += gridDim.x) {
    if (threadIdx.x < NS) s_row[threadIdx.x] = 0;
    __syncthreads();
    for (uint64_t k = ctx_off[c] + threadIdx.x; k < ctx_off[c + 1]; k += DBLOCK) {
      if (stall[k] < NS) atomicAdd(&s_row[stall[k]], count[k]);
      else atomicOr(err, ERR_STALL);
    }
    __syncthreads();
    if (threadIdx.x < NS) own[(uint64_t)c * NS + threadIdx.x] = s_row[threadIdx.x];
    __syncthreads();
  }
}

// host tree, deepest contexts first: order = contexts by descending depth,
// lvl = offsets of each depth group in `order`
__global__ void __launch_bounds__(1024)
k_host_up(const uint32_t* __restrict__ order, const uint32_t* __restrict__ lvl, uint32_t n_lvl,
          const uint32_t* __restrict__ parent, uint32_t n_ctx, unsigned long long* __restrict__ incl,
          double* __restrict__ W) {
  for (uint32_t l = 0; l < n_lvl; ++l) {
    for (uint32_t i = lvl[l] + threadIdx.x; i < lvl[l + 1]; i += 1024) {
      const uint32_t c = order[i], p = parent[c];
      if (p == NONE32) continue;
      for (int s = 0; s < NS; ++s) {
        unsigned long long v = incl[(uint64_t)c * NS + s];
        if (v) atomicAdd(&incl[(uint64_t)p * NS + s], v);
      }
    }
    __threadfence();
    __syncthreads();
  }
  for (uint32_t c = threadIdx.x; c < n_ctx; c += 1024) {
    unsigned long long S = 0, Sst = 0;
    for (int s = 0; s < NS; ++s) S += incl[(uint64_t)c * NS + s];
    for (int s = 1; s < NS; ++s) Sst += incl[(uint64_t)c * NS + s];
    W[c] = issue_rate((double)S, (double)Sst);
  }
}

// static scope roll-up per context.  Per workgroup: row_of (one word per scope
// id, NONE between contexts), row_id (scope id of each row) and the rows.
// (a) every key marks its scope and each enclosing scope; (b) a scan over the
// ids gives the marked ones dense rows in id order; (c) every key adds its
// samples along the chain; (d) rows are counted or written, and the marks are
// cleared.  Marks are atomic stores of one value; barriers order the passes.
struct ScopeArgs {
  const uint32_t* sparent;   // map scope table: parent
  uint32_t n_ids;
  const uint64_t* ctx_off;
  const uint32_t* k_scope;
  const uint8_t* k_stall;
  const unsigned long long* k_count;
  uint32_t n_ctx;
  unsigned int* ticket;
  uint8_t* ws;
  uint64_t ws_stride;
  unsigned long long* n_rows;  // counting pass
  const uint64_t* row_off;     // emission pass
  uint32_t* o_scope;
  unsigned long long* o_val;
  unsigned int* err;           // ERR_* bits
  int emit;
};


// byte offsets inside one workgroup's workspace
__host__ __device__ inline uint64_t scope_ids_off(uint32_t n_ids) { return ((uint64_t)n_ids * 4 + 255) & ~255ull; }
__host__ __device__ inline uint64_t scope_rows_off(uint32_t n_ids) { return 2 * scope_ids_off(n_ids); }
__host__ __device__ inline uint64_t scope_ws_stride(uint32_t n_ids) {
  return scope_rows_off(n_ids) + (uint64_t)n_ids * NS * 8;
}

__global__ void __launch_bounds__(DBLOCK) k_scope(ScopeArgs a) {
  __shared__ uint32_t s_c;
  __shared__ unsigned long long s_unm[NS];
  __shared__ uint32_t s_tmp[DBLOCK / WAVE + 1];
  uint8_t* ws = a.ws + (uint64_t)blockIdx.x * a.ws_stride;
  uint32_t* row_of = reinterpret_cast<uint32_t*>(ws);
  uint32_t* row_id = reinterpret_cast<uint32_t*>(ws + scope_ids_off(a.n_ids));
  unsigned long long* rows = reinterpret_cast<unsigned long long*>(ws + scope_rows_off(a.n_ids));
  while (true) {
    if (threadIdx.x == 0) s_c = atomicAdd(a.ticket, 1u);
    if (threadIdx.x < NS) s_unm[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t c = s_c;
    if (c >= a.n_ctx) break;
    const uint64_t k0 = a.ctx_off[c], k1 = a.ctx_off[c + 1];
    // (a) marks
    for (uint64_t k = k0 + threadIdx.x; k < k1; k += DBLOCK) {
      uint32_t x = a.k_scope[k];
      for (uint32_t steps = 0; x != NONE32; ++steps) {
        if (x >= a.n_ids || steps >= a.n_ids) { atomicOr(a.err, ERR_SCOPE); break; }
        __hip_atomic_store(&row_of[x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = a.sparent[x];
      }
    }
    // hand-overs of workspace words between threads: device-scope fence, then
    // the barrier (stores and atomics reach the L2; this CU's L1 is invalidated)
    __threadfence();
    __syncthreads();
    // (b) dense rows in id order
    uint32_t nrows = 0;
    for (uint32_t i0 = 0; i0 < a.n_ids; i0 += DBLOCK) {
      const uint32_t i = i0 + threadIdx.x;
      const uint32_t used =
          (i < a.n_ids && __hip_atomic_load(&row_of[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != NONE32) ? 1u
                                                                                                             : 0u;
      uint32_t t;
      const uint32_t r = nrows + block_excl_scan<DBLOCK>(used, s_tmp, &t);
      if (used) {
        row_of[i] = r;
        row_id[r] = i;
        for (int s = 0; s < NS; ++s) rows[(uint64_t)r * NS + s] = 0;
      }
      nrows += t;
    }
    __threadfence();
    __syncthreads();
    // (c) sums along the chains
    for (uint64_t k = k0 + threadIdx.x; k < k1; k += DBLOCK) {
      uint32_t x = a.k_scope[k];
      const uint32_t st = a.k_stall[k];
      const unsigned long long cnt = a.k_count[k];
      if (st >= NS) { atomicOr(a.err, ERR_STALL); continue; }
      if (x == NONE32) { atomicAdd(&s_unm[st], cnt); continue; }
      for (uint32_t steps = 0; x != NONE32 && x < a.n_ids && steps < a.n_ids; ++steps) {
        const uint32_t r = row_of[x];
        if (r >= nrows) { atomicOr(a.err, ERR_SCOPE); break; }
        atomicAdd(&rows[(uint64_t)r * NS + st], cnt);
        x = a.sparent[x];
      }
    }
    __threadfence();
    __syncthreads();
    // (d) count or write; clear the marks
    bool unm = false;
    for (int s = 0; s < NS; ++s) unm |= s_unm[s] > 0;
    const uint64_t base = a.emit ? a.row_off[c] : 0, lim = a.emit ? a.row_off[c + 1] : 0;
    for (uint32_t r = threadIdx.x; r < nrows; r += DBLOCK) {
      const uint32_t id = row_id[r];
      if (id >= a.n_ids) { atomicOr(a.err, ERR_SCOPE); continue; }
      if (a.emit) {
        const uint64_t o = base + r;
        if (o >= lim) { atomicOr(a.err, ERR_TREE); continue; }
        a.o_scope[o] = id;
        for (int s = 0; s < NS; ++s)
          a.o_val[o * NS + s] = __hip_atomic_load(&rows[(uint64_t)r * NS + s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      row_of[id] = NONE32;
    }
    if (threadIdx.x == 0) {
      if (!a.emit) {
        a.n_rows[c] = nrows + (unm ? 1 : 0);
      } else if (unm) {
        const uint64_t o = base + nrows;
        if (o < lim) {
          a.o_scope[o] = NONE32;
          for (int s = 0; s < NS; ++s) a.o_val[o * NS + s] = s_unm[s];
        } else {
          atomicOr(a.err, ERR_TREE);
        }
      }
    }
    __threadfence();
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1024) k_scan_rows(const unsigned long long* n, uint32_t n_ctx, uint64_t* off,
                                                    unsigned long long* total) {
  __shared__ unsigned long long tmp[1024 / WAVE + 1];
  unsigned long long carry = 0;
  for (uint32_t b0 = 0; b0 < n_ctx; b0 += 1024) {
    const uint32_t c = b0 + threadIdx.x;
    const unsigned long long v = c < n_ctx ? n[c] : 0;
    unsigned long long t;
    unsigned long long ex = block_excl_scan<1024>(v, tmp, &t);
    if (c < n_ctx) off[c] = carry + ex;
    carry += t;
  }
  if (threadIdx.x == 0) { off[n_ctx] = carry; *total = carry; }
}

}  // namespace
}  // namespace hpa

using namespace hpa;

struct hpa_metrics {
  hpa_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  uint64_t n_nodes = 0, n_rows = 0;
  uint32_t n_ctx = 0;
  DBuf incl, S, W, host_incl, host_W, sc_off, sc_scope, sc_val;
};

namespace {
void check_err(unsigned int err) {
  if (!err) return;
  std::string m = "metric derivation stopped on invalid data:";
  if (err & ERR_SCOPE) m += " a scope label or scope parent is out of range;";
  if (err & ERR_STALL) m += " a stall reason is out of range;";
  if (err & ERR_TREE) m += " the calling context tree layout is inconsistent;";
  fail(HPA_E_DEVICE, m);
}
}  // namespace

extern "C" hpa_status hpa_derive_metrics(hpa_ctx* ctx, const hpa_callgraph_plan* plan, const hpa_attribution* attr,
                                         const hpa_gpu_cct* cct, hipStream_t stream, hpa_metrics** out) {
  return guard([&] {
    if (!ctx || !plan || !attr || !cct || !out) fail(HPA_E_INVAL, "NULL argument");
    if (cct_plan(cct) != plan || cct_attr(cct) != attr) fail(HPA_E_INVAL, "the tree was built from other inputs");
    if (attr->ctx != ctx) fail(HPA_E_INVAL, "handles belong to another context");
#ifndef HPA_ENABLE_GPU_CCT
    fail(HPA_E_UNSUPPORTED, "derived metrics of the GPU calling context tree are compiled out with it "
                            "(build with HPA_ENABLE_GPU_CCT)");
#endif
    DeviceGuard dg(ctx->device);
    hipStream_t s = stream;
    const uint32_t C = plan_n_ctx(plan);
    const uint64_t nn = cct_n_nodes(cct);
    auto* M = new hpa_metrics();
    std::unique_ptr<hpa_metrics> hold(M);
    M->ctx = ctx;
    M->stream = s;
    M->n_nodes = nn;
    M->n_ctx = C;
    const uint64_t nn1 = std::max<uint64_t>(nn, 1);
    M->incl = DBuf(ctx, nn1 * NS * 8, s);
    M->S = DBuf(ctx, nn1 * 8, s);
    M->W = DBuf(ctx, nn1 * 8, s);
    M->host_incl = DBuf(ctx, (uint64_t)C * NS * 8, s);
    M->host_W = DBuf(ctx, (uint64_t)C * 8, s);
    M->sc_off = DBuf(ctx, ((uint64_t)C + 1) * 8, s);
    const unsigned nwg = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(C, (uint64_t)ctx->n_cu * 8));
    DBuf d_ticket(ctx, 16, s), d_err(ctx, 8, s);
    HPA_HIP(hipMemsetAsync(d_err.p, 0, 8, s));
    // GPU CCT inclusive values
    HPA_HIP(hipMemsetAsync(d_ticket.p, 0, 16, s));
    k_cct_incl<<<nwg, DBLOCK, 0, s>>>(cct_node_off(cct), cct_size(cct), cct_depth(cct), cct_excl(cct), C,
                                      d_ticket.as<unsigned int>(), M->incl.as<double>(), M->S.as<double>(),
                                      M->W.as<double>(), d_err.as<unsigned int>());
    HPA_HIP(hipGetLastError());
    // host calling-context tree
    k_host_own<<<nwg, DBLOCK, 0, s>>>(attr->ctx_offsets.as<uint64_t>(), attr->stall.as<uint8_t>(),
                                      attr->count.as<unsigned long long>(), C,
                                      M->host_incl.as<unsigned long long>(), d_err.as<unsigned int>());
    HPA_HIP(hipGetLastError());
    {
      k_host_up<<<1, 1024, 0, s>>>(plan_depth_order(plan), plan_depth_lvl(plan), plan_n_depth_lvl(plan),
                                   plan_ctx_parent(plan), C, M->host_incl.as<unsigned long long>(),
                                   M->host_W.as<double>());
      HPA_HIP(hipGetLastError());
      // static scope tree
      const uint32_t n_ids = std::max(plan_map(plan)->n_ids, 1u);
      const unsigned nwg_s = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(C, (uint64_t)ctx->n_cu * 2));
      const uint64_t stride = scope_ws_stride(n_ids);
      DBuf ws(ctx, stride * nwg_s, s);
      HPA_HIP(hipMemset2DAsync(ws.p, stride, 0xFF, (uint64_t)n_ids * 4, nwg_s, s));
      DBuf d_nrows(ctx, (uint64_t)C * 8, s), d_tot(ctx, 8, s);
      ScopeArgs sa{};
      sa.sparent = plan_map(plan)->parent.as<uint32_t>();
      sa.n_ids = n_ids;
      sa.ctx_off = attr->ctx_offsets.as<uint64_t>();
      sa.k_scope = attr->scope.as<uint32_t>();
      sa.k_stall = attr->stall.as<uint8_t>();
      sa.k_count = attr->count.as<unsigned long long>();
      sa.n_ctx = C;
      sa.ticket = d_ticket.as<unsigned int>() + 1;
      sa.ws = ws.as<uint8_t>();
      sa.ws_stride = stride;
      sa.n_rows = d_nrows.as<unsigned long long>();
      sa.err = d_err.as<unsigned int>();
      HPA_HIP(hipMemsetAsync(d_nrows.p, 0, (uint64_t)C * 8, s));
      sa.emit = 0;
      k_scope<<<nwg_s, DBLOCK, 0, s>>>(sa);
      HPA_HIP(hipGetLastError());
      k_scan_rows<<<1, 1024, 0, s>>>(d_nrows.as<unsigned long long>(), C, M->sc_off.as<uint64_t>(),
                                     d_tot.as<unsigned long long>());
      unsigned long long tot = 0;
      unsigned int err = 0;
      HPA_HIP(hipMemcpyAsync(&tot, d_tot.p, 8, hipMemcpyDeviceToHost, s));
      HPA_HIP(hipMemcpyAsync(&err, d_err.p, 4, hipMemcpyDeviceToHost, s));
      sync_stream(ctx, s);
      check_err(err);
      M->n_rows = tot;
      M->sc_scope = DBuf(ctx, std::max<uint64_t>(tot, 1) * 4, s);
      M->sc_val = DBuf(ctx, std::max<uint64_t>(tot, 1) * NS * 8, s);
      HPA_HIP(hipMemsetAsync(d_ticket.p, 0, 16, s));
      sa.emit = 1;
      sa.row_off = M->sc_off.as<uint64_t>();
      sa.o_scope = M->sc_scope.as<uint32_t>();
      sa.o_val = M->sc_val.as<unsigned long long>();
      k_scope<<<nwg_s, DBLOCK, 0, s>>>(sa);
      HPA_HIP(hipGetLastError());
      HPA_HIP(hipMemcpyAsync(&err, d_err.p, 4, hipMemcpyDeviceToHost, s));
      sync_stream(ctx, s);
      check_err(err);
    }
    *out = hold.release();
  });
}

extern "C" hpa_status hpa_metrics_view_get(const hpa_metrics* m, hpa_metrics_view* v) {
  return guard([&] {
    if (!m || !v) fail(HPA_E_INVAL, "NULL argument");
    v->n_nodes = m->n_nodes;
    v->n_ctx = m->n_ctx;
    v->incl = m->incl.as<double>();
    v->S = m->S.as<double>();
    v->W = m->W.as<double>();
    v->host_incl = m->host_incl.as<uint64_t>();
    v->host_W = m->host_W.as<double>();
    v->n_scope_rows = m->n_rows;
    v->sc_offsets = m->sc_off.as<uint64_t>();
    v->sc_scope = m->sc_scope.as<uint32_t>();
    v->sc_val = m->sc_val.as<uint64_t>();
  });
}

extern "C" void hpa_metrics_free(hpa_metrics* m) { delete m; }
