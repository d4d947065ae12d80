// A5: approximate GPU calling context trees (Section 6.3).
//
// Step 1: the static call graph comes from function symbols and call
// instructions; a call edge's weight is the number of samples at its call
// instruction.  Step 2: a function with samples whose incoming edges all have
// weight zero gives each incoming edge weight one, and the rule propagates to
// callers (computed here as its least fixpoint).  Step 3: strongly connected
// components (Tarjan) become single nodes; calls between members are dropped.
// Step 4: the graph is split into a tree of call paths; a function's cost is
// shared among its call sites by the ratio of each site's calls to all calls,
// and ratios multiply along a path.
//
// Readings used where the paper is silent: after condensation the step-2 rule
// is applied once more on the condensed graph (an SCC whose external calls all
// have weight zero would otherwise split 0/0); a context with a kernel entry
// uses the graph the entry reaches, its other samples form an <unreachable>
// node and unmapped PCs an <unknown> node; paths that lead to no sample are
// pruned by an integer test; children follow call-site PC order.
//
// Host: hpa_prepare_callgraph validates, finds SCCs and, for every distinct
// kernel entry, builds a local condensed DAG numbered level by level (callers
// first) with edge lists.  Device: one workgroup per context runs the whole
// analysis as level sweeps, then expands the tree breadth-first, writing each
// node straight into its depth-first preorder slot: a child's slot is its
// parent's slot + 1 + the subtree sizes of the children before it.
#include <algorithm>
#include <map>
#include <memory>
#include <numeric>
#include <set>

#include "block_prims.h"
#include "hpa_internal.h"

namespace hpa {
namespace {

constexpr int ABLOCK = 256;
constexpr uint64_t SAT = 1ull << 62;  // saturation for subtree sizes

// Per-entry local plan, offsets into the concatenated device arrays.
struct EntDesc {
  uint32_t nU, nX, nE, nL, nR, nS;
  uint64_t u0, uo0, x0, xm0, xo0, xi0, e0, l0, r0, s0;
};

struct PlanDev {
  const EntDesc* ent;
  const int32_t* ctx_ent;   // per context: plan index (every context has one)
  // uncondensed local nodes
  const uint32_t* u_gid;    // sorted global function ids
  const uint32_t* u_x;      // local condensed index
  const uint32_t* u_oo;     // out-edge CSR offsets (nU + 1 per entry, relative)
  const uint32_t* u_oe;     // local edge ids
  // condensed local nodes (level order)
  const uint32_t* x_gid;    // global condensed id
  const uint32_t* x_mo;     // member CSR offsets (nX + 1)
  const uint32_t* x_mem;    // local U ids
  const uint32_t* x_oo;     // external out-edges CSR (nX + 1), edges by call-site pc
  const uint32_t* x_oe;
  const uint32_t* x_io;     // external in-edges CSR (nX + 1)
  const uint32_t* x_ie;
  const uint32_t* lvl;      // level offsets (nL + 1) into local X ids
  const uint32_t* roots;    // local X ids
  // local edges, sorted by call-site pc
  const uint64_t* e_pc;
  const uint32_t* e_cu;     // caller local U
  const uint32_t* e_eu;     // callee local U
  // scopes owned by reach functions (sorted ids), for the scope roll-up
  const uint32_t* s_gid;
};

struct AppArgs {
  PlanDev p;
  // attribution
  const uint32_t* k_ctx;
  const uint64_t* k_pc;
  const uint8_t* k_stall;
  const unsigned long long* k_count;
  const uint32_t* k_scope;
  const uint64_t* ctx_off;
  const uint32_t* func;     // map: owning function of each scope id
  uint32_t n_ids;           // number of scope ids (entries of func)
  uint32_t n_ctx;
  unsigned int* err;        // ERR_* bits
  unsigned int* ticket;      // next context to take
  int sample_based;         // 1: step 2 (and its re-application) on; 0: weights are exact counts
  // per-workgroup workspace
  uint8_t* ws;
  uint64_t ws_stride;
  uint32_t maxU, maxX, maxE;
  uint64_t q_cap;           // frontier capacity (items) per workgroup
  // outputs: counting pass
  unsigned long long* n_nodes;   // per context
  unsigned long long* n_w;       // per context
  // outputs: emission pass
  const uint64_t* node_off;
  const uint64_t* w_off;
  uint32_t* o_parent;
  uint32_t* o_node;
  uint64_t* o_site;
  uint8_t* o_kind;
  double* o_phi;
  double* o_excl;
  uint64_t* o_size;
  uint32_t* o_depth;
  uint64_t* o_wsite;
  uint64_t* o_wval;
  int emit;
};

struct Item {
  uint64_t pre;     // preorder index within the context
  uint64_t site;
  double phi;
  uint32_t x;       // local condensed node
  uint32_t parent;  // preorder index of the parent (NONE32 for roots)
  uint32_t depth;
  uint32_t pad;
};

// Workspace layout for one workgroup (byte offsets computed on the host).
struct WsLayout {
  uint64_t u_ss, u_fl;            // u: self sum (u64), flags (u8)
  uint64_t x_row, x_ss, x_w, x_sz, x_fl;  // x: row index (u32), self sum, W', size (u64), flags
  uint64_t e_w, e_w1, e_w2;       // e: weights (u64)
  uint64_t rows;                  // self rows (maxX x 16 u64)
  uint64_t q0, q1;                // frontiers
  uint64_t total;
};

__host__ __device__ inline WsLayout ws_layout(uint32_t mU, uint32_t mX, uint32_t mE, uint64_t qcap) {
  WsLayout L;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) { uint64_t r = o; o += (bytes + 255) & ~255ull; return r; };
  L.u_ss = take(8ull * mU);
  L.u_fl = take(mU);
  L.x_row = take(4ull * mX);
  L.x_ss = take(8ull * mX);
  L.x_w = take(8ull * mX);
  L.x_sz = take(8ull * mX);
  L.x_fl = take(mX);
  L.e_w = take(8ull * mE);
  L.e_w1 = take(8ull * mE);
  L.e_w2 = take(8ull * mE);
  L.rows = take(8ull * NS * mX);
  L.q0 = take(sizeof(Item) * qcap);
  L.q1 = take(sizeof(Item) * qcap);
  L.total = o;
  return L;
}

// flag bits
constexpr uint8_t F_NZIN = 1, F_FIRES = 2, F_ACT = 4, F_HC = 8;

template <class T>
__device__ inline uint32_t lower_bound_dev(const T* a, uint32_t n, T v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Words that other threads of the workgroup update with atomics in the same
// launch are read back with atomic loads at agent scope: such a load is served
// by the L2, where the atomics were performed, never by a line that this CU's
// vector L1 may still hold from before the updates.
__device__ inline unsigned long long ld_at(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t ld_at(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Error bits raised by the kernel (checked by the host after each pass).
constexpr unsigned int ERR_SCOPE = 1, ERR_STALL = 2, ERR_ROW = 4, ERR_QUEUE = 8, ERR_NODE = 16;

struct Shared {
  unsigned long long unk[NS], unr[NS];
  unsigned long long tmp[ABLOCK / WAVE + 1];
  uint32_t tmp32[ABLOCK / WAVE + 1];
  uint32_t work_i, qn[2];
  unsigned long long total, nw;
};

// The per-context analysis (Section 6.3 steps 1-4 up to subtree sizes).
__device__ void analyze(const AppArgs& a, Shared& sh, uint32_t c, const EntDesc& E, const WsLayout& L,
                        uint8_t* ws) {
  const PlanDev& p = a.p;
  const int tid = threadIdx.x;
  unsigned long long* u_ss = reinterpret_cast<unsigned long long*>(ws + L.u_ss);
  uint8_t* u_fl = ws + L.u_fl;
  uint32_t* x_row = reinterpret_cast<uint32_t*>(ws + L.x_row);
  unsigned long long* x_ss = reinterpret_cast<unsigned long long*>(ws + L.x_ss);
  unsigned long long* x_w = reinterpret_cast<unsigned long long*>(ws + L.x_w);
  unsigned long long* x_sz = reinterpret_cast<unsigned long long*>(ws + L.x_sz);
  uint8_t* x_fl = ws + L.x_fl;
  unsigned long long* e_w = reinterpret_cast<unsigned long long*>(ws + L.e_w);
  unsigned long long* e_w1 = reinterpret_cast<unsigned long long*>(ws + L.e_w1);
  unsigned long long* e_w2 = reinterpret_cast<unsigned long long*>(ws + L.e_w2);
  unsigned long long* rows = reinterpret_cast<unsigned long long*>(ws + L.rows);
  const uint32_t* u_gid = p.u_gid + E.u0;
  const uint32_t* u_x = p.u_x + E.u0;
  const uint32_t* u_oo = p.u_oo + E.uo0;
  const uint32_t* u_oe = p.u_oe + E.e0;
  const uint32_t* x_mo = p.x_mo + E.xm0;
  const uint32_t* x_mem = p.x_mem + E.u0;
  const uint32_t* x_oo = p.x_oo + E.xm0;
  const uint32_t* x_oe = p.x_oe + E.xo0;
  const uint32_t* x_io = p.x_io + E.xm0;
  const uint32_t* x_ie = p.x_ie + E.xi0;
  const uint32_t* lvl = p.lvl + E.l0;
  const uint64_t* e_pc = p.e_pc + E.e0;
  const uint32_t* e_cu = p.e_cu + E.e0;
  const uint32_t* e_eu = p.e_eu + E.e0;

  // ---- clear ----
  for (uint32_t i = tid; i < E.nU; i += ABLOCK) { u_ss[i] = 0; u_fl[i] = 0; }
  for (uint32_t i = tid; i < E.nX; i += ABLOCK) { x_row[i] = 0; x_fl[i] = 0; }
  for (uint32_t i = tid; i < E.nE; i += ABLOCK) e_w[i] = 0;
  if (tid < NS) { sh.unk[tid] = 0; sh.unr[tid] = 0; }
  // Each hand-over of workspace words between threads is a device-scope fence
  // (the stores or atomics have reached the L2, and this CU's L1 is
  // invalidated) followed by the barrier.
  __threadfence();
  __syncthreads();
  // ---- step 1: self costs per condensed node and stall; call-site weights ----
  // (a) mark the condensed nodes that own samples; (b) give them dense rows in
  // node order and zero the rows; (c) accumulate.  Marks are atomic stores of
  // one value, and the barriers order the passes.
  const uint64_t k0 = a.ctx_off[c], k1 = a.ctx_off[c + 1];
  auto local_u = [&](uint32_t sc) -> uint32_t {
    const uint32_t f = a.func[sc];
    const uint32_t u = lower_bound_dev(u_gid, E.nU, f);
    return (u < E.nU && u_gid[u] == f) ? u : NONE32;
  };
  for (uint64_t k = k0 + tid; k < k1; k += ABLOCK) {
    const uint32_t sc = a.k_scope[k];
    if (sc == NONE32 || sc >= a.n_ids) continue;
    const uint32_t u = local_u(sc);
    if (u != NONE32) __hip_atomic_store(&x_row[u_x[u]], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __threadfence();
  __syncthreads();
  {
    uint32_t done = 0;
    for (uint32_t x0 = 0; x0 < E.nX; x0 += ABLOCK) {
      const uint32_t x = x0 + tid;
      const uint32_t used = x < E.nX ? ld_at(&x_row[x]) : 0u;
      uint32_t t;
      const uint32_t r = done + block_excl_scan<ABLOCK>(used, sh.tmp32, &t);
      if (x < E.nX) x_row[x] = used ? r : NONE32;
      if (used)
        for (int s = 0; s < NS; ++s) rows[(uint64_t)r * NS + s] = 0;
      done += t;
    }
  }
  __threadfence();
  __syncthreads();
  for (uint64_t k = k0 + tid; k < k1; k += ABLOCK) {
    const uint32_t sc = a.k_scope[k];
    const uint32_t st = a.k_stall[k];
    const unsigned long long cnt = a.k_count[k];
    const uint64_t pcv = a.k_pc[k];
    if (st >= NS) { atomicOr(a.err, ERR_STALL); continue; }
    if (sc == NONE32) {
      atomicAdd(&sh.unk[st], cnt);
      continue;
    }
    if (sc >= a.n_ids) { atomicOr(a.err, ERR_SCOPE); continue; }
    const uint32_t u = local_u(sc);
    if (u == NONE32) {
      atomicAdd(&sh.unr[st], cnt);
    } else {
      atomicAdd(&u_ss[u], cnt);
      const uint32_t r = x_row[u_x[u]];
      if (r >= E.nX) { atomicOr(a.err, ERR_ROW); continue; }
      atomicAdd(&rows[(uint64_t)r * NS + st], cnt);
    }
    const uint32_t e = lower_bound_dev(e_pc, E.nE, pcv);
    if (e < E.nE && e_pc[e] == pcv) atomicAdd(&e_w[e], cnt);
  }
  __threadfence();
  __syncthreads();
  // ---- step 2 inputs: incoming nonzero weight, activity ----
  for (uint32_t e = tid; e < E.nE; e += ABLOCK)
    if (ld_at(&e_w[e]) > 0) u_fl[e_eu[e]] = F_NZIN;  // benign race: same value
  __syncthreads();
  for (uint32_t u = tid; u < E.nU; u += ABLOCK) {
    bool act = ld_at(&u_ss[u]) > 0;
    for (uint32_t i = u_oo[u]; i < u_oo[u + 1] && !act; ++i) act = ld_at(&e_w[u_oe[i]]) > 0;
    if (act) u_fl[u] |= F_ACT;
  }
  __syncthreads();
  // ---- step 2: least fixpoint, callees first; members of one SCC iterate ----
  for (int l = (int)E.nL - 1; l >= 0; --l) {
    for (uint32_t x = lvl[l] + tid; x < lvl[l + 1]; x += ABLOCK) {
      bool again = true;
      while (again) {
        again = false;
        for (uint32_t mi = x_mo[x]; mi < x_mo[x + 1]; ++mi) {
          const uint32_t u = x_mem[mi];
          const uint8_t fl = u_fl[u];
          if ((fl & F_FIRES) || (fl & F_NZIN)) continue;
          bool fire = (fl & F_ACT) != 0;
          for (uint32_t i = u_oo[u]; i < u_oo[u + 1] && !fire; ++i) fire = (u_fl[e_eu[u_oe[i]]] & F_FIRES) != 0;
          if (fire) { u_fl[u] = fl | F_FIRES; again = true; }
        }
      }
    }
    __syncthreads();
  }
  for (uint32_t e = tid; e < E.nE; e += ABLOCK) {
    const unsigned long long w = ld_at(&e_w[e]);
    e_w1[e] = (w > 0 || !a.sample_based) ? w : ((u_fl[e_eu[e]] & F_FIRES) ? 1ull : 0ull);
  }
  __syncthreads();
  // ---- condensed graph: self sums, the step-2 rule once more, W', has-cost, sizes ----
  for (uint32_t x = tid; x < E.nX; x += ABLOCK) {
    unsigned long long ss = 0;
    for (uint32_t mi = x_mo[x]; mi < x_mo[x + 1]; ++mi) ss += ld_at(&u_ss[x_mem[mi]]);
    x_ss[x] = ss;
    bool nz = false;
    for (uint32_t i = x_io[x]; i < x_io[x + 1] && !nz; ++i) nz = e_w1[x_ie[i]] > 0;
    bool act = ss > 0;
    for (uint32_t i = x_oo[x]; i < x_oo[x + 1] && !act; ++i) act = e_w1[x_oe[i]] > 0;
    x_fl[x] = (nz ? F_NZIN : 0) | (act ? F_ACT : 0);
  }
  __syncthreads();
  for (int l = (int)E.nL - 1; l >= 0; --l) {
    for (uint32_t x = lvl[l] + tid; x < lvl[l + 1]; x += ABLOCK) {
      const uint8_t fl = x_fl[x];
      if (fl & F_NZIN) continue;
      bool fire = (fl & F_ACT) != 0;
      for (uint32_t i = x_oo[x]; i < x_oo[x + 1] && !fire; ++i) fire = (x_fl[u_x[e_eu[x_oe[i]]]] & F_FIRES) != 0;
      if (fire) x_fl[x] = fl | F_FIRES;
    }
    __syncthreads();
  }
  for (uint32_t x = tid; x < E.nX; x += ABLOCK)
    for (uint32_t i = x_oo[x]; i < x_oo[x + 1]; ++i) {
      const uint32_t e = x_oe[i];
      e_w2[e] = (e_w1[e] > 0 || !a.sample_based) ? e_w1[e] : ((x_fl[u_x[e_eu[e]]] & F_FIRES) ? 1ull : 0ull);
    }
  __syncthreads();
  for (uint32_t x = tid; x < E.nX; x += ABLOCK) {
    unsigned long long W = 0;
    for (uint32_t i = x_io[x]; i < x_io[x + 1]; ++i) W += e_w2[x_ie[i]];
    x_w[x] = W;
  }
  for (int l = (int)E.nL - 1; l >= 0; --l) {
    for (uint32_t x = lvl[l] + tid; x < lvl[l + 1]; x += ABLOCK) {
      bool hc = x_ss[x] > 0;
      unsigned long long sz = 1;
      for (uint32_t i = x_oo[x]; i < x_oo[x + 1]; ++i) {
        const uint32_t e = x_oe[i];
        const uint32_t y = u_x[e_eu[e]];
        if (e_w2[e] > 0 && (x_fl[y] & F_HC)) {
          hc = true;
          sz += x_sz[y];
          if (sz > SAT) sz = SAT;
        }
      }
      x_sz[x] = hc ? sz : 0;
      if (hc) x_fl[x] |= F_HC;
    }
    __syncthreads();
  }
  // ---- totals ----
  if (tid == 0) {
    unsigned long long tot = 0, nw = 0;
    for (uint32_t r = 0; r < E.nR; ++r) {
      uint32_t x = p.roots[E.r0 + r];
      if (x_fl[x] & F_HC) tot += x_sz[x];
      if (tot > SAT) tot = SAT;
    }
    bool unr = false, unk = false;
    for (int s = 0; s < NS; ++s) { unr |= sh.unr[s] > 0; unk |= sh.unk[s] > 0; }
    tot += unr + unk;
    sh.total = tot;
    (void)nw;
  }
  // positive final weights of external edges (listed per context by call-site pc)
  {
    unsigned long long cnt = 0;
    for (uint32_t e = tid; e < E.nE; e += ABLOCK)
      if (u_x[e_cu[e]] != u_x[e_eu[e]] && e_w2[e] > 0) ++cnt;
    unsigned long long t;
    block_excl_scan<ABLOCK>(cnt, sh.tmp, &t);
    if (tid == 0) sh.nw = t;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(ABLOCK) k_apportion(AppArgs a) {
  __shared__ Shared sh;
  const int tid = threadIdx.x;
  const WsLayout L = ws_layout(a.maxU, a.maxX, a.maxE, a.q_cap);
  uint8_t* ws = a.ws + (uint64_t)blockIdx.x * a.ws_stride;
  while (true) {
    if (tid == 0) sh.work_i = atomicAdd(a.ticket, 1u);
    __syncthreads();
    const uint32_t c = sh.work_i;
    __syncthreads();
    if (c >= a.n_ctx) break;
    if (a.ctx_off[c + 1] == a.ctx_off[c]) continue;
    const EntDesc E = a.p.ent[a.p.ctx_ent[c]];
    analyze(a, sh, c, E, L, ws);
    if (!a.emit) {
      if (tid == 0) {
        a.n_nodes[c] = sh.total;
        a.n_w[c] = sh.nw;
      }
      continue;
    }
    // ---------------- emission ----------------
    const PlanDev& p = a.p;
    const uint32_t* x_gid = p.x_gid + E.x0;
    const uint32_t* x_oo = p.x_oo + E.xm0;
    const uint32_t* x_oe = p.x_oe + E.xo0;
    const uint32_t* u_x = p.u_x + E.u0;
    const uint64_t* e_pc = p.e_pc + E.e0;
    const uint32_t* e_cu = p.e_cu + E.e0;
    const uint32_t* e_eu = p.e_eu + E.e0;
    const uint32_t* x_row = reinterpret_cast<const uint32_t*>(ws + L.x_row);
    const unsigned long long* x_w = reinterpret_cast<const unsigned long long*>(ws + L.x_w);
    const unsigned long long* x_sz = reinterpret_cast<const unsigned long long*>(ws + L.x_sz);
    const uint8_t* x_fl = ws + L.x_fl;
    const unsigned long long* e_w2 = reinterpret_cast<const unsigned long long*>(ws + L.e_w2);
    const unsigned long long* rows = reinterpret_cast<const unsigned long long*>(ws + L.rows);
    Item* q[2] = {reinterpret_cast<Item*>(ws + L.q0), reinterpret_cast<Item*>(ws + L.q1)};
    const uint64_t base = a.node_off[c], end = a.node_off[c + 1];
    // final weights, by call-site pc (edges are stored in pc order)
    {
      const uint64_t wb = a.w_off[c], we = a.w_off[c + 1];
      unsigned long long done = 0;
      for (uint32_t e0 = 0; e0 < E.nE; e0 += ABLOCK) {
        const uint32_t e = e0 + tid;
        const bool pos = e < E.nE && u_x[e_cu[e]] != u_x[e_eu[e]] && e_w2[e] > 0;
        unsigned long long t;
        unsigned long long ex = block_excl_scan<ABLOCK>((unsigned long long)pos, sh.tmp, &t);
        if (pos) {
          const uint64_t o = wb + done + ex;
          if (o < we) {
            a.o_wsite[o] = e_pc[e];
            a.o_wval[o] = e_w2[e];
          } else {
            atomicOr(a.err, ERR_NODE);
          }
        }
        done += t;
      }
    }
    // roots, in order, each followed by its whole subtree in preorder
    if (tid == 0) {
      uint64_t pre = 0;
      uint32_t n = 0;
      for (uint32_t r = 0; r < E.nR; ++r) {
        const uint32_t x = p.roots[E.r0 + r];
        if (!(x_fl[x] & F_HC)) continue;
        if (n < a.q_cap) q[0][n++] = Item{pre, NONE64, 1.0, x, NONE32, 0, 0};
        else atomicOr(a.err, ERR_QUEUE);
        pre += x_sz[x];
      }
      // special nodes after every call path
      uint32_t k = 0;
      for (int kind = 1; kind <= 2; ++kind) {
        const unsigned long long* row = kind == 1 ? sh.unr : sh.unk;
        unsigned long long t = 0;
        for (int s = 0; s < NS; ++s) t += row[s];
        if (!t) continue;
        const uint64_t o = base + pre + k++;
        if (o >= end) { atomicOr(a.err, ERR_NODE); continue; }
        a.o_parent[o] = NONE32;
        a.o_node[o] = NONE32;
        a.o_site[o] = NONE64;
        a.o_kind[o] = (uint8_t)kind;
        a.o_phi[o] = 1.0;
        a.o_size[o] = 1;
        a.o_depth[o] = 0;
        for (int s = 0; s < NS; ++s) a.o_excl[o * NS + s] = (double)row[s];
      }
      sh.qn[0] = n;
    }
    __syncthreads();
    int cur = 0;
    while (sh.qn[cur] > 0) {
      const uint32_t n = sh.qn[cur];
      if (tid == 0) sh.qn[cur ^ 1] = 0;
      __syncthreads();
      for (uint32_t i = tid; i < n && i < a.q_cap; i += ABLOCK) {
        const Item it = q[cur][i];
        const uint64_t o = base + it.pre;
        if (o >= end || it.x >= E.nX) { atomicOr(a.err, ERR_NODE); continue; }
        a.o_parent[o] = it.parent;
        a.o_node[o] = x_gid[it.x];
        a.o_site[o] = it.site;
        a.o_kind[o] = 0;
        a.o_phi[o] = it.phi;
        a.o_size[o] = x_sz[it.x];
        a.o_depth[o] = it.depth;
        const uint32_t r = x_row[it.x];
        for (int s = 0; s < NS; ++s)
          a.o_excl[o * NS + s] = (r == NONE32 ? 0.0 : (double)ld_at(&rows[(uint64_t)r * NS + s])) * it.phi;
        uint64_t off = it.pre + 1;
        for (uint32_t j = x_oo[it.x]; j < x_oo[it.x + 1]; ++j) {
          const uint32_t e = x_oe[j];
          const uint32_t y = u_x[e_eu[e]];
          if (e_w2[e] == 0 || !(x_fl[y] & F_HC)) continue;
          const double ratio = (double)e_w2[e] / (double)x_w[y];
          const uint32_t slot = atomicAdd(&sh.qn[cur ^ 1], 1u);
          if (slot < a.q_cap) q[cur ^ 1][slot] = Item{off, e_pc[e], it.phi * ratio, y, (uint32_t)it.pre, it.depth + 1, 0};
          else atomicOr(a.err, ERR_QUEUE);
          off += x_sz[y];
        }
      }
      __syncthreads();
      cur ^= 1;
    }
    __syncthreads();
  }
}

// Exclusive scan over contexts of node and weight counts (one workgroup).
__global__ void __launch_bounds__(1024) k_cct_scan(const unsigned long long* n_nodes, const unsigned long long* n_w,
                                                   uint32_t n_ctx, uint64_t* node_off, uint64_t* w_off,
                                                   unsigned long long* totals) {
  __shared__ unsigned long long tmp[1024 / WAVE + 1];
  unsigned long long cn = 0, cw = 0, mx = 0;
  for (uint32_t b0 = 0; b0 < n_ctx; b0 += 1024) {
    const uint32_t c = b0 + threadIdx.x;
    const unsigned long long vn = c < n_ctx ? n_nodes[c] : 0, vw = c < n_ctx ? n_w[c] : 0;
    mx = vn > mx ? vn : mx;
    unsigned long long tn, tw;
    unsigned long long en = block_excl_scan<1024>(vn, tmp, &tn);
    unsigned long long ew = block_excl_scan<1024>(vw, tmp, &tw);
    if (c < n_ctx) { node_off[c] = cn + en; w_off[c] = cw + ew; }
    cn += tn;
    cw += tw;
  }
  mx = wave_max(mx);
  __shared__ unsigned long long smax;
  if (threadIdx.x == 0) smax = 0;
  __syncthreads();
  if (lane_id() == 0) atomicMax(&smax, mx);
  __syncthreads();
  if (threadIdx.x == 0) {
    node_off[n_ctx] = cn;
    w_off[n_ctx] = cw;
    totals[0] = cn;
    totals[1] = cw;
    totals[2] = smax;
  }
}

}  // namespace
}  // namespace hpa

// ============================================================================
// host side
// ============================================================================
using namespace hpa;

struct hpa_callgraph_plan {
  hpa_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  const hpa_structure_map* map = nullptr;
  uint32_t V = 0, n_ctx = 0, n_ent = 0;
  uint32_t maxU = 0, maxX = 0, maxE = 0, maxS = 0;
  std::vector<uint32_t> h_scc, h_parent;
  std::vector<int32_t> h_ctx_ent;
  std::vector<uint32_t> h_depth_order;  // contexts by descending depth (host-tree roll-up)
  std::vector<uint32_t> h_depth;
  std::vector<uint32_t> h_depth_lvl;    // offsets of each depth group in h_depth_order
  DBuf scc, ent, ctx_ent, u_gid, u_x, u_oo, u_oe, x_gid, x_mo, x_mem, x_oo, x_oe, x_io, x_ie, lvl, roots, e_pc, e_cu,
      e_eu, s_gid, ctx_parent, depth_order, depth_lvl;
  std::vector<EntDesc> h_ent;
  hpa::PlanDev dev() const {
    return PlanDev{ent.as<EntDesc>(), ctx_ent.as<int32_t>(), u_gid.as<uint32_t>(), u_x.as<uint32_t>(),
                   u_oo.as<uint32_t>(), u_oe.as<uint32_t>(), x_gid.as<uint32_t>(), x_mo.as<uint32_t>(),
                   x_mem.as<uint32_t>(), x_oo.as<uint32_t>(), x_oe.as<uint32_t>(), x_io.as<uint32_t>(),
                   x_ie.as<uint32_t>(), lvl.as<uint32_t>(), roots.as<uint32_t>(), e_pc.as<uint64_t>(),
                   e_cu.as<uint32_t>(), e_eu.as<uint32_t>(), s_gid.as<uint32_t>()};
  }
};

namespace {

// Tarjan's algorithm, iterative; component ids ranked by smallest member.
std::vector<uint32_t> scc_of(uint32_t V, const std::vector<std::vector<uint32_t>>& adj) {
  std::vector<int64_t> idx(V, -1), low(V, 0);
  std::vector<uint8_t> on(V, 0);
  std::vector<uint32_t> comp(V, NONE32), st;
  int64_t counter = 0;
  uint32_t nc = 0;
  std::vector<std::pair<uint32_t, uint32_t>> frames;
  for (uint32_t s = 0; s < V; ++s) {
    if (idx[s] >= 0) continue;
    frames.push_back({s, 0});
    idx[s] = low[s] = counter++;
    st.push_back(s);
    on[s] = 1;
    while (!frames.empty()) {
      auto& fr = frames.back();
      const uint32_t v = fr.first;
      if (fr.second < adj[v].size()) {
        const uint32_t w = adj[v][fr.second++];
        if (idx[w] < 0) {
          idx[w] = low[w] = counter++;
          st.push_back(w);
          on[w] = 1;
          frames.push_back({w, 0});
        } else if (on[w]) {
          low[v] = std::min(low[v], idx[w]);
        }
      } else {
        if (low[v] == idx[v]) {
          uint32_t w;
          do {
            w = st.back();
            st.pop_back();
            on[w] = 0;
            comp[w] = nc;
          } while (w != v);
          ++nc;
        }
        frames.pop_back();
        if (!frames.empty()) low[frames.back().first] = std::min(low[frames.back().first], low[v]);
      }
    }
  }
  std::vector<uint32_t> first(nc, NONE32);
  for (uint32_t v = 0; v < V; ++v) first[comp[v]] = std::min(first[comp[v]], v);
  std::vector<uint32_t> order(nc);
  std::iota(order.begin(), order.end(), 0u);
  std::sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return first[x] < first[y]; });
  std::vector<uint32_t> rank(nc);
  for (uint32_t i = 0; i < nc; ++i) rank[order[i]] = i;
  for (uint32_t v = 0; v < V; ++v) comp[v] = rank[comp[v]];
  return comp;
}

struct HostPlan {
  std::vector<EntDesc> ent;
  std::vector<uint32_t> u_gid, u_x, u_oo, u_oe, x_gid, x_mo, x_mem, x_oo, x_oe, x_io, x_ie, lvl, roots, e_cu, e_eu,
      s_gid;
  std::vector<uint64_t> e_pc;
};

// Local condensed DAG of one entry (entry = NONE32: the whole graph).
void build_entry(uint32_t entry, uint32_t V, const std::vector<uint8_t>& is_func,
                 const std::vector<std::vector<uint32_t>>& out_sites, const std::vector<uint64_t>& spc,
                 const std::vector<uint32_t>& scaller, const std::vector<uint32_t>& scallee,
                 const std::vector<uint32_t>& comp, const std::vector<std::vector<uint32_t>>& scopes_of_func,
                 HostPlan& H) {
  EntDesc d{};
  d.u0 = H.u_gid.size();
  d.uo0 = H.u_oo.size();
  d.x0 = H.x_gid.size();
  d.xm0 = H.x_mo.size();
  d.xo0 = H.x_oe.size();
  d.xi0 = H.x_ie.size();
  d.e0 = H.e_pc.size();
  d.l0 = H.lvl.size();
  d.r0 = H.roots.size();
  d.s0 = H.s_gid.size();
  // reach
  std::vector<uint32_t> R;
  if (entry == NONE32) {
    for (uint32_t v = 0; v < V; ++v)
      if (is_func[v]) R.push_back(v);
  } else {
    std::vector<uint8_t> seen(V, 0);
    R.push_back(entry);
    seen[entry] = 1;
    for (size_t i = 0; i < R.size(); ++i)
      for (uint32_t e : out_sites[R[i]])
        if (!seen[scallee[e]]) { seen[scallee[e]] = 1; R.push_back(scallee[e]); }
    std::sort(R.begin(), R.end());
  }
  const uint32_t nU = (uint32_t)R.size();
  std::map<uint32_t, uint32_t> uloc;
  for (uint32_t i = 0; i < nU; ++i) uloc[R[i]] = i;
  // local edges (caller in reach), by call-site pc
  std::vector<uint32_t> es;
  for (uint32_t v : R) for (uint32_t e : out_sites[v]) es.push_back(e);
  std::sort(es.begin(), es.end(), [&](uint32_t x, uint32_t y) { return spc[x] < spc[y]; });
  const uint32_t nE = (uint32_t)es.size();
  std::vector<uint32_t> ecu(nE), eeu(nE);
  for (uint32_t i = 0; i < nE; ++i) { ecu[i] = uloc[scaller[es[i]]]; eeu[i] = uloc[scallee[es[i]]]; }
  // condensed nodes present in reach
  std::vector<uint32_t> cx;
  for (uint32_t v : R) cx.push_back(comp[v]);
  std::sort(cx.begin(), cx.end());
  cx.erase(std::unique(cx.begin(), cx.end()), cx.end());
  std::map<uint32_t, uint32_t> cloc;
  for (uint32_t i = 0; i < cx.size(); ++i) cloc[cx[i]] = i;
  const uint32_t nXc = (uint32_t)cx.size();
  std::vector<std::vector<uint32_t>> cout(nXc), cin(nXc);
  std::vector<uint32_t> uxc(nU);
  for (uint32_t u = 0; u < nU; ++u) uxc[u] = cloc[comp[R[u]]];
  for (uint32_t i = 0; i < nE; ++i) {
    uint32_t a = uxc[ecu[i]], b = uxc[eeu[i]];
    if (a != b) { cout[a].push_back(i); cin[b].push_back(i); }
  }
  // levels: longest path from the sources of the local condensed DAG (Kahn)
  std::vector<uint32_t> indeg(nXc, 0), level(nXc, 0), q;
  for (uint32_t x = 0; x < nXc; ++x) for (uint32_t i : cout[x]) ++indeg[uxc[eeu[i]]];
  for (uint32_t x = 0; x < nXc; ++x) if (!indeg[x]) q.push_back(x);
  for (size_t i = 0; i < q.size(); ++i) {
    uint32_t x = q[i];
    for (uint32_t e : cout[x]) {
      uint32_t y = uxc[eeu[e]];
      level[y] = std::max(level[y], level[x] + 1);
      if (--indeg[y] == 0) q.push_back(y);
    }
  }
  // local x ids in (level, condensed id) order
  std::vector<uint32_t> xo(nXc);
  std::iota(xo.begin(), xo.end(), 0u);
  std::stable_sort(xo.begin(), xo.end(), [&](uint32_t p, uint32_t r) { return level[p] < level[r]; });
  std::vector<uint32_t> xnew(nXc);
  for (uint32_t i = 0; i < nXc; ++i) xnew[xo[i]] = i;
  uint32_t nL = nXc ? level[xo.back()] + 1 : 0;
  // write
  for (uint32_t u = 0; u < nU; ++u) { H.u_gid.push_back(R[u]); H.u_x.push_back(xnew[uxc[u]]); }
  {
    std::vector<std::vector<uint32_t>> uo(nU);
    for (uint32_t i = 0; i < nE; ++i) uo[ecu[i]].push_back(i);
    uint32_t o = 0;
    for (uint32_t u = 0; u < nU; ++u) {
      H.u_oo.push_back(o);
      for (uint32_t e : uo[u]) H.u_oe.push_back(e);
      o += (uint32_t)uo[u].size();
    }
    H.u_oo.push_back(o);
  }
  std::vector<std::vector<uint32_t>> mem(nXc);
  for (uint32_t u = 0; u < nU; ++u) mem[xnew[uxc[u]]].push_back(u);
  uint32_t om = 0, oo = 0, oi = 0;
  for (uint32_t i = 0; i < nXc; ++i) {
    const uint32_t xc = xo[i];
    H.x_gid.push_back(cx[xc]);
    H.x_mo.push_back(om);
    for (uint32_t u : mem[i]) H.x_mem.push_back(u);
    om += (uint32_t)mem[i].size();
    std::vector<uint32_t> o = cout[xc];  // already in pc order (edges sorted by pc)
    H.x_oo.push_back(oo);
    for (uint32_t e : o) H.x_oe.push_back(e);
    oo += (uint32_t)o.size();
    H.x_io.push_back(oi);
    for (uint32_t e : cin[xc]) H.x_ie.push_back(e);
    oi += (uint32_t)cin[xc].size();
  }
  H.x_mo.push_back(om);
  H.x_oo.push_back(oo);
  H.x_io.push_back(oi);
  for (uint32_t l = 0, i = 0; l <= nL; ++l) {
    while (i < nXc && level[xo[i]] < l) ++i;
    H.lvl.push_back(i);
  }
  for (uint32_t i = 0; i < nE; ++i) { H.e_pc.push_back(spc[es[i]]); H.e_cu.push_back(ecu[i]); H.e_eu.push_back(eeu[i]); }
  // roots
  uint32_t nR = 0;
  if (entry != NONE32) {
    H.roots.push_back(xnew[cloc[comp[entry]]]);
    nR = 1;
  } else {
    std::vector<uint32_t> rs;
    for (uint32_t xc = 0; xc < nXc; ++xc) if (cin[xc].empty()) rs.push_back(xc);
    std::sort(rs.begin(), rs.end(), [&](uint32_t p, uint32_t r) { return cx[p] < cx[r]; });
    for (uint32_t xc : rs) H.roots.push_back(xnew[xc]);
    nR = (uint32_t)rs.size();
  }
  // scopes owned by the reach functions
  std::vector<uint32_t> sc;
  for (uint32_t v : R) for (uint32_t s : scopes_of_func[v]) sc.push_back(s);
  std::sort(sc.begin(), sc.end());
  for (uint32_t s : sc) H.s_gid.push_back(s);
  d.nU = nU;
  d.nX = nXc;
  d.nE = nE;
  d.nL = nL;
  d.nR = nR;
  d.nS = (uint32_t)sc.size();
  H.ent.push_back(d);
}

}  // namespace

extern "C" hpa_status hpa_prepare_callgraph(hpa_ctx* ctx, const hpa_structure_map* map, const hpa_callgraph* g,
                                            const hpa_context_table* t, hipStream_t stream,
                                            hpa_callgraph_plan** out) {
  return guard([&] {
    if (!ctx || !map || !g || !t || !out) fail(HPA_E_INVAL, "NULL argument");
    if (map->ctx != ctx) fail(HPA_E_INVAL, "map belongs to another context");
    if (map->prebuilt) fail(HPA_E_INVAL, "a call graph needs a map built from scopes");
    const uint32_t V = g->n_funcs;
    if (V != map->n_ids) fail(HPA_E_INVAL, "n_funcs must equal the map's number of scope ids");
    if (g->n_sites && (!g->site_pc || !g->site_caller || !g->site_callee)) fail(HPA_E_INVAL, "NULL site array");
    if (t->n && (!t->parent || !t->kernel_entry)) fail(HPA_E_INVAL, "NULL context array");
    if (t->n == 0) fail(HPA_E_INVAL, "empty context table");
    DeviceGuard dg(ctx->device);
    std::vector<uint8_t> is_func(V, 0);
    for (uint32_t v = 0; v < V; ++v) is_func[v] = map->h_kind[v] == HPA_FUNC;
    const uint64_t E = g->n_sites;
    std::vector<uint64_t> spc(g->site_pc, g->site_pc + E);
    std::vector<uint32_t> scaller(g->site_caller, g->site_caller + E), scallee(g->site_callee, g->site_callee + E);
    std::vector<std::vector<uint32_t>> out_sites(V), adj(V);
    {
      std::vector<uint64_t> sorted = spc;
      std::sort(sorted.begin(), sorted.end());
      if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) fail(HPA_E_INVAL, "duplicate call-site pc");
    }
    for (uint64_t e = 0; e < E; ++e) {
      const uint32_t u = scaller[e], v = scallee[e];
      if (u >= V || v >= V || !is_func[u] || !is_func[v]) fail(HPA_E_INVAL, "call edge between non-functions");
      // the call instruction must lie in the caller's addresses
      auto it = std::upper_bound(map->h_start.begin(), map->h_start.end(), spc[e]);
      bool ok = it != map->h_start.begin();
      if (ok) {
        size_t i = (size_t)(it - map->h_start.begin()) - 1;
        ok = spc[e] < map->h_end[i] && map->h_func[map->h_scope[i]] == u;
      }
      if (!ok) fail(HPA_E_INVAL, "call site " + std::to_string(e) + " is not inside its caller");
      out_sites[u].push_back((uint32_t)e);
      adj[u].push_back(v);
    }
    const uint32_t C = t->n;
    std::vector<uint32_t> depth(C, 0);
    for (uint32_t c = 0; c < C; ++c) {
      if (t->parent[c] != NONE32 && t->parent[c] >= C) fail(HPA_E_INVAL, "context parent out of range");
      const int32_t k = t->kernel_entry[c];
      if (k < -1 || (k >= 0 && ((uint32_t)k >= V || !is_func[k]))) fail(HPA_E_INVAL, "kernel entry is not a function");
    }
    for (uint32_t c = 0; c < C; ++c) {
      uint32_t x = c, d = 0;
      while (t->parent[x] != NONE32) {
        x = t->parent[x];
        if (++d > C) fail(HPA_E_INVAL, "cycle in the context table");
      }
      depth[c] = d;
    }
    auto* P = new hpa_callgraph_plan();
    std::unique_ptr<hpa_callgraph_plan> hold(P);
    P->ctx = ctx;
    P->stream = stream;
    P->map = map;
    P->V = V;
    P->n_ctx = C;
    P->h_scc = scc_of(V, adj);
    P->h_parent.assign(t->parent, t->parent + C);
    P->h_depth = depth;
    P->h_depth_order.resize(C);
    std::iota(P->h_depth_order.begin(), P->h_depth_order.end(), 0u);
    std::stable_sort(P->h_depth_order.begin(), P->h_depth_order.end(),
                     [&](uint32_t a, uint32_t b) { return depth[a] > depth[b]; });
    std::vector<std::vector<uint32_t>> scopes_of_func(V);
    for (uint32_t s = 0; s < V; ++s)
      if (map->h_func[s] != NONE32 && map->h_kind[s] != 0xFF) scopes_of_func[map->h_func[s]].push_back(s);
    // one local plan per distinct entry (and one for contexts without an entry)
    HostPlan H;
    std::map<int32_t, int32_t> plan_of;
    P->h_ctx_ent.assign(C, 0);
    for (uint32_t c = 0; c < C; ++c) {
      const int32_t k = t->kernel_entry[c];
      auto it = plan_of.find(k);
      if (it == plan_of.end()) {
        int32_t id = (int32_t)H.ent.size();
        build_entry(k < 0 ? NONE32 : (uint32_t)k, V, is_func, out_sites, spc, scaller, scallee, P->h_scc,
                    scopes_of_func, H);
        it = plan_of.emplace(k, id).first;
      }
      P->h_ctx_ent[c] = it->second;
    }
    P->n_ent = (uint32_t)H.ent.size();
    for (auto& d : H.ent) {
      P->maxU = std::max(P->maxU, d.nU);
      P->maxX = std::max(P->maxX, d.nX);
      P->maxE = std::max(P->maxE, d.nE);
      P->maxS = std::max(P->maxS, d.nS);
    }
    P->h_ent = H.ent;
    auto up32 = [&](const std::vector<uint32_t>& v) { return upload(ctx, v, stream); };
    P->scc = up32(P->h_scc);
    P->ent = upload(ctx, H.ent, stream);
    P->ctx_ent = upload(ctx, P->h_ctx_ent, stream);
    P->u_gid = up32(H.u_gid); P->u_x = up32(H.u_x); P->u_oo = up32(H.u_oo); P->u_oe = up32(H.u_oe);
    P->x_gid = up32(H.x_gid); P->x_mo = up32(H.x_mo); P->x_mem = up32(H.x_mem); P->x_oo = up32(H.x_oo);
    P->x_oe = up32(H.x_oe); P->x_io = up32(H.x_io); P->x_ie = up32(H.x_ie); P->lvl = up32(H.lvl);
    P->roots = up32(H.roots); P->e_cu = up32(H.e_cu); P->e_eu = up32(H.e_eu); P->s_gid = up32(H.s_gid);
    P->e_pc = upload(ctx, H.e_pc, stream);
    P->ctx_parent = up32(P->h_parent);
    P->depth_order = up32(P->h_depth_order);
    P->h_depth_lvl.push_back(0);
    for (uint32_t i = 1; i <= C; ++i)
      if (i == C || depth[P->h_depth_order[i]] != depth[P->h_depth_order[i - 1]]) P->h_depth_lvl.push_back(i);
    P->depth_lvl = up32(P->h_depth_lvl);
    sync_stream(ctx, stream);
    *out = hold.release();
  });
}

extern "C" void hpa_callgraph_plan_free(hpa_callgraph_plan* p) { delete p; }

struct hpa_gpu_cct {
  hpa_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  const hpa_callgraph_plan* plan = nullptr;
  const hpa_attribution* attr = nullptr;
  uint64_t n_nodes = 0, n_w = 0;
  DBuf node_off, parent, node, site, kind, phi, excl, size, depth, w_off, w_site, w_val;
};

namespace hpa {
// accessors used by derive.hip
const uint64_t* cct_node_off(const hpa_gpu_cct* t) { return t->node_off.as<uint64_t>(); }
const uint32_t* cct_parent(const hpa_gpu_cct* t) { return t->parent.as<uint32_t>(); }
const uint64_t* cct_size(const hpa_gpu_cct* t) { return t->size.as<uint64_t>(); }
const uint32_t* cct_depth(const hpa_gpu_cct* t) { return t->depth.as<uint32_t>(); }
const double* cct_excl(const hpa_gpu_cct* t) { return t->excl.as<double>(); }
uint64_t cct_n_nodes(const hpa_gpu_cct* t) { return t->n_nodes; }
const hpa_callgraph_plan* cct_plan(const hpa_gpu_cct* t) { return t->plan; }
const hpa_attribution* cct_attr(const hpa_gpu_cct* t) { return t->attr; }
PlanDev plan_dev(const hpa_callgraph_plan* p) { return p->dev(); }
uint32_t plan_max_scopes(const hpa_callgraph_plan* p) { return p->maxS; }
uint32_t plan_n_ctx(const hpa_callgraph_plan* p) { return p->n_ctx; }
const hpa_structure_map* plan_map(const hpa_callgraph_plan* p) { return p->map; }
const uint32_t* plan_ctx_parent(const hpa_callgraph_plan* p) { return p->ctx_parent.as<uint32_t>(); }
const uint32_t* plan_depth_order(const hpa_callgraph_plan* p) { return p->depth_order.as<uint32_t>(); }
const std::vector<uint32_t>& plan_h_depth(const hpa_callgraph_plan* p) { return p->h_depth; }
const std::vector<uint32_t>& plan_h_depth_order(const hpa_callgraph_plan* p) { return p->h_depth_order; }
const uint32_t* plan_depth_lvl(const hpa_callgraph_plan* p) { return p->depth_lvl.as<uint32_t>(); }
uint32_t plan_n_depth_lvl(const hpa_callgraph_plan* p) { return (uint32_t)p->h_depth_lvl.size() - 1; }
}  // namespace hpa

namespace {
void check_err(unsigned int err) {
  if (!err) return;
  std::string m = "apportioning stopped on invalid data:";
  if (err & ERR_SCOPE) m += " a scope label is out of range;";
  if (err & ERR_STALL) m += " a stall reason is out of range;";
  if (err & (ERR_ROW | ERR_QUEUE | ERR_NODE)) m += " internal capacity check failed;";
  fail(HPA_E_DEVICE, m);
}
}  // namespace

extern "C" hpa_status hpa_apportion_callpaths(hpa_ctx* ctx, const hpa_callgraph_plan* plan,
                                              const hpa_attribution* attr, const hpa_apportion_opts* opts,
                                              hipStream_t stream, hpa_gpu_cct** out) {
  return guard([&] {
    if (!ctx || !plan || !attr || !out) fail(HPA_E_INVAL, "NULL argument");
    if (plan->ctx != ctx || attr->ctx != ctx) fail(HPA_E_INVAL, "handles belong to another context");
    if (attr->map != plan->map) fail(HPA_E_INVAL, "attribution and plan use different structure maps");
    if (attr->n_ctx != plan->n_ctx) fail(HPA_E_INVAL, "attribution and plan have different context counts");
    const int sample_based = opts ? opts->sample_based : 1;
#ifndef HPA_ENABLE_GPU_CCT
    fail(HPA_E_UNSUPPORTED, "GPU call-path apportioning is compiled out (build with HPA_ENABLE_GPU_CCT): its kernels "
                            "stopped making progress on the device on a 4-context, 500-sample case, cause not found");
#endif
    DeviceGuard dg(ctx->device);
    hipStream_t s = stream;
    const uint32_t C = plan->n_ctx;
    auto* T = new hpa_gpu_cct();
    std::unique_ptr<hpa_gpu_cct> hold(T);
    T->ctx = ctx;
    T->stream = s;
    T->plan = plan;
    T->attr = attr;
    DBuf d_nn(ctx, (uint64_t)C * 8, s), d_nw(ctx, (uint64_t)C * 8, s), d_tot(ctx, 32, s), d_ticket(ctx, 8, s),
        d_err(ctx, 8, s);
    HPA_HIP(hipMemsetAsync(d_err.p, 0, 8, s));
    HPA_HIP(hipMemsetAsync(d_nn.p, 0, (uint64_t)C * 8, s));
    HPA_HIP(hipMemsetAsync(d_nw.p, 0, (uint64_t)C * 8, s));
    HPA_HIP(hipMemsetAsync(d_ticket.p, 0, 8, s));
    T->node_off = DBuf(ctx, ((uint64_t)C + 1) * 8, s);
    T->w_off = DBuf(ctx, ((uint64_t)C + 1) * 8, s);
    const uint32_t n_wg = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(C, (uint64_t)ctx->n_cu * 8));
    AppArgs a{};
    a.p = plan->dev();
    a.k_ctx = attr->ctx_id.as<uint32_t>();
    a.k_pc = attr->pc.as<uint64_t>();
    a.k_stall = attr->stall.as<uint8_t>();
    a.k_count = attr->count.as<unsigned long long>();
    a.k_scope = attr->scope.as<uint32_t>();
    a.ctx_off = attr->ctx_offsets.as<uint64_t>();
    a.func = plan->map->func.as<uint32_t>();
    a.n_ids = plan->map->n_ids;
    a.err = d_err.as<unsigned int>();
    a.n_ctx = C;
    a.ticket = d_ticket.as<unsigned int>();
    a.sample_based = sample_based ? 1 : 0;
    a.maxU = std::max(plan->maxU, 1u);
    a.maxX = std::max(plan->maxX, 1u);
    a.maxE = std::max(plan->maxE, 1u);
    a.q_cap = 1;
    a.n_nodes = d_nn.as<unsigned long long>();
    a.n_w = d_nw.as<unsigned long long>();
    // counting pass
    {
      WsLayout L = ws_layout(a.maxU, a.maxX, a.maxE, a.q_cap);
      a.ws_stride = L.total;
      DBuf ws(ctx, L.total * n_wg, s);
      a.ws = ws.as<uint8_t>();
      a.emit = 0;
      k_apportion<<<n_wg, ABLOCK, 0, s>>>(a);
      HPA_HIP(hipGetLastError());
      k_cct_scan<<<1, 1024, 0, s>>>(d_nn.as<unsigned long long>(), d_nw.as<unsigned long long>(), C,
                                    T->node_off.as<uint64_t>(), T->w_off.as<uint64_t>(),
                                    d_tot.as<unsigned long long>());
      HPA_HIP(hipGetLastError());
    }
    unsigned long long tot[3];
    unsigned int err = 0;
    HPA_HIP(hipMemcpyAsync(tot, d_tot.p, sizeof(tot), hipMemcpyDeviceToHost, s));
    HPA_HIP(hipMemcpyAsync(&err, d_err.p, sizeof(err), hipMemcpyDeviceToHost, s));
    sync_stream(ctx, s);
    check_err(err);
    if (opts && opts->required_nodes) *opts->required_nodes = tot[0];
    if (tot[0] >= SAT) fail(HPA_E_BUDGET, "the calling context tree has more than 2^62 nodes");
    if (opts && opts->max_cct_nodes && tot[0] > opts->max_cct_nodes)
      fail(HPA_E_BUDGET, "the calling context tree needs " + std::to_string(tot[0]) + " nodes");
    T->n_nodes = tot[0];
    T->n_w = tot[1];
    const uint64_t nn = std::max<uint64_t>(tot[0], 1), nw = std::max<uint64_t>(tot[1], 1);
    T->parent = DBuf(ctx, nn * 4, s);
    T->node = DBuf(ctx, nn * 4, s);
    T->site = DBuf(ctx, nn * 8, s);
    T->kind = DBuf(ctx, nn, s);
    T->phi = DBuf(ctx, nn * 8, s);
    T->excl = DBuf(ctx, nn * 8 * NS, s);
    T->size = DBuf(ctx, nn * 8, s);
    T->depth = DBuf(ctx, nn * 4, s);
    T->w_site = DBuf(ctx, nw * 8, s);
    T->w_val = DBuf(ctx, nw * 8, s);
    // emission pass
    if (tot[0] || tot[1]) {
      a.q_cap = std::max<uint64_t>(tot[2], 1);
      WsLayout L = ws_layout(a.maxU, a.maxX, a.maxE, a.q_cap);
      a.ws_stride = L.total;
      DBuf ws(ctx, L.total * n_wg, s);
      a.ws = ws.as<uint8_t>();
      HPA_HIP(hipMemsetAsync(d_ticket.p, 0, 8, s));
      a.emit = 1;
      a.node_off = T->node_off.as<uint64_t>();
      a.w_off = T->w_off.as<uint64_t>();
      a.o_parent = T->parent.as<uint32_t>();
      a.o_node = T->node.as<uint32_t>();
      a.o_site = T->site.as<uint64_t>();
      a.o_kind = T->kind.as<uint8_t>();
      a.o_phi = T->phi.as<double>();
      a.o_excl = T->excl.as<double>();
      a.o_size = T->size.as<uint64_t>();
      a.o_depth = T->depth.as<uint32_t>();
      a.o_wsite = T->w_site.as<uint64_t>();
      a.o_wval = T->w_val.as<uint64_t>();
      k_apportion<<<n_wg, ABLOCK, 0, s>>>(a);
      HPA_HIP(hipGetLastError());
      HPA_HIP(hipMemcpyAsync(&err, d_err.p, sizeof(err), hipMemcpyDeviceToHost, s));
      sync_stream(ctx, s);
      check_err(err);
    }
    *out = hold.release();
  });
}

extern "C" hpa_status hpa_gpu_cct_view_get(const hpa_gpu_cct* t, hpa_gpu_cct_view* v) {
  return guard([&] {
    if (!t || !v) fail(HPA_E_INVAL, "NULL argument");
    v->n_nodes = t->n_nodes;
    v->n_ctx = t->plan->n_ctx;
    v->n_funcs = t->plan->V;
    v->scc = t->plan->scc.as<uint32_t>();
    v->node_offsets = t->node_off.as<uint64_t>();
    v->parent = t->parent.as<uint32_t>();
    v->node = t->node.as<uint32_t>();
    v->site = t->site.as<uint64_t>();
    v->kind = t->kind.as<uint8_t>();
    v->phi = t->phi.as<double>();
    v->excl = t->excl.as<double>();
    v->n_weights = t->n_w;
    v->w_offsets = t->w_off.as<uint64_t>();
    v->w_site = t->w_site.as<uint64_t>();
    v->w_val = t->w_val.as<uint64_t>();
  });
}

extern "C" void hpa_gpu_cct_free(hpa_gpu_cct* t) { delete t; }
