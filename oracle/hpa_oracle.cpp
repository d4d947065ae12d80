// Plain CPU oracle for GPU PC-sample attribution (test infrastructure only).
//
// This file is the slow, obviously-correct reference that the GPU library is
// checked against.  It is single-threaded, uses std::sort / std::map / plain
// loops, and shares no source with the GPU path.  Only the tests, the smoke
// check and the CPU-baseline leg of the benchmark load it.
//
// Paper: Zhou et al., "Measurement and Analysis of GPU-accelerated
// Applications with HPCToolkit", Parallel Computing 2021 (arXiv 2109.06931).
//
//   Structure map ......... Section 5 (relocating and splitting overlapping GPU
//                           functions; line map and inlined code from DWARF;
//                           loop nests) and Section 6.1 "Calling Context
//                           Expansion" (instruction -> lines, inlined code, loops).
//   Attribution ........... Section 4.2 (a PC sample = instruction address,
//                           stall reason, count, under a kernel placeholder) and
//                           Section 4.5 (a raw metric is the sum of measured values).
//   Apportioning .......... Section 6.3, steps 1-4 (static call graph weighted by
//                           call-instruction samples; zero-in-weight propagation;
//                           Tarjan SCCs; gprof-style splitting into a CCT).
//   Derived metrics ....... Section 6.1 "Statistic Generation" (propagate values
//                           up the tree) and Section 7.1 (warp issue rate
//                           W = (S - S_stall) / S).
//
// Where the paper is silent, ambiguous or self-contradictory, these readings
// are used:
//   R1 a record without a weight counts once;
//   R2 stall reason 0 is "not stalled", 1..15 are stalls;
//   R3 unmapped PCs are kept under scope UNMAPPED and an <unknown> CCT node;
//   R4 overlapping functions: an address belongs to the containing function
//      with the largest start, then the smallest end, then the smallest id;
//   R5 inline/loop ranges form a laminar family, each inside one function's
//      owned addresses; equal ranges nest FUNC > INLINE > LOOP, lower id outer;
//   R6 step 2 is the least fixpoint of its rule;
//   R7 after SCC condensation the step-2 rule is applied once more on the
//      condensed graph (fixes an SCC left with 0/0);
//   R8 a context with a kernel entry uses the graph restricted to the entry's
//      reach; samples outside it go to an <unreachable> node;
//   R9 multi-level splitting multiplies the per-level ratios;
//   R10 an SCC is one CCT node carrying the sum over its members;
//   R11 zero-cost paths are pruned by an integer has-cost test;
//   R12 floating point is evaluated in the fixed orders written below;
//   R13 canonical orders: keys by (ctx, pc, stall); CCT in DFS preorder with
//       children by call-site PC; SCC ids by smallest member.

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <utility>
#include <vector>

namespace {

constexpr int ORC_OK = 0, ORC_INVAL = -1, ORC_UNSORTED = -2, ORC_OVERLAP = -3,
              ORC_NOT_LAMINAR = -4, ORC_BUDGET = -6;
constexpr uint32_t NONE32 = 0xFFFFFFFFu;
constexpr uint64_t NONE64 = 0xFFFFFFFFFFFFFFFFull;
constexpr int NS = 16;  // stall reasons
constexpr uint32_t K_FUNC = 0, K_INLINE = 1, K_LOOP = 2, K_UNUSED = 0xFF;

using Row = std::array<uint64_t, NS>;

// ----------------------------------------------------------------------------
// Structure map
// ----------------------------------------------------------------------------
struct Map {
  std::vector<uint64_t> start, end;           // elementary intervals [start, end)
  std::vector<uint32_t> scope, file, line;    // label of each interval
  std::vector<uint32_t> parent, func;         // scope table, indexed by scope id
  std::vector<uint8_t> kind;
};

struct Rng {
  uint64_t s, e;
  uint32_t id, kind;
};

// Elementary segment owner / innermost computation (Section 5; readings R4, R5).
int build_map(const uint64_t* ss, const uint64_t* se, const uint32_t* sid, const uint32_t* sk,
              uint64_t ns, const uint64_t* ls, const uint64_t* le, const uint32_t* lf,
              const uint32_t* ll, uint64_t nl, Map& m) {
  uint32_t n_ids = 0;
  std::map<uint32_t, uint32_t> kind_of;
  std::vector<Rng> funcs, others;
  for (uint64_t i = 0; i < ns; ++i) {
    if (ss[i] >= se[i] || sk[i] > K_LOOP || sid[i] >= 0x7FFFFFFFu) return ORC_INVAL;
    auto it = kind_of.find(sid[i]);
    if (it != kind_of.end() && it->second != sk[i]) return ORC_INVAL;
    kind_of[sid[i]] = sk[i];
    n_ids = std::max(n_ids, sid[i] + 1);
    Rng r{ss[i], se[i], sid[i], sk[i]};
    (sk[i] == K_FUNC ? funcs : others).push_back(r);
  }
  // line ranges: non-overlapping (an overlap is an error, not a tie to break)
  std::vector<Rng> lines;
  for (uint64_t i = 0; i < nl; ++i) {
    if (ls[i] >= le[i]) return ORC_INVAL;
    lines.push_back(Rng{ls[i], le[i], (uint32_t)i, 0});
  }
  std::sort(lines.begin(), lines.end(), [](const Rng& a, const Rng& b) { return a.s < b.s; });
  for (size_t i = 1; i < lines.size(); ++i)
    if (lines[i].s < lines[i - 1].e) return ORC_OVERLAP;

  // all boundaries
  std::vector<uint64_t> B;
  for (auto& r : funcs) { B.push_back(r.s); B.push_back(r.e); }
  for (auto& r : others) { B.push_back(r.s); B.push_back(r.e); }
  for (auto& r : lines) { B.push_back(r.s); B.push_back(r.e); }
  std::sort(B.begin(), B.end());
  B.erase(std::unique(B.begin(), B.end()), B.end());
  size_t nseg = B.empty() ? 0 : B.size() - 1;

  // owner function of each segment: max start, then min end, then min id (R4)
  auto fcmp = [](const Rng& a, const Rng& b) {
    if (a.s != b.s) return a.s > b.s;
    if (a.e != b.e) return a.e < b.e;
    return a.id < b.id;
  };
  // innermost non-function scope: max start, then min end, then kind LOOP
  // inside INLINE, then higher id inside lower id (R5)
  auto icmp = [](const Rng& a, const Rng& b) {
    if (a.s != b.s) return a.s > b.s;
    if (a.e != b.e) return a.e < b.e;
    if (a.kind != b.kind) return a.kind > b.kind;
    return a.id > b.id;
  };
  std::vector<uint32_t> seg_owner(nseg, NONE32), seg_inner(nseg, NONE32), seg_file(nseg, 0),
      seg_line(nseg, 0);
  {
    // events: at each boundary index, ranges starting / ending there
    std::vector<std::vector<Rng>> fstart(B.size()), fend(B.size()), ostart(B.size()), oend(B.size());
    auto idx = [&](uint64_t a) { return (size_t)(std::lower_bound(B.begin(), B.end(), a) - B.begin()); };
    for (auto& r : funcs) { fstart[idx(r.s)].push_back(r); fend[idx(r.e)].push_back(r); }
    for (auto& r : others) { ostart[idx(r.s)].push_back(r); oend[idx(r.e)].push_back(r); }
    std::multiset<Rng, decltype(fcmp)> af(fcmp);
    std::multiset<Rng, decltype(icmp)> ao(icmp);
    size_t li = 0;
    for (size_t i = 0; i < nseg; ++i) {
      for (auto& r : fend[i]) af.erase(af.find(r));
      for (auto& r : oend[i]) ao.erase(ao.find(r));
      for (auto& r : fstart[i]) af.insert(r);
      for (auto& r : ostart[i]) ao.insert(r);
      if (!af.empty()) seg_owner[i] = af.begin()->id;
      if (!ao.empty()) seg_inner[i] = ao.begin()->id;
      while (li < lines.size() && lines[li].e <= B[i]) ++li;
      if (li < lines.size() && lines[li].s <= B[i] && B[i] < lines[li].e) {
        seg_file[i] = lf[lines[li].id];
        seg_line[i] = ll[lines[li].id];
      }
    }
  }

  // scope table and laminarity (R5)
  m.kind.assign(n_ids, (uint8_t)K_UNUSED);
  m.parent.assign(n_ids, NONE32);
  m.func.assign(n_ids, NONE32);
  for (auto& kv : kind_of) m.kind[kv.first] = (uint8_t)kv.second;
  for (auto& r : funcs) m.func[r.id] = r.id;
  std::vector<uint8_t> seen(n_ids, 0);
  {
    std::vector<Rng> o = others;
    std::sort(o.begin(), o.end(), [](const Rng& a, const Rng& b) {
      if (a.s != b.s) return a.s < b.s;
      if (a.e != b.e) return a.e > b.e;
      if (a.kind != b.kind) return a.kind < b.kind;
      return a.id < b.id;
    });
    std::vector<Rng> stack;
    for (auto& r : o) {
      while (!stack.empty() && stack.back().e <= r.s) stack.pop_back();
      if (!stack.empty() && (r.e > stack.back().e || stack.back().id == r.id)) return ORC_NOT_LAMINAR;
      // owner must be one function over the whole range
      size_t a = (size_t)(std::lower_bound(B.begin(), B.end(), r.s) - B.begin());
      size_t b = (size_t)(std::lower_bound(B.begin(), B.end(), r.e) - B.begin());
      uint32_t own = seg_owner[a];
      if (own == NONE32) return ORC_NOT_LAMINAR;
      for (size_t k = a; k < b; ++k)
        if (seg_owner[k] != own) return ORC_NOT_LAMINAR;
      uint32_t par = stack.empty() ? own : stack.back().id;
      if (seen[r.id]) {
        if (m.parent[r.id] != par || m.func[r.id] != own) return ORC_NOT_LAMINAR;
      } else {
        seen[r.id] = 1;
        m.parent[r.id] = par;
        m.func[r.id] = own;
      }
      stack.push_back(r);
    }
  }

  // label each owned segment and merge equal touching neighbours
  for (size_t i = 0; i < nseg; ++i) {
    if (seg_owner[i] == NONE32) continue;
    uint32_t sc = seg_inner[i] != NONE32 ? seg_inner[i] : seg_owner[i];
    if (!m.start.empty() && m.end.back() == B[i] && m.scope.back() == sc &&
        m.file.back() == seg_file[i] && m.line.back() == seg_line[i]) {
      m.end.back() = B[i + 1];
    } else {
      m.start.push_back(B[i]);
      m.end.push_back(B[i + 1]);
      m.scope.push_back(sc);
      m.file.push_back(seg_file[i]);
      m.line.push_back(seg_line[i]);
    }
  }
  return ORC_OK;
}

// Interval containing pc, or NONE32 (Section 6.1, calling-context expansion).
uint32_t lookup(const Map& m, uint64_t pc) {
  auto it = std::upper_bound(m.start.begin(), m.start.end(), pc);
  if (it == m.start.begin()) return NONE32;
  size_t i = (size_t)(it - m.start.begin()) - 1;
  return pc < m.end[i] ? (uint32_t)i : NONE32;
}

// ----------------------------------------------------------------------------
// Attribution: count[(ctx, pc, stall)] += weight  (Sections 4.2, 4.5)
// ----------------------------------------------------------------------------
struct Attr {
  uint32_t n_ctx = 0;
  std::vector<uint32_t> ctx, scope;
  std::vector<uint64_t> pc, count, ctx_off;
  std::vector<uint8_t> stall;
};

struct Key {
  uint32_t ctx;
  uint64_t pc;
  uint8_t stall;
  bool operator<(const Key& o) const {
    if (ctx != o.ctx) return ctx < o.ctx;
    if (pc != o.pc) return pc < o.pc;
    return stall < o.stall;
  }
  bool operator==(const Key& o) const { return ctx == o.ctx && pc == o.pc && stall == o.stall; }
};

int attribute(const Map& m, const uint64_t* pc, const uint32_t* ctx, const uint8_t* stall,
              const uint32_t* weight, uint64_t n, uint32_t n_ctx, const uint8_t* ctx_mask, Attr& a) {
  std::vector<std::pair<Key, uint64_t>> v;
  for (uint64_t i = 0; i < n; ++i) {
    if (stall[i] >= NS || ctx[i] >= n_ctx) return ORC_INVAL;
    if (ctx_mask && !ctx_mask[ctx[i]]) continue;
    v.push_back({Key{ctx[i], pc[i], stall[i]}, weight ? (uint64_t)weight[i] : 1ull});
  }
  std::sort(v.begin(), v.end(), [](const std::pair<Key, uint64_t>& x, const std::pair<Key, uint64_t>& y) {
    return x.first < y.first;
  });
  a.n_ctx = n_ctx;
  for (size_t i = 0; i < v.size(); ++i) {
    if (i > 0 && v[i].first == v[i - 1].first) {
      a.count.back() += v[i].second;
      continue;
    }
    a.ctx.push_back(v[i].first.ctx);
    a.pc.push_back(v[i].first.pc);
    a.stall.push_back(v[i].first.stall);
    a.count.push_back(v[i].second);
    uint32_t iv = lookup(m, v[i].first.pc);
    a.scope.push_back(iv == NONE32 ? NONE32 : m.scope[iv]);
  }
  a.ctx_off.assign((size_t)n_ctx + 1, 0);
  for (uint32_t c : a.ctx) a.ctx_off[(size_t)c + 1]++;
  for (uint32_t c = 0; c < n_ctx; ++c) a.ctx_off[c + 1] += a.ctx_off[c];
  return ORC_OK;
}

// ----------------------------------------------------------------------------
// GPU calling context tree (Section 6.3)
// ----------------------------------------------------------------------------
struct Cct {
  std::vector<uint32_t> scc;                      // condensed id per function node
  std::vector<uint64_t> node_off;                 // CSR over host contexts
  std::vector<uint32_t> parent, node;             // parent: ctx-local index or NONE32
  std::vector<uint64_t> site;                     // call site pc of the edge into the node
  std::vector<uint8_t> kind;                      // 0 call path node, 1 unreachable, 2 unknown
  std::vector<double> phi, excl;                  // excl: nodes x 16
  std::vector<uint64_t> w_off, w_site, w_val;     // final edge weights per context (w' > 0)
};

struct Graph {
  uint32_t V = 0;
  std::vector<uint64_t> pc;
  std::vector<uint32_t> caller, callee;
  std::vector<std::vector<uint32_t>> out, in;  // site indices
};

// Tarjan's algorithm, iterative (Section 6.3 step 3); ids then renumbered by
// smallest member so that the labelling does not depend on visit order.
std::vector<uint32_t> tarjan(const Graph& g) {
  const uint32_t V = g.V;
  std::vector<int64_t> index(V, -1), low(V, 0);
  std::vector<uint8_t> on(V, 0);
  std::vector<uint32_t> comp(V, NONE32), st;
  int64_t next = 0;
  uint32_t ncomp = 0;
  for (uint32_t root = 0; root < V; ++root) {
    if (index[root] >= 0) continue;
    std::vector<std::pair<uint32_t, size_t>> call;  // (node, next out-edge position)
    call.push_back({root, 0});
    index[root] = low[root] = next++;
    st.push_back(root);
    on[root] = 1;
    while (!call.empty()) {
      uint32_t v = call.back().first;
      size_t& k = call.back().second;
      if (k < g.out[v].size()) {
        uint32_t w = g.callee[g.out[v][k++]];
        if (index[w] < 0) {
          index[w] = low[w] = next++;
          st.push_back(w);
          on[w] = 1;
          call.push_back({w, 0});
        } else if (on[w]) {
          low[v] = std::min(low[v], index[w]);
        }
      } else {
        if (low[v] == index[v]) {
          while (true) {
            uint32_t w = st.back();
            st.pop_back();
            on[w] = 0;
            comp[w] = ncomp;
            if (w == v) break;
          }
          ++ncomp;
        }
        call.pop_back();
        if (!call.empty()) {
          uint32_t u = call.back().first;
          low[u] = std::min(low[u], low[v]);
        }
      }
    }
  }
  std::vector<uint32_t> minm(ncomp, NONE32);
  for (uint32_t v = 0; v < V; ++v) minm[comp[v]] = std::min(minm[comp[v]], v);
  std::vector<uint32_t> ord(ncomp);
  for (uint32_t i = 0; i < ncomp; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return minm[a] < minm[b]; });
  std::vector<uint32_t> rank(ncomp);
  for (uint32_t i = 0; i < ncomp; ++i) rank[ord[i]] = i;
  for (uint32_t v = 0; v < V; ++v) comp[v] = rank[comp[v]];
  return comp;
}

int apportion(const Map& m, const Graph& g, uint32_t n_ctx, const uint32_t* cpar, const int32_t* centry,
              const Attr& a, int sample_based, uint64_t max_nodes, uint64_t* required, Cct& out) {
  const uint32_t V = g.V;
  out.scc = tarjan(g);
  const std::vector<uint32_t>& comp = out.scc;
  uint32_t nC = 0;
  for (uint32_t v = 0; v < V; ++v) nC = std::max(nC, comp[v] + 1);
  // static zero-in-degree condensed nodes (roots when a context has no entry)
  std::vector<uint8_t> has_ext_in(nC, 0);
  for (size_t e = 0; e < g.pc.size(); ++e)
    if (comp[g.caller[e]] != comp[g.callee[e]]) has_ext_in[comp[g.callee[e]]] = 1;
  // members of each condensed node
  std::vector<std::vector<uint32_t>> members(nC);
  for (uint32_t v = 0; v < V; ++v) members[comp[v]].push_back(v);

  out.node_off.assign((size_t)n_ctx + 1, 0);
  out.w_off.assign((size_t)n_ctx + 1, 0);
  std::vector<uint32_t> stamp(V, NONE32);  // stamp[v] == c  <=>  v in reach for context c
  for (uint32_t c = 0; c < n_ctx; ++c) {
    out.node_off[c] = out.parent.size();
    out.w_off[c] = out.w_site.size();
    uint64_t k0 = a.ctx_off[c], k1 = a.ctx_off[c + 1];
    if (k0 == k1) continue;
    // ---- self costs and call-instruction sample totals (step 1) ----
    std::map<uint32_t, Row> self;   // function -> per-stall sample sums
    std::map<uint64_t, uint64_t> pc_total;
    Row unknown{}, unreach{};
    for (uint64_t k = k0; k < k1; ++k) {
      pc_total[a.pc[k]] += a.count[k];
      if (a.scope[k] == NONE32) { unknown[a.stall[k]] += a.count[k]; continue; }
      uint32_t f = m.func[a.scope[k]];
      self[f][a.stall[k]] += a.count[k];
    }
    // ---- reach restriction (R8) ----
    int32_t entry = centry[c];
    if (entry >= 0) {
      std::vector<uint32_t> q{(uint32_t)entry};
      stamp[entry] = c;
      for (size_t qi = 0; qi < q.size(); ++qi)
        for (uint32_t e : g.out[q[qi]])
          if (stamp[g.callee[e]] != c) { stamp[g.callee[e]] = c; q.push_back(g.callee[e]); }
    } else {
      for (uint32_t v = 0; v < V; ++v) stamp[v] = c;
    }
    auto inR = [&](uint32_t v) { return stamp[v] == c; };
    for (auto it = self.begin(); it != self.end();) {
      if (!inR(it->first)) {
        for (int s = 0; s < NS; ++s) unreach[s] += it->second[s];
        it = self.erase(it);
      } else {
        ++it;
      }
    }
    std::vector<uint32_t> R;
    for (uint32_t v = 0; v < V; ++v) if (inR(v)) R.push_back(v);
    auto rowsum = [](const Row& r) { uint64_t t = 0; for (auto x : r) t += x; return t; };
    // edge weights w(e) for sites whose caller is in reach
    std::map<uint32_t, uint64_t> w;  // site index -> weight
    for (uint32_t v : R)
      for (uint32_t e : g.out[v]) {
        auto it = pc_total.find(g.pc[e]);
        w[e] = it == pc_total.end() ? 0 : it->second;
      }
    // ---- step 2: least fixpoint of the zero-in-weight rule (R6) ----
    std::map<uint32_t, uint64_t> w1 = w;
    if (sample_based) {
      std::set<uint32_t> fires;
      auto inzero = [&](uint32_t f) {
        for (uint32_t e : g.in[f]) if (inR(g.caller[e]) && w.at(e) != 0) return false;
        return true;
      };
      auto active0 = [&](uint32_t f) {
        auto it = self.find(f);
        if (it != self.end() && rowsum(it->second) > 0) return true;
        for (uint32_t e : g.out[f]) if (w.at(e) > 0) return true;
        return false;
      };
      bool changed = true;
      while (changed) {
        changed = false;
        for (uint32_t f : R) {
          if (fires.count(f) || !inzero(f)) continue;
          bool act = active0(f);
          for (uint32_t e : g.out[f]) if (fires.count(g.callee[e])) act = true;
          if (act) { fires.insert(f); changed = true; }
        }
      }
      for (auto& kv : w1)
        if (kv.second == 0 && fires.count(g.callee[kv.first])) kv.second = 1;
    }
    // ---- step 3: condensation; R7 re-applies the step-2 rule on it ----
    std::map<uint32_t, Row> selfX;
    for (auto& kv : self)
      for (int s = 0; s < NS; ++s) selfX[comp[kv.first]][s] += kv.second[s];
    std::vector<uint32_t> RX;  // condensed nodes in reach, ascending
    for (uint32_t v : R) RX.push_back(comp[v]);
    std::sort(RX.begin(), RX.end());
    RX.erase(std::unique(RX.begin(), RX.end()), RX.end());
    auto external = [&](uint32_t e) { return comp[g.caller[e]] != comp[g.callee[e]]; };
    std::map<uint32_t, uint64_t> w2 = w1;  // only external edges matter below
    if (sample_based) {
      std::set<uint32_t> firesX;
      auto inzeroX = [&](uint32_t X) {
        for (uint32_t v : members[X])
          for (uint32_t e : g.in[v])
            if (inR(g.caller[e]) && external(e) && w1.at(e) != 0) return false;
        return true;
      };
      auto active0X = [&](uint32_t X) {
        auto it = selfX.find(X);
        if (it != selfX.end() && rowsum(it->second) > 0) return true;
        for (uint32_t v : members[X])
          for (uint32_t e : g.out[v]) if (inR(v) && external(e) && w1.at(e) > 0) return true;
        return false;
      };
      bool changed = true;
      while (changed) {
        changed = false;
        for (uint32_t X : RX) {
          if (firesX.count(X) || !inzeroX(X)) continue;
          bool act = active0X(X);
          for (uint32_t v : members[X])
            for (uint32_t e : g.out[v])
              if (inR(v) && external(e) && firesX.count(comp[g.callee[e]])) act = true;
          if (act) { firesX.insert(X); changed = true; }
        }
      }
      for (auto& kv : w2)
        if (kv.second == 0 && external(kv.first) && firesX.count(comp[g.callee[kv.first]])) kv.second = 1;
    }
    // W'(X): total weight of external in-edges from inside reach
    std::map<uint32_t, uint64_t> WX;
    for (auto& kv : w2)
      if (external(kv.first)) WX[comp[g.callee[kv.first]]] += kv.second;
    // ---- has-cost (R11): integer, decided before any floating point ----
    std::set<uint32_t> hc;
    {
      bool changed = true;
      while (changed) {
        changed = false;
        for (uint32_t X : RX) {
          if (hc.count(X)) continue;
          auto it = selfX.find(X);
          bool h = it != selfX.end() && rowsum(it->second) > 0;
          for (uint32_t v : members[X])
            for (uint32_t e : g.out[v])
              if (inR(v) && external(e) && w2.at(e) > 0 && hc.count(comp[g.callee[e]])) h = true;
          if (h) { hc.insert(X); changed = true; }
        }
      }
    }
    // ---- step 4: unfold into a CCT (R9, R10, R12, R13) ----
    std::vector<uint32_t> roots;
    if (entry >= 0) roots.push_back(comp[entry]);
    else for (uint32_t X : RX) if (!has_ext_in[X]) roots.push_back(X);
    struct Frame { uint32_t X; uint32_t parent; uint64_t site; double phi; };
    for (uint32_t r : roots) {
      if (!hc.count(r)) continue;
      std::vector<Frame> stk{Frame{r, NONE32, NONE64, 1.0}};
      while (!stk.empty()) {
        Frame f = stk.back();
        stk.pop_back();
        uint32_t me = (uint32_t)(out.parent.size() - out.node_off[c]);
        out.parent.push_back(f.parent);
        out.node.push_back(f.X);
        out.site.push_back(f.site);
        out.kind.push_back(0);
        out.phi.push_back(f.phi);
        auto it = selfX.find(f.X);
        for (int s = 0; s < NS; ++s)
          out.excl.push_back((double)(it == selfX.end() ? 0 : it->second[s]) * f.phi);
        // children: external call sites out of the members, w' > 0, callee has cost,
        // ordered by call-site pc; pushed in reverse so they pop in order
        std::vector<uint32_t> kids;
        for (uint32_t v : members[f.X])
          for (uint32_t e : g.out[v])
            if (inR(v) && external(e) && w2.at(e) > 0 && hc.count(comp[g.callee[e]])) kids.push_back(e);
        std::sort(kids.begin(), kids.end(), [&](uint32_t x, uint32_t y) { return g.pc[x] < g.pc[y]; });
        for (size_t i = kids.size(); i-- > 0;) {
          uint32_t e = kids[i];
          uint32_t Y = comp[g.callee[e]];
          double ratio = (double)w2.at(e) / (double)WX.at(Y);
          stk.push_back(Frame{Y, me, g.pc[e], f.phi * ratio});
        }
      }
    }
    auto special = [&](const Row& r, uint8_t kind) {
      if (rowsum(r) == 0) return;
      out.parent.push_back(NONE32);
      out.node.push_back(NONE32);
      out.site.push_back(NONE64);
      out.kind.push_back(kind);
      out.phi.push_back(1.0);
      for (int s = 0; s < NS; ++s) out.excl.push_back((double)r[s]);
    };
    special(unreach, 1);
    special(unknown, 2);
    // final edge weights, by call-site pc
    std::vector<std::pair<uint64_t, uint64_t>> ws;
    for (auto& kv : w2)
      if (external(kv.first) && kv.second > 0) ws.push_back({g.pc[kv.first], kv.second});
    std::sort(ws.begin(), ws.end());
    for (auto& p : ws) { out.w_site.push_back(p.first); out.w_val.push_back(p.second); }
  }
  out.node_off[n_ctx] = out.parent.size();
  out.w_off[n_ctx] = out.w_site.size();
  if (required) *required = out.parent.size();
  if (max_nodes && out.parent.size() > max_nodes) return ORC_BUDGET;
  return ORC_OK;
}

// ----------------------------------------------------------------------------
// Derived metrics (Sections 6.1 and 7.1)
// ----------------------------------------------------------------------------
struct Derived {
  std::vector<double> incl, S, W;                   // per CCT node (incl: x16)
  std::vector<uint64_t> host_incl;                  // per host context x16
  std::vector<double> host_W;
  std::vector<uint64_t> sc_off, sc_val;             // static scope roll-up CSR (x16)
  std::vector<uint32_t> sc_scope;
};

double issue_rate(double S, double Sst) { return S == 0.0 ? 0.0 : (S - Sst) / S; }

void derive(const Map& m, const Attr& a, const Cct& t, uint32_t n_ctx, const uint32_t* cpar, Derived& d) {
  // GPU CCT: I(p,s) = E(p,s) + sum over children in child order (reverse preorder walk)
  size_t nn = t.parent.size();
  d.incl.assign(nn * NS, 0.0);
  d.S.assign(nn, 0.0);
  d.W.assign(nn, 0.0);
  for (uint32_t c = 0; c < n_ctx; ++c) {
    uint64_t b = t.node_off[c], e = t.node_off[c + 1];
    std::vector<std::vector<uint64_t>> kids(e - b);
    for (uint64_t i = b; i < e; ++i)
      if (t.parent[i] != NONE32) kids[t.parent[i]].push_back(i);
    for (uint64_t i = e; i-- > b;) {
      for (int s = 0; s < NS; ++s) {
        double v = t.excl[i * NS + s];
        for (uint64_t k : kids[i - b]) v = v + d.incl[k * NS + s];
        d.incl[i * NS + s] = v;
      }
      double S = 0.0, Sst = 0.0;
      for (int s = 0; s < NS; ++s) S = S + d.incl[i * NS + s];
      for (int s = 1; s < NS; ++s) Sst = Sst + d.incl[i * NS + s];
      d.S[i] = S;
      d.W[i] = issue_rate(S, Sst);
    }
  }
  // host calling-context tree: integer inclusive sums
  d.host_incl.assign((size_t)n_ctx * NS, 0);
  for (uint64_t k = 0; k < a.ctx.size(); ++k) d.host_incl[(size_t)a.ctx[k] * NS + a.stall[k]] += a.count[k];
  std::vector<uint32_t> depth(n_ctx, 0);
  for (uint32_t c = 0; c < n_ctx; ++c) {
    uint32_t x = c, dd = 0;
    while (cpar[x] != NONE32) { x = cpar[x]; ++dd; }
    depth[c] = dd;
  }
  std::vector<uint32_t> ord(n_ctx);
  for (uint32_t c = 0; c < n_ctx; ++c) ord[c] = c;
  std::stable_sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) { return depth[x] > depth[y]; });
  for (uint32_t c : ord)
    if (cpar[c] != NONE32)
      for (int s = 0; s < NS; ++s) d.host_incl[(size_t)cpar[c] * NS + s] += d.host_incl[(size_t)c * NS + s];
  d.host_W.assign(n_ctx, 0.0);
  for (uint32_t c = 0; c < n_ctx; ++c) {
    uint64_t S = 0, Sst = 0;
    for (int s = 0; s < NS; ++s) S += d.host_incl[(size_t)c * NS + s];
    for (int s = 1; s < NS; ++s) Sst += d.host_incl[(size_t)c * NS + s];
    d.host_W[c] = issue_rate((double)S, (double)Sst);
  }
  // static scope tree per context: every key adds to its scope and all ancestors
  std::map<std::pair<uint32_t, uint32_t>, Row> acc;
  for (uint64_t k = 0; k < a.ctx.size(); ++k) {
    uint32_t x = a.scope[k];
    if (x == NONE32) { acc[{a.ctx[k], NONE32}][a.stall[k]] += a.count[k]; continue; }
    while (x != NONE32) {
      acc[{a.ctx[k], x}][a.stall[k]] += a.count[k];
      x = m.parent[x];
    }
  }
  d.sc_off.assign((size_t)n_ctx + 1, 0);
  for (auto& kv : acc) {
    d.sc_off[(size_t)kv.first.first + 1]++;
    d.sc_scope.push_back(kv.first.second);
    for (int s = 0; s < NS; ++s) d.sc_val.push_back(kv.second[s]);
  }
  for (uint32_t c = 0; c < n_ctx; ++c) d.sc_off[c + 1] += d.sc_off[c];
}

template <class T>
void put(const std::vector<T>& v, T* dst) {
  if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(T));
}

}  // namespace

// ============================================================================
// C interface for the Python wrapper (names prefixed orc_, unrelated to the
// library's own ABI).
// ============================================================================
extern "C" {

int orc_map_build(const uint64_t* ss, const uint64_t* se, const uint32_t* sid, const uint32_t* sk,
                  uint64_t ns, const uint64_t* ls, const uint64_t* le, const uint32_t* lf,
                  const uint32_t* ll, uint64_t nl, void** out) {
  Map* m = new Map();
  int rc = build_map(ss, se, sid, sk, ns, ls, le, lf, ll, nl, *m);
  if (rc != ORC_OK) { delete m; return rc; }
  *out = m;
  return ORC_OK;
}

// A map made of given sorted, disjoint intervals; interval i is labelled i.
int orc_map_from_intervals(const uint64_t* s, const uint64_t* e, uint64_t n, void** out) {
  for (uint64_t i = 0; i < n; ++i) {
    if (s[i] >= e[i]) return ORC_INVAL;
    if (i && s[i] <= s[i - 1]) return ORC_UNSORTED;
    if (i && s[i] < e[i - 1]) return ORC_OVERLAP;
  }
  Map* m = new Map();
  m->start.assign(s, s + n);
  m->end.assign(e, e + n);
  m->scope.resize(n);
  for (uint64_t i = 0; i < n; ++i) m->scope[i] = (uint32_t)i;
  m->file.assign(n, 0);
  m->line.assign(n, 0);
  *out = m;
  return ORC_OK;
}

void orc_map_sizes(void* h, uint64_t* n_iv, uint64_t* n_ids) {
  Map* m = (Map*)h;
  *n_iv = m->start.size();
  *n_ids = m->kind.size();
}

void orc_map_get(void* h, uint64_t* s, uint64_t* e, uint32_t* sc, uint32_t* f, uint32_t* l,
                 uint32_t* parent, uint8_t* kind, uint32_t* func) {
  Map* m = (Map*)h;
  put(m->start, s); put(m->end, e); put(m->scope, sc); put(m->file, f); put(m->line, l);
  put(m->parent, parent); put(m->kind, kind); put(m->func, func);
}

void orc_lookup(void* h, const uint64_t* pc, uint64_t n, uint32_t* out) {
  Map* m = (Map*)h;
  for (uint64_t i = 0; i < n; ++i) out[i] = lookup(*m, pc[i]);
}

void orc_map_free(void* h) { delete (Map*)h; }

int orc_attribute(void* hm, const uint64_t* pc, const uint32_t* ctx, const uint8_t* stall,
                  const uint32_t* weight, uint64_t n, uint32_t n_ctx, const uint8_t* ctx_mask, void** out) {
  Attr* a = new Attr();
  int rc = attribute(*(Map*)hm, pc, ctx, stall, weight, n, n_ctx, ctx_mask, *a);
  if (rc != ORC_OK) { delete a; return rc; }
  *out = a;
  return ORC_OK;
}

uint64_t orc_attr_size(void* h) { return ((Attr*)h)->ctx.size(); }

void orc_attr_get(void* h, uint32_t* ctx, uint64_t* pc, uint8_t* stall, uint64_t* count, uint32_t* scope,
                  uint64_t* ctx_off) {
  Attr* a = (Attr*)h;
  put(a->ctx, ctx); put(a->pc, pc); put(a->stall, stall); put(a->count, count); put(a->scope, scope);
  put(a->ctx_off, ctx_off);
}

void orc_attr_free(void* h) { delete (Attr*)h; }

// Validates the call graph and context table, then apportions (Section 6.3).
int orc_apportion(void* hm, uint32_t n_funcs, const uint64_t* site_pc, const uint32_t* site_caller,
                  const uint32_t* site_callee, uint64_t n_sites, uint32_t n_ctx, const uint32_t* cpar,
                  const int32_t* centry, void* ha, int sample_based, uint64_t max_nodes,
                  uint64_t* required, void** out) {
  const Map& m = *(Map*)hm;
  const Attr& a = *(Attr*)ha;
  if (n_funcs != m.kind.size() || a.n_ctx != n_ctx) return ORC_INVAL;
  Graph g;
  g.V = n_funcs;
  g.out.resize(n_funcs);
  g.in.resize(n_funcs);
  std::set<uint64_t> pcs;
  for (uint64_t e = 0; e < n_sites; ++e) {
    uint32_t u = site_caller[e], v = site_callee[e];
    if (u >= n_funcs || v >= n_funcs || m.kind[u] != K_FUNC || m.kind[v] != K_FUNC) return ORC_INVAL;
    if (!pcs.insert(site_pc[e]).second) return ORC_INVAL;
    uint32_t iv = lookup(m, site_pc[e]);
    if (iv == NONE32 || m.func[m.scope[iv]] != u) return ORC_INVAL;
    g.pc.push_back(site_pc[e]);
    g.caller.push_back(u);
    g.callee.push_back(v);
    g.out[u].push_back((uint32_t)e);
    g.in[v].push_back((uint32_t)e);
  }
  for (uint32_t c = 0; c < n_ctx; ++c) {
    if (cpar[c] != NONE32 && cpar[c] >= n_ctx) return ORC_INVAL;
    if (centry[c] < -1 || (centry[c] >= 0 && ((uint32_t)centry[c] >= n_funcs || m.kind[centry[c]] != K_FUNC)))
      return ORC_INVAL;
    uint32_t x = c;
    for (uint32_t steps = 0; cpar[x] != NONE32; ++steps) {
      if (steps > n_ctx) return ORC_INVAL;  // cycle in the context table
      x = cpar[x];
    }
  }
  Cct* t = new Cct();
  int rc = apportion(m, g, n_ctx, cpar, centry, a, sample_based, max_nodes, required, *t);
  if (rc != ORC_OK) { delete t; return rc; }
  *out = t;
  return ORC_OK;
}

void orc_cct_sizes(void* h, uint64_t* n_nodes, uint64_t* n_w, uint64_t* n_scc) {
  Cct* t = (Cct*)h;
  *n_nodes = t->parent.size();
  *n_w = t->w_site.size();
  *n_scc = t->scc.size();
}

void orc_cct_get(void* h, uint32_t* scc, uint64_t* node_off, uint32_t* parent, uint32_t* node, uint64_t* site,
                 uint8_t* kind, double* phi, double* excl, uint64_t* w_off, uint64_t* w_site, uint64_t* w_val) {
  Cct* t = (Cct*)h;
  put(t->scc, scc); put(t->node_off, node_off); put(t->parent, parent); put(t->node, node);
  put(t->site, site); put(t->kind, kind); put(t->phi, phi); put(t->excl, excl);
  put(t->w_off, w_off); put(t->w_site, w_site); put(t->w_val, w_val);
}

void orc_cct_free(void* h) { delete (Cct*)h; }

int orc_derive(void* hm, void* ha, void* ht, uint32_t n_ctx, const uint32_t* cpar, void** out) {
  Derived* d = new Derived();
  derive(*(Map*)hm, *(Attr*)ha, *(Cct*)ht, n_ctx, cpar, *d);
  *out = d;
  return ORC_OK;
}

uint64_t orc_derived_nscope(void* h) { return ((Derived*)h)->sc_scope.size(); }

void orc_derived_get(void* h, double* incl, double* S, double* W, uint64_t* host_incl, double* host_W,
                     uint64_t* sc_off, uint32_t* sc_scope, uint64_t* sc_val) {
  Derived* d = (Derived*)h;
  put(d->incl, incl); put(d->S, S); put(d->W, W); put(d->host_incl, host_incl); put(d->host_W, host_W);
  put(d->sc_off, sc_off); put(d->sc_scope, sc_scope); put(d->sc_val, sc_val);
}

void orc_derived_free(void* h) { delete (Derived*)h; }

}  // extern "C"
