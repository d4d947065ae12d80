"""Brute-force formulations used to pin the C++ oracle on tiny inputs.

Each function here restates a definition from the paper in the most direct
form available, deliberately different from the oracle's algorithm:

* per-address scope resolution by scanning every range (smallest container)
  instead of a boundary sweep (Section 5; Section 6.1 calling-context expansion);
* attribution with a Python dict (Section 4.5: a raw metric is a sum);
* SCCs from mutual reachability of the transitive closure instead of Tarjan
  (Section 6.3, step 3);
* the step-2 rule executed literally, one function at a time, in a caller
  supplied order (Section 6.3, step 2);
* has-cost from plain reachability and the CCT by enumerating every call path
  (Section 6.3, step 4);
* inclusive metrics by summing over path prefixes (Section 6.1, statistic
  generation) and W = (S - S_stall) / S (Section 7.1).

Pure Python: only for inputs of a few dozen functions / thousands of samples.
"""
from __future__ import annotations

from collections import defaultdict

FUNC, INLINE, LOOP = 0, 1, 2
NONE32 = 0xFFFFFFFF
NS = 16


# ----------------------------------------------------------------------------
# structure
# ----------------------------------------------------------------------------

def owner_of(addr, scopes):
    """Function owning addr: containing function with largest start, then
    smallest end, then smallest id (functions split into disjoint ranges)."""
    best = None
    for s, e, i, k in scopes:
        if k == FUNC and s <= addr < e:
            key = (-s, e, i)
            if best is None or key < best[0]:
                best = (key, i)
    return None if best is None else best[1]


def innermost_of(addr, scopes):
    """Smallest non-function range containing addr; among equal ranges a loop is
    inside an inline scope and a higher id inside a lower id."""
    best = None
    for s, e, i, k in scopes:
        if k != FUNC and s <= addr < e:
            key = (e - s, -k, -i)
            if best is None or key < best[0]:
                best = (key, i)
    return None if best is None else best[1]


def line_of(addr, lines):
    for s, e, f, ln in lines:
        if s <= addr < e:
            return f, ln
    return 0, 0


def label_of(addr, scopes, lines):
    """(scope, file, line) of an address, or None if no function covers it."""
    own = owner_of(addr, scopes)
    if own is None:
        return None
    inner = innermost_of(addr, scopes)
    f, ln = line_of(addr, lines)
    return (own if inner is None else inner, f, ln)


def ancestors(scope_id, scopes):
    """Chain scope, enclosing scopes ..., owning function, by range containment."""
    rngs = [(s, e, i, k) for s, e, i, k in scopes if i == scope_id]
    s0, e0, _, k0 = rngs[0]
    if k0 == FUNC:
        return [scope_id]
    chain = [scope_id]
    own = owner_of(s0, scopes)
    enclosing = []
    for s, e, i, k in scopes:
        if k != FUNC and i != scope_id and s <= s0 and e0 <= e:
            if (s, e) == (s0, e0) and (k, i) >= (k0, scope_id):
                continue  # equal range but not outer
            enclosing.append((e - s, -k, -i, i))
    enclosing.sort()
    chain += [t[3] for t in enclosing]
    chain.append(own)
    return chain


# ----------------------------------------------------------------------------
# attribution
# ----------------------------------------------------------------------------

def attribute(pc, ctx, stall, weight=None):
    acc = {}
    for i in range(len(pc)):
        k = (int(ctx[i]), int(pc[i]), int(stall[i]))
        acc[k] = acc.get(k, 0) + (1 if weight is None else int(weight[i]))
    return acc


# ----------------------------------------------------------------------------
# call graph
# ----------------------------------------------------------------------------

def closure(nodes, edges):
    """Reachability matrix (Warshall) over node list; edges = (u, v) pairs."""
    idx = {v: j for j, v in enumerate(nodes)}
    n = len(nodes)
    R = [[False] * n for _ in range(n)]
    for u, v in edges:
        R[idx[u]][idx[v]] = True
    for k in range(n):
        for i in range(n):
            if R[i][k]:
                rk = R[k]
                ri = R[i]
                for j in range(n):
                    if rk[j]:
                        ri[j] = True
    return idx, R


def scc_ids(nodes, edges):
    """Canonical SCC id per node: components by mutual reachability, ranked by
    smallest member."""
    idx, R = closure(nodes, edges)
    comp = {}
    for v in nodes:
        mem = [w for w in nodes if w == v or (R[idx[v]][idx[w]] and R[idx[w]][idx[v]])]
        comp[v] = min(mem)
    reps = sorted(set(comp.values()))
    rank = {r: j for j, r in enumerate(reps)}
    return {v: rank[comp[v]] for v in nodes}


def step2_literal(order, sites, weight, selfsum):
    """Section 6.3 step 2, executed literally in the given function order.

    sites: list of (site_id, caller, callee); weight: site_id -> call samples;
    selfsum: function -> samples.  A function that has samples, or calls along
    an edge that now has weight, and whose incoming edges all have zero weight,
    gets weight one on every incoming edge; passes repeat until nothing changes.
    """
    w = dict(weight)
    changed = True
    while changed:
        changed = False
        for f in order:
            inc = [sid for sid, u, v in sites if v == f]
            if not inc or any(w[sid] != 0 for sid in inc):
                continue
            active = selfsum.get(f, 0) > 0 or any(w[sid] > 0 for sid, u, v in sites if u == f)
            if active:
                for sid in inc:
                    w[sid] = 1
                changed = True
    return w


def reach(entry, sites):
    seen = {entry}
    stack = [entry]
    while stack:
        u = stack.pop()
        for _, a, b in sites:
            if a == u and b not in seen:
                seen.add(b)
                stack.append(b)
    return seen


def cct_paths(funcs, sites, site_pc, samples_by_func, pc_samples, entry, sample_based=True, order=None):
    """GPU CCT of one context by explicit path enumeration.

    funcs: function ids; sites: list of (site_id, caller, callee);
    samples_by_func: function -> [16 counts]; pc_samples: pc -> call samples.
    Returns (paths, unreachable_row): paths maps a tuple of call-site pcs from
    the root (prefixed by the root's condensed id) to (phi, condensed node, row).
    """
    R = set(funcs) if entry is None else reach(entry, sites)
    rs = [(sid, u, v) for sid, u, v in sites if u in R]
    self_in = {f: r for f, r in samples_by_func.items() if f in R}
    unreach = [0] * NS
    for f, r in samples_by_func.items():
        if f not in R:
            unreach = [a + b for a, b in zip(unreach, r)]
    w0 = {sid: pc_samples.get(site_pc[sid], 0) for sid, _, _ in rs}
    ssum = {f: sum(r) for f, r in self_in.items()}
    w1 = step2_literal(order or sorted(R), rs, w0, ssum) if sample_based else w0
    nodes = sorted(R)
    comp = scc_ids(sorted(funcs), [(u, v) for _, u, v in sites])
    ext = [(sid, u, v) for sid, u, v in rs if comp[u] != comp[v]]
    # step-2 rule once more on the condensed graph
    cself = defaultdict(lambda: [0] * NS)
    for f, r in self_in.items():
        cself[comp[f]] = [a + b for a, b in zip(cself[comp[f]], r)]
    X_nodes = sorted({comp[v] for v in nodes})
    csites = [(sid, comp[u], comp[v]) for sid, u, v in ext]
    if sample_based:
        w2 = step2_literal(X_nodes, csites, {sid: w1[sid] for sid, _, _ in csites},
                           {X: sum(r) for X, r in cself.items()})
    else:
        w2 = {sid: w1[sid] for sid, _, _ in csites}
    Wp = defaultdict(int)
    for sid, U, V in csites:
        Wp[V] += w2[sid]
    # has cost: reaches a node with samples along positive edges
    pos = [(U, V) for sid, U, V in csites if w2[sid] > 0]
    idx, Rm = closure(X_nodes, pos)

    def has_cost(X):
        if sum(cself[X]) > 0:
            return True
        return any(Rm[idx[X]][idx[Y]] and sum(cself[Y]) > 0 for Y in X_nodes)

    if entry is not None:
        roots = [comp[entry]]
    else:
        indeg = {X: 0 for X in X_nodes}
        for _, u, v in sites:
            if comp[u] != comp[v] and comp[v] in indeg:
                indeg[comp[v]] += 1
        roots = [X for X in X_nodes if indeg[X] == 0]
    paths = {}

    def walk(X, key, phi):
        paths[key] = (phi, X, [float(c) * phi for c in cself[X]])
        kids = sorted([(site_pc[sid], sid, V) for sid, U, V in csites if U == X and w2[sid] > 0 and has_cost(V)])
        for pc, sid, V in kids:
            walk(V, key + (pc,), phi * (float(w2[sid]) / float(Wp[V])))

    for r in roots:
        if has_cost(r):
            walk(r, (r,), 1.0)
    return paths, unreach, w2, comp


def inclusive_by_prefix(paths):
    """I(p) = sum of E over every path that extends p (Section 6.1)."""
    out = {}
    for k in paths:
        row = [0.0] * NS
        for k2, (_, _, e) in paths.items():
            if k2[:len(k)] == k:
                row = [a + b for a, b in zip(row, e)]
        out[k] = row
    return out


def issue_rate(row):
    """Warp issue rate W = (S - S_stall) / S with reason 0 = not stalled (Section 7.1)."""
    S = sum(row)
    Sst = sum(row[1:])
    return 0.0 if S == 0 else (S - Sst) / S
