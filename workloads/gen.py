"""Seeded synthetic workload generator.

Every array is drawn from numpy's Philox counter-based generator keyed by
(master seed, component, chunk), so any chunk of a sample stream can be
regenerated on its own and two machines produce identical bytes.

Shapes follow the paper's description of the measured data:

* PC samples arrive per kernel invocation, in one buffer whose samples all sit
  under that invocation's placeholder context (Section 4.2), so the stream is a
  sequence of segments with a constant context id.
* Each sample is (instruction address, stall reason, count); a record here
  carries one observation (count 1) unless a weight array is supplied.
* GPU binaries hold many functions, some device functions embedded inside
  global functions (Section 5), with line maps, inlined code and loops.
* The static call graph comes from function symbols and call instructions
  (Section 6.3, step 1); recursion appears as strongly connected components.

Nothing here computes an attribution result.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

FUNC, INLINE, LOOP = 0, 1, 2
UNMAPPED = 0xFFFFFFFF
N_STALL = 16
STRIDE = 16  # bytes between instruction addresses
STALL_TABLE = 64  # quantisation of each instruction's stall distribution

# component tags for the Philox key
_C_STRUCT, _C_GRAPH, _C_CTX, _C_SEG, _C_SAMPLE, _C_STALLTAB, _C_ZIPF, _C_LEARN = range(1, 9)


def _rng(seed: int, component: int, chunk: int = 0) -> np.random.Generator:
    key = ((seed & 0xFFFFFFFFFFFFFFFF) << 64) | ((component & 0xFFFFFFFF) << 32) | (chunk & 0xFFFFFFFF)
    return np.random.Generator(np.random.Philox(key=key))


@dataclass
class Workload:
    """One synthetic profile: structure, call graph, contexts and samples."""

    name: str
    seed: int
    # structure (host arrays; ranges are [start, end) byte addresses)
    scope_start: np.ndarray
    scope_end: np.ndarray
    scope_id: np.ndarray
    scope_kind: np.ndarray
    line_start: np.ndarray
    line_end: np.ndarray
    line_file: np.ndarray
    line_line: np.ndarray
    n_scope_ids: int
    # call graph: node ids are function scope ids
    site_pc: np.ndarray
    site_caller: np.ndarray
    site_callee: np.ndarray
    # host calling-context table
    ctx_parent: np.ndarray
    ctx_entry: np.ndarray
    # samples (filled by make_samples)
    pc: np.ndarray | None = None
    ctx: np.ndarray | None = None
    stall: np.ndarray | None = None
    weight: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n_ctx(self) -> int:
        return int(self.ctx_parent.shape[0])

    @property
    def n_samples(self) -> int:
        return 0 if self.pc is None else int(self.pc.shape[0])


# ----------------------------------------------------------------------------
# program structure
# ----------------------------------------------------------------------------

class _Node:
    __slots__ = ("lo", "hi", "depth", "kids", "scope_kids", "fid")

    def __init__(self, lo, hi, depth, fid):
        self.lo, self.hi, self.depth, self.fid = lo, hi, depth, fid
        self.kids = []  # (lo, hi) blocked sub-ranges, sorted
        self.scope_kids = []  # child _Node objects that are scopes

    def gaps(self):
        out, cur = [], self.lo
        for a, b in sorted(self.kids):
            if a > cur:
                out.append((cur, a))
            cur = max(cur, b)
        if cur < self.hi:
            out.append((cur, self.hi))
        return out


def _pick_subrange(rng, node, max_frac=0.7):
    gaps = node.gaps()
    if not gaps:
        return None
    lens = np.array([b - a for a, b in gaps], dtype=np.float64)
    g = int(rng.choice(len(gaps), p=lens / lens.sum()))
    a, b = gaps[g]
    glen = b - a
    ln = 1 + int(rng.integers(0, max(1, int(glen * max_frac))))
    ln = min(ln, glen)
    s = a + int(rng.integers(0, glen - ln + 1))
    return s, s + ln


def _build_structure(rng, bins, n_embedded, n_inline, inline_depth, n_loops, n_lines,
                     line_cover=0.95, multi_range_loop_frac=0.1, geometric_q=0.5):
    """Lay out binaries and their scopes.

    bins: list of (base address, array of top-level function sizes in instructions).
    Returns a dict with scope/line arrays plus per-instruction ownership.
    """
    # global instruction numbering: binaries concatenated
    inst_pc_parts, bin_of_fn = [], []
    fn_ranges = []  # (global lo, global hi) per top-level function
    g0 = 0
    bin_bounds = []
    for b, (base, sizes) in enumerate(bins):
        n = int(np.sum(sizes))
        inst_pc_parts.append(np.uint64(base) + np.arange(n, dtype=np.uint64) * np.uint64(STRIDE))
        off = g0
        for s in sizes:
            fn_ranges.append((off, off + int(s)))
            bin_of_fn.append(b)
            off += int(s)
        bin_bounds.append((g0, g0 + n))
        g0 += n
    inst_pc = np.concatenate(inst_pc_parts)
    n_inst = g0
    n_top = len(fn_ranges)

    # embedded device functions: strictly inside a host function
    hosts = [i for i, (lo, hi) in enumerate(fn_ranges) if hi - lo >= 12]
    emb_host = rng.choice(hosts, size=min(n_embedded, len(hosts)), replace=False) if n_embedded else []
    emb_ranges = []
    for h in emb_host:
        lo, hi = fn_ranges[h]
        size = hi - lo
        ln = 2 + int(rng.integers(0, max(1, size // 3)))
        a = 2 + int(rng.integers(0, size - ln - 2))
        emb_ranges.append((lo + a, lo + a + ln, int(h)))
    n_funcs = n_top + len(emb_ranges)

    owner = np.empty(n_inst, dtype=np.int64)
    for f, (lo, hi) in enumerate(fn_ranges):
        owner[lo:hi] = f
    for j, (lo, hi, h) in enumerate(emb_ranges):
        owner[lo:hi] = n_top + j

    # containers per function (blocked by embedded ranges)
    fnodes = []
    for f, (lo, hi) in enumerate(fn_ranges):
        fnodes.append(_Node(lo, hi, 0, f))
    for j, (lo, hi, h) in enumerate(emb_ranges):
        fnodes[h].kids.append((lo, hi))
        fnodes.append(_Node(lo, hi, 0, n_top + j))
    fsizes = np.array([nd.hi - nd.lo for nd in fnodes], dtype=np.float64)
    fprob = fsizes / fsizes.sum()

    scopes = []  # (lo, hi, kind, local index)

    def descend(max_depth):
        nd = fnodes[int(rng.choice(n_funcs, p=fprob))]
        while nd.scope_kids and nd.depth < max_depth and rng.random() < geometric_q:
            nd = nd.scope_kids[int(rng.integers(0, len(nd.scope_kids)))]
        return nd

    def add_scope(kind, idx, max_depth, tries=20):
        for _ in range(tries):
            nd = descend(max_depth - 1)
            if nd.depth >= max_depth:
                continue
            r = _pick_subrange(rng, nd)
            if r is None:
                continue
            child = _Node(r[0], r[1], nd.depth + 1, nd.fid)
            nd.kids.append(r)
            nd.scope_kids.append(child)
            scopes.append((r[0], r[1], kind, idx))
            return nd
        return None

    for i in range(n_inline):
        add_scope(INLINE, i, inline_depth)
    for i in range(n_loops):
        parent = add_scope(LOOP, i, inline_depth + 4)
        if parent is not None and rng.random() < multi_range_loop_frac:
            r = _pick_subrange(rng, parent)
            if r is not None:
                parent.kids.append(r)
                parent.scope_kids.append(_Node(r[0], r[1], parent.depth + 1, parent.fid))
                scopes.append((r[0], r[1], LOOP, i))

    n_inl_made = 1 + max([s[3] for s in scopes if s[2] == INLINE], default=-1)
    n_loop_made = 1 + max([s[3] for s in scopes if s[2] == LOOP], default=-1)

    def pc_of(g):  # address of instruction g (a range start)
        b = int(np.searchsorted([bb[1] for bb in bin_bounds], g, side="right"))
        b = min(b, len(bins) - 1)
        return np.uint64(bins[b][0]) + np.uint64(g - bin_bounds[b][0]) * np.uint64(STRIDE)

    s_start, s_end, s_id, s_kind = [], [], [], []
    for f, (lo, hi) in enumerate(fn_ranges):
        s_start.append(pc_of(lo)); s_end.append(pc_of(lo) + np.uint64((hi - lo) * STRIDE))
        s_id.append(f); s_kind.append(FUNC)
    for j, (lo, hi, h) in enumerate(emb_ranges):
        s_start.append(pc_of(lo)); s_end.append(pc_of(lo) + np.uint64((hi - lo) * STRIDE))
        s_id.append(n_top + j); s_kind.append(FUNC)
    for lo, hi, kind, idx in scopes:
        sid = n_funcs + idx if kind == INLINE else n_funcs + n_inl_made + idx
        s_start.append(pc_of(lo)); s_end.append(pc_of(lo) + np.uint64((hi - lo) * STRIDE))
        s_id.append(sid); s_kind.append(kind)
    n_scope_ids = n_funcs + n_inl_made + n_loop_made

    # line ranges: cut at every function / embedded boundary and binary boundary
    cuts = set()
    for lo, hi in fn_ranges:
        cuts.add(lo); cuts.add(hi)
    for lo, hi, _ in emb_ranges:
        cuts.add(lo); cuts.add(hi)
    n_seg_target = int(math.ceil(n_lines / line_cover))
    extra = max(0, n_seg_target - len(cuts) + 1)
    if extra:
        cuts.update(int(x) for x in rng.choice(n_inst, size=min(extra, n_inst), replace=False))
    cuts = np.array(sorted(c for c in cuts if 0 <= c <= n_inst), dtype=np.int64)
    seg_lo, seg_hi = cuts[:-1], cuts[1:]
    keep = np.ones(seg_lo.shape[0], dtype=bool)
    n_drop = max(0, seg_lo.shape[0] - n_lines)
    if n_drop:
        keep[rng.choice(seg_lo.shape[0], size=n_drop, replace=False)] = False
    seg_lo, seg_hi = seg_lo[keep], seg_hi[keep]
    l_start = inst_pc[seg_lo]
    l_end = inst_pc[seg_hi - 1] + np.uint64(STRIDE)
    l_file = (1 + owner[seg_lo] % 64).astype(np.uint32)
    l_line = rng.integers(1, 20000, size=seg_lo.shape[0]).astype(np.uint32)

    # owned instruction lists per function (CSR), used for sampling
    order = np.argsort(owner, kind="stable")
    owned_cnt = np.bincount(owner, minlength=n_funcs).astype(np.int64)
    owned_ptr = np.zeros(n_funcs + 1, dtype=np.int64)
    np.cumsum(owned_cnt, out=owned_ptr[1:])

    return dict(
        scope_start=np.array(s_start, dtype=np.uint64), scope_end=np.array(s_end, dtype=np.uint64),
        scope_id=np.array(s_id, dtype=np.uint32), scope_kind=np.array(s_kind, dtype=np.uint32),
        line_start=l_start.astype(np.uint64), line_end=l_end.astype(np.uint64),
        line_file=l_file, line_line=l_line, n_scope_ids=n_scope_ids,
        n_funcs=n_funcs, inst_pc=inst_pc, owner=owner, owned_list=order.astype(np.int64),
        owned_ptr=owned_ptr, bin_of_fn=np.array(bin_of_fn + [bin_of_fn[h] for _, _, h in emb_ranges]),
        n_bins=len(bins),
    )


# ----------------------------------------------------------------------------
# call graph
# ----------------------------------------------------------------------------

def _er_dag_edges(rng, nodes, mean_out):
    """Erdos-Renyi DAG over a random topological order of `nodes`."""
    n = len(nodes)
    if n < 2:
        return []
    perm = rng.permutation(nodes)
    p = 2.0 * mean_out / n
    n_pairs = n * (n - 1) // 2
    m = int(rng.binomial(n_pairs, min(1.0, p)))
    edges = set()
    while len(edges) < m:
        k = m - len(edges)
        i = rng.integers(0, n, size=2 * k)
        j = rng.integers(0, n, size=2 * k)
        for a, b in zip(i.tolist(), j.tolist()):
            if a == b:
                continue
            if a > b:
                a, b = b, a
            edges.add((a, b))
            if len(edges) >= m:
                break
    return [(int(perm[a]), int(perm[b])) for a, b in sorted(edges)]


def _build_callgraph(rng, st, per_bin_mean_out, scc_frac, scc_size):
    n_funcs = st["n_funcs"]
    bin_of_fn = st["bin_of_fn"]
    edges = []
    for b in range(st["n_bins"]):
        nodes = np.nonzero(bin_of_fn == b)[0]
        edges += _er_dag_edges(rng, nodes, per_bin_mean_out)
    indeg = np.zeros(n_funcs, dtype=np.int64)
    for a, c in edges:
        indeg[c] += 1
    # recursion: cycles among non-kernel nodes of one binary
    if scc_frac > 0:
        for b in range(st["n_bins"]):
            cand = [int(v) for v in np.nonzero((bin_of_fn == b) & (indeg > 0))[0]]
            rng.shuffle(cand)
            budget = int(round(scc_frac * np.sum(bin_of_fn == b)))
            pos = 0
            while budget >= 2 and pos + 2 <= len(cand):
                k = int(rng.integers(scc_size[0], scc_size[1] + 1))
                k = max(2, min(k, budget, len(cand) - pos))
                mem = cand[pos:pos + k]
                pos += k
                budget -= k
                for i in range(k):
                    edges.append((mem[i], mem[(i + 1) % k]))
    # one call instruction per edge, at a distinct owned instruction of the caller
    owned_ptr, owned_list, inst_pc = st["owned_ptr"], st["owned_list"], st["inst_pc"]
    used = {}
    site_pc, site_caller, site_callee = [], [], []
    for a, c in edges:
        lo, hi = owned_ptr[a], owned_ptr[a + 1]
        taken = used.setdefault(a, set())
        if len(taken) >= hi - lo:
            continue
        while True:
            g = int(owned_list[lo + int(rng.integers(0, hi - lo))])
            if g not in taken:
                break
        taken.add(g)
        site_pc.append(inst_pc[g]); site_caller.append(a); site_callee.append(c)
    site_pc = np.array(site_pc, dtype=np.uint64)
    site_caller = np.array(site_caller, dtype=np.uint32)
    site_callee = np.array(site_callee, dtype=np.uint32)
    order = np.argsort(site_pc, kind="stable")
    return site_pc[order], site_caller[order], site_callee[order]


def _kernels(n_funcs, site_callee):
    indeg = np.bincount(site_callee.astype(np.int64), minlength=n_funcs)
    return np.nonzero(indeg == 0)[0]


def _reach(n_funcs, site_caller, site_callee, k, _cache={}):
    """Functions reachable from k over call edges (k included), ascending."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import breadth_first_order
    key = (id(site_caller), id(site_callee), n_funcs)
    g = _cache.get(key)
    if g is None or g[0] is not site_caller:
        m = csr_matrix((np.ones(len(site_caller), np.int8), (site_caller.astype(np.int64),
                                                             site_callee.astype(np.int64))),
                       shape=(n_funcs, n_funcs))
        _cache.clear()
        _cache[key] = g = (site_caller, m)
    order = breadth_first_order(g[1], int(k), directed=True, return_predecessors=False)
    return np.sort(order).astype(np.int64)


# ----------------------------------------------------------------------------
# host calling contexts
# ----------------------------------------------------------------------------

def _recursive_tree(rng, n, max_depth):
    parent = np.full(n, UNMAPPED, dtype=np.uint32)
    depth = np.zeros(n, dtype=np.int64)
    for i in range(1, n):
        while True:
            p = int(rng.integers(0, i))
            if depth[p] < max_depth:
                break
        parent[i] = p
        depth[i] = depth[p] + 1
    return parent, depth


def _leaf_tree(rng, n_internal, n_leaves, max_depth):
    parent, depth = _recursive_tree(rng, n_internal, max_depth - 1)
    lp = np.empty(n_leaves, dtype=np.uint32)
    for i in range(n_leaves):
        lp[i] = int(rng.integers(0, n_internal))
    return np.concatenate([parent, lp]), n_internal


# ----------------------------------------------------------------------------
# samples
# ----------------------------------------------------------------------------

def _zipf_blocks(rng, item_lists, s):
    """Concatenated, slot-shifted Zipf CDFs over each list (item order = hotness)."""
    cdfs, items, starts = [], [], [0]
    for slot, lst in enumerate(item_lists):
        n = len(lst)
        w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
        c = np.cumsum(w)
        c /= c[-1]
        c[-1] = 1.0
        cdfs.append(c + slot)
        items.append(np.asarray(lst, dtype=np.int64)[rng.permutation(n)])
        starts.append(starts[-1] + n)
    return np.concatenate(cdfs), np.concatenate(items), np.array(starts, dtype=np.int64)


def _stall_tables(rng, n_inst, alpha=0.5):
    """Per instruction, a Dirichlet(alpha) distribution over the 16 stall
    reasons, quantised to a STALL_TABLE-entry inverse-CDF table: entry j holds
    the reason whose CDF interval contains (j + 0.5) / STALL_TABLE."""
    if alpha == 0.5:
        # Gamma(1/2, 1) is Z^2 / 2 for a standard normal Z; the factor cancels below
        g = rng.standard_normal(size=(n_inst, N_STALL))
        g *= g
    else:
        g = rng.standard_gamma(alpha, size=(n_inst, N_STALL))
    g /= np.maximum(g.sum(axis=1, keepdims=True), 1e-300)
    cdf = np.cumsum(g, axis=1)
    # first table entry j with (j + 0.5) / T > cdf[s]; entry j's reason counts those s
    first = np.clip(np.ceil(cdf * STALL_TABLE - 0.5), 0, STALL_TABLE).astype(np.int64)
    flat = (first * n_inst + np.arange(n_inst, dtype=np.int64)[:, None]).ravel()
    cnt = np.bincount(flat, minlength=n_inst * (STALL_TABLE + 1)).astype(np.uint8)
    cnt = cnt.reshape(STALL_TABLE + 1, n_inst)[:STALL_TABLE]
    tab = np.minimum(np.cumsum(cnt, axis=0, dtype=np.uint8), N_STALL - 1)
    return np.ascontiguousarray(tab.T)


def make_samples(w: Workload, n: int, seg_mean: float, zipf_s: float, mode: str,
                 seg_sigma: float = 1.0, p_stray: float = 5e-4, p_unmapped: float = 5e-4,
                 weighted: bool = False, shuffled: bool = False, chunk: int = 1 << 22,
                 threads: int = 8) -> None:
    """Draw n samples into w.pc / w.ctx / w.stall (and w.weight if weighted).

    mode "instr": PC ~ Zipf(zipf_s) over the owned instructions of reach(entry).
    mode "func":  function ~ Zipf(zipf_s) over reach(entry), instruction uniform
                  among the function's owned instructions.
    A fraction p_stray of samples land on a random instruction anywhere (so
    some fall outside the entry's reach) and p_unmapped on addresses that no
    function covers.
    """
    st = w.meta["st"]
    seed = w.seed
    rs = _rng(seed, _C_SEG)
    leaves = np.nonzero(w.ctx_entry >= 0)[0]
    mu = math.log(seg_mean) - 0.5 * seg_sigma * seg_sigma
    lens = []
    tot = 0
    while tot < n:
        L = np.maximum(1, np.rint(rs.lognormal(mu, seg_sigma, size=max(16, int(2 * (n - tot) / seg_mean) + 16)))).astype(np.int64)
        lens.append(L)
        tot += int(L.sum())
    lens = np.concatenate(lens)
    cs = np.cumsum(lens)
    nseg = int(np.searchsorted(cs, n, side="left")) + 1
    lens = lens[:nseg].copy()
    lens[-1] -= int(cs[nseg - 1] - n)
    seg_ctx = leaves[rs.integers(0, leaves.shape[0], size=nseg)].astype(np.uint32)
    seg_start = np.zeros(nseg + 1, dtype=np.int64)
    np.cumsum(lens, out=seg_start[1:])

    entries = np.unique(w.ctx_entry[leaves])
    slot_of_entry = {int(k): i for i, k in enumerate(entries)}
    seg_slot = np.array([slot_of_entry[int(w.ctx_entry[c])] for c in seg_ctx], dtype=np.int64)

    rz = _rng(seed, _C_ZIPF)
    n_funcs = st["n_funcs"]
    reach = [_reach(n_funcs, w.site_caller, w.site_callee, int(k)) for k in entries]
    owned_ptr, owned_list = st["owned_ptr"], st["owned_list"]
    if mode == "instr":
        lists = [np.concatenate([owned_list[owned_ptr[f]:owned_ptr[f + 1]] for f in r]) for r in reach]
    elif mode == "func":
        lists = reach
    else:
        raise ValueError(mode)
    cdf, items, _ = _zipf_blocks(rz, lists, zipf_s)
    tab = _stall_tables(_rng(seed, _C_STALLTAB), st["inst_pc"].shape[0])
    inst_pc = st["inst_pc"]
    n_inst = inst_pc.shape[0]
    owned_cnt = np.diff(owned_ptr)
    unm_base = inst_pc[0]

    pc = np.empty(n, dtype=np.uint64)
    ctx = np.empty(n, dtype=np.uint32)
    stall = np.empty(n, dtype=np.uint8)
    weight = np.empty(n, dtype=np.uint32) if weighted else None

    def work(ci):
        lo = ci * chunk
        hi = min(n, lo + chunk)
        m = hi - lo
        r = _rng(seed, _C_SAMPLE, ci)
        seg = np.searchsorted(seg_start, np.arange(lo, hi, dtype=np.int64), side="right") - 1
        u = r.random(m)
        idx = np.searchsorted(cdf, u + seg_slot[seg], side="left")
        idx = np.minimum(idx, cdf.shape[0] - 1)
        it = items[idx]
        if mode == "instr":
            g = it
        else:
            u2 = r.random(m)
            off = np.minimum((u2 * owned_cnt[it]).astype(np.int64), owned_cnt[it] - 1)
            g = owned_list[owned_ptr[it] + off]
        u3 = r.random(m)
        stray = u3 < p_stray
        if stray.any():
            g = g.copy()
            g[stray] = r.integers(0, n_inst, size=int(stray.sum()))
        p = inst_pc[g].copy()
        sidx = (r.random(m) * STALL_TABLE).astype(np.int64)
        s = tab[g, np.minimum(sidx, STALL_TABLE - 1)]
        unm = (u3 >= p_stray) & (u3 < p_stray + p_unmapped)
        if unm.any():
            p[unm] = unm_base - np.uint64(STRIDE) * (np.uint64(1) + r.integers(0, 1024, size=int(unm.sum())).astype(np.uint64))
        pc[lo:hi] = p
        ctx[lo:hi] = seg_ctx[seg]
        stall[lo:hi] = s
        if weighted:
            weight[lo:hi] = 1 + r.integers(0, 8, size=m).astype(np.uint32)

    n_chunks = (n + chunk - 1) // chunk
    if threads > 1 and n_chunks > 1:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(work, range(n_chunks)))
    else:
        for ci in range(n_chunks):
            work(ci)
    if shuffled:
        perm = _rng(seed, _C_SAMPLE, 0xFFFFFFFF).permutation(n)
        pc, ctx, stall = pc[perm], ctx[perm], stall[perm]
        if weighted:
            weight = weight[perm]
    w.pc, w.ctx, w.stall, w.weight = pc, ctx, stall, weight
    w.meta.update(n_segments=nseg, seg_mean=seg_mean, zipf_s=zipf_s, mode=mode, shuffled=shuffled)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

def _assemble(name, seed, st, cg, parent, entry):
    sp, sc, se = cg
    return Workload(
        name=name, seed=seed,
        scope_start=st["scope_start"], scope_end=st["scope_end"], scope_id=st["scope_id"],
        scope_kind=st["scope_kind"], line_start=st["line_start"], line_end=st["line_end"],
        line_file=st["line_file"], line_line=st["line_line"], n_scope_ids=st["n_scope_ids"],
        site_pc=sp, site_caller=sc, site_callee=se, ctx_parent=parent, ctx_entry=entry,
        meta={"st": st},
    )


def config1(seed: int = 2109069311, n_samples: int = 1_000_000, **kw) -> Workload:
    """Tiny plain-method profile: one binary, 64 functions, 4,096 instructions."""
    rs = _rng(seed, _C_STRUCT)
    n_top, n_emb = 62, 2
    sizes = 8 + rs.multinomial(4096 - 8 * n_top, [1.0 / n_top] * n_top)
    st = _build_structure(rs, [(0x1000_0000, sizes)], n_emb, n_inline=32, inline_depth=3,
                          n_loops=8, n_lines=1000)
    cg = _build_callgraph(_rng(seed, _C_GRAPH), st, per_bin_mean_out=2.0, scc_frac=0.0, scc_size=(2, 2))
    rc = _rng(seed, _C_CTX)
    parent, n_int = _leaf_tree(rc, 13, 32, 4)
    kern = _kernels(st["n_funcs"], cg[2])
    entry = np.full(parent.shape[0], -1, dtype=np.int32)
    entry[n_int:] = kern[rc.integers(0, kern.shape[0], size=32)]
    w = _assemble("config1", seed, st, cg, parent, entry)
    if n_samples:
        make_samples(w, n_samples, seg_mean=4096, zipf_s=1.2, mode="instr", **kw)
    return w


def config2(seed: int = 2109069312, n_samples: int = 256_000_000, n_funcs: int = 20_000,
            n_inst: int = 2_000_000, n_lines: int = 200_000, n_loops: int = 5_000,
            n_inline: int = 20_000, n_ctx: int = 100_000, **kw) -> Workload:
    """Medium plain-method profile: 4 binaries, 20k functions, 2M instructions."""
    rs = _rng(seed, _C_STRUCT)
    bins = []
    per = n_funcs // 4
    for b in range(4):
        x = rs.lognormal(0.0, 1.0, size=per)
        sizes = np.maximum(4, np.floor(x / x.sum() * (n_inst // 4))).astype(np.int64)
        bins.append(((b + 1) << 40, sizes))
    st = _build_structure(rs, bins, 0, n_inline=n_inline, inline_depth=8, n_loops=n_loops,
                          n_lines=n_lines)
    cg = _build_callgraph(_rng(seed, _C_GRAPH), st, per_bin_mean_out=3.0, scc_frac=0.02,
                          scc_size=(2, 50))
    rc = _rng(seed, _C_CTX)
    parent, _ = _recursive_tree(rc, n_ctx, 40)
    has_kid = np.zeros(n_ctx, dtype=bool)
    has_kid[parent[parent != UNMAPPED].astype(np.int64)] = True
    kern = _kernels(st["n_funcs"], cg[2])
    entry = np.full(n_ctx, -1, dtype=np.int32)
    leaves = np.nonzero(~has_kid)[0]
    entry[leaves] = kern[rc.integers(0, kern.shape[0], size=leaves.shape[0])]
    w = _assemble("config2", seed, st, cg, parent, entry)
    if n_samples:
        make_samples(w, n_samples, seg_mean=2048, zipf_s=1.1, mode="func", **kw)
    return w


def small_config(seed: int, n_samples: int = 200_000, n_funcs: int = 400, n_inst: int = 24_000,
                 n_ctx: int = 600, seg_mean: float = 700, mode: str = "func", n_bins: int = 2,
                 scc_frac: float = 0.05, **kw) -> Workload:
    """Config-2-shaped profile at a size the oracle finishes in a second."""
    rs = _rng(seed, _C_STRUCT)
    bins = []
    per = n_funcs // n_bins
    for b in range(n_bins):
        x = rs.lognormal(0.0, 1.0, size=per)
        sizes = np.maximum(4, np.floor(x / x.sum() * (n_inst // n_bins))).astype(np.int64)
        bins.append(((b + 1) << 40, sizes))
    st = _build_structure(rs, bins, 3, n_inline=n_funcs, inline_depth=8, n_loops=n_funcs // 4,
                          n_lines=n_inst // 10)
    cg = _build_callgraph(_rng(seed, _C_GRAPH), st, per_bin_mean_out=3.0, scc_frac=scc_frac,
                          scc_size=(2, 8))
    rc = _rng(seed, _C_CTX)
    parent, _ = _recursive_tree(rc, n_ctx, 12)
    has_kid = np.zeros(n_ctx, dtype=bool)
    has_kid[parent[parent != UNMAPPED].astype(np.int64)] = True
    kern = _kernels(st["n_funcs"], cg[2])
    entry = np.full(n_ctx, -1, dtype=np.int32)
    leaves = np.nonzero(~has_kid)[0]
    entry[leaves] = kern[rc.integers(0, kern.shape[0], size=leaves.shape[0])]
    w = _assemble(f"small{seed}", seed, st, cg, parent, entry)
    if n_samples:
        make_samples(w, n_samples, seg_mean=seg_mean, zipf_s=1.1, mode=mode, **kw)
    return w


def tiny_random_case(seed: int, n_funcs: int = 6, n_samples: int = 300, cycles: bool = True,
                     n_ctx: int = 4, weighted: bool = False) -> Workload:
    """A few functions, a dense random call graph with cycles, a handful of contexts.

    Sized for brute-force checks (path enumeration, all node orders)."""
    rs = _rng(seed, _C_STRUCT)
    sizes = 4 + rs.integers(0, 6, size=n_funcs)
    st = _build_structure(rs, [(0x4000, sizes)], 1 if n_funcs >= 4 else 0, n_inline=n_funcs,
                          inline_depth=3, n_loops=max(1, n_funcs // 2), n_lines=int(sizes.sum()) // 2)
    rg = _rng(seed, _C_GRAPH)
    nf = st["n_funcs"]
    edges = []
    for a in range(nf):
        for c in range(nf):
            if a != c and rg.random() < (0.35 if cycles else 0.0) + (0.3 if a < c else 0.0):
                edges.append((a, c))
    owned_ptr, owned_list, inst_pc = st["owned_ptr"], st["owned_list"], st["inst_pc"]
    sp, sc, se, used = [], [], [], set()
    for a, c in edges:
        cand = [int(g) for g in owned_list[owned_ptr[a]:owned_ptr[a + 1]] if int(g) not in used]
        if not cand:
            continue
        g = cand[int(rg.integers(0, len(cand)))]
        used.add(g)
        sp.append(inst_pc[g]); sc.append(a); se.append(c)
    sp = np.array(sp, dtype=np.uint64); sc = np.array(sc, dtype=np.uint32); se = np.array(se, dtype=np.uint32)
    o = np.argsort(sp)
    sp, sc, se = sp[o], sc[o], se[o]
    rc = _rng(seed, _C_CTX)
    parent, _ = _recursive_tree(rc, n_ctx, 3)
    entry = np.full(n_ctx, -1, dtype=np.int32)
    for i in range(n_ctx):
        x = rc.random()
        entry[i] = -1 if x < 0.25 else int(rc.integers(0, nf))
    w = _assemble(f"tiny{seed}", seed, st, (sp, sc, se), parent, entry)
    # samples: any owned instruction, skewed, plus a few unmapped addresses
    r = _rng(seed, _C_SAMPLE)
    n_inst = inst_pc.shape[0]
    gi = np.minimum((r.random(n_samples) ** 2 * n_inst).astype(np.int64), n_inst - 1)
    pc = inst_pc[gi].copy()
    unm = r.random(n_samples) < 0.03
    pc[unm] = np.uint64(0x4000 - STRIDE)
    ctxs = r.integers(0, n_ctx, size=n_samples).astype(np.uint32)
    w.pc, w.ctx = pc, ctxs
    w.stall = r.integers(0, N_STALL, size=n_samples).astype(np.uint8)
    w.weight = (1 + r.integers(0, 5, size=n_samples)).astype(np.uint32) if weighted else None
    return w


# ----------------------------------------------------------------------------
# learned-index workload and batched profiles (filled in by their own builders)
# ----------------------------------------------------------------------------

def learned_intervals(seed: int = 2109069314, n: int = 50_000_000, base: int = 1 << 32):
    """Sorted, disjoint [start, end) intervals with lognormal(4, 2) start gaps.

    Start-to-start delta d = 1 + floor(lognormal(4, 2)); the interval length is
    d with probability 1/2 (touching the next start), else uniform in [1, d],
    so holes exist."""
    r = _rng(seed, _C_LEARN, 0)
    d = 1 + np.floor(r.lognormal(4.0, 2.0, size=n)).astype(np.uint64)
    d = np.minimum(d, np.uint64(1 << 32))
    start = np.empty(n, dtype=np.uint64)
    start[0] = base
    np.cumsum(d[:-1], out=start[1:])
    start[1:] += np.uint64(base)
    full = r.random(n) < 0.5
    ln = np.where(full, d, 1 + np.floor(r.random(n) * d.astype(np.float64)).astype(np.uint64))
    ln = np.minimum(ln, d)
    end = start + ln
    return start, end


def learned_queries(start: np.ndarray, end: np.ndarray, n: int, seed: int = 2109069314,
                    zipf_frac: float = 0.7, zipf_s: float = 1.05, chunk: int = 1 << 22,
                    threads: int = 8) -> np.ndarray:
    """Query PCs: a Zipf-picked interval plus a uniform offset inside it, or a
    uniform address over the whole span (these may hit holes)."""
    m = start.shape[0]
    rz = _rng(seed, _C_LEARN, 1)
    perm = rz.permutation(m)
    w = np.arange(1, m + 1, dtype=np.float64) ** (-zipf_s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    lo_all, hi_all = int(start[0]), int(end[-1])
    out = np.empty(n, dtype=np.uint64)

    def work(ci):
        lo = ci * chunk
        hi = min(n, lo + chunk)
        k = hi - lo
        r = _rng(seed, _C_LEARN, 2 + ci)
        pick = r.random(k) < zipf_frac
        iv = perm[np.minimum(np.searchsorted(cdf, r.random(k)), m - 1)]
        span = (end[iv] - start[iv]).astype(np.float64)
        q_in = start[iv] + np.floor(r.random(k) * span).astype(np.uint64)
        q_un = np.uint64(lo_all) + np.floor(r.random(k) * float(hi_all - lo_all)).astype(np.uint64)
        out[lo:hi] = np.where(pick, q_in, q_un)

    nc = (n + chunk - 1) // chunk
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(work, range(nc)))
    return out


def learned_queries_gpu(start: np.ndarray, end: np.ndarray, n: int, seed: int = 2109069314,
                        zipf_frac: float = 0.7, zipf_s: float = 1.05, device="cuda"):
    """The query mix of learned_queries drawn on the GPU with torch's seeded
    generator (for sizes where host drawing is slow): a Zipf-picked interval
    plus a uniform offset inside it, or a uniform address over the whole span.
    Returns a uint64 CUDA tensor."""
    import torch
    m = start.shape[0]
    rz = _rng(seed, _C_LEARN, 1)
    perm = torch.from_numpy(rz.permutation(m).astype(np.int64)).to(device)
    w = torch.arange(1, m + 1, dtype=torch.float64, device=device).pow_(-zipf_s)
    cdf = torch.cumsum(w, 0)
    cdf /= cdf[-1].clone()
    del w
    s = torch.from_numpy(start.view(np.int64)).to(device)
    e = torch.from_numpy(end.view(np.int64)).to(device)
    lo_all, hi_all = int(start[0]), int(end[-1])
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty(n, dtype=torch.int64, device=device)
    step = 1 << 26
    for a in range(0, n, step):
        k = min(step, n - a)
        pick = torch.rand(k, generator=g, device=device) < zipf_frac
        iv = perm[torch.clamp(torch.searchsorted(cdf, torch.rand(k, generator=g, device=device,
                                                                  dtype=torch.float64)), max=m - 1)]
        span = (e[iv] - s[iv]).to(torch.float64)
        q_in = s[iv] + torch.floor(torch.rand(k, generator=g, device=device, dtype=torch.float64) * span).to(torch.int64)
        q_un = lo_all + torch.floor(torch.rand(k, generator=g, device=device, dtype=torch.float64)
                                    * float(hi_all - lo_all)).to(torch.int64)
        out[a:a + k] = torch.where(pick, q_in, q_un)
    return out.view(torch.uint64)
