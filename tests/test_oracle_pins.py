"""Pins of the CPU oracle against brute force, closed forms and hand-worked cases.

These run without a GPU.  Each test names the passage of the paper it checks.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from workloads import config1, small_config, tiny_random_case
from workloads import handmade
from workloads.gen import FUNC, INLINE, LOOP

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NONE32 = oracle.NONE32


def _scopes(w):
    return list(zip(w.scope_start.tolist(), w.scope_end.tolist(), w.scope_id.tolist(), w.scope_kind.tolist()))


def _lines(w):
    return list(zip(w.line_start.tolist(), w.line_end.tolist(), w.line_file.tolist(), w.line_line.tolist()))


# ---------------------------------------------------------------------------
# structure map (Section 5; Section 6.1 calling-context expansion)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", list(range(12)))
def test_map_matches_per_address_scan(seed):
    w = tiny_random_case(seed, n_funcs=5 + seed % 4)
    m = oracle.build_map_workload(w)
    sc, ln = _scopes(w), _lines(w)
    lo = int(w.scope_start.min()) - 32
    hi = int(w.scope_end.max()) + 32
    probes = np.arange(lo, hi, 4, dtype=np.uint64)
    iv = oracle.lookup(m, probes)
    for a, i in zip(probes.tolist(), iv.tolist()):
        lab = brute.label_of(a, sc, ln)
        if lab is None:
            assert i == NONE32, hex(a)
        else:
            assert i != NONE32, hex(a)
            assert (int(m.scope[i]), int(m.file[i]), int(m.line[i])) == lab, hex(a)
    # maximal merge: touching neighbours never share a label
    for i in range(1, len(m.start)):
        if m.start[i] == m.end[i - 1]:
            assert (m.scope[i], m.file[i], m.line[i]) != (m.scope[i - 1], m.file[i - 1], m.line[i - 1])
    # scope table: parent chain equals the chain of containing ranges
    for sid in set(w.scope_id.tolist()):
        chain = [sid]
        while m.parent[chain[-1]] != NONE32:
            chain.append(int(m.parent[chain[-1]]))
        assert chain == brute.ancestors(sid, sc)


def test_map_owner_matches_generator_layout():
    # Every instruction the generator assigned to function f resolves to f.
    w = config1(n_samples=0)
    st = w.meta["st"]
    m = oracle.build_map_workload(w)
    iv = oracle.lookup(m, st["inst_pc"])
    assert (iv != NONE32).all()
    assert np.array_equal(m.func[m.scope[iv]], st["owner"].astype(np.uint32))


def test_map_split_overlapping_functions():
    # Section 5: overlapping functions become disjoint ranges.  F=[0x100,0x200),
    # G=[0x140,0x180) embedded in F, H=[0x1c0,0x240) overlapping F's tail:
    # the later start owns each shared address.
    m = oracle.build_map([0x100, 0x140, 0x1C0], [0x200, 0x180, 0x240], [0, 1, 2], [FUNC] * 3)
    assert m.start.tolist() == [0x100, 0x140, 0x180, 0x1C0]
    assert m.end.tolist() == [0x140, 0x180, 0x1C0, 0x240]
    assert m.scope.tolist() == [0, 1, 0, 2]
    # equal start: the shorter function owns; equal range: the smaller id owns
    m = oracle.build_map([0x100, 0x100, 0x100], [0x200, 0x180, 0x180], [4, 7, 5], [FUNC] * 3)
    assert m.scope.tolist() == [5, 4]


def test_map_equal_ranges_nest():
    # Reading: equal ranges nest function > inline > loop, lower id outer.
    m = oracle.build_map([0, 0, 0, 0], [64, 64, 64, 64], [0, 5, 3, 7], [FUNC, INLINE, LOOP, INLINE])
    assert m.scope.tolist() == [3]
    assert m.parent[3] == 7 and m.parent[7] == 5 and m.parent[5] == 0 and m.parent[0] == NONE32
    assert m.func[3] == 0 and m.func[7] == 0


def test_map_lines_and_gaps():
    m = oracle.build_map([0x100], [0x200], [0], [FUNC], [0x120, 0x180], [0x140, 0x1A0], [3, 3], [10, 11])
    assert m.start.tolist() == [0x100, 0x120, 0x140, 0x180, 0x1A0]
    assert m.file.tolist() == [0, 3, 0, 3, 0]
    assert m.line.tolist() == [0, 10, 0, 11, 0]
    assert oracle.lookup(m, np.array([0xFF, 0x200, 0x100, 0x1FF], np.uint64)).tolist() == [NONE32, NONE32, 0, 4]


@pytest.mark.parametrize("case,code", [
    # crossing loops
    (dict(s=[0, 16, 48], e=[256, 96, 128], i=[0, 1, 2], k=[FUNC, LOOP, LOOP]), oracle.E_NOT_LAMINAR),
    # inline scope straddling an embedded function's range
    (dict(s=[0, 64, 32], e=[256, 128, 96], i=[0, 1, 2], k=[FUNC, FUNC, INLINE]), oracle.E_NOT_LAMINAR),
    # inline scope outside every function
    (dict(s=[0, 300], e=[256, 310], i=[0, 1], k=[FUNC, INLINE]), oracle.E_NOT_LAMINAR),
    # empty range
    (dict(s=[0, 32], e=[256, 32], i=[0, 1], k=[FUNC, LOOP]), oracle.E_INVAL),
    # one id, two kinds
    (dict(s=[0, 32], e=[256, 64], i=[0, 0], k=[FUNC, LOOP]), oracle.E_INVAL),
])
def test_map_errors(case, code):
    with pytest.raises(oracle.OracleError) as ei:
        oracle.build_map(case["s"], case["e"], case["i"], case["k"])
    assert ei.value.code == code


def test_map_loop_parent_mismatch():
    # loop 2 has one range inside inline 1 and one outside it
    with pytest.raises(oracle.OracleError) as ei:
        oracle.build_map([0, 0, 16, 128], [256, 64, 32, 160], [0, 1, 2, 2], [FUNC, INLINE, LOOP, LOOP])
    assert ei.value.code == oracle.E_NOT_LAMINAR


def test_map_overlapping_lines():
    with pytest.raises(oracle.OracleError) as ei:
        oracle.build_map([0], [256], [0], [FUNC], [0, 32], [64, 96], [1, 1], [1, 2])
    assert ei.value.code == oracle.E_OVERLAP


def test_prebuilt_intervals():
    m = oracle.map_from_intervals([10, 20, 40], [15, 40, 41])
    q = np.array([9, 10, 14, 15, 19, 20, 39, 40, 41, 1 << 40], np.uint64)
    assert oracle.lookup(m, q).tolist() == [NONE32, 0, 0, NONE32, NONE32, 1, 1, 2, NONE32, NONE32]
    for s, e, code in [([10, 5], [12, 8], oracle.E_UNSORTED), ([10, 11], [12, 13], oracle.E_OVERLAP),
                       ([10], [10], oracle.E_INVAL)]:
        with pytest.raises(oracle.OracleError) as ei:
            oracle.map_from_intervals(s, e)
        assert ei.value.code == code


# ---------------------------------------------------------------------------
# attribution (Section 4.2 sample record; Section 4.5 raw metric = sum)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_attribute_matches_dict(seed, weighted):
    w = tiny_random_case(seed, n_samples=3000, n_ctx=6, weighted=weighted)
    m = oracle.build_map_workload(w)
    a = oracle.attribute(m, w.pc, w.ctx, w.stall, w.weight, w.n_ctx)
    ref = brute.attribute(w.pc, w.ctx, w.stall, w.weight)
    keys = sorted(ref)
    assert list(zip(a.ctx.tolist(), a.pc.tolist(), a.stall.tolist())) == keys
    assert a.count.tolist() == [ref[k] for k in keys]
    sc, ln = _scopes(w), _lines(w)
    for p, s in zip(a.pc.tolist(), a.scope.tolist()):
        lab = brute.label_of(p, sc, ln)
        assert s == (NONE32 if lab is None else lab[0])
    # every sample attributed exactly once; per-context histogram
    tot = w.n_samples if w.weight is None else int(w.weight.sum())
    assert int(a.count.sum()) == tot
    per = np.bincount(w.ctx, weights=None if w.weight is None else w.weight.astype(np.float64),
                      minlength=w.n_ctx)
    got = [int(a.count[a.ctx_offsets[c]:a.ctx_offsets[c + 1]].sum()) for c in range(w.n_ctx)]
    assert got == [int(x) for x in per]


def test_attribute_config1_invariants():
    w = config1()
    m = oracle.build_map_workload(w)
    a = oracle.attribute(m, w.pc, w.ctx, w.stall, None, w.n_ctx)
    assert int(a.count.sum()) == w.n_samples
    # keys strictly increasing by (ctx, pc, stall)
    k = (a.ctx.astype(object) << 72) | (a.pc.astype(object) << 8) | a.stall.astype(object)
    assert all(k[i] < k[i + 1] for i in range(len(k) - 1))
    # independent aggregation with numpy unique over packed keys
    ks = np.stack([w.ctx.astype(np.uint64), w.pc, w.stall.astype(np.uint64)], axis=1)
    uk, cnt = np.unique(ks, axis=0, return_counts=True)
    assert np.array_equal(uk[:, 0], a.ctx.astype(np.uint64))
    assert np.array_equal(uk[:, 1], a.pc)
    assert np.array_equal(cnt.astype(np.uint64), a.count)


def test_attribute_errors():
    m = oracle.build_map([0], [256], [0], [FUNC])
    with pytest.raises(oracle.OracleError) as ei:
        oracle.attribute(m, np.array([0], np.uint64), np.array([0], np.uint32), np.array([16], np.uint8), None, 1)
    assert ei.value.code == oracle.E_INVAL
    with pytest.raises(oracle.OracleError) as ei:
        oracle.attribute(m, np.array([0], np.uint64), np.array([1], np.uint32), np.array([0], np.uint8), None, 1)
    assert ei.value.code == oracle.E_INVAL


# ---------------------------------------------------------------------------
# GPU calling context tree (Section 6.3)
# ---------------------------------------------------------------------------

def _oracle_paths(t, ci):
    b, e = int(t.node_off[ci]), int(t.node_off[ci + 1])
    keys = []
    out = {}
    for i in range(b, e):
        if t.kind[i] != 0:
            continue
        p = int(t.parent[i])
        key = (int(t.node[i]),) if p == NONE32 else keys[p] + (int(t.site[i]),)
        keys.append(key)
        out[key] = (float(t.phi[i]), int(t.node[i]), t.excl[i].tolist())
    return out


def _brute_case(w, ci, sample_based=True, order=None):
    m = oracle.build_map_workload(w)
    sc, ln = _scopes(w), _lines(w)
    sel = w.ctx == ci
    funcs = [f for f in range(w.n_scope_ids) if m.kind[f] == FUNC]
    by_func, pc_samples, unknown = {}, {}, [0] * 16
    for p, s, c in zip(w.pc[sel].tolist(), w.stall[sel].tolist(),
                       (w.weight[sel] if w.weight is not None else np.ones(int(sel.sum()), np.int64)).tolist()):
        pc_samples[p] = pc_samples.get(p, 0) + c
        own = brute.owner_of(p, sc)
        if own is None:
            unknown[s] += c
            continue
        by_func.setdefault(own, [0] * 16)[s] += c
    sites = [(i, int(u), int(v)) for i, (u, v) in enumerate(zip(w.site_caller, w.site_callee))]
    site_pc = {i: int(p) for i, p in enumerate(w.site_pc)}
    entry = int(w.ctx_entry[ci])
    return brute.cct_paths(funcs, sites, site_pc, by_func, pc_samples, None if entry < 0 else entry,
                           sample_based, order), unknown


@pytest.mark.parametrize("seed", list(range(16)))
def test_cct_matches_path_enumeration(seed):
    w = tiny_random_case(seed, n_funcs=4 + seed % 4, n_samples=400, n_ctx=4, weighted=seed % 3 == 0)
    m, a, t, d = oracle.run_all(w)
    # SCCs by mutual reachability
    funcs = [f for f in range(w.n_scope_ids) if m.kind[f] == FUNC]
    comp = brute.scc_ids(list(range(w.n_scope_ids)), list(zip(w.site_caller.tolist(), w.site_callee.tolist())))
    assert [comp[v] for v in range(w.n_scope_ids)] == t.scc.tolist()
    for ci in range(w.n_ctx):
        if a.ctx_offsets[ci] == a.ctx_offsets[ci + 1]:
            assert t.node_off[ci] == t.node_off[ci + 1]
            continue
        (paths, unreach, w2, _), unknown = _brute_case(w, ci)
        got = _oracle_paths(t, ci)
        assert set(got) == set(paths)
        for k, (phi, X, row) in paths.items():
            gphi, gX, grow = got[k]
            assert gX == X
            assert gphi == pytest.approx(phi, rel=1e-12)
            assert grow == pytest.approx(row, rel=1e-12)
        b, e = int(t.node_off[ci]), int(t.node_off[ci + 1])
        specials = {int(t.kind[i]): t.excl[i].tolist() for i in range(b, e) if t.kind[i] != 0}
        assert specials.get(1, [0.0] * 16) == [float(x) for x in unreach]
        assert specials.get(2, [0.0] * 16) == [float(x) for x in unknown]
        # final positive edge weights
        wb, we = int(t.w_off[ci]), int(t.w_off[ci + 1])
        got_w = dict(zip(t.w_site[wb:we].tolist(), t.w_val[wb:we].tolist()))
        exp_w = {int(w.site_pc[sid]): v for sid, v in w2.items() if v > 0}
        assert got_w == exp_w
        # conservation: exclusive costs of the context sum to its samples
        n_c = int(a.count[a.ctx_offsets[ci]:a.ctx_offsets[ci + 1]].sum())
        assert t.excl[b:e].sum() == pytest.approx(n_c, rel=1e-12)
        # inclusive metrics equal sums over path extensions
        inc = brute.inclusive_by_prefix(paths)
        keys = []
        for i in range(b, e):
            if t.kind[i] != 0:
                continue
            p = int(t.parent[i])
            key = (int(t.node[i]),) if p == NONE32 else keys[p] + (int(t.site[i]),)
            keys.append(key)
            assert d.incl[i].tolist() == pytest.approx(inc[key], rel=1e-12)
            assert d.W[i] == pytest.approx(brute.issue_rate(inc[key]), rel=1e-12)


@pytest.mark.parametrize("seed", list(range(10)))
def test_exact_counts_match_path_enumeration(seed):
    # Exact-count call graphs (Section 4.2 instrumentation; Section 6.3 step 1
    # with exact counts of call instructions): the weights are the counts as
    # given, step 2 and its re-application are off, the unfolding is the same.
    w = tiny_random_case(300 + seed, n_funcs=4 + seed % 4, n_samples=400, n_ctx=3, weighted=True)
    m = oracle.build_map_workload(w)
    a = oracle.attribute(m, w.pc, w.ctx, w.stall, w.weight, w.n_ctx)
    t = oracle.apportion_workload(m, w, a, sample_based=0)
    for ci in range(w.n_ctx):
        if a.ctx_offsets[ci] == a.ctx_offsets[ci + 1]:
            continue
        (paths, _, w2, _), _ = _brute_case(w, ci, sample_based=False)
        got = _oracle_paths(t, ci)
        assert list(got) == list(paths)
        for k, (phi, X, row) in paths.items():
            assert got[k][0] == pytest.approx(phi, rel=1e-12)
            assert got[k][2] == pytest.approx(row, rel=1e-12)
        wb, we = int(t.w_off[ci]), int(t.w_off[ci + 1])
        assert dict(zip(t.w_site[wb:we].tolist(), t.w_val[wb:we].tolist())) == \
            {int(w.site_pc[sid]): v for sid, v in w2.items() if v > 0}


def test_exact_counts_skip_step2():
    # With exact counts an unsampled call edge stays at zero: B's samples have no
    # call path into them from the entry, so only the entry's own path remains
    # (the sample-based rule would set the A -> B edge to one, Section 6.3 step 2).
    w = handmade.build(3, [(2, 0, 0), (0, 1, 0)], {1: [(0, 6)], 2: [(0, 1)]}, entry=2)
    m = oracle.build_map_workload(w)
    a = oracle.attribute(m, w.pc, w.ctx, w.stall, w.weight, w.n_ctx)
    t = oracle.apportion_workload(m, w, a, sample_based=0)
    assert t.w_val.tolist() == []
    assert [int(x) for x in t.node] == [2]
    ts = oracle.apportion_workload(m, w, a, sample_based=1)
    assert [int(x) for x in ts.node] == [2, 0, 1]
    # exact counts split a callee in proportion to its call counts, as gprof does
    w = handmade.build(4, [(0, 3, 3), (1, 3, 1), (2, 3, 4)], {3: [(0, 80)]}, entry=None)
    m = oracle.build_map_workload(w)
    a = oracle.attribute(m, w.pc, w.ctx, w.stall, w.weight, w.n_ctx)
    t = oracle.apportion_workload(m, w, a, sample_based=0)
    rows = sorted((float(t.phi[i]), float(t.excl[i][0])) for i in range(len(t.node)) if t.node[i] == t.scc[3])
    assert rows == [(1 / 8, 10.0), (3 / 8, 30.0), (4 / 8, 40.0)]


@pytest.mark.parametrize("seed", list(range(10)))
def test_step2_order_independent(seed):
    # The literal step-2 rule gives one result whatever order functions are visited in.
    w = tiny_random_case(100 + seed, n_funcs=5 + seed % 3, n_samples=120, n_ctx=2)
    m = oracle.build_map_workload(w)
    nf = sum(1 for k in m.kind if k == FUNC)
    ci = 0
    results = set()
    for order in itertools.permutations(range(nf)):
        (paths, unreach, w2, _), _ = _brute_case(w, ci, order=list(order))
        results.add(tuple(sorted(w2.items())))
    assert len(results) == 1


def test_fig4_shape_golden():
    g = json.load(open(os.path.join(GOLDEN, "fig4_shape.json")))
    names = g["functions"]
    fid = {n: i for i, n in enumerate(names)}
    sites = [(fid[s["caller"]], fid[s["callee"]], s["call_samples"]) for s in g["sites"]]
    self_rows = {fid[n]: [(0, c)] for n, c in g["self_noncall"].items() if c}
    w = handmade.build(len(names), sites, self_rows, entry=fid[g["entry"]])
    m, a, t, d = oracle.run_all(w)
    pc_of = {}
    k = {}
    for s in g["sites"]:
        u = fid[s["caller"]]
        k[u] = k.get(u, 0) + 1
        pc_of[s["name"]] = handmade.func_start(u) + k[u] * 16
    exp = g["expected_preorder"]
    assert int(t.node_off[1]) == len(exp)
    keys = []
    for i, row in enumerate(exp):
        p = int(t.parent[i])
        key = (int(t.node[i]),) if p == NONE32 else keys[p] + (int(t.site[i]),)
        keys.append(key)
        want = (fid[row["path"][0]],) + tuple(pc_of[x] for x in row["path"][1:])
        assert key == want
        assert t.phi[i] == row["phi"]
        assert t.excl[i].sum() == row["excl"]
        assert d.incl[i].sum() == row["incl"]
    # D and E collapse into one SCC node, the others stay singletons
    assert t.scc[fid["D"]] == t.scc[fid["E"]]
    assert len(set(t.scc.tolist())) == 4


def _preorder_keys(t, ci):
    """Path keys of context ci's call-path nodes in the order the tree stores them."""
    b, e = int(t.node_off[ci]), int(t.node_off[ci + 1])
    keys = []
    for i in range(b, e):
        if t.kind[i] != 0:
            continue
        p = int(t.parent[i])
        keys.append((int(t.node[i]),) if p == NONE32 else keys[p] + (int(t.site[i]),))
    return keys


def test_cct_children_follow_call_site_pc_order():
    # Section 6.3 step 4 unfolds the graph into a tree of call paths; the stored
    # tree is in depth-first preorder with the children of a node ordered by the
    # call-site PC of their edge.  Here call-site PC order, callee-id order and
    # the order the sites are listed in all differ, at two levels:
    #   caller 0: sites listed to callees 1, 3, 2 at instructions 2, 1, 3
    #             -> PC order 3, 1, 2 (callee order 1, 2, 3; listing 1, 3, 2)
    #   caller 2: sites listed to callees 5, 4 at instructions 1, 2
    #   caller 3: sites listed to callees 4, 5 at instructions 2, 1
    sites = [(0, 1, 2), (0, 3, 3), (0, 2, 5), (2, 5, 1), (2, 4, 2), (3, 4, 4), (3, 5, 1)]
    slots = [2, 1, 3, 1, 2, 2, 1]
    w = handmade.build(6, sites, {1: [(0, 3)], 4: [(2, 8)], 5: [(1, 6)]}, entry=0, site_slots=slots)
    m, a, t, d = oracle.run_all(w)
    got = _preorder_keys(t, 0)
    (paths, _, _, _), _ = _brute_case(w, 0)
    assert got == list(paths)  # brute force walks children in call-site PC order
    pc = {(u, v): int(p) for (u, v, _), p in zip(sites, w.site_pc.tolist())}
    want = [(0,), (0, pc[0, 3]), (0, pc[0, 3], pc[3, 5]), (0, pc[0, 3], pc[3, 4]), (0, pc[0, 1]),
            (0, pc[0, 2]), (0, pc[0, 2], pc[2, 5]), (0, pc[0, 2], pc[2, 4])]
    assert got == want
    # children of the root by callee: 3, 1, 2 (neither callee-id nor listing order)
    assert [int(t.node[i]) for i in range(int(t.node_off[1])) if len(got[i]) == 2] == [3, 1, 2]


def test_tree_has_unit_ratios():
    # A call tree: every function has one call site, so every phi is 1 (gprof split of one).
    sites = [(0, 1, 3), (0, 2, 1), (1, 3, 0), (2, 4, 2)]
    w = handmade.build(5, sites, {3: [(1, 4)], 4: [(0, 2)], 0: [(2, 5)]}, entry=0)
    m, a, t, d = oracle.run_all(w)
    assert (t.phi == 1.0).all()
    assert t.excl.sum() == w.n_samples


def test_diamond_equal_weights_half():
    # 0 -> 1 -> 3 and 0 -> 2 -> 3 with equal call samples: 3's cost splits exactly in half.
    w = handmade.build(4, [(0, 1, 2), (0, 2, 2), (1, 3, 5), (2, 3, 5)], {3: [(3, 10)]}, entry=0)
    m, a, t, d = oracle.run_all(w)
    node3 = [i for i in range(len(t.node)) if t.node[i] == t.scc[3]]
    assert [t.phi[i] for i in node3] == [0.5, 0.5]
    assert [t.excl[i][3] for i in node3] == [5.0, 5.0]


def test_gprof_single_level_split():
    # Section 6.3 step 4: a callee's samples are apportioned by the ratio of
    # each call site's calls to all calls.  Weights 1, 2, 5 -> 1/8, 2/8, 5/8.
    w = handmade.build(4, [(0, 3, 1), (1, 3, 2), (2, 3, 5)], {3: [(0, 64)]}, entry=None)
    m, a, t, d = oracle.run_all(w)
    rows = sorted((float(t.phi[i]), float(t.excl[i][0])) for i in range(len(t.node)) if t.node[i] == t.scc[3])
    assert rows == [(1 / 8, 8.0), (2 / 8, 16.0), (5 / 8, 40.0)]


def test_power_of_two_weights_exact():
    # chain of splits with power-of-two weights: phi = product of exact binary fractions
    w = handmade.build(5, [(0, 1, 1), (0, 2, 3), (1, 3, 1), (2, 3, 1), (3, 4, 4), (1, 4, 4)],
                       {4: [(5, 64)]}, entry=0)
    m, a, t, d = oracle.run_all(w)
    assert t.excl.sum() == w.n_samples
    for x in t.phi:
        assert x * 64 == int(x * 64)


def test_step2_fires_on_unsampled_call_site():
    # Section 6.3 step 2: B is sampled but no call site into it is, so A->B gets weight 1;
    # the rule then climbs through callers: C -> A is unsampled too and A is now active.
    w = handmade.build(3, [(2, 0, 0), (0, 1, 0)], {1: [(0, 6)]}, entry=2)
    m, a, t, d = oracle.run_all(w)
    assert t.w_val.tolist() == [1, 1]
    assert t.phi.tolist() == [1.0, 1.0, 1.0]
    assert t.excl.sum() == 6


def test_scc_left_at_zero_over_zero_is_reweighted():
    # D <-> E both sampled with call samples on the internal edges; the external
    # edge X -> D is unsampled.  Step 2 does not fire (D's in-edge from E weighs 1),
    # condensation drops the internal edges and the SCC would be 0/0: the step-2
    # rule applied once more on the condensed graph gives X -> D weight 1.
    X, D, E = 0, 1, 2
    w = handmade.build(3, [(X, D, 0), (D, E, 1), (E, D, 1)], {D: [(0, 3)], E: [(1, 2)], X: [(0, 1)]}, entry=X)
    m, a, t, d = oracle.run_all(w)
    assert t.scc[D] == t.scc[E]
    assert t.node_off[1] == 2
    assert t.phi.tolist() == [1.0, 1.0]
    assert t.excl[1].sum() == 3 + 2 + 2  # D, E and the two call-site samples


def test_reach_restriction_and_specials():
    # context entry 0 reaches 1 only; samples in 2 go to <unreachable>, unmapped PCs to <unknown>.
    # Function 1 has no samples and calls nothing, so its path carries no cost and is pruned.
    w = handmade.build(3, [(0, 1, 1), (2, 1, 1)], {0: [(0, 2)], 2: [(4, 3)]}, entry=0,
                       unknown_row=[(7, 5)])
    m, a, t, d = oracle.run_all(w)
    kinds = t.kind.tolist()
    assert kinds == [0, 1, 2]
    assert t.excl[0].sum() == 3  # two samples + the call-site sample in function 0
    assert t.excl[1][4] == 3 and t.excl[1].sum() == 4  # function 2: 3 samples + its call site
    assert t.excl[2][7] == 5
    assert t.excl.sum() == w.n_samples


def test_no_entry_uses_static_roots():
    # entry -1: roots are the condensed nodes with no incoming call edge, ascending
    w = handmade.build(4, [(0, 2, 1), (1, 2, 3)], {2: [(0, 8)], 3: [(0, 1)]}, entry=None)
    m, a, t, d = oracle.run_all(w)
    roots = [int(t.node[i]) for i in range(len(t.node)) if t.parent[i] == NONE32]
    assert roots == [0, 1, 3]
    assert t.excl.sum() == w.n_samples


def test_budget_reports_required_nodes():
    w = small_config(7, n_samples=20000, n_funcs=120, n_inst=4000, n_ctx=60)
    m = oracle.build_map_workload(w)
    a = oracle.attribute(m, w.pc, w.ctx, w.stall, None, w.n_ctx)
    t = oracle.apportion_workload(m, w, a)
    need = len(t.parent)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.apportion_workload(m, w, a, max_nodes=need - 1)
    assert ei.value.code == oracle.E_BUDGET and ei.value.required == need


def test_callgraph_validation():
    w = handmade.build(3, [(0, 1, 1)], {1: [(0, 1)]}, entry=0)
    m = oracle.build_map_workload(w)
    a = oracle.attribute(m, w.pc, w.ctx, w.stall, None, w.n_ctx)
    bad_pc = w.site_pc.copy(); bad_pc[0] = handmade.func_start(2) + 16  # site not inside its caller
    for sp, sc, se, ent in [
        (np.concatenate([w.site_pc, w.site_pc]), np.array([0, 0], np.uint32), np.array([1, 2], np.uint32), [0]),
        (bad_pc, w.site_caller, w.site_callee, [0]),
        (w.site_pc, w.site_caller, np.array([7], np.uint32), [0]),
        (w.site_pc, w.site_caller, w.site_callee, [5]),
    ]:
        with pytest.raises(oracle.OracleError) as ei:
            oracle.apportion(m, w.n_scope_ids, sp, sc, se, w.ctx_parent, np.array(ent, np.int32), a)
        assert ei.value.code == oracle.E_INVAL


# ---------------------------------------------------------------------------
# derived metrics (Section 6.1 statistic generation; Section 7.1 W)
# ---------------------------------------------------------------------------

def test_warp_issue_rate_closed_form():
    # W = (S - S_stall) / S: 6 issued of 16 samples -> 0.375
    w = handmade.build(1, [], {0: [(0, 6), (3, 4), (9, 6)]}, entry=0)
    m, a, t, d = oracle.run_all(w)
    assert d.W.tolist() == [0.375]
    assert d.S.tolist() == [16.0]
    assert d.host_W.tolist() == [0.375]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_host_and_scope_rollups(seed):
    w = small_config(seed, n_samples=30000, n_funcs=80, n_inst=3000, n_ctx=40)
    m, a, t, d = oracle.run_all(w)
    # host tree: inclusive at a context = samples of its subtree (brute descendant scan)
    par = w.ctx_parent.tolist()
    own = np.zeros((w.n_ctx, 16), np.uint64)
    np.add.at(own, (w.ctx.astype(np.int64), w.stall.astype(np.int64)), 1)
    for c in range(w.n_ctx):
        sub = [x for x in range(w.n_ctx) if _is_desc(x, c, par)]
        assert np.array_equal(d.host_incl[c], own[sub].sum(axis=0))
    roots = [c for c in range(w.n_ctx) if par[c] == NONE32]
    assert int(sum(d.host_incl[r].sum() for r in roots)) == w.n_samples
    # static scope tree: inclusive over the scope's ancestors chain
    sc = _scopes(w)
    exp = {}
    for c, s, st, cnt in zip(a.ctx.tolist(), a.scope.tolist(), a.stall.tolist(), a.count.tolist()):
        chain = [NONE32] if s == NONE32 else brute.ancestors(s, sc)
        for y in chain:
            exp.setdefault((c, y), [0] * 16)[st] += cnt
    got = {}
    for c in range(w.n_ctx):
        for i in range(int(d.sc_off[c]), int(d.sc_off[c + 1])):
            got[(c, int(d.sc_scope[i]))] = d.sc_val[i].tolist()
    assert got == exp


def _is_desc(x, c, par):
    while x != NONE32:
        if x == c:
            return True
        x = par[x]
    return False


def test_conservation_small_and_config1():
    for w in [small_config(11), config1()]:
        m, a, t, d = oracle.run_all(w)
        for ci in range(w.n_ctx):
            b, e = int(t.node_off[ci]), int(t.node_off[ci + 1])
            n_c = int(a.count[a.ctx_offsets[ci]:a.ctx_offsets[ci + 1]].sum())
            assert abs(t.excl[b:e].sum() - n_c) <= 1e-9 * max(1, n_c)


# ---------------------------------------------------------------------------
# learned index: FP64 reference of the root network (no passage in the paper;
# the answer itself is the plain search, pinned by the lookup tests above)
# ---------------------------------------------------------------------------

def test_learned_ref_gradient_matches_central_differences():
    from oracle import learned_ref as L
    r = np.random.default_rng(5)
    p = r.normal(0.0, 0.5, size=L.NPARAM)
    X = r.random((7, 2))
    T = r.random(7)
    g = L.grad(p, X, T)
    idx = list(range(0, L.NPARAM, 7)) + [L.NPARAM - 1]
    fd = L.central_differences(p, X, T, idx)
    np.testing.assert_allclose(g[idx], fd, rtol=1e-5, atol=1e-9)


def test_learned_ref_forward_closed_form():
    # one active path: h1_0 = x0, h2_0 = 2 * h1_0, y = 3 * h2_0 + 0.5 -> y = 6 x0 + 0.5
    from oracle import learned_ref as L
    p = np.zeros(L.NPARAM)
    p[0] = 1.0                                  # W1[0][0]
    p[2 * 64 + 64 + 0] = 2.0                    # W2[0][0]
    p[2 * 64 + 64 + 64 * 64 + 64 + 0] = 3.0     # w3[0]
    p[-1] = 0.5                                 # b3
    X = np.array([[0.25, 0.9], [0.0, 0.3], [1.0, 0.0]])
    y, _ = L.forward(p, X)
    assert y.tolist() == [2.0, 0.5, 6.5]
    # a negative input is cut by the first ReLU
    y, _ = L.forward(p, np.array([[-0.5, 0.0]]))
    assert y.tolist() == [0.5]


# ---------------------------------------------------------------------------
# several profiles: statistics (Section 4.5), sparse layouts (Section 6.2),
# combination of runs (Section 4.7)
# ---------------------------------------------------------------------------

class _A:
    def __init__(self, keys):
        ks = sorted(keys)
        self.ctx = np.array([k[0] for k in ks], np.uint32)
        self.pc = np.array([k[1] for k in ks], np.uint64)
        self.stall = np.array([k[2] for k in ks], np.uint8)
        self.count = np.array([keys[k] for k in ks], np.uint64)


def test_unify_identical_profiles_have_no_spread():
    from oracle import unify_ref as U
    keys = {(0, 0x100, 0): 5, (0, 0x100, 3): 2, (1, 0x80, 1): 7}
    r = U.unify([_A(keys)] * 4)
    assert r["st_sum"].tolist() == [20, 8, 28]
    assert r["st_min"].tolist() == r["st_max"].tolist() == [5, 2, 7]
    assert r["st_mean"].tolist() == [5.0, 2.0, 7.0]
    assert r["st_std"].tolist() == [0.0] * 3 and r["st_cov"].tolist() == [0.0] * 3


def test_unify_single_holder_closed_form():
    # one of P profiles holds x, the others nothing: mean x/P, std x sqrt(P-1)/P, CoV sqrt(P-1)
    from oracle import unify_ref as U
    P, x = 5, 40
    profs = [_A({})] * (P - 1) + [_A({(2, 0x40, 9): x})]
    r = U.unify(profs)
    assert r["st_min"].tolist() == [0] and r["st_max"].tolist() == [x]
    assert r["st_mean"][0] == pytest.approx(x / P, rel=1e-15)
    assert r["st_std"][0] == pytest.approx(x * np.sqrt(P - 1) / P, rel=1e-15)
    assert r["st_cov"][0] == pytest.approx(np.sqrt(P - 1), rel=1e-15)
    assert r["cms_pid"].tolist() == [P - 1]


def test_unify_layouts_transpose_and_space():
    # CMS and PMS hold the same (profile, context, metric, value) entries; the CMS
    # size is 2 nnz (pids, vals) + metric pairs + contexts + 1 (Section 6.2)
    from oracle import unify_ref as U
    r0 = np.random.default_rng(3)
    profs = []
    for p in range(4):
        keys = {}
        for _ in range(60):
            keys[(int(r0.integers(0, 5)), 0x1000 + 16 * int(r0.integers(0, 9)), int(r0.integers(0, 16)))] = \
                int(r0.integers(1, 50))
        profs.append(_A(keys))
    r = U.unify(profs)
    cms = set()
    for c in range(len(r["ctx"])):
        for j in range(int(r["cms_m_off"][c]), int(r["cms_m_off"][c + 1])):
            a = int(r["cms_mstart"][j])
            b = int(r["cms_mstart"][j + 1]) if j + 1 < len(r["cms_mstart"]) else len(r["cms_pid"])
            for i in range(a, b):
                cms.add((int(r["cms_pid"][i]), c, int(r["cms_mid"][j]), int(r["cms_val"][i])))
    pms = set()
    for p in range(4):
        hs = range(int(r["pms_c_off"][p]), int(r["pms_c_off"][p + 1]))
        for h in hs:
            a = int(r["pms_cstart"][h])
            b = int(r["pms_cstart"][h + 1]) if h + 1 < hs.stop else int(r["pms_off"][p + 1])
            for i in range(a, b):
                pms.add((p, int(r["pms_ctx"][h]), int(r["pms_mid"][i]), int(r["pms_val"][i])))
    nnz = sum(len(a.count) for a in profs)
    assert cms == pms and len(cms) == nnz
    size = 2 * len(r["cms_pid"]) + len(r["cms_mid"]) + len(r["ctx"]) + 1
    assert size == 2 * nnz + len(r["cms_mid"]) + len(r["ctx"]) + 1
    # the statistics' sums equal the per-key totals of the combination
    comb = U.combine(profs)
    tot = {(int(c), int(p), int(s)): int(n) for c, p, s, n in zip(comb["ctx"], comb["pc"], comb["stall"],
                                                                 comb["count"])}
    for j in range(len(r["st_sum"])):
        c = int(r["st_ctx"][j])
        assert tot[(int(r["ctx"][c]), int(r["pc"][c]), int(r["st_mid"][j]))] == int(r["st_sum"][j])


def test_combine_equals_attribution_of_all_samples():
    # Section 4.7: combining runs sums their raw metrics; attributing the union of
    # the runs' samples at once gives the same keys (Section 4.5: a raw metric is a sum)
    from oracle import unify_ref as U
    w = small_config(21, n_samples=30000)
    m = oracle.build_map_workload(w)
    cuts = [0, 7000, 19000, 30000]
    runs = [oracle.attribute(m, w.pc[a:b], w.ctx[a:b], w.stall[a:b], None, w.n_ctx) for a, b in zip(cuts, cuts[1:])]
    allr = oracle.attribute(m, w.pc, w.ctx, w.stall, None, w.n_ctx)
    comb = U.combine(runs)
    for f in ["ctx", "pc", "stall", "count"]:
        assert np.array_equal(comb[f], getattr(allr, f))
