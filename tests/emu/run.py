"""Run the CPU build of the kernel sources (build.py) through the C ABI on
small seeded cases and compare every output with the oracle: attribution
(dense and general pipelines), and the calling-context tree with its derived
metrics (integer fields exactly, FP64 fields within 1e-9 relative).  "Device"
pointers of the CPU build are host pointers, so outputs are read in place.

usage: python tests/emu/run.py LIBRARY CASE...   (cases: see CASES)
Prints one line per case; exits 1 if any case differs from the oracle.
"""
import ctypes as C
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
import numpy as np  # noqa: E402

import oracle  # noqa: E402
import paper_2109_06931_amd as hpa  # noqa: E402
from workloads import handmade, small_config, tiny_random_case  # noqa: E402

RTOL = 1e-9


def load(path):
    """The CPU build exports the attribution and call-path entry points only."""
    L = C.CDLL(path)
    P, PP, I, U32 = C.c_void_p, C.POINTER(C.c_void_p), C.c_int, C.c_uint32
    L.hpa_last_error.restype = C.c_char_p
    L.hpa_ctx_create.argtypes = [I, P, PP]
    L.hpa_ctx_destroy.argtypes = [P]
    L.hpa_ctx_destroy.restype = None
    L.hpa_build_structure_map.argtypes = [P, C.POINTER(hpa._StructureDesc), P, PP]
    L.hpa_structure_map_view_get.argtypes = [P, C.POINTER(hpa._MapView)]
    L.hpa_structure_map_free.argtypes = [P]
    L.hpa_structure_map_free.restype = None
    L.hpa_attribute.argtypes = [P, P, C.POINTER(hpa._Samples), P, PP]
    L.hpa_attribution_view_get.argtypes = [P, C.POINTER(hpa._AttrView)]
    L.hpa_attribution_free.argtypes = [P]
    L.hpa_attribution_free.restype = None
    L.hpa_prepare_callgraph.argtypes = [P, P, C.POINTER(hpa._CallGraph), C.POINTER(hpa._ContextTable), P, PP]
    L.hpa_callgraph_plan_free.argtypes = [P]
    L.hpa_callgraph_plan_free.restype = None
    L.hpa_apportion_callpaths.argtypes = [P, P, P, C.POINTER(hpa._ApportionOpts), P, PP]
    L.hpa_gpu_cct_view_get.argtypes = [P, C.POINTER(hpa._CctView)]
    L.hpa_gpu_cct_free.argtypes = [P]
    L.hpa_gpu_cct_free.restype = None
    L.hpa_derive_metrics.argtypes = [P, P, P, P, P, PP]
    L.hpa_metrics_view_get.argtypes = [P, C.POINTER(hpa._MetricsView)]
    L.hpa_metrics_free.argtypes = [P]
    L.hpa_metrics_free.restype = None
    hpa._lib = L
    hpa._stream = lambda s=None: 0  # one in-order "stream"
    return L


def view(ptr, shape, dt):
    n = int(np.prod(shape))
    if n == 0:
        return np.zeros(shape, dt)
    buf = (C.c_char * (n * np.dtype(dt).itemsize)).from_address(ptr)
    return np.frombuffer(buf, dtype=dt).reshape(shape).copy()


def _ok(rc, L, what):
    if rc != 0:
        raise RuntimeError(f"{what}: status {rc}: {L.hpa_last_error().decode(errors='replace')}")


def attribute(L, ctx, m, w):
    pc = np.ascontiguousarray(w.pc, np.uint64)
    cx = np.ascontiguousarray(w.ctx, np.uint32)
    st = np.ascontiguousarray(w.stall, np.uint8)
    wt = None if w.weight is None else np.ascontiguousarray(w.weight, np.uint32)
    s = hpa._Samples(pc.ctypes.data, cx.ctypes.data, st.ctypes.data, None if wt is None else wt.ctypes.data,
                     len(pc), w.n_ctx)
    h = C.c_void_p()
    _ok(L.hpa_attribute(ctx.h, m.h, C.byref(s), None, C.byref(h)), L, "hpa_attribute")
    v = hpa._AttrView()
    _ok(L.hpa_attribution_view_get(h, C.byref(v)), L, "hpa_attribution_view_get")
    u = v.n_keys
    got = dict(ctx=view(v.ctx, (u,), np.uint32), pc=view(v.pc, (u,), np.uint64),
               stall=view(v.stall, (u,), np.uint8), count=view(v.count, (u,), np.uint64),
               scope=view(v.scope, (u,), np.uint32), ctx_offsets=view(v.ctx_offsets, (w.n_ctx + 1,), np.uint64))
    return h, got


def check_attribution(got, oa):
    bad = []
    if len(got["ctx"]) != len(oa.ctx):
        return [f"key count {len(got['ctx'])} vs {len(oa.ctx)}"]
    for f in ["ctx", "pc", "stall", "count", "scope", "ctx_offsets"]:
        if not np.array_equal(got[f], getattr(oa, f)):
            bad.append(f)
    return bad


def run_attr(L, w):
    ctx = hpa.Context(0)
    m = hpa.build_structure_map_workload(ctx, w)
    h, got = attribute(L, ctx, m, w)
    L.hpa_attribution_free(h)
    om = oracle.build_map_workload(w)
    oa = oracle.attribute(om, w.pc, w.ctx, w.stall, w.weight, w.n_ctx)
    return check_attribution(got, oa), f"{len(w.pc)} samples, {len(oa.ctx)} keys"


def run_cct(L, w, sample_based=1):
    ctx = hpa.Context(0)
    m = hpa.build_structure_map_workload(ctx, w)
    ah, got = attribute(L, ctx, m, w)
    sp, sc, se = (np.ascontiguousarray(w.site_pc, np.uint64), np.ascontiguousarray(w.site_caller, np.uint32),
                  np.ascontiguousarray(w.site_callee, np.uint32))
    cp, ce = np.ascontiguousarray(w.ctx_parent, np.uint32), np.ascontiguousarray(w.ctx_entry, np.int32)
    g = hpa._CallGraph(w.n_scope_ids, len(sp), sp.ctypes.data, sc.ctypes.data, se.ctypes.data)
    t = hpa._ContextTable(len(cp), cp.ctypes.data, ce.ctypes.data)
    plan = C.c_void_p()
    _ok(L.hpa_prepare_callgraph(ctx.h, m.h, C.byref(g), C.byref(t), None, C.byref(plan)), L, "hpa_prepare_callgraph")
    req = C.c_uint64(0)
    o = hpa._ApportionOpts(sample_based, 0, C.cast(C.byref(req), C.c_void_p))
    th = C.c_void_p()
    _ok(L.hpa_apportion_callpaths(ctx.h, plan, ah, C.byref(o), None, C.byref(th)), L, "hpa_apportion_callpaths")
    dh = C.c_void_p()
    _ok(L.hpa_derive_metrics(ctx.h, plan, ah, th, None, C.byref(dh)), L, "hpa_derive_metrics")
    tv, dv = hpa._CctView(), hpa._MetricsView()
    _ok(L.hpa_gpu_cct_view_get(th, C.byref(tv)), L, "hpa_gpu_cct_view_get")
    _ok(L.hpa_metrics_view_get(dh, C.byref(dv)), L, "hpa_metrics_view_get")
    n, c, r, ns = tv.n_nodes, tv.n_ctx, dv.n_scope_rows, hpa.N_STALL
    tt = dict(scc=view(tv.scc, (tv.n_funcs,), np.uint32), node_offsets=view(tv.node_offsets, (c + 1,), np.uint64),
              parent=view(tv.parent, (n,), np.uint32), node=view(tv.node, (n,), np.uint32),
              site=view(tv.site, (n,), np.uint64), kind=view(tv.kind, (n,), np.uint8),
              phi=view(tv.phi, (n,), np.float64), excl=view(tv.excl, (n, ns), np.float64),
              w_offsets=view(tv.w_offsets, (c + 1,), np.uint64), w_site=view(tv.w_site, (tv.n_weights,), np.uint64),
              w_val=view(tv.w_val, (tv.n_weights,), np.uint64))
    dd = dict(incl=view(dv.incl, (n, ns), np.float64), S=view(dv.S, (n,), np.float64),
              W=view(dv.W, (n,), np.float64), host_incl=view(dv.host_incl, (c, ns), np.uint64),
              host_W=view(dv.host_W, (c,), np.float64), sc_offsets=view(dv.sc_offsets, (c + 1,), np.uint64),
              sc_scope=view(dv.sc_scope, (r,), np.uint32), sc_val=view(dv.sc_val, (r, ns), np.uint64))
    L.hpa_metrics_free(dh)
    L.hpa_gpu_cct_free(th)
    L.hpa_callgraph_plan_free(plan)
    L.hpa_attribution_free(ah)
    om, oa, ot, od = oracle.run_all(w, sample_based=sample_based)
    bad = check_attribution(got, oa)
    exact = [("scc", ot.scc), ("node_offsets", ot.node_off), ("parent", ot.parent), ("node", ot.node),
             ("site", ot.site), ("kind", ot.kind), ("w_offsets", ot.w_off), ("w_site", ot.w_site),
             ("w_val", ot.w_val)]
    bad += [f for f, e in exact if not np.array_equal(tt[f], e)]
    close = [("phi", tt["phi"], ot.phi), ("excl", tt["excl"], ot.excl), ("incl", dd["incl"], od.incl),
             ("S", dd["S"], od.S), ("W", dd["W"], od.W), ("host_W", dd["host_W"], od.host_W)]
    for f, a, e in close:
        a, e = np.asarray(a), np.asarray(e)
        if a.shape != e.shape or not np.allclose(a, e, rtol=RTOL, atol=0):
            bad.append(f)
    exact2 = [("host_incl", od.host_incl), ("sc_offsets", od.sc_off), ("sc_scope", od.sc_scope),
              ("sc_val", od.sc_val)]
    bad += [f for f, e in exact2 if not np.array_equal(dd[f], e)]
    return bad, f"{len(w.pc)} samples, {n} tree nodes"


def _tiny(seed):
    return tiny_random_case(seed, n_funcs=4 + seed % 5, n_samples=500 + 50 * seed, n_ctx=4 + seed % 3,
                            weighted=seed % 4 == 3)


def _fig4():
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "fig4_shape.json")))
    names = g["functions"]
    fid = {nm: i for i, nm in enumerate(names)}
    sites = [(fid[s["caller"]], fid[s["callee"]], s["call_samples"]) for s in g["sites"]]
    self_rows = {fid[nm]: [(0, c)] for nm, c in g["self_noncall"].items() if c}
    return handmade.build(len(names), sites, self_rows, entry=fid[g["entry"]])


CASES = {f"cct_tiny{s}": (run_cct, lambda s=s: _tiny(s)) for s in range(12)}
CASES.update({
    "cct_fig4": (run_cct, _fig4),
    "cct_small1": (run_cct, lambda: small_config(1, n_samples=20_000, n_funcs=120, n_inst=4000, n_ctx=60)),
    "attr_tiny0": (run_attr, lambda: _tiny(0)),
    "attr_tiny3w": (run_attr, lambda: _tiny(3)),
    "attr_small2w": (run_attr, lambda: small_config(2, n_samples=30_000, weighted=True)),
    "attr_small3s": (run_attr, lambda: small_config(3, n_samples=30_000, shuffled=True)),
})


def main(argv):
    L = load(argv[0])
    failed = 0
    for name in argv[1:]:
        fn, make = CASES[name]
        t0 = time.time()
        print(f"case {name}", flush=True)
        bad, what = fn(L, make())
        failed += bool(bad)
        print(f"{name}: {'OK' if not bad else 'MISMATCH ' + ','.join(bad)} ({what}, {time.time() - t0:.1f} s)",
              flush=True)
    return 1 if failed else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
