"""CPU oracle for GPU PC-sample attribution -- test infrastructure only.

`hpa_oracle.cpp` is a plain single-threaded C++ reference of every step of the
path (structure map, attribution, apportioning into a GPU calling-context tree,
derived metrics); `brute.py` holds pure-Python brute-force formulations used to
pin the oracle on tiny inputs.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark use this package; the library never does.
Nothing here is shared with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hpa_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVAL, E_UNSORTED, E_OVERLAP, E_NOT_LAMINAR, E_NOMEM, E_BUDGET = 0, -1, -2, -3, -4, -5, -6
NONE32 = 0xFFFFFFFF
NONE64 = 0xFFFFFFFFFFFFFFFF
NS = 16


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (no vector FMA contraction, plain -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P, U64, U32, I32, I = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int32, C.c_int
        PP = C.POINTER(C.c_void_p)
        PU64 = C.POINTER(C.c_uint64)
        L.orc_map_build.argtypes = [P, P, P, P, U64, P, P, P, P, U64, PP]
        L.orc_map_from_intervals.argtypes = [P, P, U64, PP]
        L.orc_map_sizes.argtypes = [P, PU64, PU64]
        L.orc_map_get.argtypes = [P] + [P] * 8
        L.orc_lookup.argtypes = [P, P, U64, P]
        L.orc_map_free.argtypes = [P]
        L.orc_attribute.argtypes = [P, P, P, P, P, U64, U32, P, PP]
        L.orc_attr_size.argtypes = [P]
        L.orc_attr_size.restype = U64
        L.orc_attr_get.argtypes = [P] * 7
        L.orc_attr_free.argtypes = [P]
        L.orc_apportion.argtypes = [P, U32, P, P, P, U64, U32, P, P, P, I, U64, PU64, PP]
        L.orc_cct_sizes.argtypes = [P, PU64, PU64, PU64]
        L.orc_cct_get.argtypes = [P] * 12
        L.orc_cct_free.argtypes = [P]
        L.orc_derive.argtypes = [P, P, P, U32, P, PP]
        L.orc_derived_nscope.argtypes = [P]
        L.orc_derived_nscope.restype = U64
        L.orc_derived_get.argtypes = [P] * 9
        L.orc_derived_free.argtypes = [P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


class _Handle:
    _free = None

    def __init__(self, h):
        self.h = h

    def __del__(self):
        if self.h and _lib is not None:
            getattr(_lib, self._free)(self.h)
            self.h = None


class Map(_Handle):
    """Elementary intervals [start, end) with labels, and the scope table."""

    _free = "orc_map_free"

    def _load(self):
        n_iv, n_ids = C.c_uint64(), C.c_uint64()
        lib().orc_map_sizes(self.h, C.byref(n_iv), C.byref(n_ids))
        m, k = n_iv.value, n_ids.value
        self.start = np.empty(m, np.uint64); self.end = np.empty(m, np.uint64)
        self.scope = np.empty(m, np.uint32); self.file = np.empty(m, np.uint32)
        self.line = np.empty(m, np.uint32)
        self.parent = np.empty(k, np.uint32); self.kind = np.empty(k, np.uint8)
        self.func = np.empty(k, np.uint32)
        lib().orc_map_get(self.h, *map(_p, [self.start, self.end, self.scope, self.file, self.line,
                                            self.parent, self.kind, self.func]))
        return self

    @property
    def n_ids(self):
        return int(self.kind.shape[0])


def build_map(scope_start, scope_end, scope_id, scope_kind, line_start=None, line_end=None,
              line_file=None, line_line=None) -> Map:
    ss, se = _c(scope_start, np.uint64), _c(scope_end, np.uint64)
    si, sk = _c(scope_id, np.uint32), _c(scope_kind, np.uint32)
    nl = 0 if line_start is None else len(line_start)
    ls = _c(line_start if nl else np.zeros(0), np.uint64)
    le = _c(line_end if nl else np.zeros(0), np.uint64)
    lf = _c(line_file if nl else np.zeros(0), np.uint32)
    ll = _c(line_line if nl else np.zeros(0), np.uint32)
    h = C.c_void_p()
    rc = lib().orc_map_build(_p(ss), _p(se), _p(si), _p(sk), len(ss), _p(ls), _p(le), _p(lf), _p(ll),
                             nl, C.byref(h))
    if rc != OK:
        raise OracleError(rc, "structure map")
    return Map(h)._load()


def build_map_workload(w) -> Map:
    return build_map(w.scope_start, w.scope_end, w.scope_id, w.scope_kind, w.line_start, w.line_end,
                     w.line_file, w.line_line)


def map_from_intervals(start, end) -> Map:
    s, e = _c(start, np.uint64), _c(end, np.uint64)
    h = C.c_void_p()
    rc = lib().orc_map_from_intervals(_p(s), _p(e), len(s), C.byref(h))
    if rc != OK:
        raise OracleError(rc, "interval map")
    return Map(h)._load()


def lookup(m: Map, pc) -> np.ndarray:
    q = _c(pc, np.uint64)
    out = np.empty(len(q), np.uint32)
    lib().orc_lookup(m.h, _p(q), len(q), _p(out))
    return out


class Attribution(_Handle):
    _free = "orc_attr_free"


def attribute(m: Map, pc, ctx, stall, weight, n_ctx: int, ctx_mask=None) -> Attribution:
    pc, ctx, stall = _c(pc, np.uint64), _c(ctx, np.uint32), _c(stall, np.uint8)
    weight = _c(weight, np.uint32)
    mask = _c(ctx_mask, np.uint8)
    h = C.c_void_p()
    rc = lib().orc_attribute(m.h, _p(pc), _p(ctx), _p(stall), _p(weight), len(pc), n_ctx, _p(mask),
                             C.byref(h))
    if rc != OK:
        raise OracleError(rc, "attribution")
    a = Attribution(h)
    u = int(lib().orc_attr_size(h))
    a.ctx = np.empty(u, np.uint32); a.pc = np.empty(u, np.uint64); a.stall = np.empty(u, np.uint8)
    a.count = np.empty(u, np.uint64); a.scope = np.empty(u, np.uint32)
    a.ctx_offsets = np.empty(n_ctx + 1, np.uint64)
    lib().orc_attr_get(h, *map(_p, [a.ctx, a.pc, a.stall, a.count, a.scope, a.ctx_offsets]))
    a.n_ctx = n_ctx
    return a


class Cct(_Handle):
    _free = "orc_cct_free"


def apportion(m: Map, n_funcs, site_pc, site_caller, site_callee, ctx_parent, ctx_entry,
              a: Attribution, sample_based: int = 1, max_nodes: int = 0) -> Cct:
    sp, sc, se = _c(site_pc, np.uint64), _c(site_caller, np.uint32), _c(site_callee, np.uint32)
    cp, ce = _c(ctx_parent, np.uint32), _c(ctx_entry, np.int32)
    h = C.c_void_p()
    req = C.c_uint64()
    rc = lib().orc_apportion(m.h, n_funcs, _p(sp), _p(sc), _p(se), len(sp), len(cp), _p(cp), _p(ce),
                             a.h, sample_based, max_nodes, C.byref(req), C.byref(h))
    if rc != OK:
        err = OracleError(rc, "apportion")
        err.required = req.value
        raise err
    t = Cct(h)
    nn, nw, nscc = C.c_uint64(), C.c_uint64(), C.c_uint64()
    lib().orc_cct_sizes(h, C.byref(nn), C.byref(nw), C.byref(nscc))
    nn, nw, nscc = nn.value, nw.value, nscc.value
    nc = len(cp)
    t.scc = np.empty(nscc, np.uint32); t.node_off = np.empty(nc + 1, np.uint64)
    t.parent = np.empty(nn, np.uint32); t.node = np.empty(nn, np.uint32)
    t.site = np.empty(nn, np.uint64); t.kind = np.empty(nn, np.uint8)
    t.phi = np.empty(nn, np.float64); t.excl = np.empty((nn, NS), np.float64)
    t.w_off = np.empty(nc + 1, np.uint64); t.w_site = np.empty(nw, np.uint64)
    t.w_val = np.empty(nw, np.uint64)
    lib().orc_cct_get(h, *map(_p, [t.scc, t.node_off, t.parent, t.node, t.site, t.kind, t.phi, t.excl,
                                   t.w_off, t.w_site, t.w_val]))
    t.required = req.value
    return t


def apportion_workload(m: Map, w, a: Attribution, **kw) -> Cct:
    return apportion(m, w.n_scope_ids, w.site_pc, w.site_caller, w.site_callee, w.ctx_parent,
                     w.ctx_entry, a, **kw)


class Derived(_Handle):
    _free = "orc_derived_free"


def derive(m: Map, a: Attribution, t: Cct, ctx_parent) -> Derived:
    cp = _c(ctx_parent, np.uint32)
    h = C.c_void_p()
    lib().orc_derive(m.h, a.h, t.h, len(cp), _p(cp), C.byref(h))
    d = Derived(h)
    nn = t.parent.shape[0]
    nc = len(cp)
    k = int(lib().orc_derived_nscope(h))
    d.incl = np.empty((nn, NS), np.float64); d.S = np.empty(nn, np.float64); d.W = np.empty(nn, np.float64)
    d.host_incl = np.empty((nc, NS), np.uint64); d.host_W = np.empty(nc, np.float64)
    d.sc_off = np.empty(nc + 1, np.uint64); d.sc_scope = np.empty(k, np.uint32)
    d.sc_val = np.empty((k, NS), np.uint64)
    lib().orc_derived_get(h, *map(_p, [d.incl, d.S, d.W, d.host_incl, d.host_W, d.sc_off, d.sc_scope,
                                       d.sc_val]))
    return d


def run_all(w, sample_based: int = 1, ctx_mask=None):
    """Structure map -> attribution -> apportioning -> derived metrics for a workload."""
    m = build_map_workload(w)
    a = attribute(m, w.pc, w.ctx, w.stall, w.weight, w.n_ctx, ctx_mask=ctx_mask)
    t = apportion_workload(m, w, a, sample_based=sample_based)
    d = derive(m, a, t, w.ctx_parent)
    return m, a, t, d
