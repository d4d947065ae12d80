"""Hand-specified small profiles (explicit functions, call sites and samples).

Function f occupies `size` instructions starting at base + f * size * 16.
Instruction 0 of each function carries its non-call samples; call site k of a
caller sits at instruction 1 + k.  This module only lays out inputs.
"""
from __future__ import annotations

import numpy as np

from .gen import FUNC, STRIDE, UNMAPPED, Workload

BASE = 0x10000


def func_start(f: int, size: int = 16) -> int:
    return BASE + f * size * STRIDE


def build(n_funcs: int, sites, self_rows, entry=0, size: int = 16, n_ctx: int = 1,
          ctx_parent=None, ctx_entry=None, ctx_of=None, unknown_row=None, site_slots=None) -> Workload:
    """sites: list of (caller, callee, call_samples[, stall]); self_rows: f -> list of
    (stall, count) non-call samples.  All samples go to context 0 unless ctx_of
    maps a function to another context.  site_slots, if given, places site i at
    instruction site_slots[i] of its caller instead of 1 + its rank among the
    caller's sites (the call-site arrays keep the listing order)."""
    s_start = np.array([func_start(f, size) for f in range(n_funcs)], dtype=np.uint64)
    s_end = s_start + np.uint64(size * STRIDE)
    per_caller = {}
    site_pc, site_caller, site_callee, pcs, stalls, ctxs = [], [], [], [], [], []
    ctx_of = ctx_of or {}
    for t in sites:
        u, v, c = t[0], t[1], t[2]
        st = t[3] if len(t) > 3 else 0
        k = per_caller.get(u, 0)
        per_caller[u] = k + 1
        slot = (1 + k) if site_slots is None else site_slots[len(site_pc)]
        pc = func_start(u, size) + slot * STRIDE
        site_pc.append(pc); site_caller.append(u); site_callee.append(v)
        pcs += [pc] * c; stalls += [st] * c; ctxs += [ctx_of.get(u, 0)] * c
    for f, rows in self_rows.items():
        for st, c in rows:
            pcs += [func_start(f, size)] * c; stalls += [st] * c; ctxs += [ctx_of.get(f, 0)] * c
    if unknown_row:
        for st, c in unknown_row:
            pcs += [BASE - STRIDE] * c; stalls += [st] * c; ctxs += [0] * c
    parent = np.full(n_ctx, UNMAPPED, np.uint32) if ctx_parent is None else np.asarray(ctx_parent, np.uint32)
    if ctx_entry is None:
        ctx_entry = [entry if entry is not None else -1] * n_ctx
    w = Workload(
        name="handmade", seed=0, scope_start=s_start, scope_end=s_end,
        scope_id=np.arange(n_funcs, dtype=np.uint32), scope_kind=np.full(n_funcs, FUNC, np.uint32),
        line_start=np.zeros(0, np.uint64), line_end=np.zeros(0, np.uint64),
        line_file=np.zeros(0, np.uint32), line_line=np.zeros(0, np.uint32), n_scope_ids=n_funcs,
        site_pc=np.array(site_pc, np.uint64), site_caller=np.array(site_caller, np.uint32),
        site_callee=np.array(site_callee, np.uint32), ctx_parent=parent,
        ctx_entry=np.asarray(ctx_entry, np.int32),
    )
    w.pc = np.array(pcs, np.uint64)
    w.ctx = np.array(ctxs, np.uint32)
    w.stall = np.array(stalls, np.uint8)
    w.meta["site_names"] = None
    return w
