"""Python binding of libhpa (GPU PC-sample attribution on MI355X).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory (inputs as CUDA tensors) and the stream
(`torch.cuda.current_stream()` unless one is given).  Names follow the C ABI
in include/hpa.h.  The library must be built (`paper_2109_06931_amd.build`);
importing this module on a machine without it raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HPA_LIBRARY") or os.path.join(_HERE, "libhpa.so")

OK, E_INVAL, E_UNSORTED, E_OVERLAP, E_NOT_LAMINAR, E_NOMEM, E_BUDGET, E_DEVICE, E_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
UNMAPPED = 0xFFFFFFFF
NO_SITE = 0xFFFFFFFFFFFFFFFF
N_STALL = 16
LOOKUP_PLAIN, LOOKUP_LEARNED = 0, 1
NOALLOC_SCRATCH_BYTES = 128 << 20
NODE_PATH, NODE_UNREACHABLE, NODE_UNKNOWN = 0, 1, 2

SCOPE_DTYPE = np.dtype([("start", "<u8"), ("end", "<u8"), ("id", "<u4"), ("kind", "<u4")])
LINE_DTYPE = np.dtype([("start", "<u8"), ("end", "<u8"), ("file", "<u4"), ("line", "<u4")])


class HpaError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what}: status {code}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# ctypes declarations
# ---------------------------------------------------------------------------
P = C.c_void_p
U64, U32, I32, I = C.c_uint64, C.c_uint32, C.c_int32, C.c_int


class _StructureDesc(C.Structure):
    _fields_ = [("scopes", P), ("n_scopes", U64), ("lines", P), ("n_lines", U64), ("iv_start", P),
                ("iv_end", P), ("n_iv", U64), ("learned", I)]


class _MapView(C.Structure):
    _fields_ = [("n_intervals", U64), ("n_scope_ids", U32), ("start", P), ("end", P), ("scope", P),
                ("file", P), ("line", P), ("parent", P), ("kind", P), ("func", P)]


class _Samples(C.Structure):
    _fields_ = [("pc", P), ("ctx", P), ("stall", P), ("weight", P), ("n", U64), ("n_ctx", U32)]


class _AttrView(C.Structure):
    _fields_ = [("n_keys", U64), ("n_ctx", U32), ("ctx", P), ("pc", P), ("stall", P), ("count", P),
                ("scope", P), ("ctx_offsets", P)]


class _CallGraph(C.Structure):
    _fields_ = [("n_funcs", U32), ("n_sites", U64), ("site_pc", P), ("site_caller", P), ("site_callee", P)]


class _ContextTable(C.Structure):
    _fields_ = [("n", U32), ("parent", P), ("kernel_entry", P)]


class _ApportionOpts(C.Structure):
    _fields_ = [("sample_based", I), ("max_cct_nodes", U64), ("required_nodes", P)]


class _CctView(C.Structure):
    _fields_ = [("n_nodes", U64), ("n_ctx", U32), ("n_funcs", U32), ("scc", P), ("node_offsets", P),
                ("parent", P), ("node", P), ("site", P), ("kind", P), ("phi", P), ("excl", P),
                ("n_weights", U64), ("w_offsets", P), ("w_site", P), ("w_val", P)]


class _MetricsView(C.Structure):
    _fields_ = [("n_nodes", U64), ("n_ctx", U32), ("incl", P), ("S", P), ("W", P), ("host_incl", P),
                ("host_W", P), ("n_scope_rows", U64), ("sc_offsets", P), ("sc_scope", P), ("sc_val", P)]


class _LearnedOpts(C.Structure):
    _fields_ = [("n_leaves", U32), ("train_steps", U32), ("batch", U32), ("train_rows", U32), ("lr", C.c_float),
                ("window_cap", U32), ("seed", U64)]


class _LearnedStats(C.Structure):
    _fields_ = [("n_leaves", U32), ("train_steps", U32), ("train_mse", C.c_double), ("mean_window", C.c_double),
                ("max_window", U32), ("uncovered", U64), ("params", P)]


LEARNED_NPARAM = 4417


class _ServerOpts(C.Structure):
    _fields_ = [("n_profiles", U32), ("n_ctx", U32), ("table_slots", U64), ("pc_slots", U64),
                ("max_batch_bytes", U64), ("n_slots", U32), ("max_batch_buffers", U32), ("hbm_budget", U64)]


class _ServerStats(C.Structure):
    _fields_ = [("buffers", U64), ("samples", U64), ("bytes", U64), ("batches", U64), ("errors", U64),
                ("max_inflight_bytes", U64), ("p50_us", C.c_double), ("p99_us", C.c_double),
                ("max_us", C.c_double), ("mean_us", C.c_double), ("span_s", C.c_double)]


class _UnifiedView(C.Structure):
    _fields_ = [("n_profiles", U32), ("n_contexts", U64), ("n_nonzeros", U64), ("n_metric_entries", U64),
                ("n_profile_contexts", U64)] + [(n, P) for n in (
                    "ctx", "pc", "scope", "cms_ctx_off", "cms_m_off", "cms_mid", "cms_mstart", "cms_mctx", "cms_pid",
                    "cms_val", "pms_off", "pms_c_off", "pms_ctx", "pms_cstart", "pms_mid", "pms_val", "st_sum",
                    "st_min", "st_max", "st_mean", "st_std", "st_cov")]


SPARSE_CMS, SPARSE_PMS = 0, 1


class _ProfileDesc(C.Structure):
    _fields_ = [("map", P), ("n_samples", U64), ("n_ctx", U32)]


class _BatchOpts(C.Structure):
    _fields_ = [("max_round_samples", U64), ("autotune", I), ("merge_rounds", U32), ("scan_wg_per_cu", U32)]


class _BatchInfo(C.Structure):
    _fields_ = [("n_rounds", U32), ("merge_rounds", U32), ("scan_wg_per_cu", U32), ("autotuned", U32),
                ("total_keys", U64), ("tune_ms", C.c_double)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", P)]


class _StageTime(C.Structure):
    _fields_ = [("name", C.c_char_p), ("ms", C.c_double), ("calls", U64), ("items_in", U64), ("items_out", U64)]


_lib = None


def lib():
    """Load libhpa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libhpa.so is not built at {LIB_PATH}; run paper_2109_06931_amd/build.py")
        L = C.CDLL(LIB_PATH)
        PP = C.POINTER(C.c_void_p)
        L.hpa_last_error.restype = C.c_char_p
        L.hpa_ctx_create.argtypes = [I, P, PP]
        L.hpa_ctx_destroy.argtypes = [P]
        L.hpa_ctx_destroy.restype = None
        L.hpa_ctx_set_timing.argtypes = [P, I]
        L.hpa_ctx_get_sync_count.argtypes = [P, C.POINTER(U64)]
        L.hpa_ctx_get_timing.argtypes = [P, C.POINTER(_StageTime), U32, C.POINTER(U32)]
        L.hpa_build_structure_map.argtypes = [P, C.POINTER(_StructureDesc), P, PP]
        L.hpa_structure_map_view_get.argtypes = [P, C.POINTER(_MapView)]
        L.hpa_structure_map_free.argtypes = [P]
        L.hpa_structure_map_free.restype = None
        L.hpa_lookup_intervals.argtypes = [P, P, P, U64, P, I, P]
        L.hpa_attribute.argtypes = [P, P, C.POINTER(_Samples), P, PP]
        L.hpa_learned_train.argtypes = [P, P, C.POINTER(_LearnedOpts), P]
        L.hpa_attribute_noalloc.argtypes = [P, P, C.POINTER(_Samples), P, P, P, P, P, P, C.POINTER(U64),
                                            C.POINTER(U64), P]
        L.hpa_attribute_batched.argtypes = [P, U32, P, C.POINTER(_Samples), C.POINTER(_BatchOpts), P, PP]
        L.hpa_batch_profile_view.argtypes = [P, U32, C.POINTER(_AttrView)]
        L.hpa_batch_info_get.argtypes = [P, C.POINTER(_BatchInfo)]
        L.hpa_batch_free.argtypes = [P]
        L.hpa_batch_free.restype = None
        L.hpa_unify_profiles.argtypes = [P, U32, P, P, PP]
        L.hpa_unified_view_get.argtypes = [P, C.POINTER(_UnifiedView)]
        L.hpa_unified_free.argtypes = [P]
        L.hpa_unified_free.restype = None
        L.hpa_unified_write.argtypes = [P, C.c_char_p, I, U64, P]
        L.hpa_combine_runs.argtypes = [P, U32, P, P, PP]
        L.hpa_server_create.argtypes = [P, P, C.POINTER(_ServerOpts), PP]
        L.hpa_server_submit.argtypes = [P, U32, P, U64, C.POINTER(U64)]
        L.hpa_server_wait.argtypes = [P, U64, C.POINTER(C.c_double)]
        L.hpa_server_drain.argtypes = [P]
        L.hpa_server_stats_get.argtypes = [P, I, C.POINTER(_ServerStats)]
        L.hpa_server_snapshot.argtypes = [P, U32, P, PP]
        L.hpa_server_destroy.argtypes = [P]
        L.hpa_server_destroy.restype = None
        L.hpa_learned_stats_get.argtypes = [P, C.POINTER(_LearnedStats)]
        L.hpa_lookup_learned_counted.argtypes = [P, P, P, U64, P, P, P]
        L.hpa_learned_grad.argtypes = [P, P, P, P, U64, P, P]
        L.hpa_attribution_view_get.argtypes = [P, C.POINTER(_AttrView)]
        L.hpa_attribution_free.argtypes = [P]
        L.hpa_attribution_free.restype = None
        if hasattr(L, "hpa_prepare_callgraph"):
            L.hpa_prepare_callgraph.argtypes = [P, P, C.POINTER(_CallGraph), C.POINTER(_ContextTable), P, PP]
            L.hpa_callgraph_plan_free.argtypes = [P]
            L.hpa_callgraph_plan_free.restype = None
            L.hpa_apportion_callpaths.argtypes = [P, P, P, C.POINTER(_ApportionOpts), P, PP]
            L.hpa_gpu_cct_view_get.argtypes = [P, C.POINTER(_CctView)]
            L.hpa_gpu_cct_free.argtypes = [P]
            L.hpa_gpu_cct_free.restype = None
            L.hpa_derive_metrics.argtypes = [P, P, P, P, P, PP]
            L.hpa_metrics_view_get.argtypes = [P, C.POINTER(_MetricsView)]
            L.hpa_metrics_free.argtypes = [P]
            L.hpa_metrics_free.restype = None
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != OK:
        raise HpaError(rc, what, lib().hpa_last_error().decode(errors="replace"))


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream if hasattr(s, "cuda_stream") else int(s)


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------------------
# device views -> torch tensors
# ---------------------------------------------------------------------------
_TYPESTR = {np.dtype(np.uint8): "|u1", np.dtype(np.uint32): "<u4", np.dtype(np.int32): "<i4",
            np.dtype(np.uint64): "<u8", np.dtype(np.float64): "<f8", np.dtype(np.float32): "<f4"}
_hip = None


def _hip_memcpy_d2d(dst: int, src: int, nbytes: int):
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [P, P, C.c_size_t, I]
    rc = _hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), nbytes, 3)  # device to device
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")


class _DevArray:
    def __init__(self, ptr, shape, dtype):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": _TYPESTR[np.dtype(dtype)],
                                         "data": (int(ptr or 0), False), "version": 3, "strides": None}


def device_view(ptr, shape, dtype, owner=None):
    """A torch tensor over library-owned device memory (copied if torch cannot alias it)."""
    import torch
    shape = tuple(int(x) for x in shape)
    n = int(np.prod(shape)) if shape else 1
    tdt = {np.dtype(np.uint8): torch.uint8, np.dtype(np.uint32): torch.uint32, np.dtype(np.int32): torch.int32,
           np.dtype(np.uint64): torch.uint64, np.dtype(np.float64): torch.float64,
           np.dtype(np.float32): torch.float32}[np.dtype(dtype)]
    if n == 0 or not ptr:
        return torch.empty(shape, dtype=tdt, device="cuda")
    try:
        t = torch.as_tensor(_DevArray(ptr, shape, dtype), device="cuda")
        if t.dtype != tdt:
            t = t.view(tdt)
        t._hpa_owner = owner  # keep the handle alive
        return t
    except Exception:
        t = torch.empty(shape, dtype=tdt, device="cuda")
        torch.cuda.synchronize()
        _hip_memcpy_d2d(t.data_ptr(), int(ptr), n * np.dtype(dtype).itemsize)
        return t


# ---------------------------------------------------------------------------
# API
# ---------------------------------------------------------------------------
class Context:
    """hpa_ctx on one device.

    Without `allocator` the library allocates from the device's stream-ordered
    pool.  An allocator is an object with `alloc(nbytes, stream) -> int` (a
    device address, 0 on failure) and `free(ptr, stream)`; the library calls
    them for every device buffer it needs (hpa_allocator)."""

    def __init__(self, device: int = 0, allocator=None):
        self.h = C.c_void_p()
        self._alloc = None
        if allocator is not None:
            def _a(nbytes, stream, user):
                return int(allocator.alloc(int(nbytes), stream)) or None

            def _f(ptr, stream, user):
                allocator.free(int(ptr), stream)

            # the callbacks must outlive the context
            self._alloc = _Allocator(_ALLOC_FN(_a), _FREE_FN(_f), None)
        _check(lib().hpa_ctx_create(device, C.byref(self._alloc) if self._alloc else None, C.byref(self.h)),
               "hpa_ctx_create")
        self.device = device

    def sync_count(self) -> int:
        """hpa_ctx_get_sync_count: host synchronisations the library has made on this context."""
        n = U64(0)
        _check(lib().hpa_ctx_get_sync_count(self.h, C.byref(n)), "hpa_ctx_get_sync_count")
        return n.value

    def set_timing(self, on: bool = True):
        """hpa_ctx_set_timing: per-stage device timing of later calls (clears the table)."""
        _check(lib().hpa_ctx_set_timing(self.h, int(bool(on))), "hpa_ctx_set_timing")

    def timing(self) -> dict:
        """hpa_ctx_get_timing: {stage name: dict(ms, calls, items_in, items_out)}."""
        n = U32(0)
        _check(lib().hpa_ctx_get_timing(self.h, None, 0, C.byref(n)), "hpa_ctx_get_timing")
        rows = (_StageTime * max(n.value, 1))()
        _check(lib().hpa_ctx_get_timing(self.h, rows, n.value, C.byref(n)), "hpa_ctx_get_timing")
        return {r.name.decode(): dict(ms=r.ms, calls=r.calls, items_in=r.items_in, items_out=r.items_out)
                for r in rows[:n.value]}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpa_ctx_destroy(self.h)
            self.h = None


class StructureMap:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h
        v = _MapView()
        _check(lib().hpa_structure_map_view_get(h, C.byref(v)), "hpa_structure_map_view_get")
        self.n_intervals, self.n_scope_ids = v.n_intervals, v.n_scope_ids
        self._v = v

    def tensors(self):
        v, m, k = self._v, self.n_intervals, self.n_scope_ids
        return dict(start=device_view(v.start, (m,), np.uint64, self), end=device_view(v.end, (m,), np.uint64, self),
                    scope=device_view(v.scope, (m,), np.uint32, self), file=device_view(v.file, (m,), np.uint32, self),
                    line=device_view(v.line, (m,), np.uint32, self), parent=device_view(v.parent, (k,), np.uint32, self),
                    kind=device_view(v.kind, (k,), np.uint8, self), func=device_view(v.func, (k,), np.uint32, self))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpa_structure_map_free(self.h)
            self.h = None


def build_structure_map(ctx: Context, scope_start=None, scope_end=None, scope_id=None, scope_kind=None,
                        line_start=None, line_end=None, line_file=None, line_line=None,
                        iv_start=None, iv_end=None, learned: bool = False, stream=None) -> StructureMap:
    """hpa_build_structure_map from host (numpy) arrays."""
    d = _StructureDesc()
    keep = []
    if iv_start is not None:
        s, e = _np(iv_start, np.uint64), _np(iv_end, np.uint64)
        keep += [s, e]
        d.iv_start, d.iv_end, d.n_iv = s.ctypes.data, e.ctypes.data, len(s)
    else:
        sc = np.empty(len(scope_start), SCOPE_DTYPE)
        sc["start"], sc["end"], sc["id"], sc["kind"] = scope_start, scope_end, scope_id, scope_kind
        keep.append(sc)
        d.scopes, d.n_scopes = sc.ctypes.data if len(sc) else None, len(sc)
        if line_start is not None and len(line_start):
            ln = np.empty(len(line_start), LINE_DTYPE)
            ln["start"], ln["end"], ln["file"], ln["line"] = line_start, line_end, line_file, line_line
            keep.append(ln)
            d.lines, d.n_lines = ln.ctypes.data, len(ln)
    d.learned = 1 if learned else 0
    h = C.c_void_p()
    _check(lib().hpa_build_structure_map(ctx.h, C.byref(d), C.c_void_p(_stream(stream)), C.byref(h)),
           "hpa_build_structure_map")
    return StructureMap(ctx, h)


def build_structure_map_workload(ctx: Context, w, **kw) -> StructureMap:
    return build_structure_map(ctx, w.scope_start, w.scope_end, w.scope_id, w.scope_kind, w.line_start, w.line_end,
                               w.line_file, w.line_line, **kw)


def _device_arrays(*specs):
    """Check that each (tensor, name, itemsize, n, optional) can be handed to the
    library as n contiguous integers of `itemsize` bytes in device memory.  Shapes
    and types are checked for every array before placement, and everything before
    any library call; a mismatch raises ValueError."""
    for t, name, itemsize, n, optional in specs:
        if t is None:
            if optional:
                continue
            raise ValueError(f"{name} is required")
        if not hasattr(t, "data_ptr") or not hasattr(t, "element_size"):
            raise ValueError(f"{name} must be a torch tensor, got {type(t).__name__}")
        if t.dtype.is_floating_point or t.dtype.is_complex or str(t.dtype) == "torch.bool":
            raise ValueError(f"{name} must hold integers, got {t.dtype}")
        if t.element_size() != itemsize:
            raise ValueError(f"{name} must have {itemsize}-byte elements, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if n is not None and t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    for t, name, _, _, _ in specs:
        if t is not None and not t.is_cuda:
            raise ValueError(f"{name} must be in GPU memory (a CUDA tensor)")


def lookup_intervals(ctx: Context, m: StructureMap, pc, out, mode: int = LOOKUP_PLAIN, stream=None):
    """hpa_lookup_intervals on CUDA tensors pc (uint64) -> out (uint32, same length)."""
    _device_arrays((pc, "pc", 8, None, False), (out, "out", 4, pc.numel() if hasattr(pc, "numel") else None, False))
    _check(lib().hpa_lookup_intervals(ctx.h, m.h, _ptr(pc), pc.numel(), _ptr(out), mode,
                                      C.c_void_p(_stream(stream))), "hpa_lookup_intervals")
    return out


def learned_train(ctx: Context, m: StructureMap, n_leaves: int = 0, train_steps: int = 2000, batch: int = 0,
                  train_rows: int = 0, lr: float = 0.0, window_cap: int = 0, seed: int = 0, stream=None):
    """hpa_learned_train: (re)train the map's learned index (train_steps=0 keeps the untrained root)."""
    o = _LearnedOpts(int(n_leaves), int(train_steps), int(batch), int(train_rows), float(lr), int(window_cap),
                     int(seed))
    _check(lib().hpa_learned_train(ctx.h, m.h, C.byref(o), C.c_void_p(_stream(stream))), "hpa_learned_train")
    return learned_stats(m)


def learned_stats(m: StructureMap) -> dict:
    """hpa_learned_stats_get as a dict; 'params' is a device tensor view of the root's parameters."""
    st = _LearnedStats()
    _check(lib().hpa_learned_stats_get(m.h, C.byref(st)), "hpa_learned_stats_get")
    return dict(n_leaves=st.n_leaves, train_steps=st.train_steps, train_mse=st.train_mse,
                mean_window=st.mean_window, max_window=st.max_window, uncovered=st.uncovered,
                params=device_view(st.params, (LEARNED_NPARAM,), np.float32, m))


def lookup_learned_counted(ctx: Context, m: StructureMap, pc, out, counts, stream=None):
    """hpa_lookup_learned_counted: learned lookup that adds (probes, fallbacks) into counts (2 x uint64)."""
    _device_arrays((pc, "pc", 8, None, False), (out, "out", 4, pc.numel(), False), (counts, "counts", 8, 2, False))
    _check(lib().hpa_lookup_learned_counted(ctx.h, m.h, _ptr(pc), pc.numel(), _ptr(out), _ptr(counts),
                                            C.c_void_p(_stream(stream))), "hpa_lookup_learned_counted")
    return out


def learned_grad(ctx: Context, params, x, t, stream=None):
    """hpa_learned_grad: gradient (and summed squared error) of the root's mean squared error."""
    import torch
    n = t.numel()
    for a, name, k in ((params, "params", LEARNED_NPARAM), (x, "x", 2 * n), (t, "t", n)):
        if a.dtype != torch.float32 or not a.is_contiguous() or a.numel() != k or not a.is_cuda:
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of {k} elements")
    g = torch.empty(LEARNED_NPARAM + 1, dtype=torch.float32, device=params.device)
    _check(lib().hpa_learned_grad(ctx.h, _ptr(params), _ptr(x), _ptr(t), n, _ptr(g), C.c_void_p(_stream(stream))),
           "hpa_learned_grad")
    return g


class Attribution:
    def __init__(self, ctx, m, h):
        self.ctx, self.map, self.h = ctx, m, h
        v = _AttrView()
        _check(lib().hpa_attribution_view_get(h, C.byref(v)), "hpa_attribution_view_get")
        self.n_keys, self.n_ctx, self._v = v.n_keys, v.n_ctx, v

    def tensors(self):
        v, u = self._v, self.n_keys
        return dict(ctx=device_view(v.ctx, (u,), np.uint32, self), pc=device_view(v.pc, (u,), np.uint64, self),
                    stall=device_view(v.stall, (u,), np.uint8, self),
                    count=device_view(v.count, (u,), np.uint64, self),
                    scope=device_view(v.scope, (u,), np.uint32, self),
                    ctx_offsets=device_view(v.ctx_offsets, (self.n_ctx + 1,), np.uint64, self))

    def numpy(self):
        return {k: t.cpu().numpy() for k, t in self.tensors().items()}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpa_attribution_free(self.h)
            self.h = None


def attribute(ctx: Context, m: StructureMap, pc, ctx_ids, stall, weight=None, n_ctx: int = None,
              stream=None) -> Attribution:
    """hpa_attribute on CUDA tensors (uint64 pc, uint32/int32 ctx, uint8 stall, optional uint32 weight),
    all of one length.  n_ctx defaults to max(ctx) + 1."""
    n = pc.numel() if hasattr(pc, "numel") else None
    _device_arrays((pc, "pc", 8, None, False), (ctx_ids, "ctx_ids", 4, n, False), (stall, "stall", 1, n, False),
                   (weight, "weight", 4, n, True))
    if n_ctx is None:
        import torch
        n_ctx = int(ctx_ids.view(torch.int32).max().item()) + 1 if n else 1
    if not 0 < int(n_ctx) < 2 ** 32:
        raise ValueError(f"n_ctx must be in [1, 2^32), got {n_ctx}")
    s = _Samples()
    s.pc, s.ctx, s.stall, s.weight = _ptr(pc), _ptr(ctx_ids), _ptr(stall), _ptr(weight)
    s.n, s.n_ctx = pc.numel(), int(n_ctx)
    h = C.c_void_p()
    _check(lib().hpa_attribute(ctx.h, m.h, C.byref(s), C.c_void_p(_stream(stream)), C.byref(h)), "hpa_attribute")
    return Attribution(ctx, m, h)


class CallgraphPlan:
    def __init__(self, ctx, m, h, n_ctx):
        self.ctx, self.map, self.h, self.n_ctx = ctx, m, h, n_ctx

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpa_callgraph_plan_free(self.h)
            self.h = None


def prepare_callgraph(ctx: Context, m: StructureMap, n_funcs, site_pc, site_caller, site_callee, ctx_parent,
                      ctx_entry, stream=None) -> CallgraphPlan:
    sp, sc, se = _np(site_pc, np.uint64), _np(site_caller, np.uint32), _np(site_callee, np.uint32)
    cp, ce = _np(ctx_parent, np.uint32), _np(ctx_entry, np.int32)
    g = _CallGraph(int(n_funcs), len(sp), sp.ctypes.data if len(sp) else None, sc.ctypes.data if len(sc) else None,
                   se.ctypes.data if len(se) else None)
    t = _ContextTable(len(cp), cp.ctypes.data, ce.ctypes.data)
    h = C.c_void_p()
    _check(lib().hpa_prepare_callgraph(ctx.h, m.h, C.byref(g), C.byref(t), C.c_void_p(_stream(stream)), C.byref(h)),
           "hpa_prepare_callgraph")
    return CallgraphPlan(ctx, m, h, len(cp))


def prepare_callgraph_workload(ctx: Context, m: StructureMap, w, **kw) -> CallgraphPlan:
    return prepare_callgraph(ctx, m, w.n_scope_ids, w.site_pc, w.site_caller, w.site_callee, w.ctx_parent,
                             w.ctx_entry, **kw)


class GpuCct:
    def __init__(self, ctx, plan, attr, h):
        self.ctx, self.plan, self.attr, self.h = ctx, plan, attr, h
        v = _CctView()
        _check(lib().hpa_gpu_cct_view_get(h, C.byref(v)), "hpa_gpu_cct_view_get")
        self._v = v
        self.n_nodes, self.n_ctx, self.n_funcs, self.n_weights = v.n_nodes, v.n_ctx, v.n_funcs, v.n_weights

    def tensors(self):
        v, n, c = self._v, self.n_nodes, self.n_ctx
        return dict(scc=device_view(v.scc, (self.n_funcs,), np.uint32, self),
                    node_offsets=device_view(v.node_offsets, (c + 1,), np.uint64, self),
                    parent=device_view(v.parent, (n,), np.uint32, self), node=device_view(v.node, (n,), np.uint32, self),
                    site=device_view(v.site, (n,), np.uint64, self), kind=device_view(v.kind, (n,), np.uint8, self),
                    phi=device_view(v.phi, (n,), np.float64, self),
                    excl=device_view(v.excl, (n, N_STALL), np.float64, self),
                    w_offsets=device_view(v.w_offsets, (c + 1,), np.uint64, self),
                    w_site=device_view(v.w_site, (self.n_weights,), np.uint64, self),
                    w_val=device_view(v.w_val, (self.n_weights,), np.uint64, self))

    def numpy(self):
        return {k: t.cpu().numpy() for k, t in self.tensors().items()}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpa_gpu_cct_free(self.h)
            self.h = None


def apportion_callpaths(ctx: Context, plan: CallgraphPlan, attr: Attribution, sample_based: int = 1,
                        max_cct_nodes: int = 0, stream=None) -> GpuCct:
    req = C.c_uint64(0)
    o = _ApportionOpts(int(sample_based), int(max_cct_nodes), C.cast(C.byref(req), C.c_void_p))
    h = C.c_void_p()
    rc = lib().hpa_apportion_callpaths(ctx.h, plan.h, attr.h, C.byref(o), C.c_void_p(_stream(stream)), C.byref(h))
    if rc != OK:
        err = HpaError(rc, "hpa_apportion_callpaths", lib().hpa_last_error().decode(errors="replace"))
        err.required = req.value
        raise err
    t = GpuCct(ctx, plan, attr, h)
    t.required = req.value
    return t


class Metrics:
    def __init__(self, ctx, cct, h):
        self.ctx, self.cct, self.h = ctx, cct, h
        v = _MetricsView()
        _check(lib().hpa_metrics_view_get(h, C.byref(v)), "hpa_metrics_view_get")
        self._v = v
        self.n_nodes, self.n_ctx, self.n_scope_rows = v.n_nodes, v.n_ctx, v.n_scope_rows

    def tensors(self):
        v, n, c, r = self._v, self.n_nodes, self.n_ctx, self.n_scope_rows
        return dict(incl=device_view(v.incl, (n, N_STALL), np.float64, self),
                    S=device_view(v.S, (n,), np.float64, self), W=device_view(v.W, (n,), np.float64, self),
                    host_incl=device_view(v.host_incl, (c, N_STALL), np.uint64, self),
                    host_W=device_view(v.host_W, (c,), np.float64, self),
                    sc_offsets=device_view(v.sc_offsets, (c + 1,), np.uint64, self),
                    sc_scope=device_view(v.sc_scope, (r,), np.uint32, self),
                    sc_val=device_view(v.sc_val, (r, N_STALL), np.uint64, self))

    def numpy(self):
        return {k: t.cpu().numpy() for k, t in self.tensors().items()}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpa_metrics_free(self.h)
            self.h = None


def derive_metrics(ctx: Context, plan: CallgraphPlan, attr: Attribution, cct: GpuCct, stream=None) -> Metrics:
    h = C.c_void_p()
    _check(lib().hpa_derive_metrics(ctx.h, plan.h, attr.h, cct.h, C.c_void_p(_stream(stream)), C.byref(h)),
           "hpa_derive_metrics")
    return Metrics(ctx, cct, h)


def samples_to_device(w, device="cuda"):
    """Copy a workload's sample arrays into CUDA tensors (uint64/uint32/uint8)."""
    import torch
    pc = torch.from_numpy(w.pc.view(np.int64)).to(device).view(torch.uint64)
    cx = torch.from_numpy(w.ctx.view(np.int32)).to(device).view(torch.uint32)
    st = torch.from_numpy(w.stall).to(device)
    wt = None if w.weight is None else torch.from_numpy(w.weight.view(np.int32)).to(device).view(torch.uint32)
    return pc, cx, st, wt


# ---------------------------------------------------------------------------
# serving ingest
# ---------------------------------------------------------------------------
def sample_buffer(pc, ctx_ids, stall, pinned: bool = True):
    """A host buffer in the layout hpa_server_submit reads: pc u64[n], ctx u32[n],
    stall u8[n] back to back (a uint8 torch tensor, pinned by default)."""
    import torch
    pc = np.ascontiguousarray(pc, np.uint64)
    cx = np.ascontiguousarray(ctx_ids, np.uint32)
    st = np.ascontiguousarray(stall, np.uint8)
    n = len(pc)
    if len(cx) != n or len(st) != n:
        raise ValueError("pc, ctx and stall must have the same length")
    t = torch.empty(13 * n + 8, dtype=torch.uint8, pin_memory=pinned)
    a = t.numpy()
    a[:8 * n] = pc.view(np.uint8)
    a[8 * n:12 * n] = cx.view(np.uint8)
    a[12 * n:13 * n] = st
    t.n_samples = n
    return t


class Server:
    """hpa_server: continuous ingest of sample buffers into per-profile device state."""

    def __init__(self, ctx: Context, m: StructureMap, n_profiles: int, n_ctx: int, table_slots: int = 0,
                 pc_slots: int = 0, max_batch_bytes: int = 0, n_slots: int = 0, max_batch_buffers: int = 0,
                 hbm_budget: int = 0):
        self.ctx, self.map = ctx, m
        o = _ServerOpts(int(n_profiles), int(n_ctx), int(table_slots), int(pc_slots), int(max_batch_bytes),
                        int(n_slots), int(max_batch_buffers), int(hbm_budget))
        self.h = C.c_void_p()
        _check(lib().hpa_server_create(ctx.h, m.h, C.byref(o), C.byref(self.h)), "hpa_server_create")
        self._held = {}

    def submit(self, profile: int, buf) -> int:
        """Queue a buffer made by sample_buffer(); it is kept alive until its ticket completes."""
        t = U64(0)
        _check(lib().hpa_server_submit(self.h, int(profile), C.c_void_p(buf.data_ptr()), int(buf.n_samples),
                                       C.byref(t)), "hpa_server_submit")
        self._held[t.value] = buf
        return t.value

    def wait(self, ticket: int) -> float:
        lat = C.c_double(0.0)
        try:
            _check(lib().hpa_server_wait(self.h, int(ticket), C.byref(lat)), "hpa_server_wait")
        finally:
            self._held.pop(ticket, None)
        return lat.value

    def drain(self):
        _check(lib().hpa_server_drain(self.h), "hpa_server_drain")
        self._held.clear()

    def stats(self, reset: bool = False) -> dict:
        st = _ServerStats()
        _check(lib().hpa_server_stats_get(self.h, int(bool(reset)), C.byref(st)), "hpa_server_stats_get")
        return {k: getattr(st, k) for k, _ in _ServerStats._fields_}

    def snapshot(self, profile: int, stream=None) -> Attribution:
        h = C.c_void_p()
        _check(lib().hpa_server_snapshot(self.h, int(profile), C.c_void_p(_stream(stream)), C.byref(h)),
               "hpa_server_snapshot")
        return Attribution(self.ctx, self.map, h)

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpa_server_destroy(self.h)
            self.h = None
            self._held.clear()

    def __del__(self):
        self.close()


# ---------------------------------------------------------------------------
# several profiles: unification, statistics, sparse layouts, combined runs
# ---------------------------------------------------------------------------
class Unified:
    """hpa_unified: unified contexts of several profiles, CMS/PMS layouts and statistics."""

    def __init__(self, ctx, profiles, h):
        self.ctx, self.profiles, self.h = ctx, profiles, h
        v = _UnifiedView()
        _check(lib().hpa_unified_view_get(h, C.byref(v)), "hpa_unified_view_get")
        self._v = v

    def tensors(self):
        v = self._v
        U, K, NM, NH, P_ = v.n_contexts, v.n_nonzeros, v.n_metric_entries, v.n_profile_contexts, v.n_profiles
        d = lambda p, n, dt: device_view(p, (n,), dt, self)  # noqa: E731
        return dict(ctx=d(v.ctx, U, np.uint32), pc=d(v.pc, U, np.uint64), scope=d(v.scope, U, np.uint32),
                    cms_ctx_off=d(v.cms_ctx_off, U + 1, np.uint64), cms_m_off=d(v.cms_m_off, U + 1, np.uint64),
                    cms_mid=d(v.cms_mid, NM, np.uint8), cms_mstart=d(v.cms_mstart, NM, np.uint64),
                    cms_mctx=d(v.cms_mctx, NM, np.uint32), cms_pid=d(v.cms_pid, K, np.uint32),
                    cms_val=d(v.cms_val, K, np.uint64), pms_off=d(v.pms_off, P_ + 1, np.uint64),
                    pms_c_off=d(v.pms_c_off, P_ + 1, np.uint64), pms_ctx=d(v.pms_ctx, NH, np.uint32),
                    pms_cstart=d(v.pms_cstart, NH, np.uint64), pms_mid=d(v.pms_mid, K, np.uint8),
                    pms_val=d(v.pms_val, K, np.uint64), st_sum=d(v.st_sum, NM, np.uint64),
                    st_min=d(v.st_min, NM, np.uint64), st_max=d(v.st_max, NM, np.uint64),
                    st_mean=d(v.st_mean, NM, np.float64), st_std=d(v.st_std, NM, np.float64),
                    st_cov=d(v.st_cov, NM, np.float64))

    def numpy(self):
        return {k: t.cpu().numpy() for k, t in self.tensors().items()}

    def write(self, path: str, fmt: int = SPARSE_CMS, round_bytes: int = 0, stream=None):
        _check(lib().hpa_unified_write(self.h, str(path).encode(), int(fmt), int(round_bytes),
                                       C.c_void_p(_stream(stream))), "hpa_unified_write")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpa_unified_free(self.h)
            self.h = None


def _handles(attrs):
    arr = (C.c_void_p * len(attrs))(*[a.h.value if hasattr(a.h, "value") else a.h for a in attrs])
    return arr


def unify_profiles(ctx: Context, profiles, stream=None) -> Unified:
    """hpa_unify_profiles over a list of Attribution objects."""
    h = C.c_void_p()
    arr = _handles(profiles)
    _check(lib().hpa_unify_profiles(ctx.h, len(profiles), C.cast(arr, C.c_void_p), C.c_void_p(_stream(stream)),
                                    C.byref(h)), "hpa_unify_profiles")
    return Unified(ctx, list(profiles), h)


def combine_runs(ctx: Context, runs, stream=None) -> Attribution:
    """hpa_combine_runs: per key, the sum of the runs' counts."""
    h = C.c_void_p()
    arr = _handles(runs)
    _check(lib().hpa_combine_runs(ctx.h, len(runs), C.cast(arr, C.c_void_p), C.c_void_p(_stream(stream)),
                                  C.byref(h)), "hpa_combine_runs")
    return Attribution(ctx, runs[0].map, h)


# ---------------------------------------------------------------------------
# batches of profiles
# ---------------------------------------------------------------------------
class _BatchProfile(Attribution):
    """One profile's result inside a batch (views into the batch's arrays)."""

    def __init__(self, batch, p):
        self.ctx, self.map, self.h, self._batch = batch.ctx, batch.maps[p], None, batch
        v = _AttrView()
        _check(lib().hpa_batch_profile_view(batch.h, p, C.byref(v)), "hpa_batch_profile_view")
        self.n_keys, self.n_ctx, self._v = v.n_keys, v.n_ctx, v

    def __del__(self):
        pass


class Batch:
    """hpa_batch: the results of hpa_attribute_batched, one view per profile."""

    def __init__(self, ctx, maps, h):
        self.ctx, self.maps, self.h = ctx, maps, h

    def profile(self, p: int) -> Attribution:
        return _BatchProfile(self, p)

    def info(self) -> dict:
        i = _BatchInfo()
        _check(lib().hpa_batch_info_get(self.h, C.byref(i)), "hpa_batch_info_get")
        return {k: getattr(i, k) for k, _ in _BatchInfo._fields_}

    def __len__(self):
        return len(self.maps)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpa_batch_free(self.h)
            self.h = None


def attribute_batched(ctx: Context, maps, n_samples, n_ctx, pc, ctx_ids, stall, weight=None,
                      max_round_samples: int = 0, autotune: bool = False, merge_rounds: int = 2,
                      scan_wg_per_cu: int = 0, stream=None) -> Batch:
    """hpa_attribute_batched: maps / n_samples / n_ctx per profile; pc, ctx_ids (local per profile), stall
    (and weight) are the profiles' records back to back as CUDA tensors."""
    n = pc.numel() if hasattr(pc, "numel") else None
    _device_arrays((pc, "pc", 8, None, False), (ctx_ids, "ctx_ids", 4, n, False), (stall, "stall", 1, n, False),
                   (weight, "weight", 4, n, True))
    P_ = len(maps)
    if len(n_samples) != P_ or len(n_ctx) != P_:
        raise ValueError("maps, n_samples and n_ctx must have one entry per profile")
    if int(sum(int(x) for x in n_samples)) != n:
        raise ValueError("the profiles' sample counts must add up to the records given")
    descs = (_ProfileDesc * P_)(*[_ProfileDesc(m.h, int(k), int(c)) for m, k, c in zip(maps, n_samples, n_ctx)])
    s = _Samples()
    s.pc, s.ctx, s.stall, s.weight = _ptr(pc), _ptr(ctx_ids), _ptr(stall), _ptr(weight)
    s.n, s.n_ctx = n, 1
    o = _BatchOpts(int(max_round_samples), int(bool(autotune)), int(merge_rounds), int(scan_wg_per_cu))
    h = C.c_void_p()
    _check(lib().hpa_attribute_batched(ctx.h, P_, C.cast(descs, C.c_void_p), C.byref(s), C.byref(o),
                                       C.c_void_p(_stream(stream)), C.byref(h)), "hpa_attribute_batched")
    return Batch(ctx, list(maps), h)


def attribute_noalloc(ctx: Context, m: StructureMap, pc, ctx_ids, stall, weight, n_ctx: int, out: dict,
                      stream=None):
    """hpa_attribute_noalloc into caller tensors out = dict(ctx, pc, stall, count, scope, ctx_offsets);
    returns (n_keys, scratch bytes used)."""
    n = pc.numel() if hasattr(pc, "numel") else None
    _device_arrays((pc, "pc", 8, None, False), (ctx_ids, "ctx_ids", 4, n, False), (stall, "stall", 1, n, False),
                   (weight, "weight", 4, n, True), (out["ctx"], "out ctx", 4, None, False),
                   (out["pc"], "out pc", 8, None, False), (out["stall"], "out stall", 1, None, False),
                   (out["count"], "out count", 8, None, False), (out["scope"], "out scope", 4, None, False),
                   (out["ctx_offsets"], "out ctx_offsets", 8, int(n_ctx) + 1, False))
    for k in ("ctx", "pc", "stall", "count", "scope"):
        if out[k].numel() < n:
            raise ValueError(f"out {k} has room for {out[k].numel()} keys, need {n}")
    s = _Samples()
    s.pc, s.ctx, s.stall, s.weight = _ptr(pc), _ptr(ctx_ids), _ptr(stall), _ptr(weight)
    s.n, s.n_ctx = n, int(n_ctx)
    nk, used = U64(0), U64(0)
    _check(lib().hpa_attribute_noalloc(ctx.h, m.h, C.byref(s), *[_ptr(out[k]) for k in
                                       ("ctx", "pc", "stall", "count", "scope", "ctx_offsets")],
                                       C.byref(nk), C.byref(used), C.c_void_p(_stream(stream))),
           "hpa_attribute_noalloc")
    return nk.value, used.value
