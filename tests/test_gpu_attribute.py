"""GPU parity of the structure map, interval lookup and attribution (A1-A4)
against the CPU oracle, through the C ABI.  Integer results must match bit for bit."""
import numpy as np
import pytest

import oracle
from workloads import config1, small_config, tiny_random_case
from workloads import handmade
from workloads.gen import FUNC

from .parity import assert_attribution_equal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hpa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_06931_amd as hpa
    hpa.lib()
    return hpa


@pytest.fixture(scope="module")
def hctx(hpa):
    return hpa.Context(0)


def _run(hpa, hctx, w, weighted=None):
    m = hpa.build_structure_map_workload(hctx, w)
    om = oracle.build_map_workload(w)
    pc, cx, st, wt = hpa.samples_to_device(w)
    a = hpa.attribute(hctx, m, pc, cx, st, wt, w.n_ctx)
    torch.cuda.synchronize()
    oa = oracle.attribute(om, w.pc, w.ctx, w.stall, w.weight, w.n_ctx)
    return m, om, a, oa


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_structure_map_matches_oracle(hpa, hctx, seed):
    w = small_config(seed, n_samples=0) if seed else config1(n_samples=0)
    m = hpa.build_structure_map_workload(hctx, w)
    om = oracle.build_map_workload(w)
    t = {k: v.cpu().numpy() for k, v in m.tensors().items()}
    for f in ["start", "end", "scope", "file", "line", "parent", "kind", "func"]:
        assert np.array_equal(t[f], getattr(om, f)), f


def test_structure_map_errors(hpa, hctx):
    cases = [
        (dict(scope_start=[0, 16, 48], scope_end=[256, 96, 128], scope_id=[0, 1, 2], scope_kind=[0, 2, 2]),
         hpa.E_NOT_LAMINAR),
        (dict(scope_start=[0, 64, 32], scope_end=[256, 128, 96], scope_id=[0, 1, 2], scope_kind=[0, 0, 1]),
         hpa.E_NOT_LAMINAR),
        (dict(scope_start=[0, 32], scope_end=[256, 32], scope_id=[0, 1], scope_kind=[0, 2]), hpa.E_INVAL),
        (dict(scope_start=[0], scope_end=[256], scope_id=[0], scope_kind=[0], line_start=[0, 32],
              line_end=[64, 96], line_file=[1, 1], line_line=[1, 2]), hpa.E_OVERLAP),
        (dict(iv_start=[10, 5], iv_end=[12, 8]), hpa.E_UNSORTED),
        (dict(iv_start=[10, 11], iv_end=[12, 13]), hpa.E_OVERLAP),
    ]
    for kw, code in cases:
        kw = {k: np.array(v) for k, v in kw.items()}
        with pytest.raises(hpa.HpaError) as ei:
            hpa.build_structure_map(hctx, **kw)
        assert ei.value.code == code, kw


@pytest.mark.parametrize("seed", [0, 1])
def test_lookup_plain_matches_oracle(hpa, hctx, seed):
    w = small_config(10 + seed, n_samples=0, n_funcs=3000, n_inst=200_000)
    m = hpa.build_structure_map_workload(hctx, w)
    om = oracle.build_map_workload(w)
    r = np.random.default_rng(seed)
    lo, hi = int(w.scope_start.min()) - 4096, int(w.scope_end.max()) + 4096
    q = np.concatenate([r.integers(lo, hi, 200_000, dtype=np.uint64), om.start, om.end, om.start - np.uint64(1),
                        np.array([0, 2**64 - 1], np.uint64)])
    qt = torch.from_numpy(q.view(np.int64)).cuda().view(torch.uint64)
    out = torch.empty(len(q), dtype=torch.int32, device="cuda").view(torch.uint32)
    hpa.lookup_intervals(hctx, m, qt, out)
    assert np.array_equal(out.cpu().numpy(), oracle.lookup(om, q))


def test_lookup_prebuilt_intervals(hpa, hctx):
    s = np.array([10, 20, 40], np.uint64)
    e = np.array([15, 40, 41], np.uint64)
    m = hpa.build_structure_map(hctx, iv_start=s, iv_end=e)
    q = np.array([9, 10, 14, 15, 19, 20, 39, 40, 41, 1 << 40], np.uint64)
    qt = torch.from_numpy(q.view(np.int64)).cuda().view(torch.uint64)
    out = torch.empty(len(q), dtype=torch.int32, device="cuda").view(torch.uint32)
    hpa.lookup_intervals(hctx, m, qt, out)
    assert out.cpu().numpy().tolist() == [0xFFFFFFFF, 0, 0, 0xFFFFFFFF, 0xFFFFFFFF, 1, 1, 2, 0xFFFFFFFF, 0xFFFFFFFF]


@pytest.mark.parametrize("seed", list(range(6)))
def test_attribute_tiny(hpa, hctx, seed):
    w = tiny_random_case(seed, n_samples=2000 + 700 * seed, n_ctx=3 + seed, weighted=seed % 2 == 1)
    m, om, a, oa = _run(hpa, hctx, w)
    assert_attribution_equal(a.numpy(), oa, f"tiny{seed}")


@pytest.mark.parametrize("seed,kw", [
    (1, {}),
    (2, dict(weighted=True)),
    (3, dict(shuffled=True)),
    (4, dict(seg_mean=20000.0)),
    (5, dict(seg_mean=30.0)),
    # runs of about 10 samples: still the run path, but a unit spans more runs
    # than its workgroup copies to LDS, so it walks the global run list
    (6, dict(seg_mean=10.0)),
    (7, dict(seg_mean=10.0, weighted=True)),
])
def test_attribute_small(hpa, hctx, seed, kw):
    w = small_config(seed, n_samples=300_000, **kw)
    m, om, a, oa = _run(hpa, hctx, w)
    assert_attribution_equal(a.numpy(), oa, f"small{seed}{kw}")


@pytest.mark.parametrize("weighted", [False, True])
def test_attribute_last_unit_counted(hpa, hctx, weighted):
    # the last context is big and all its samples sit on one pc: its only
    # part is a counted one, and it is the last unit, which closes the
    # context offsets and reports the key count
    w = tiny_random_case(7, n_funcs=5, n_samples=30_000, n_ctx=2, weighted=weighted)
    w.ctx[:] = 1
    w.ctx[:50] = 0
    w.pc[50:] = np.max(w.pc[w.ctx == 1])
    m, om, a, oa = _run(hpa, hctx, w)
    assert a.n_keys == len(oa.ctx) > 0
    assert_attribution_equal(a.numpy(), oa, "last unit counted")


@pytest.mark.parametrize("seed,n_bins,weighted", [
    # one address window per binary: a unit whose keys fall in up to four
    # windows finds a key's window among registers, more windows take the
    # search over the window table; few contexts, so units span all windows
    (12, 3, False),
    (13, 7, False),
    (14, 7, True),
    (15, 12, False),
])
def test_attribute_many_windows(hpa, hctx, seed, n_bins, weighted):
    w = small_config(seed, n_samples=250_000, n_ctx=40, n_bins=n_bins, weighted=weighted)
    m, om, a, oa = _run(hpa, hctx, w)
    assert_attribution_equal(a.numpy(), oa, f"windows{n_bins}")


@pytest.mark.parametrize("seed,kw,fallback", [
    # contexts of ~37k samples: most are cut into parts by coordinate range,
    # a few keep the chunk path (one coordinate bucket over 16,384 samples)
    (8, dict(n_ctx=8), True),
    (9, dict(n_ctx=12, weighted=True), None),
    (11, dict(n_ctx=20, seg_mean=300.0), None),
    # every context too concentrated to split: the chunk path only
    (10, dict(n_ctx=6, n_samples=600_000), True),
])
def test_attribute_split_big_contexts(hpa, hctx, seed, kw, fallback):
    """Contexts over 16,384 samples, on both pipelines.  The dense pipeline
    cuts them into coordinate-bucket parts (a bucket over 16,384 samples is
    counted).  A few far pcs in one small context send the same call to the
    general pipeline, whose split and chunk paths the stage timer shows."""
    kw = dict(kw)
    w = small_config(seed, n_samples=kw.pop("n_samples", 300_000), **kw)
    for far in (False, True):
        if far:
            hist = np.bincount(w.ctx, minlength=w.n_ctx)
            smallest = int(np.argmin(np.where(hist > 0, hist, np.iinfo(np.int64).max)))
            idx = np.flatnonzero(w.ctx == smallest)[:3]
            w.pc[idx] += np.uint64(1 << 50)
        hctx.set_timing(True)
        try:
            m, om, a, oa = _run(hpa, hctx, w)
            stages = hctx.timing()
        finally:
            hctx.set_timing(False)
        assert_attribution_equal(a.numpy(), oa, f"split{seed}{kw} far={far}")
        if not far:
            assert stages.get("d_split", {}).get("items_out", 0) > 0, "no big context on the dense pipeline"
            continue
        assert "d_split" not in stages, "the dense pipeline finished despite far pcs"
        split_in = stages.get("split_plan", {}).get("items_in", 0)
        if seed == 10:
            assert split_in == 0
        else:
            assert split_in > 0, "no context was split"
        if fallback:
            assert stages.get("big_sort", {}).get("items_in", 0) > 0, "no context kept the chunk path"


def test_attribute_config1(hpa, hctx):
    w = config1()
    m, om, a, oa = _run(hpa, hctx, w)
    assert_attribution_equal(a.numpy(), oa, "config1")


def test_attribute_one_giant_context(hpa, hctx):
    # every sample under one placeholder: the chunk-sort and merge path only
    w = small_config(21, n_samples=200_000, n_ctx=3, seg_mean=5000)
    w.ctx[:] = 1
    m, om, a, oa = _run(hpa, hctx, w)
    assert_attribution_equal(a.numpy(), oa, "giant")


def test_attribute_edge_cases(hpa, hctx):
    w = tiny_random_case(7, n_samples=5000, n_ctx=5)
    # all samples at unmapped PCs
    w.pc[:] = np.uint64(0x10)
    m, om, a, oa = _run(hpa, hctx, w)
    assert_attribution_equal(a.numpy(), oa, "unmapped")
    # a single key
    w.pc[:] = w.scope_start[0]
    w.ctx[:] = 2
    w.stall[:] = 9
    m, om, a, oa = _run(hpa, hctx, w)
    assert_attribution_equal(a.numpy(), oa, "single key")
    assert a.n_keys == 1
    # many empty contexts around a few busy ones
    w2 = tiny_random_case(8, n_samples=3000, n_ctx=4)
    w2.ctx_parent = np.full(70_000, 0xFFFFFFFF, np.uint32)
    w2.ctx_entry = np.full(70_000, -1, np.int32)
    w2.ctx = (w2.ctx.astype(np.int64) * 17_000 + 3).astype(np.uint32)
    m, om, a, oa = _run(hpa, hctx, w2)
    assert_attribution_equal(a.numpy(), oa, "sparse contexts")


def test_attribute_empty(hpa, hctx):
    w = tiny_random_case(9, n_samples=10, n_ctx=3)
    m = hpa.build_structure_map_workload(hctx, w)
    e64 = torch.empty(0, dtype=torch.int64, device="cuda").view(torch.uint64)
    e32 = torch.empty(0, dtype=torch.int32, device="cuda").view(torch.uint32)
    e8 = torch.empty(0, dtype=torch.uint8, device="cuda")
    a = hpa.attribute(hctx, m, e64, e32, e8, None, 3)
    assert a.n_keys == 0
    assert a.numpy()["ctx_offsets"].tolist() == [0, 0, 0, 0]


def test_attribute_rejects_bad_records(hpa, hctx):
    w = tiny_random_case(10, n_samples=1000, n_ctx=3)
    m = hpa.build_structure_map_workload(hctx, w)
    pc, cx, st, wt = hpa.samples_to_device(w)
    st2 = st.clone()
    st2[500] = 16
    with pytest.raises(hpa.HpaError) as ei:
        hpa.attribute(hctx, m, pc, cx, st2, None, 3)
    assert ei.value.code == hpa.E_INVAL
    cx2 = cx.clone()
    cx2[10] = 3
    with pytest.raises(hpa.HpaError) as ei:
        hpa.attribute(hctx, m, pc, cx2, st, None, 3)
    assert ei.value.code == hpa.E_INVAL


def test_attribute_deterministic(hpa, hctx):
    w = small_config(31, n_samples=200_000, shuffled=True)
    m = hpa.build_structure_map_workload(hctx, w)
    pc, cx, st, wt = hpa.samples_to_device(w)
    r1 = hpa.attribute(hctx, m, pc, cx, st, None, w.n_ctx).numpy()
    r2 = hpa.attribute(hctx, m, pc, cx, st, None, w.n_ctx).numpy()
    for k in r1:
        assert np.array_equal(r1[k], r2[k]), k


@pytest.mark.parametrize("weighted", [False, True])
def test_attribute_far_and_offgrid_pcs(hpa, hctx, weighted):
    """PCs far outside the code (keys wider than 32 bits: the unit pass reruns
    with the general kernel) and PCs off the instruction grid (raw-pc keys)."""
    w = tiny_random_case(11, n_samples=20_000, n_ctx=6, weighted=weighted)
    w.pc[::7] += np.uint64(1 << 50)
    m, om, a, oa = _run(hpa, hctx, w)
    assert_attribution_equal(a.numpy(), oa, "far")
    w = tiny_random_case(12, n_samples=20_000, n_ctx=6, weighted=weighted)
    w.pc[::5] += np.uint64(3)
    m, om, a, oa = _run(hpa, hctx, w)
    assert_attribution_equal(a.numpy(), oa, "off-grid")


def test_attribute_giant_context_far_pcs(hpa, hctx):
    # one context over many chunks, some chunks with far PCs (general chunk kernel)
    w = small_config(22, n_samples=120_000, n_ctx=3, seg_mean=5000)
    w.ctx[:] = 2
    w.pc[50_000:50_100] += np.uint64(1 << 52)
    m, om, a, oa = _run(hpa, hctx, w)
    assert_attribution_equal(a.numpy(), oa, "giant far")


def test_attribute_map_without_dense_coordinates(hpa, hctx):
    """Functions scattered far apart: the map has no dense coordinates, so
    every key is labelled by the separate binary-search pass."""
    r = np.random.default_rng(5)
    n_f = 200
    starts = (np.arange(n_f, dtype=np.uint64) << np.uint64(36)) + np.uint64(0x1000)
    w = tiny_random_case(13, n_samples=10, n_ctx=4)
    w.scope_start = starts
    w.scope_end = starts + np.uint64(256)
    w.scope_id = np.arange(n_f, dtype=np.uint32)
    w.scope_kind = np.zeros(n_f, dtype=np.uint32)
    w.line_start = w.line_end = w.line_file = w.line_line = None
    w.n_scope_ids = n_f
    n = 50_000
    f = r.integers(0, n_f, n).astype(np.uint64)
    w.pc = starts[f] + (r.integers(0, 16, n).astype(np.uint64) << np.uint64(4))
    w.pc[::97] = np.uint64(5)
    w.ctx = np.repeat(r.integers(0, 4, n // 500), 500).astype(np.uint32)
    w.stall = r.integers(0, 16, n).astype(np.uint8)
    w.weight = None
    m, om, a, oa = _run(hpa, hctx, w)
    assert_attribution_equal(a.numpy(), oa, "no dense map")


def test_attribute_reuses_cached_blocks(hpa):
    # one context, calls of different sizes in a row: the library reuses the
    # blocks of earlier calls, which still hold their data, so any buffer read
    # before it is written would show up here as a wrong result
    ctx = hpa.Context(0)
    big = small_config(8, n_samples=300_000, n_ctx=8)
    small = small_config(2, n_samples=60_000)
    for name, w in [("big", big), ("small", small), ("big again", big), ("small again", small)]:
        m, om, a, oa = _run(hpa, ctx, w)
        assert_attribution_equal(a.numpy(), oa, f"cached blocks: {name}")
        del a, m


class _TorchAllocator:
    """Caller allocator for hpa_ctx_create: device blocks from torch, counted."""

    def __init__(self, refuse=False):
        self.live = {}
        self.n_alloc = self.n_free = 0
        self.refuse = refuse

    def alloc(self, nbytes, stream):
        if self.refuse:
            return 0
        t = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
        self.live[t.data_ptr()] = t
        self.n_alloc += 1
        return t.data_ptr()

    def free(self, ptr, stream):
        assert ptr in self.live, "the library freed a block it did not get from this allocator"
        del self.live[ptr]
        self.n_free += 1


def test_attribute_with_caller_allocator(hpa):
    """Every device buffer of the call comes from the caller's allocator and goes
    back to it when the handles are freed; the result is the oracle's."""
    al = _TorchAllocator()
    c = hpa.Context(0, allocator=al)
    w = small_config(21, n_samples=150_000)
    m, om, a, oa = _run(hpa, c, w)
    assert_attribution_equal(a.numpy(), oa)
    assert al.n_alloc > 0 and al.live, "no buffer came from the caller's allocator"
    torch.cuda.synchronize()
    del a, m
    torch.cuda.synchronize()
    assert al.n_free == al.n_alloc and not al.live, (al.n_alloc, al.n_free)
    del c


def test_attribute_allocator_returning_null(hpa):
    """An allocator that returns NULL makes the call fail with HPA_E_NOMEM."""
    al = _TorchAllocator(refuse=True)
    c = hpa.Context(0, allocator=al)
    w = small_config(22, n_samples=20_000)
    with pytest.raises(hpa.HpaError) as ei:
        _run(hpa, c, w)
    assert ei.value.code == hpa.E_NOMEM
    del c


def test_attribute_synchronises_once(hpa, hctx):
    """With dense coordinates and every pc on them, hpa_attribute waits for the
    stream exactly once (to learn the key count); a pc off the coordinates
    makes the call redo the work on the general path, which waits more."""
    w = small_config(23, n_samples=200_000)
    m = hpa.build_structure_map_workload(hctx, w)
    pc, cx, st, wt = hpa.samples_to_device(w)
    torch.cuda.synchronize()
    n0 = hctx.sync_count()
    a = hpa.attribute(hctx, m, pc, cx, st, wt, w.n_ctx)
    assert hctx.sync_count() - n0 == 1
    om = oracle.build_map_workload(w)
    assert_attribution_equal(a.numpy(), oracle.attribute(om, w.pc, w.ctx, w.stall, w.weight, w.n_ctx), "dense")
    w.pc[::9] += np.uint64(1 << 50)
    pc, cx, st, wt = hpa.samples_to_device(w)
    torch.cuda.synchronize()
    n0 = hctx.sync_count()
    a = hpa.attribute(hctx, m, pc, cx, st, wt, w.n_ctx)
    assert hctx.sync_count() - n0 > 1
    assert_attribution_equal(a.numpy(), oracle.attribute(om, w.pc, w.ctx, w.stall, w.weight, w.n_ctx), "far")


def _wide_coordinates(seed, weighted):
    """400 functions 256 KiB apart (one window) on a 16-byte grid: about
    6.7M dense coordinates, more than 2^22."""
    r = np.random.default_rng(seed)
    n_f, n = 400, 300_000
    starts = np.uint64(0x5000_0000) + (np.arange(n_f, dtype=np.uint64) << np.uint64(18))
    w = tiny_random_case(seed, n_samples=10, n_ctx=4)
    w.scope_start, w.scope_end = starts, starts + np.uint64(272)
    w.scope_id = np.arange(n_f, dtype=np.uint32)
    w.scope_kind = np.zeros(n_f, dtype=np.uint32)
    w.line_start = w.line_end = w.line_file = w.line_line = None
    w.n_scope_ids = n_f
    f = np.minimum(r.zipf(1.3, n) - 1, n_f - 1).astype(np.uint64)
    w.pc = starts[f] + (r.integers(0, 17, n).astype(np.uint64) << np.uint64(4))
    n_ctx = 300
    w.ctx_parent = np.full(n_ctx, 0xFFFFFFFF, dtype=np.uint32)
    w.ctx_entry = np.full(n_ctx, -1, dtype=np.int32)
    w.ctx = np.repeat(r.integers(0, n_ctx, n // 500), 500).astype(np.uint32)
    w.stall = r.integers(0, 16, n).astype(np.uint8)
    w.weight = (1 + r.integers(0, 9, n)).astype(np.uint32) if weighted else None
    return w


@pytest.mark.parametrize("weighted", [False, True])
def test_attribute_wide_coordinates(hpa, hctx, weighted):
    """Over 2^22 dense coordinates (records hold 26 bits): the dense pipeline,
    with fewer local contexts per unit so that keys fit 31 bits."""
    print(f"case wide coordinates weighted={weighted}", flush=True)
    w = _wide_coordinates(40 + weighted, weighted)
    m = hpa.build_structure_map_workload(hctx, w)
    pc, cx, st, wt = hpa.samples_to_device(w)
    torch.cuda.synchronize()
    n0 = hctx.sync_count()
    a = hpa.attribute(hctx, m, pc, cx, st, wt, w.n_ctx)
    assert hctx.sync_count() - n0 == 1  # the dense pipeline
    om = oracle.build_map_workload(w)
    assert_attribution_equal(a.numpy(), oracle.attribute(om, w.pc, w.ctx, w.stall, w.weight, w.n_ctx), "wide")


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 63, 255, 256, 257, 1023, 1025, 4099])
def test_attribute_ragged_sizes(hpa, hctx, n):
    """Sample counts around the lane groups (4 samples) and wave steps (256
    samples) of the dense pipeline's histogram and scatter, from aligned
    arrays (vector loads) and from arrays one element into a larger buffer
    (scalar loads)."""
    print(f"case ragged n={n}", flush=True)
    w = tiny_random_case(50 + n % 7, n_samples=n, n_ctx=3, weighted=n % 2 == 1)
    m = hpa.build_structure_map_workload(hctx, w)
    om = oracle.build_map_workload(w)
    oa = oracle.attribute(om, w.pc, w.ctx, w.stall, w.weight, w.n_ctx)
    pc, cx, st, wt = hpa.samples_to_device(w)
    a = hpa.attribute(hctx, m, pc, cx, st, wt, w.n_ctx)
    assert_attribution_equal(a.numpy(), oa, f"ragged{n} aligned")

    def shifted(t):
        buf = torch.empty(t.numel() + 1, dtype=t.dtype, device=t.device)
        buf[1:] = t
        return buf[1:]

    p1 = shifted(pc.view(torch.int64)).view(torch.uint64)
    c1 = shifted(cx.view(torch.int32)).view(torch.uint32)
    w1 = None if wt is None else shifted(wt.view(torch.int32)).view(torch.uint32)
    a = hpa.attribute(hctx, m, p1, c1, shifted(st), w1, w.n_ctx)
    assert_attribution_equal(a.numpy(), oa, f"ragged{n} unaligned")
