"""GPU parity of batched attribution: every profile's result from one batched
call must equal hpa_attribute on that profile alone, byte for byte (and the
oracle, on a sample of profiles), across rounds, profiles of very different
sizes and maps, weighted records, and autotuned run-time parameters."""
import numpy as np
import pytest

import oracle
from workloads import small_config, tiny_random_case

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


def _no_dense_profile(seed):
    r = np.random.default_rng(seed)
    n_f = 120
    starts = (np.arange(n_f, dtype=np.uint64) << np.uint64(36)) + np.uint64(0x1000)
    w = tiny_random_case(13, n_samples=10, n_ctx=4)
    w.scope_start, w.scope_end = starts, starts + np.uint64(256)
    w.scope_id = np.arange(n_f, dtype=np.uint32)
    w.scope_kind = np.zeros(n_f, dtype=np.uint32)
    w.line_start = w.line_end = w.line_file = w.line_line = None
    w.n_scope_ids = n_f
    n = 30_000
    f = r.integers(0, n_f, n).astype(np.uint64)
    w.pc = starts[f] + (r.integers(0, 16, n).astype(np.uint64) << np.uint64(4))
    w.ctx = np.repeat(r.integers(0, 4, n // 300), 300).astype(np.uint32)
    w.stall = r.integers(0, 16, n).astype(np.uint8)
    w.weight = None
    return w


def _profiles(weighted):
    ws = []
    for i, n in enumerate([40_000, 3_000, 150_000, 10, 70_000, 0, 25_000]):
        if n == 0:
            w = small_config(200 + i, n_samples=0, n_ctx=50)
            w.pc = np.zeros(0, np.uint64); w.ctx = np.zeros(0, np.uint32); w.stall = np.zeros(0, np.uint8)
            w.weight = np.zeros(0, np.uint32) if weighted else None
        else:
            w = small_config(200 + i, n_samples=n, n_ctx=[300, 40, 5, 3, 900, 50, 60][i], weighted=weighted)
        ws.append(w)
    # a giant context (chunk path), and a profile whose map has no dense coordinates
    g = small_config(230, n_samples=60_000, n_ctx=3, seg_mean=5000, weighted=weighted)
    g.ctx[:] = 1
    g.pc[1000:1100] += np.uint64(1 << 50)
    ws.append(g)
    nd = _no_dense_profile(231)
    if weighted:
        nd.weight = (1 + np.arange(len(nd.pc)) % 7).astype(np.uint32)
    ws.append(nd)
    return ws


def _cat(ws, weighted):
    pc = np.concatenate([w.pc for w in ws]).astype(np.uint64)
    cx = np.concatenate([w.ctx for w in ws]).astype(np.uint32)
    st = np.concatenate([w.stall for w in ws]).astype(np.uint8)
    d = lambda a, t: torch.from_numpy(a.view(t)).cuda()  # noqa: E731
    wt = d(np.concatenate([w.weight for w in ws]).astype(np.uint32), np.int32).view(torch.uint32) if weighted \
        else None
    return d(pc, np.int64).view(torch.uint64), d(cx, np.int32).view(torch.uint32), torch.from_numpy(st).cuda(), wt


@pytest.mark.parametrize("weighted, round_cap, autotune", [(False, 0, False), (False, 120_000, True),
                                                           (True, 90_000, False)])
def test_batch_equals_single_calls(hpa, hctx, weighted, round_cap, autotune):
    print(f"case batch weighted={weighted} round_cap={round_cap} autotune={autotune}", flush=True)
    ws = _profiles(weighted)
    maps = [hpa.build_structure_map_workload(hctx, w) for w in ws]
    pc, cx, st, wt = _cat(ws, weighted)
    b = hpa.attribute_batched(hctx, maps, [len(w.pc) for w in ws], [w.n_ctx for w in ws], pc, cx, st, wt,
                              max_round_samples=round_cap, autotune=autotune)
    info = b.info()
    assert info["n_rounds"] >= (2 if round_cap else 1)
    for i, (w, m) in enumerate(zip(ws, maps)):
        got = b.profile(i).numpy()
        if len(w.pc):
            p2, c2, s2, w2 = hpa.samples_to_device(w)
            one = hpa.attribute(hctx, m, p2, c2, s2, w2, w.n_ctx).numpy()
        else:
            one = None
        if one is not None:
            for f in ["ctx", "pc", "stall", "count", "scope", "ctx_offsets"]:
                assert np.array_equal(got[f], one[f]), f"profile {i}: {f}"
        else:
            assert len(got["ctx"]) == 0 and not got["ctx_offsets"].any()
        if i in (0, 6, 7, 8):
            om = oracle.build_map_workload(w)
            oa = oracle.attribute(om, w.pc, w.ctx, w.stall, w.weight, w.n_ctx)
            assert_attribution_equal(got, oa, f"profile {i} vs oracle")


def test_batch_rejects_bad_counts(hpa, hctx):
    ws = _profiles(False)[:2]
    maps = [hpa.build_structure_map_workload(hctx, w) for w in ws]
    pc, cx, st, _ = _cat(ws, False)
    with pytest.raises(ValueError):
        hpa.attribute_batched(hctx, maps, [len(ws[0].pc), 5], [w.n_ctx for w in ws], pc, cx, st)
    # a record whose ctx is beyond its own profile's count (but below the other's)
    cx2 = cx.clone()
    cx2[0] = ws[1].n_ctx + ws[0].n_ctx
    with pytest.raises(hpa.HpaError) as ei:
        hpa.attribute_batched(hctx, maps, [len(w.pc) for w in ws], [w.n_ctx for w in ws], pc, cx2, st)
    assert ei.value.code == hpa.E_INVAL


def _shared_map_profiles(weighted):
    """Profiles drawn from three program structures, interleaved in the batch:
    slices of three sample streams (one whose map has no dense coordinates),
    one slice with pcs off the dense coordinates, one empty profile."""
    wa = small_config(300, n_samples=200_000, n_ctx=400, weighted=weighted)
    wb = small_config(301, n_samples=150_000, n_ctx=250, weighted=weighted)
    wc = _no_dense_profile(232)
    if weighted:
        wc.weight = (1 + np.arange(len(wc.pc)) % 5).astype(np.uint32)
    cuts = [(wa, 0, 50_000), (wb, 0, 40_000), (wc, 0, 12_000), (wa, 50_000, 120_000), (wb, 40_000, 41_000),
            (wa, 120_000, 200_000), (wc, 12_000, 30_000), (wb, 41_000, 150_000), (wa, 0, 0), (wb, 0, 5)]
    out = []
    for k, (w, a, b) in enumerate(cuts):
        prof = dict(w=w, pc=w.pc[a:b].copy(), ctx=w.ctx[a:b].copy(), stall=w.stall[a:b].copy(),
                    weight=None if w.weight is None else w.weight[a:b].copy())
        if k == 5:  # a pc off the dense coordinates: its batch round takes the general pipeline
            prof["pc"][100:140] += np.uint64(1 << 50)
        out.append(prof)
    return wa, wb, out


@pytest.mark.parametrize("weighted, round_cap, autotune", [(False, 0, False), (True, 0, False),
                                                           (False, 100_000, False), (True, 100_000, True)])
def test_batch_grouped_by_shared_maps(hpa, hctx, weighted, round_cap, autotune):
    print(f"case grouped weighted={weighted} round_cap={round_cap} autotune={autotune}", flush=True)
    wa, wb, profs = _shared_map_profiles(weighted)
    ma, mb = hpa.build_structure_map_workload(hctx, wa), hpa.build_structure_map_workload(hctx, wb)
    mc = hpa.build_structure_map_workload(hctx, profs[2]["w"])
    maps = [ma if p["w"] is wa else mb if p["w"] is wb else mc for p in profs]
    d = lambda a, t: torch.from_numpy(np.ascontiguousarray(a).view(t)).cuda()  # noqa: E731
    pc = d(np.concatenate([p["pc"] for p in profs]).astype(np.uint64), np.int64).view(torch.uint64)
    cx = d(np.concatenate([p["ctx"] for p in profs]).astype(np.uint32), np.int32).view(torch.uint32)
    st = torch.from_numpy(np.concatenate([p["stall"] for p in profs]).astype(np.uint8)).cuda()
    wt = d(np.concatenate([p["weight"] for p in profs]).astype(np.uint32), np.int32).view(torch.uint32) \
        if weighted else None
    b = hpa.attribute_batched(hctx, maps, [len(p["pc"]) for p in profs], [p["w"].n_ctx for p in profs], pc, cx,
                              st, wt, max_round_samples=round_cap, autotune=autotune)
    info = b.info()
    # one map per round: at least one round per map, more under the cap
    assert info["n_rounds"] >= (5 if round_cap else 3)
    for i, p in enumerate(profs):
        got = b.profile(i).numpy()
        w, n = p["w"], len(p["pc"])
        if n:
            dv = lambda a, t: torch.from_numpy(np.ascontiguousarray(a).view(t)).cuda()  # noqa: E731
            one = hpa.attribute(hctx, maps[i], dv(p["pc"], np.int64).view(torch.uint64),
                                dv(p["ctx"], np.int32).view(torch.uint32), torch.from_numpy(p["stall"]).cuda(),
                                None if p["weight"] is None else dv(p["weight"], np.int32).view(torch.uint32),
                                w.n_ctx).numpy()
            for f in ["ctx", "pc", "stall", "count", "scope", "ctx_offsets"]:
                assert np.array_equal(got[f], one[f]), f"profile {i}: {f}"
        else:
            assert len(got["ctx"]) == 0 and not got["ctx_offsets"].any()
        if i in (1, 2, 5, 9):
            om = oracle.build_map_workload(w)
            oa = oracle.attribute(om, p["pc"], p["ctx"], p["stall"], p["weight"], w.n_ctx)
            assert_attribution_equal(got, oa, f"profile {i} vs oracle")


def test_batch_grouped_rejects_bad_ctx(hpa, hctx):
    wa, wb, profs = _shared_map_profiles(False)
    ma, mb = hpa.build_structure_map_workload(hctx, wa), hpa.build_structure_map_workload(hctx, wb)
    mc = hpa.build_structure_map_workload(hctx, profs[2]["w"])
    maps = [ma if p["w"] is wa else mb if p["w"] is wb else mc for p in profs]
    cx_np = np.concatenate([p["ctx"] for p in profs]).astype(np.uint32)
    cx_np[len(profs[0]["ctx"]) + 3] = wb.n_ctx  # a record of profile 1 beyond its profile's count
    pc = torch.from_numpy(np.concatenate([p["pc"] for p in profs]).astype(np.uint64).view(np.int64)).cuda()
    st = torch.from_numpy(np.concatenate([p["stall"] for p in profs]).astype(np.uint8)).cuda()
    cx = torch.from_numpy(cx_np.view(np.int32)).cuda().view(torch.uint32)
    with pytest.raises(hpa.HpaError) as ei:
        hpa.attribute_batched(hctx, maps, [len(p["pc"]) for p in profs], [p["w"].n_ctx for p in profs],
                              pc.view(torch.uint64), cx, st)
    assert ei.value.code == hpa.E_INVAL
