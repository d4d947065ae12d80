"""The attribution entry point that allocates nothing, against hpa_attribute:
bit-exact outputs on two calls in a row (the second smaller, so the scratch
array still holds the first call's data), and the size limits."""
import numpy as np
import pytest

from workloads import small_config

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hpa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_06931_amd as hpa
    hpa.lib()
    return hpa


def _out(n, n_ctx):
    e = lambda dt, k: torch.empty(k, dtype=dt, device="cuda")  # noqa: E731
    return dict(ctx=e(torch.int32, n), pc=e(torch.int64, n), stall=e(torch.uint8, n), count=e(torch.int64, n),
                scope=e(torch.int32, n), ctx_offsets=e(torch.int64, n_ctx + 1))


def test_noalloc_matches_attribute_twice(hpa):
    ctx = hpa.Context(0)
    for i, (n, weighted, giant) in enumerate([(1_000_000, True, True), (120_000, False, False)]):
        w = small_config(40 + i, n_samples=n, n_ctx=500, weighted=weighted)
        if giant:  # most samples in one context: the chunk path's buffers too
            w.ctx[: n // 2] = 3
        print(f"case noalloc call {i}: n={n}", flush=True)
        m = hpa.build_structure_map_workload(ctx, w)
        pc, cx, st, wt = hpa.samples_to_device(w)
        ref = hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx).numpy()
        out = _out(n, w.n_ctx)
        nk, used = hpa.attribute_noalloc(ctx, m, pc, cx, st, wt, w.n_ctx, out)
        assert nk == len(ref["ctx"])
        got = {k: v.cpu().numpy() for k, v in out.items()}
        for f, dt in [("ctx", np.uint32), ("pc", np.uint64), ("stall", np.uint8), ("count", np.uint64),
                      ("scope", np.uint32)]:
            assert np.array_equal(got[f][:nk].view(dt), ref[f]), f"call {i}: {f}"
        assert np.array_equal(got["ctx_offsets"].view(np.uint64), ref["ctx_offsets"])
        assert 0 < used <= hpa.NOALLOC_SCRATCH_BYTES
        print(f"call {i}: {nk} keys, scratch {used} bytes", flush=True)


def test_noalloc_rejects_sizes(hpa):
    ctx = hpa.Context(0)
    w = small_config(45, n_samples=1000, n_ctx=10)
    m = hpa.build_structure_map_workload(ctx, w)
    n = (1 << 20) + 1
    pc = torch.zeros(n, dtype=torch.int64, device="cuda").view(torch.uint64)
    cx = torch.zeros(n, dtype=torch.int32, device="cuda").view(torch.uint32)
    st = torch.zeros(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(hpa.HpaError) as ei:
        hpa.attribute_noalloc(ctx, m, pc, cx, st, None, 10, _out(n, 10))
    assert ei.value.code == hpa.E_INVAL and "samples without allocation" in str(ei.value)
    with pytest.raises(hpa.HpaError) as ei:
        hpa.attribute_noalloc(ctx, m, pc[:10], cx[:10], st[:10], None, (1 << 16) + 1, _out(10, (1 << 16) + 1))
    assert ei.value.code == hpa.E_INVAL
