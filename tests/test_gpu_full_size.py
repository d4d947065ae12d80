"""Attribution at the full size of the medium workload (256M samples, 100k
contexts), in the launch configuration the benchmark times, compared element
by element with the oracle over the whole batch: all six output arrays
(ctx, pc, stall, count, scope of every key and the context CSR) must be equal.
Two sample orders are run: the generator's per-kernel-invocation segments (the
benchmark's input) and the same records shuffled, which leaves no runs of one
context and so takes the scatter path.  Properties that hold at any size
(every sample counted once, per-context totals, strict key order) are checked
on the device first, so a failure names the broken property."""
import numpy as np
import pytest

import oracle
from workloads import config2

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

FIELDS = [("ctx", np.uint32), ("pc", np.uint64), ("stall", np.uint8), ("count", np.uint64), ("scope", np.uint32)]


@pytest.fixture(scope="module", params=["segments", "shuffled"])
def full(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_06931_amd as hpa
    shuffled = request.param == "shuffled"
    print(f"\n[full-size] generating the medium workload (256M samples, {request.param})", flush=True)
    w = config2(threads=16, shuffled=shuffled)
    ctx = hpa.Context(0)
    m = hpa.build_structure_map_workload(ctx, w)
    pc, cx, st, wt = hpa.samples_to_device(w)
    print("[full-size] attributing on the GPU", flush=True)
    a = hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx)
    torch.cuda.synchronize()
    del pc, cx, st
    yield hpa, w, a
    del a, m, ctx
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_full_size_invariants(full):
    hpa, w, a = full
    t = a.tensors()
    N, C, U = w.n_samples, w.n_ctx, a.n_keys
    count = t["count"].view(torch.int64)
    assert int(count.sum().item()) == N, "every sample attributed exactly once"
    assert int(count.min().item()) >= 1
    off = t["ctx_offsets"].view(torch.int64)
    assert int(off[0].item()) == 0 and int(off[-1].item()) == U
    assert bool((off[1:] >= off[:-1]).all().item())
    # per-context totals equal the per-context sample histogram
    cs = torch.cat([torch.zeros(1, dtype=torch.int64, device="cuda"), torch.cumsum(count, 0)])
    per_ctx = (cs[off[1:]] - cs[off[:-1]]).cpu().numpy()
    assert np.array_equal(per_ctx, np.bincount(w.ctx, minlength=C).astype(np.int64))
    # keys strictly increasing in (ctx, pc, stall); ctx agrees with the CSR
    kc = t["ctx"].view(torch.int32).to(torch.int64)
    kp = t["pc"].view(torch.int64)
    ks = t["stall"].to(torch.int64)
    assert int(ks.max().item()) < 16
    same = kc[1:] == kc[:-1]
    assert bool((kc[1:] >= kc[:-1]).all().item())
    # pcs compare as unsigned: flip the sign bit
    kpu = kp ^ torch.tensor(-(2**63), dtype=torch.int64, device="cuda")
    up = (kpu[1:] > kpu[:-1]) | ((kp[1:] == kp[:-1]) & (ks[1:] > ks[:-1]))
    assert bool((~same | up).all().item()), "keys within a context are not strictly increasing"
    sizes = torch.bincount(kc, minlength=C)
    assert torch.equal(sizes, off[1:] - off[:-1])


@pytest.mark.timeout(900)
def test_full_size_equals_oracle_everywhere(full):
    hpa, w, a = full
    print(f"\n[full-size] oracle over all {w.n_samples} samples", flush=True)
    om = oracle.build_map_workload(w)
    oa = oracle.attribute(om, w.pc, w.ctx, w.stall, w.weight, w.n_ctx)
    print(f"[full-size] oracle: {len(oa.count)} keys; comparing", flush=True)
    t = a.tensors()
    assert a.n_keys == len(oa.count), f"{a.n_keys} keys, oracle {len(oa.count)}"
    got_off = t["ctx_offsets"].cpu().numpy().view(np.uint64)
    assert np.array_equal(got_off, oa.ctx_offsets), "context CSR differs"
    for f, dt in FIELDS:
        got = t[f].cpu().numpy().view(dt)
        exp = getattr(oa, f)
        if not np.array_equal(got, exp):
            bad = np.flatnonzero(got != exp)
            k = int(bad[0])
            c = int(np.searchsorted(oa.ctx_offsets, k, side="right") - 1)
            raise AssertionError(f"field {f}: {len(bad)} keys differ; first at key {k} (context {c}): "
                                 f"got {got[k]}, oracle {exp[k]}")
        del got
