"""Attribution at the full size of the medium workload (256M samples, 100k
contexts), in the launch configuration the benchmark times.  The oracle cannot
redo the whole batch in test time, so the check is: properties that hold at any
size over every key (every sample counted once, per-context totals, strict key
order, the context CSR), plus bit-exact equality with the oracle on sampled
contexts (the largest ones, which take the chunk-sort path, and random ones,
which take the unit path) and on sampled keys' scope labels."""
import numpy as np
import pytest

import oracle
from workloads import config2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_06931_amd as hpa
    print("[full-size] generating the medium workload (256M samples)", flush=True)
    w = config2(threads=16)
    ctx = hpa.Context(0)
    m = hpa.build_structure_map_workload(ctx, w)
    pc, cx, st, wt = hpa.samples_to_device(w)
    print("[full-size] attributing", flush=True)
    a = hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx)
    torch.cuda.synchronize()
    del pc, cx, st
    return hpa, w, a


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
    up = (kp[1:] > kp[:-1]) | ((kp[1:] == kp[:-1]) & (ks[1:] > ks[:-1]))
    assert bool((~same | up).all().item()), "keys within a context are not strictly increasing"
    sizes = torch.bincount(kc, minlength=C)
    assert torch.equal(sizes, off[1:] - off[:-1])


def test_full_size_sampled_contexts_match_oracle(full):
    hpa, w, a = full
    C = w.n_ctx
    hist = np.bincount(w.ctx, minlength=C)
    r = np.random.default_rng(2109)
    big = np.argsort(hist)[-4:]
    rnd = r.choice(np.flatnonzero(hist > 0), 60, replace=False)
    pick = np.unique(np.concatenate([big, rnd, [0, C - 1]]))
    mask = np.zeros(C, np.uint8)
    mask[pick] = 1
    om = oracle.build_map_workload(w)
    print(f"[full-size] oracle on {len(pick)} contexts", flush=True)
    oa = oracle.attribute(om, w.pc, w.ctx, w.stall, w.weight, C, ctx_mask=mask)
    t = a.tensors()
    off = t["ctx_offsets"].cpu().numpy().view(np.uint64)
    for c in pick:
        b, e = int(off[c]), int(off[c + 1])
        ob, oe = int(oa.ctx_offsets[c]), int(oa.ctx_offsets[c + 1])
        assert e - b == oe - ob, f"context {c}: {e - b} keys, oracle {oe - ob}"
        if e == b:
            continue
        for f, dt in [("ctx", np.uint32), ("pc", np.uint64), ("stall", np.uint8), ("count", np.uint64),
                      ("scope", np.uint32)]:
            got = t[f][b:e].cpu().numpy().view(dt)
            assert np.array_equal(got, getattr(oa, f)[ob:oe]), f"context {c}: field {f}"


def test_full_size_sampled_scope_labels(full):
    hpa, w, a = full
    t = a.tensors()
    U = a.n_keys
    idx = np.random.default_rng(7).integers(0, U, 200_000)
    it = torch.from_numpy(idx).cuda()
    pcs = t["pc"].view(torch.int64)[it].cpu().numpy().view(np.uint64)
    got = t["scope"].view(torch.int32)[it].cpu().numpy().view(np.uint32)
    om = oracle.build_map_workload(w)
    iv = oracle.lookup(om, pcs)
    exp = np.where(iv == 0xFFFFFFFF, np.uint32(0xFFFFFFFF), om.scope[np.minimum(iv, len(om.scope) - 1)])
    assert np.array_equal(got, exp.astype(np.uint32))
