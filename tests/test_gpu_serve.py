"""GPU tests of the serving ingest through the C ABI.

Each profile's state, read back as an attribution, must equal the oracle's
attribution of exactly the buffers submitted to that profile (bit-exact), and
must be the same whether the profile's buffers arrive alone or interleaved
with other profiles' buffers, in any order.
"""
import numpy as np
import pytest

import oracle
from workloads import config1

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from .parity import assert_attribution_equal  # noqa: E402


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


@pytest.fixture(scope="module")
def w1():
    return config1(n_samples=1_500_000)


def _cut(w, seed, n_profiles, n_buffers):
    """Cut the workload's samples into buffers of log-uniform size and deal
    them to profiles; returns [(profile, lo, hi)]."""
    r = np.random.default_rng(seed)
    sizes = np.exp(r.uniform(np.log(300), np.log(60_000), size=n_buffers)).astype(np.int64)
    cuts, lo = [], 0
    for s in sizes:
        hi = min(w.n_samples, lo + int(s))
        if hi <= lo:
            break
        cuts.append((int(r.integers(0, n_profiles)), lo, hi))
        lo = hi
    return cuts


def _oracle_for(m, w, cuts, p):
    idx = np.concatenate([np.arange(lo, hi) for q, lo, hi in cuts if q == p] or [np.zeros(0, np.int64)])
    return oracle.attribute(m, w.pc[idx], w.ctx[idx], w.stall[idx], None, w.n_ctx)


def test_server_matches_oracle_alone_and_mixed(hpa, hctx, w1):
    w = w1
    m = hpa.build_structure_map_workload(hctx, w)
    om = oracle.build_map_workload(w)
    P = 6
    cuts = _cut(w, 1, P, 120)
    bufs = [hpa.sample_buffer(w.pc[lo:hi], w.ctx[lo:hi], w.stall[lo:hi]) for _, lo, hi in cuts]
    srv = hpa.Server(hctx, m, n_profiles=P, n_ctx=w.n_ctx, table_slots=1 << 18, n_slots=3,
                     max_batch_bytes=8 << 20)
    tickets = [srv.submit(p, b) for (p, _, _), b in zip(cuts, bufs)]
    lat = [srv.wait(t) for t in tickets]
    assert all(x > 0 for x in lat)
    st = srv.stats()
    assert st["buffers"] == len(cuts) and st["errors"] == 0 and st["p99_us"] >= st["p50_us"] > 0
    mixed = {}
    for p in range(P):
        got = srv.snapshot(p).numpy()
        assert_attribution_equal(got, _oracle_for(om, w, cuts, p), f"profile {p} mixed")
        mixed[p] = got
    srv.close()
    # alone: a fresh server receives only profile 2's buffers, in reverse order
    alone = hpa.Server(hctx, m, n_profiles=P, n_ctx=w.n_ctx, table_slots=1 << 18, n_slots=2,
                       max_batch_bytes=8 << 20)
    for (p, _, _), b in reversed(list(zip(cuts, bufs))):
        if p == 2:
            alone.submit(2, b)
    alone.drain()
    got = alone.snapshot(2).numpy()
    for f in ["ctx", "pc", "stall", "count", "scope", "ctx_offsets"]:
        assert np.array_equal(got[f], mixed[2][f]), f"alone vs mixed: {f}"
    # an untouched profile is empty
    empty = alone.snapshot(0).numpy()
    assert len(empty["ctx"]) == 0 and int(empty["ctx_offsets"][-1]) == 0
    alone.close()


def test_server_state_accumulates_across_snapshots(hpa, hctx, w1):
    w = w1
    m = hpa.build_structure_map_workload(hctx, w)
    om = oracle.build_map_workload(w)
    cuts = [(0, 0, 5000), (0, 5000, 90_000), (0, 90_000, 91_000)]
    srv = hpa.Server(hctx, m, n_profiles=1, n_ctx=w.n_ctx, table_slots=1 << 17)
    bufs = [hpa.sample_buffer(w.pc[lo:hi], w.ctx[lo:hi], w.stall[lo:hi]) for _, lo, hi in cuts]
    srv.wait(srv.submit(0, bufs[0]))
    assert_attribution_equal(srv.snapshot(0).numpy(), _oracle_for(om, w, cuts[:1], 0), "after one")
    for b in bufs[1:]:
        srv.submit(0, b)
    srv.drain()
    assert_attribution_equal(srv.snapshot(0).numpy(), _oracle_for(om, w, cuts, 0), "after three")
    srv.close()


def test_server_rejects_bad_input(hpa, hctx, w1):
    w = w1
    m = hpa.build_structure_map_workload(hctx, w)
    with pytest.raises(hpa.HpaError) as ei:
        hpa.Server(hctx, m, n_profiles=4, n_ctx=w.n_ctx, table_slots=1 << 20, hbm_budget=1 << 20)
    assert ei.value.code == hpa.E_BUDGET
    srv = hpa.Server(hctx, m, n_profiles=2, n_ctx=w.n_ctx, table_slots=1 << 12, max_batch_bytes=1 << 20)
    big = hpa.sample_buffer(w.pc[:100_000], w.ctx[:100_000], w.stall[:100_000])
    with pytest.raises(hpa.HpaError) as ei:
        srv.submit(0, big)
    assert ei.value.code == hpa.E_BUDGET
    with pytest.raises(hpa.HpaError) as ei:
        srv.submit(5, big)
    assert ei.value.code == hpa.E_INVAL
    bad = hpa.sample_buffer(w.pc[:100], np.full(100, w.n_ctx, np.uint32), w.stall[:100])
    t = srv.submit(1, bad)
    with pytest.raises(hpa.HpaError) as ei:
        srv.wait(t)
    assert ei.value.code == hpa.E_INVAL
    srv.close()
