"""GPU tests of the learned interval index through the C ABI.

- Answers: the learned lookup must equal the plain binary search and the
  oracle's upper-bound search bit for bit (trained and untrained roots, maps
  built from scopes and from prebuilt intervals, edge addresses).
- Training kernels: the device gradient of the root's mean squared error is
  compared with the FP64 reference (itself pinned by central differences).
- Training helps: the trained root's windows and probes per lookup are
  smaller than the untrained root's.
"""
import numpy as np
import pytest

import oracle
from oracle import learned_ref
from workloads import config1, learned_intervals, learned_queries

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


def _dev_u64(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.uint64).view(np.int64)).cuda().view(torch.uint64)


def _lookup(hpa, hctx, m, q, mode):
    out = torch.empty(q.numel(), dtype=torch.uint32, device="cuda")
    hpa.lookup_intervals(hctx, m, q, out, mode=mode)
    return out


def _edge_queries(start, end):
    s, e = start.astype(np.uint64), end.astype(np.uint64)
    one = np.uint64(1)
    parts = [s, e, e - one, s[1:] - one, s[:1] - one, np.array([0, 2**64 - 1, int(e[-1]), int(s[-1])], np.uint64)]
    return np.concatenate(parts)


def _check_identity(hpa, hctx, m, qh, start, end, label):
    q = _dev_u64(qh)
    plain = _lookup(hpa, hctx, m, q, hpa.LOOKUP_PLAIN)
    counts = torch.zeros(2, dtype=torch.uint64, device="cuda")
    learned = torch.empty_like(plain)
    hpa.lookup_learned_counted(hctx, m, q, learned, counts)
    ref = oracle.lookup(oracle.map_from_intervals(start, end), qh)
    assert np.array_equal(plain.cpu().numpy(), ref), f"{label}: plain search differs from the oracle"
    got = learned.cpu().numpy()
    if not np.array_equal(got, ref):
        bad = np.nonzero(got != ref)[0]
        i = int(bad[0])
        raise AssertionError(f"{label}: learned lookup differs at {len(bad)} queries; first q={int(qh[i]):#x} "
                             f"got {got[i]} want {ref[i]}")
    c = counts.cpu().numpy().view(np.uint64)
    return int(c[0]), int(c[1])


@pytest.mark.parametrize("steps", [0, 400])
def test_learned_matches_plain_and_oracle(hpa, hctx, steps):
    start, end = learned_intervals(seed=11, n=300_000)
    m = hpa.build_structure_map(hctx, iv_start=start, iv_end=end)
    st = hpa.learned_train(hctx, m, train_steps=steps)
    assert st["n_leaves"] == 4096 and st["train_steps"] == steps
    q = np.concatenate([learned_queries(start, end, 2_000_003, seed=12), _edge_queries(start, end)])
    probes, fallbacks = _check_identity(hpa, hctx, m, q, start, end, f"steps={steps}")
    assert probes > 0 and fallbacks <= len(q)


def test_training_shrinks_windows_and_probes(hpa, hctx):
    start, end = learned_intervals(seed=13, n=400_000)
    q = learned_queries(start, end, 1_000_000, seed=14)
    res = {}
    for steps in (0, 1500):
        m = hpa.build_structure_map(hctx, iv_start=start, iv_end=end)
        st = hpa.learned_train(hctx, m, train_steps=steps, n_leaves=1024)
        probes, fallbacks = _check_identity(hpa, hctx, m, q, start, end, f"steps={steps}")
        res[steps] = (st["mean_window"], probes / len(q), fallbacks)
    assert res[1500][0] < res[0][0], res
    assert res[1500][1] < res[0][1], res


def test_learned_on_structure_map(hpa, hctx):
    # the learned index over a map built from scopes (every instruction address)
    w = config1(n_samples=0)
    m = hpa.build_structure_map_workload(hctx, w, learned=True)
    v = m.tensors()
    start, end = v["start"].cpu().numpy(), v["end"].cpu().numpy()
    lo, hi = int(start[0]) - 64, int(end[-1]) + 64
    q = np.arange(lo, hi, 4, dtype=np.uint64)
    _check_identity(hpa, hctx, m, q, start, end, "config1")


@pytest.mark.parametrize("n", [2, 3, 5, 17, 4097])
def test_learned_tiny_maps(hpa, hctx, n):
    start, end = learned_intervals(seed=20 + n, n=n)
    m = hpa.build_structure_map(hctx, iv_start=start, iv_end=end, learned=True)
    q = np.concatenate([_edge_queries(start, end), learned_queries(start, end, 5000, seed=n)])
    _check_identity(hpa, hctx, m, q, start, end, f"n={n}")


def test_learned_needs_two_intervals(hpa, hctx):
    m = hpa.build_structure_map(hctx, iv_start=np.array([16], np.uint64), iv_end=np.array([32], np.uint64))
    with pytest.raises(hpa.HpaError) as ei:
        hpa.learned_train(hctx, m)
    assert ei.value.code == hpa.E_UNSUPPORTED


@pytest.mark.parametrize("seed, n", [(1, 1000), (2, 128), (3, 1)])
def test_learned_gradient_matches_fp64(hpa, hctx, seed, n):
    r = np.random.default_rng(seed)
    p = r.normal(0.0, 0.3, size=learned_ref.NPARAM).astype(np.float32)
    X = r.random((n, 2)).astype(np.float32)
    T = r.random(n).astype(np.float32)
    g = hpa.learned_grad(hctx, torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(),
                         torch.from_numpy(T).cuda()).cpu().numpy().astype(np.float64)
    ref = learned_ref.grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    # FP32 arithmetic against FP64: error relative to each block's largest gradient
    scale = np.abs(ref).max()
    np.testing.assert_allclose(g[:-1], ref, rtol=2e-3, atol=2e-5 * scale)
    sse = float(np.sum((learned_ref.forward(p.astype(np.float64), X.astype(np.float64))[0] - T) ** 2))
    assert g[-1] == pytest.approx(sse, rel=1e-4)


@pytest.mark.slow
def test_learned_full_size(hpa, hctx):
    """5e7 intervals, 1e9 queries: learned == plain on every query, and the
    oracle agrees on 1e7 of them."""
    start, end = learned_intervals()
    print("case learned full size: intervals ready", flush=True)
    m = hpa.build_structure_map(hctx, iv_start=start, iv_end=end, learned=True)
    n_total = 1_000_000_000
    chunk = 100_000_000
    out_p = torch.empty(chunk, dtype=torch.uint32, device="cuda")
    out_l = torch.empty_like(out_p)
    for c in range(n_total // chunk):
        qh = learned_queries(start, end, chunk, seed=2109069314 + 1000 * (c + 1), threads=16)
        q = _dev_u64(qh)
        hpa.lookup_intervals(hctx, m, q, out_p, mode=hpa.LOOKUP_PLAIN)
        hpa.lookup_intervals(hctx, m, q, out_l, mode=hpa.LOOKUP_LEARNED)
        assert torch.equal(out_p, out_l), f"chunk {c}: learned differs from plain"
        if c == 0:
            ref = oracle.lookup(oracle.map_from_intervals(start, end), qh[:10_000_000])
            assert np.array_equal(out_l[:10_000_000].cpu().numpy(), ref)
        print(f"chunk {c} identical", flush=True)
