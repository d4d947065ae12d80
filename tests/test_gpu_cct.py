"""GPU parity of the GPU calling context tree (A5) and derived metrics (A6)
against the CPU oracle through the C ABI.  Integer fields bit-exact; FP64
fields (phi, exclusive and inclusive costs, W) within 1e-9 relative."""
import json
import os

import numpy as np
import pytest

import oracle
from workloads import config1, small_config, tiny_random_case
from workloads import handmade

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
RTOL = 1e-9
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# The device path of A5/A6 is compiled out.  Its first version took a GPU
# memory fault on test_cct_tiny[0] (twice, the second time after a first fix);
# its rewrite, which matches the oracle when the kernel source runs on the CPU,
# stopped making progress on the device on the same case (no output for 180 s,
# no fault).  The cause is not found, so these cases stay off the device.
DISABLED = pytest.mark.skip(reason="GPU call-path apportioning is compiled out: its rewrite stopped making "
                                   "progress on the device on test_cct_tiny[0]; cause not found")



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


def _gpu_all(hpa, hctx, w, max_nodes=0, sample_based=1):
    m = hpa.build_structure_map_workload(hctx, w)
    pc, cx, st, wt = hpa.samples_to_device(w)
    a = hpa.attribute(hctx, m, pc, cx, st, wt, w.n_ctx)
    plan = hpa.prepare_callgraph_workload(hctx, m, w)
    t = hpa.apportion_callpaths(hctx, plan, a, sample_based=sample_based, max_cct_nodes=max_nodes)
    d = hpa.derive_metrics(hctx, plan, a, t)
    return m, a, plan, t, d


def _close(got, exp, what):
    got, exp = np.asarray(got), np.asarray(exp)
    assert got.shape == exp.shape, what
    np.testing.assert_allclose(got, exp, rtol=RTOL, atol=0, err_msg=what)


def check_against_oracle(hpa, hctx, w, label="", sample_based=1):
    print(f"case {label}", flush=True)
    m, a, plan, t, d = _gpu_all(hpa, hctx, w, sample_based=sample_based)
    om, oa, ot, od = oracle.run_all(w, sample_based=sample_based)
    tt, dd = t.numpy(), d.numpy()
    assert np.array_equal(tt["scc"], ot.scc), f"{label}: scc"
    assert np.array_equal(tt["node_offsets"], ot.node_off), f"{label}: node offsets"
    for f, of in [("parent", "parent"), ("node", "node"), ("site", "site"), ("kind", "kind")]:
        assert np.array_equal(tt[f], getattr(ot, of)), f"{label}: {f}"
    _close(tt["phi"], ot.phi, f"{label}: phi")
    _close(tt["excl"], ot.excl, f"{label}: excl")
    assert np.array_equal(tt["w_offsets"], ot.w_off), f"{label}: weight offsets"
    assert np.array_equal(tt["w_site"], ot.w_site) and np.array_equal(tt["w_val"], ot.w_val), f"{label}: weights"
    _close(dd["incl"], od.incl, f"{label}: incl")
    _close(dd["S"], od.S, f"{label}: S")
    _close(dd["W"], od.W, f"{label}: W")
    assert np.array_equal(dd["host_incl"], od.host_incl), f"{label}: host tree"
    _close(dd["host_W"], od.host_W, f"{label}: host W")
    assert np.array_equal(dd["sc_offsets"], od.sc_off), f"{label}: scope offsets"
    assert np.array_equal(dd["sc_scope"], od.sc_scope), f"{label}: scope ids"
    assert np.array_equal(dd["sc_val"], od.sc_val), f"{label}: scope values"
    # conservation: every context's exclusive costs add up to its samples
    # (sample-based weights only: exact counts may leave a function unreached)
    off = a.numpy()["ctx_offsets"]
    cnt = a.numpy()["count"]
    for c in range(w.n_ctx if sample_based else 0):
        b, e = int(tt["node_offsets"][c]), int(tt["node_offsets"][c + 1])
        n_c = int(cnt[off[c]:off[c + 1]].sum())
        assert abs(tt["excl"][b:e].sum() - n_c) <= 1e-9 * max(1, n_c)
    return t, d


@DISABLED
@pytest.mark.parametrize("seed", list(range(12)))
def test_cct_tiny(hpa, hctx, seed):
    w = tiny_random_case(seed, n_funcs=4 + seed % 5, n_samples=500 + 50 * seed, n_ctx=4 + seed % 3,
                         weighted=seed % 4 == 3)
    check_against_oracle(hpa, hctx, w, f"tiny{seed}")


@DISABLED
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cct_small(hpa, hctx, seed):
    w = small_config(seed, n_samples=200_000)
    check_against_oracle(hpa, hctx, w, f"small{seed}")


@DISABLED
def test_cct_config1(hpa, hctx):
    check_against_oracle(hpa, hctx, config1(), "config1")


@DISABLED
def test_cct_handmade_cases(hpa, hctx):
    g = json.load(open(os.path.join(GOLDEN, "fig4_shape.json")))
    names = g["functions"]
    fid = {n: i for i, n in enumerate(names)}
    sites = [(fid[s["caller"]], fid[s["callee"]], s["call_samples"]) for s in g["sites"]]
    self_rows = {fid[n]: [(0, c)] for n, c in g["self_noncall"].items() if c}
    t, d = check_against_oracle(hpa, hctx, handmade.build(len(names), sites, self_rows, entry=fid[g["entry"]]), "fig4")
    assert t.numpy()["phi"].tolist() == [r["phi"] for r in g["expected_preorder"]]
    cases = [
        handmade.build(3, [(0, 1, 0), (1, 2, 1), (2, 1, 1)], {1: [(0, 3)], 2: [(1, 2)], 0: [(0, 1)]}, entry=0),
        handmade.build(3, [(0, 1, 1), (2, 1, 1)], {0: [(0, 2)], 2: [(4, 3)]}, entry=0, unknown_row=[(7, 5)]),
        handmade.build(4, [(0, 2, 1), (1, 2, 3)], {2: [(0, 8)], 3: [(0, 1)]}, entry=None),
        handmade.build(4, [(0, 1, 2), (0, 2, 2), (1, 3, 5), (2, 3, 5)], {3: [(3, 10)]}, entry=0),
        handmade.build(3, [(2, 0, 0), (0, 1, 0)], {1: [(0, 6)]}, entry=2),
    ]
    for i, w in enumerate(cases):
        check_against_oracle(hpa, hctx, w, f"handmade{i}")


@DISABLED
def test_cct_budget(hpa, hctx):
    w = small_config(7, n_samples=20000, n_funcs=120, n_inst=4000, n_ctx=60)
    m, a, plan, t, d = _gpu_all(hpa, hctx, w)
    need = t.n_nodes
    with pytest.raises(hpa.HpaError) as ei:
        _gpu_all(hpa, hctx, w, max_nodes=need - 1)
    assert ei.value.code == hpa.E_BUDGET and ei.value.required == need


def test_prepare_callgraph_validation(hpa, hctx):
    w = handmade.build(3, [(0, 1, 1)], {1: [(0, 1)]}, entry=0)
    m = hpa.build_structure_map_workload(hctx, w)
    bad_pc = w.site_pc.copy()
    bad_pc[0] = handmade.func_start(2) + 16
    for sp, sc, se, ent in [
        (np.concatenate([w.site_pc, w.site_pc]), np.array([0, 0], np.uint32), np.array([1, 2], np.uint32), [0]),
        (bad_pc, w.site_caller, w.site_callee, [0]),
        (w.site_pc, w.site_caller, np.array([7], np.uint32), [0]),
        (w.site_pc, w.site_caller, w.site_callee, [5]),
    ]:
        with pytest.raises(hpa.HpaError) as ei:
            hpa.prepare_callgraph(hctx, m, w.n_scope_ids, sp, sc, se, w.ctx_parent, np.array(ent, np.int32))
        assert ei.value.code == hpa.E_INVAL


@DISABLED
@pytest.mark.parametrize("seed", list(range(6)))
def test_cct_exact_counts(hpa, hctx, seed):
    """Exact-count call graphs: weights taken as given, step 2 off."""
    w = tiny_random_case(300 + seed, n_funcs=4 + seed % 4, n_samples=400, n_ctx=3, weighted=True)
    check_against_oracle(hpa, hctx, w, f"exact{seed}", sample_based=0)


@DISABLED
def test_cct_exact_counts_small(hpa, hctx):
    check_against_oracle(hpa, hctx, small_config(11, n_samples=50_000, weighted=True), "exact-small", sample_based=0)


def test_cct_entry_points_compiled_out(hpa, hctx):
    """Until the device path is verified, both entry points fail with
    HPA_E_UNSUPPORTED before any kernel is launched."""
    w = handmade.build(3, [(0, 1, 1)], {1: [(0, 1)]}, entry=0)
    m = hpa.build_structure_map_workload(hctx, w)
    pc, cx, st, wt = hpa.samples_to_device(w)
    a = hpa.attribute(hctx, m, pc, cx, st, wt, w.n_ctx)
    plan = hpa.prepare_callgraph_workload(hctx, m, w)
    with pytest.raises(hpa.HpaError) as ei:
        hpa.apportion_callpaths(hctx, plan, a)
    assert ei.value.code == hpa.E_UNSUPPORTED
