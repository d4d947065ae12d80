"""GPU parity of cross-profile unification, statistics, the sparse layouts and
the combination of runs against the plain reference (integers bit-exact, FP64
statistics within 1e-9 relative), and of the sparse file against the arrays."""
import numpy as np
import pytest

import oracle
from oracle import unify_ref
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


@pytest.fixture(scope="module")
def hctx(hpa):
    return hpa.Context(0)


def _profiles(hpa, hctx, seed, P, n):
    w = small_config(seed, n_samples=n * P, n_ctx=300)
    m = hpa.build_structure_map_workload(hctx, w)
    pc, cx, st, _ = hpa.samples_to_device(w)
    r = np.random.default_rng(seed)
    cuts = np.sort(r.choice(np.arange(1, n * P), size=P - 1, replace=False))
    bounds = [0] + cuts.tolist() + [n * P]
    gpu = [hpa.attribute(hctx, m, pc[a:b].contiguous(), cx[a:b].contiguous(), st[a:b].contiguous(), None, w.n_ctx)
           for a, b in zip(bounds, bounds[1:])]
    return w, m, gpu


class _Np:
    def __init__(self, d):
        for k in ("ctx", "pc", "stall", "count"):
            setattr(self, k, d[k])


@pytest.mark.parametrize("seed, P", [(31, 1), (32, 3), (33, 9)])
def test_unify_matches_reference(hpa, hctx, seed, P, tmp_path):
    print(f"case unify seed={seed} P={P}", flush=True)
    w, m, gpu = _profiles(hpa, hctx, seed, P, 20_000)
    u = hpa.unify_profiles(hctx, gpu)
    got = u.numpy()
    ref = unify_ref.unify([_Np(a.numpy()) for a in gpu])
    for k in ["ctx", "pc", "cms_ctx_off", "cms_m_off", "cms_mid", "cms_mstart", "cms_pid", "cms_val", "pms_off",
              "pms_c_off", "pms_ctx", "pms_cstart", "pms_mid", "pms_val", "st_sum", "st_min", "st_max"]:
        assert np.array_equal(got[k], ref[k]), k
    assert np.array_equal(got["cms_mctx"], ref["st_ctx"])
    for k in ["st_mean", "st_std", "st_cov"]:
        np.testing.assert_allclose(got[k], ref[k], rtol=1e-9, atol=0, err_msg=k)
    # the files hold the same arrays, written through a small bounce buffer
    for fmt, names in [(hpa.SPARSE_CMS, ["ctx", "pc", "cms_ctx_off", "cms_m_off", "cms_mid", "cms_mstart",
                                          "cms_pid", "cms_val"]),
                       (hpa.SPARSE_PMS, ["ctx", "pc", "pms_off", "pms_c_off", "pms_ctx", "pms_cstart", "pms_mid",
                                          "pms_val"])]:
        path = tmp_path / f"out{fmt}.bin"
        u.write(path, fmt, round_bytes=4096)
        raw = path.read_bytes()
        hdr = np.frombuffer(raw[:64], np.uint64)
        assert int(hdr[0]) == 0x45535241505350 and int(hdr[1]) == fmt and int(hdr[7]) == len(names)
        offs = np.frombuffer(raw[64:64 + 8 * len(names)], np.uint64)
        for o, name in zip(offs.tolist(), names):
            a = got[name]
            assert np.array_equal(np.frombuffer(raw[o:o + a.nbytes], a.dtype), a), (fmt, name)


def test_combine_runs_matches_attribution_of_all(hpa, hctx):
    w, m, gpu = _profiles(hpa, hctx, 34, 4, 25_000)
    comb = hpa.combine_runs(hctx, gpu).numpy()
    om = oracle.build_map_workload(w)
    allr = oracle.attribute(om, w.pc, w.ctx, w.stall, None, w.n_ctx)
    for f in ["ctx", "pc", "stall", "count", "scope"]:
        assert np.array_equal(comb[f], getattr(allr, f)), f
    assert np.array_equal(comb["ctx_offsets"], allr.ctx_offsets)
