"""Comparison helpers shared by the GPU parity tests (no method arithmetic)."""
import numpy as np

NONE32 = 0xFFFFFFFF


def assert_attribution_equal(got: dict, exp, label=""):
    """Bit-exact comparison of a GPU attribution (numpy dict) with the oracle's."""
    n = len(exp.ctx)
    assert len(got["ctx"]) == n, f"{label}: {len(got['ctx'])} keys vs {n}"
    for f in ["ctx", "pc", "stall", "count", "scope"]:
        g, e = got[f], getattr(exp, f)
        if not np.array_equal(g, e):
            bad = np.nonzero(g != e)[0]
            i = int(bad[0])
            raise AssertionError(f"{label}: field {f} differs at {len(bad)} keys; first {i}: "
                                 f"got {g[i]} want {e[i]} (ctx {exp.ctx[i]} pc {exp.pc[i]:#x} stall {exp.stall[i]})")
    assert np.array_equal(got["ctx_offsets"], exp.ctx_offsets), f"{label}: ctx_offsets differ"
