"""The binding rejects malformed device arrays before any call into the library.

These checks run without a GPU: every case fails validation (wrong element
size, floating point, non-contiguous, length mismatch, or host memory) and so
never reaches a kernel.
"""
import pytest
import torch

import paper_2109_06931_amd as hpa


def _samples(n=8):
    return (torch.zeros(n, dtype=torch.int64), torch.zeros(n, dtype=torch.int32),
            torch.zeros(n, dtype=torch.uint8), torch.ones(n, dtype=torch.int32))


@pytest.mark.parametrize("case, match", [
    ("ctx_int64", "ctx_ids must have 4-byte"),
    ("stall_int32", "stall must have 1-byte"),
    ("pc_float", "pc must hold integers"),
    ("ctx_short", "ctx_ids has 7 elements"),
    ("weight_short", "weight has 4 elements"),
    ("stall_strided", "stall must be contiguous"),
    ("host_memory", "must be in GPU memory"),
])
def test_attribute_rejects_bad_arrays(case, match):
    pc, cx, st, wt = _samples()
    n_ctx = 4
    if case == "ctx_int64":
        cx = torch.zeros(8, dtype=torch.int64)
    elif case == "stall_int32":
        st = torch.zeros(8, dtype=torch.int32)
    elif case == "pc_float":
        pc = torch.zeros(8, dtype=torch.float64)
    elif case == "ctx_short":
        cx = cx[:7]
    elif case == "weight_short":
        wt = wt[:4]
    elif case == "stall_strided":
        st = torch.zeros(16, dtype=torch.uint8)[::2]
    with pytest.raises(ValueError, match=match):
        hpa.attribute(None, None, pc, cx, st, wt, n_ctx)


def test_lookup_rejects_short_output():
    pc = torch.zeros(10, dtype=torch.int64)
    out = torch.zeros(9, dtype=torch.int32)
    with pytest.raises(ValueError, match="out has 9 elements"):
        hpa.lookup_intervals(None, None, pc, out)
    with pytest.raises(ValueError, match="out must have 4-byte"):
        hpa.lookup_intervals(None, None, pc, torch.zeros(10, dtype=torch.int64))
