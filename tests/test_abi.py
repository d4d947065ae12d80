"""The C-ABI library loads and exports every function include/hpa.h declares
(no GPU work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hpa.h")
LIB = os.path.join(ROOT, "paper_2109_06931_amd", "libhpa.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hpa_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["hpa_build_structure_map", "hpa_attribute", "hpa_apportion_callpaths", "hpa_derive_metrics",
              "hpa_lookup_intervals", "hpa_prepare_callgraph"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhpa.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhpa.so not built")
def test_last_error_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.hpa_last_error.restype = ctypes.c_char_p
    lib.hpa_ctx_create.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    rc = lib.hpa_ctx_create(0, None, None)
    assert rc == -1  # NULL out-parameter is rejected before any device call
    assert b"NULL" in lib.hpa_last_error()
