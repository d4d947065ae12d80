"""The library's kernel sources built for the host against a CPU stand-in for
HIP (build.py) and run through the C ABI on small seeded cases, compared with
the oracle (run.py): the calling-context tree and derived metrics, whose
device path is compiled out of the GPU build, and the attribution pipelines.
One build runs under AddressSanitizer, so an out-of-bounds access of any
kernel on these cases fails the test.  This checks the kernels' logic and
indexing, not the GPU's memory model or concurrent workgroups."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
import build  # noqa: E402

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++ for the CPU build")

# (each emulated launch starts a thread per lane, so the cases stay small;
# run.py runs any other case of its table by name)
CCT = ["cct_tiny0", "cct_tiny1", "cct_tiny2", "cct_tiny3", "cct_fig4", "cct_small1"]
ATTR = ["attr_tiny0", "attr_tiny3w", "attr_small2w"]
ASAN = ["cct_tiny0", "cct_fig4", "attr_tiny3w"]


def _run(lib, cases, env=None):
    r = subprocess.run([sys.executable, os.path.join(HERE, "run.py"), lib, *cases], capture_output=True, text=True,
                       env=env, timeout=1200)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for c in cases:
        assert f"{c}: OK" in out, out[-4000:]


@pytest.fixture(scope="module")
def lib():
    return build.build()


@pytest.mark.timeout(1200)
def test_cct_and_metrics_emulated_equal_oracle(lib):
    _run(lib, CCT)


@pytest.mark.timeout(1200)
def test_attribution_emulated_equals_oracle(lib):
    _run(lib, ATTR)


@pytest.mark.timeout(1800)
def test_emulated_kernels_in_bounds_under_asan():
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.isabs(asan):
        pytest.skip("no AddressSanitizer runtime")
    lib = build.build(asan=True)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    _run(lib, ASAN, env=env)
