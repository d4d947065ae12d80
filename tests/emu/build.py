"""Build the library's kernel sources for the host against the CPU stand-in
for HIP (include/hip/hip_runtime.h here): each .hip file is copied with its
kernel launches `k<<<grid, block, lds, stream>>>(args)` rewritten as
`emu_launch(grid, block, lds, stream, [&] { k(args); })`, and compiled with
g++ into _build/libhpa_emu.so (or, with --asan, into libhpa_emu_asan.so
under AddressSanitizer).  The learned index is left out (its entry points
fail).  Test infrastructure only: nothing in the library uses it.

usage: python tests/emu/build.py [--asan]
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2109_06931_amd", "csrc")
BUILD = os.path.join(HERE, "_build")
FILES = ["core.hip", "attribute.hip", "attribute_dense.hip", "apportion.hip", "derive.hip"]


def _match_back(text, k, open_c, close_c):
    """Index of the bracket that opens the group closing at text[k]."""
    depth = 0
    while True:
        c = text[k]
        if c == close_c:
            depth += 1
        elif c == open_c:
            depth -= 1
            if depth == 0:
                return k
        k -= 1


def rewrite_launches(text):
    out, i = [], 0
    while True:
        j = text.find("<<<", i)
        if j < 0:
            out.append(text[i:])
            return "".join(out)
        k = j
        if text[k - 1] == ">":  # template arguments of the kernel name
            k = _match_back(text, k - 1, "<", ">")
        while k > 0 and (text[k - 1].isalnum() or text[k - 1] in "_:"):
            k -= 1
        kern = text[k:j]
        e = text.find(">>>", j)
        cfg = text[j + 3:e]
        p = e + 3
        if text[p] != "(":
            raise ValueError(f"unexpected launch syntax near: {text[j - 40:p + 10]!r}")
        depth, q = 0, p
        while True:
            c = text[q]
            if c == "(":
                depth += 1
            elif c == ")":
                depth -= 1
                if depth == 0:
                    break
            q += 1
        out.append(text[i:k])
        out.append(f"emu_launch({cfg}, [&] {{ {kern}({text[p + 1:q]}); }})")
        i = q + 1


STUBS = '''#include "hpa_internal.h"
namespace hpa {
void launch_lookup_learned(const hpa_structure_map*, const uint64_t*, uint64_t, uint32_t*, hipStream_t) {
  fail(HPA_E_UNSUPPORTED, "learned index: not part of the CPU build");
}
void learned_free(LearnedModel*) {}
void learned_train(hpa_structure_map*, const hpa_learned_opts*, hipStream_t) {
  fail(HPA_E_UNSUPPORTED, "learned index: not part of the CPU build");
}
void learned_train(hpa_structure_map*, hipStream_t) {
  fail(HPA_E_UNSUPPORTED, "learned index: not part of the CPU build");
}
}  // namespace hpa
'''


def build(asan=False):
    src = os.path.join(BUILD, "src_asan" if asan else "src")
    os.makedirs(src, exist_ok=True)
    for f in os.listdir(CSRC):
        text = open(os.path.join(CSRC, f)).read()
        if f.endswith(".hip"):
            open(os.path.join(src, f[:-4] + ".cpp"), "w").write(rewrite_launches(text))
        elif f.endswith(".h"):
            open(os.path.join(src, f), "w").write(text)
    open(os.path.join(src, "stubs.cpp"), "w").write(STUBS)
    flags = ["-std=c++20", "-O1", "-g", "-fPIC", "-pthread", "-ffp-contract=off", "-w",
             "-I", os.path.join(HERE, "include"), "-I", os.path.join(ROOT, "include"), "-I", src,
             "-DHPA_ENABLE_GPU_CCT"]
    if asan:
        flags += ["-fsanitize=address", "-fno-omit-frame-pointer"]
    objs, procs = [], []
    for f in [x[:-4] + ".cpp" for x in FILES] + ["stubs.cpp"]:
        o = os.path.join(src, f[:-4] + ".o")
        procs.append(subprocess.Popen(["g++", *flags, "-c", os.path.join(src, f), "-o", o]))
        objs.append(o)
    if any(p.wait() for p in procs):
        raise RuntimeError("g++ failed on the CPU build of the kernel sources")
    out = os.path.join(BUILD, "libhpa_emu_asan.so" if asan else "libhpa_emu.so")
    subprocess.check_call(["g++", *flags, "-shared", *objs, "-o", out])
    return out


if __name__ == "__main__":
    print("built", build(asan="--asan" in sys.argv))
