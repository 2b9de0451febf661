"""Build libqsv.so in-tree with hipcc for gfx950.

Run as ``python -m paper_2404_09213_amd.build_lib`` or through
``__graft_entry__.build()``. Always recompiles.

``--sanitize`` builds libqsv_san.so instead: the same sources with the host
code (planner, code generator, argument checks) instrumented by
AddressSanitizer and UndefinedBehaviorSanitizer; device code is unchanged.
It is for CPU test runs only (load it with QSV_LIB=<path> and the clang ASan
runtime in LD_PRELOAD); nothing on a GPU loads it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = [os.path.join(HERE, "csrc", "qsv.hip"), os.path.join(HERE, "csrc", "planner.cpp"),
           os.path.join(HERE, "csrc", "jit.cpp")]
OUT = os.path.join(HERE, "libqsv.so")
OUT_SAN = os.path.join(HERE, "libqsv_san.so")
# host-only sanitizers: every -fsanitize= applies to the host compilation only
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined", "-g"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-I" + os.path.join(ROOT, "include"),
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = OUT_SAN if sanitize else OUT
    tmp = out + ".tmp"
    extra = SAN_FLAGS if sanitize else []
    cmd = [HIPCC, *FLAGS, *extra, "-o", tmp, *SOURCES, "-lhiprtc", "-lrocprofiler-sdk-roctx", "-pthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    msgs = [l for l in (res.stdout + res.stderr).splitlines() if noise not in l and l.strip()]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
