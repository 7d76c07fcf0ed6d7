"""Build libfjgpu.so (the HIP C-ABI library) in-tree for gfx950.

    python -m paper_2101_08143_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfjgpu.so")
SOURCES = [os.path.join(CSRC, "fj_api.hip")]
HEADERS = [os.path.join(CSRC, "fj_guard.hpp"), os.path.join(CSRC, "fj_kernels.hpp"), os.path.join(CSRC, "fj_batched.hpp"),
           os.path.join(CSRC, "fj_blockcg.hpp"), os.path.join(CSRC, "fj_multilevel.hpp"),
           os.path.join(CSRC, "fj_aids.hpp"), os.path.join(CSRC, "fj_hierarchy.hpp"),
           os.path.join(CSRC, "fj_reorder.hpp"), os.path.join(CSRC, "fj_phased.hpp"),
           os.path.join(CSRC, "fj_server.hpp"), os.path.join(os.path.dirname(HERE), "include", "fj.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *HIPCC_FLAGS, "-o", LIB + ".tmp", *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(ln for ln in (res.stdout + res.stderr).splitlines()
                     if "packed-fp32-ops" not in ln and ln.strip())
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{msgs}")
    if verbose and msgs:
        print(msgs, file=sys.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
