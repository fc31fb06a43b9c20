"""Builds the gfx950 shared library behind include/lb.h.

    python -m paper_1703_00186_amd.build

compiles csrc/*.hip with hipcc for gfx950 into paper_1703_00186_amd/libd2q37_lb.so
(in-tree).  Packed-FP32 VALU instructions are disabled for all device code.
"""

from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libd2q37_lb.so")
SOURCES = [os.path.join(CSRC, "d2q37_kernels.hip"), os.path.join(CSRC, "d2q37_variants.hip"),
           os.path.join(CSRC, "lb_api.hip"), os.path.join(CSRC, "lb_scratch.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    sys.path.insert(0, CSRC)
    try:
        import gen_constants
    finally:
        sys.path.pop(0)
    if not gen_constants.check():
        gen_constants.write()
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
