"""Builds lb_driver (a host program that uses the library only through
include/lb.h) next to this file.  Needs the library built first."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "lb_driver.cpp")
EXE = os.path.join(HERE, "lb_driver")
PKG = os.path.join(ROOT, "paper_1703_00186_amd")


def build(force: bool = True) -> str:
    if not force and os.path.exists(EXE) and os.path.getmtime(EXE) >= os.path.getmtime(SRC):
        return EXE
    tmp = EXE + ".tmp%d" % os.getpid()
    subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I" + os.path.join(ROOT, "include"), SRC, "-L" + PKG, "-l:libd2q37_lb.so",
                    "-Wl,-rpath,$ORIGIN/../../paper_1703_00186_amd", "-o", tmp], check=True)
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build())
