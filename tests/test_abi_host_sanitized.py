"""The C ABI's host logic under AddressSanitizer and UBSan, without a GPU.

tests/abi_driver/host_abi_check.cpp drives every entry point of include/lb.h
(argument checks, workspace carving, call-order rules, success paths over
host buffers, the thread-local error message) against lb_api.hip built for the
host only, with the kernel launchers replaced by stand-ins that touch no
memory (tests/abi_driver/host_stub_launchers.cpp).  The sanitizers are
applied to host code only; nothing here runs on a GPU.
"""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "abi_driver")
CSRC = os.path.join(ROOT, "paper_1703_00186_amd", "csrc")


def test_host_abi_under_address_and_ub_sanitizers(tmp_path):
    if not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "host_abi_check")
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(CSRC, "lb_api.hip"), os.path.join(DRIVER, "host_stub_launchers.cpp"),
           "-x", "c++", os.path.join(DRIVER, "host_abi_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failure(s)" in r.stdout
