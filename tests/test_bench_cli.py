"""The benchmark's command line on the CPU: a request for more than one GPU
is refused with a message (this build measures one GPU), and the accounting
helpers give the bytes per site of every storage form."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bytes_per_site_of_every_form():
    # 37 populations read and written once; the local-reference forms also
    # read and write the site's packed 4-byte reference
    assert bench.bytes_per_site("fp64") == 592
    assert bench.bytes_per_site("fp32s") == 296
    assert bench.bytes_per_site("fp32s_f32sum") == 296
    assert bench.bytes_per_site("fp32c") == 304
    assert bench.bytes_per_site("fp32l") == 304


def test_mlups():
    assert abs(bench.mlups(3932160 * 20, 20 * 0.4e-3) - 9830.4) < 1e-9
