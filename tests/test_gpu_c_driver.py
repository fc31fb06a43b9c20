"""The C ABI used on its own: a host program (tests/abi_driver/lb_driver.cpp)
allocates with hipMalloc, runs the step through include/lb.h on a stream of
its own and writes Eq. (2) moments; they must match the oracle to 1e-12, for
the fused and the split kernels.  It also checks that lb_init rejects a short
and a misaligned workspace."""

import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from helpers import field_errors, worst
from paper_1703_00186_amd import workload

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "abi_driver"))
import build_driver  # noqa: E402


@pytest.mark.parametrize("kernel", [0, 1])
def test_c_driver_matches_oracle(tmp_path, kernel):
    exe = build_driver.EXE
    assert os.path.exists(exe), "tests/abi_driver/lb_driver is not built (run __graft_entry__.build())"
    lx, ly, steps = 96, 70, 20
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=workload.config_seed(1))
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    np.concatenate([a.ravel() for a in (rho, ux, uy, T)]).astype(np.float64).tofile(inp)
    print("lb_driver %dx%d %d steps kernel %d" % (lx, ly, steps, kernel), flush=True)
    r = subprocess.run([exe, str(inp), str(out), str(lx), str(ly), str(steps), str(kernel)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    got = np.fromfile(out, dtype=np.float64).reshape(4, lx, ly)
    P = oracle.Params(tau=0.7, gx=0.0, gy=-1e-4, t_bottom=1.5, t_top=0.5)
    ref = oracle.run_moments_extended(oracle.init_feq(rho, ux, uy, T), P, steps)
    errs = field_errors(list(got), ref)
    print("C driver vs extended oracle:", errs)
    assert worst(errs) <= 1e-12, errs
