"""The optimised CPU step against the oracle (CPU only).

Same workload inputs on both sides; several steps with walls and with
periodic y, regularized and plain BGK, at sizes spanning several vector chunks
and a ragged tail.
"""

import numpy as np
import pytest

import cpu_step
import oracle
from paper_1703_00186_amd import workload


@pytest.mark.parametrize("shape", [(6, 6), (17, 37), (64, 100)])
@pytest.mark.parametrize("ybc,regularize", [(0, 1), (0, 0), (1, 1)])
def test_cpu_step_matches_oracle(shape, ybc, regularize):
    lx, ly = shape
    f0 = oracle.init_feq(*workload.rt_fields(lx, ly, seed=5)[:4])
    kw = dict(tau=0.7, gx=1e-3, gy=-2e-3, t_bottom=1.5, t_top=0.5, regularize=regularize, ybc=ybc)
    lat = cpu_step.CpuLattice(lx, ly, f0, **kw)
    lat.step(6)
    ref = oracle.run(f0, oracle.Params(**kw), 6)
    assert np.abs(lat.get() - ref).max() <= 1e-13 * np.abs(ref).max()
