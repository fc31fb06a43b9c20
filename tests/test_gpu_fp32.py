"""FP32 "shifted populations" form on the GPU.

Storage and sums in FP32 of g_l = f_l - w_l rho_ref (rho_ref = 1), with the
equilibrium coefficients and the relaxation in FP64.  Checked per field
(rho, u, T; the metric of tests/helpers.py) against the FP64 oracle on a
256 x 256 Rayleigh-Taylor rerun over 2000 steps, and against the FP64 GPU
step on the 4096 x 4096 lattice over 2000 steps: both within 1e-5.
"""

import numpy as np
import pytest

import oracle
from helpers import field_errors, gpu_available, worst
from paper_1703_00186_amd import workload

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1703_00186_amd.lb import LB


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def oparams():
    return oracle.Params(tau=0.7, gx=0.0, gy=-1e-4, t_bottom=1.5, t_top=0.5)


def test_fp32_state_is_shifted_and_propagate_exact():
    lx, ly = 40, 70
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=1)
    lb = LB(lx, ly, rho, ux, uy, T, precision="fp32s")
    f64 = oracle.init_feq(rho, ux, uy, T)
    _, _, w, _ = oracle.model()
    g = host(lb.get_state())
    assert g.dtype == np.float32
    ref = f64 - w[:, None, None]
    assert np.abs(g.astype(np.float64) - ref).max() <= 2e-7 * np.abs(ref).max()
    rng = np.random.default_rng(0)
    g0 = rng.standard_normal((37, lx, ly)).astype(np.float32)
    lb.set_state(torch.from_numpy(g0))
    lb.propagate()
    got = host(lb.get_scratch())
    ref = oracle.propagate(g0.astype(np.float64), ybc=0)
    known = ~np.isnan(ref)
    assert np.array_equal(got[known], ref[known].astype(np.float32))


@pytest.mark.parametrize("layout", ["column", "soa"])
@pytest.mark.parametrize("precision,tol", [("fp32s", 2e-7), ("fp32s_f32sum", 1e-6)])
@pytest.mark.parametrize("kernel", ["fused", "split"])
def test_fp32_single_step_close_to_oracle(kernel, precision, tol, layout):
    """One step from the same FP32-rounded state: the FP64-sum form adds one
    FP32 rounding per population (6e-8) to the oracle's step; FP32 sums of 37
    terms add up to ~20 more ulp of the largest term."""
    lx, ly = 64, 80
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=2)
    f = oracle.run(oracle.init_feq(rho, ux, uy, T), oparams(), 5)
    lb = LB(lx, ly, rho, ux, uy, T, precision=precision, kernel=kernel, layout=layout)
    _, _, w, _ = oracle.model()
    g0 = (f - w[:, None, None]).astype(np.float32)
    lb.set_state(torch.from_numpy(g0))
    lb.step(1)
    ref = oracle.run(g0.astype(np.float64) + w[:, None, None], oparams(), 1)
    got = host(lb.populations())
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


def test_fp32_vs_oracle_256_2000_steps():
    lx, ly, steps = 256, 256, 2000
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=workload.config_seed(3))
    lb = LB(lx, ly, rho, ux, uy, T, precision="fp32s")
    lb.step(steps)
    m32 = [host(t) for t in lb.moments()]
    ref = oracle.moments(oracle.run(oracle.init_feq(rho, ux, uy, T), oparams(), steps))
    errs = field_errors(m32, ref)
    print("fp32s vs oracle 256x256x2000:", errs)
    assert worst(errs) <= 1e-5, errs


def test_fp32_vs_fp64_gpu_4096_2000_steps():
    lx, ly, steps = 4096, 4096, 2000
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=workload.config_seed(3))
    lb64 = LB(lx, ly, rho, ux, uy, T, precision="fp64")
    lb64.step(steps)
    m64 = [host(t) for t in lb64.moments()]
    del lb64
    torch.cuda.empty_cache()
    lb32 = LB(lx, ly, rho, ux, uy, T, precision="fp32s")
    lb32.step(steps)
    m32 = [host(t) for t in lb32.moments()]
    errs = field_errors(m32, m64)
    print("fp32s vs fp64 GPU 4096x4096x2000:", errs)
    assert worst(errs) <= 1e-5, errs
