"""FP32 forms on the GPU.

  fp32c         FP32 storage of each population's deviation from the rest
                Maxwellian of the site that wrote it (plus that site's FP16
                density and temperature), and the FP32 collision (FP32 Hermite
                sums; FP64 for the collision invariants, the equilibrium
                coefficients and a conservation correction);
  fp32s         FP32 storage of the shifted populations g_l = f_l - w_l rho_ref
                (rho_ref = 1 unless a test says otherwise), FP64 collision;
  fp32s_f32sum  the same storage with the collision's Hermite sums in FP32
                (ablation).
Checked per field (rho, u, T; u as max|du| / max|u|, tests/helpers.py)
against the FP64 oracle on a 256 x 256 Rayleigh-Taylor rerun over 2000 steps
and against the FP64 GPU step on the 4096 x 4096 lattice over 2000 steps.
fp32c meets 1e-5 with two orders of magnitude to spare; the shifted storage is
held to the bounds its measured errors state (its rounding floor in u over
the slow flow of the 4096 x 4096 lattice is above 1e-5).
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


def oparams(**kw):
    p = dict(tau=0.7, gx=0.0, gy=-1e-4, t_bottom=1.5, t_top=0.5)
    p.update(kw)
    return oracle.Params(**p)


@pytest.mark.parametrize("precision", ["fp32c", "fp32l"])
def test_fp32_local_state_encodes_the_equilibrium(precision):
    """The local-reference form of f^eq(rho0, u0, T0): 38 FP32 planes, and the
    populations it decodes to equal the oracle's f^eq to the rounding of the
    deviations from the FP16 reference (far below an FP32 rounding of f)."""
    lx, ly = 40, 70
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=1)
    lb = LB(lx, ly, rho, ux, uy, T, precision=precision)
    st = host(lb.get_state())
    assert st.shape == (38, lx, ly) and st.dtype == np.float32
    ref = oracle.init_feq(rho, ux, uy, T)
    got = host(lb.populations())
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("%s init decode error %.2e" % (precision, err))
    assert err <= 1e-9
    # a state round trip through get_state / set_state is exact
    lb.set_state(torch.from_numpy(st))
    assert np.array_equal(host(lb.get_state()).view(np.uint32), st.view(np.uint32))


@pytest.mark.parametrize("precision", ["fp32c", "fp32l"])
def test_fp32_local_is_fused_only(precision):
    from paper_1703_00186_amd.lb import LBError
    lx, ly = 16, 16
    f = workload.rt_fields(lx, ly, seed=1)[:4]
    with pytest.raises(LBError) as e:
        LB(lx, ly, *f, precision=precision, kernel="split")
    assert e.value.code == -1
    lb = LB(lx, ly, *f, precision=precision)
    for stage in (lb.propagate, lb.bc, lb.collide):
        with pytest.raises(LBError) as e:
            stage()
        assert e.value.code == -4
    with pytest.raises(LBError):
        lb.set_params(kernel="split")


def test_fp32_state_is_shifted_and_propagate_exact():
    precision = "fp32s"
    lx, ly = 40, 70
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=1)
    lb = LB(lx, ly, rho, ux, uy, T, precision=precision)
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


# One step from the same FP32 state.  fp32s adds one FP32 rounding per
# population (2^-24) to the oracle's step.  FP32 Hermite sums of f itself add
# ~20 ulp of the largest term (coefficients up to He_4(3r) = 92).  fp32c's
# FP32 sums round relative to the deviation from the rest Maxwellian (at
# most the size of f, at the interface), and its stored deviations are
# rounded relative to their own size.
ONE_STEP_TOL = {"fp32s": 2e-7, "fp32c": 1e-7, "fp32l": 1e-7, "fp32s_f32sum": 1e-6}


@pytest.mark.parametrize("layout", ["column", "soa"])
@pytest.mark.parametrize("precision", ["fp32s", "fp32s_f32sum"])
@pytest.mark.parametrize("kernel", ["fused", "split"])
@pytest.mark.parametrize("regularize", [1, 0])
def test_fp32_single_step_close_to_oracle(kernel, precision, layout, regularize):
    lx, ly = 64, 80
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=2)
    P = oparams(regularize=regularize)
    f = oracle.run(oracle.init_feq(rho, ux, uy, T), P, 5)
    lb = LB(lx, ly, rho, ux, uy, T, precision=precision, kernel=kernel, layout=layout,
            regularize=regularize)
    _, _, w, _ = oracle.model()
    g0 = (f - w[:, None, None]).astype(np.float32)
    lb.set_state(torch.from_numpy(g0))
    lb.step(1)
    ref = oracle.run(g0.astype(np.float64) + w[:, None, None], P, 1)
    got = host(lb.populations())
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("%s %s %s reg=%d one step: %.2e" % (precision, kernel, layout, regularize, err))
    assert err <= ONE_STEP_TOL[precision]


@pytest.mark.parametrize("shape", [(64, 80), (7, 65), (130, 257)])
@pytest.mark.parametrize("layout", ["column", "soa"])
@pytest.mark.parametrize("regularize", [1, 0])
@pytest.mark.parametrize("precision", ["fp32c", "fp32l"])
def test_fp32_local_single_step_close_to_oracle(precision, layout, regularize, shape):
    """One fused step of the local-reference form from the state it holds
    after 5 steps (decoded to FP64 populations) against the oracle's step
    from those populations; ragged tiles and the smallest odd sizes too."""
    lx, ly = shape
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=2)
    P = oparams(regularize=regularize)
    lb = LB(lx, ly, rho, ux, uy, T, precision=precision, layout=layout, regularize=regularize)
    lb.step(5)
    f = host(lb.populations())
    lb.step(1)
    ref = oracle.run(f, P, 1)
    got = host(lb.populations())
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("%s %dx%d %s reg=%d one step: %.2e" % (precision, lx, ly, layout, regularize, err))
    assert err <= ONE_STEP_TOL[precision]


@pytest.mark.parametrize("precision", ["fp32c", "fp32l"])
def test_fp32_local_periodic_y_single_step(precision):
    lx, ly = 40, 70
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=3)
    P = oparams(ybc=1)
    lb = LB(lx, ly, rho, ux, uy, T, precision=precision, ybc="periodic")
    lb.step(3)
    f = host(lb.populations())
    lb.step(1)
    ref = oracle.run(f, P, 1)
    err = np.abs(host(lb.populations()) - ref).max() / np.abs(ref).max()
    print("%s periodic y one step: %.2e" % (precision, err))
    assert err <= ONE_STEP_TOL[precision]


@pytest.mark.parametrize("rho_ref", [0.0, 1.3])
@pytest.mark.parametrize("precision", ["fp32s", "fp32s_f32sum"])
def test_fp32_shift_density_single_step(precision, rho_ref):
    """The shift density is a free parameter of the storage: one step from the
    same stored values g = f - w rho_ref must match the oracle for any
    rho_ref (rho_ref = 0: plain FP32 populations)."""
    lx, ly = 64, 80
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=2)
    f = oracle.run(oracle.init_feq(rho, ux, uy, T), oparams(), 5)
    lb = LB(lx, ly, rho, ux, uy, T, precision=precision, rho_ref=rho_ref)
    _, _, w, _ = oracle.model()
    g0 = (f - rho_ref * w[:, None, None]).astype(np.float32)
    lb.set_state(torch.from_numpy(g0))
    lb.step(1)
    ref = oracle.run(g0.astype(np.float64) + rho_ref * w[:, None, None], oparams(), 1)
    got = host(lb.populations())
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("%s rho_ref=%g one step: %.2e" % (precision, rho_ref, err))
    assert err <= ONE_STEP_TOL[precision]


@pytest.fixture(scope="module")
def oracle_256_2000():
    lx = ly = 256
    f = workload.rt_fields(lx, ly, seed=workload.config_seed(3))[:4]
    return f, oracle.moments(oracle.run(oracle.init_feq(*f), oparams(), 2000))


# per-field bounds after 2000 steps: the 1e-5 target for fp32c (measured
# ~1e-7); the shifted storage's measured rounding floor for fp32s
BOUND_256 = {"fp32c": 1e-5, "fp32l": 1e-5, "fp32s": 1e-5}


@pytest.mark.parametrize("precision", ["fp32c", "fp32l", "fp32s"])
def test_fp32_vs_oracle_256_2000_steps(precision, oracle_256_2000):
    fields, ref = oracle_256_2000
    lb = LB(256, 256, *fields, precision=precision)
    lb.step(2000)
    errs = field_errors([host(t) for t in lb.moments()], ref)
    print("%s vs oracle 256x256x2000:" % precision, errs)
    assert worst(errs) <= BOUND_256[precision], errs


def test_fp32_f32sum_ablation_stated_bound(oracle_256_2000):
    """The FP32-sum ablation misses 1e-5; it is held to the bound stated for
    it (per field, 256 x 256 x 2000 against the oracle)."""
    fields, ref = oracle_256_2000
    lb = LB(256, 256, *fields, precision="fp32s_f32sum")
    lb.step(2000)
    errs = field_errors([host(t) for t in lb.moments()], ref)
    print("fp32s_f32sum vs oracle 256x256x2000:", errs)
    assert max(errs["rho_max"], errs["T_max"]) <= 1e-4, errs
    assert errs["u_max"] <= 3e-3, errs


@pytest.mark.parametrize("rho_ref", [0.0, 1.3])
@pytest.mark.parametrize("precision", ["fp32s"])
def test_fp32_shift_density_vs_oracle_256_200_steps(precision, rho_ref):
    lx = ly = 256
    f = workload.rt_fields(lx, ly, seed=workload.config_seed(3))[:4]
    ref = oracle.moments(oracle.run(oracle.init_feq(*f), oparams(), 200))
    lb = LB(lx, ly, *f, precision=precision, rho_ref=rho_ref)
    lb.step(200)
    errs = field_errors([host(t) for t in lb.moments()], ref)
    print("%s rho_ref=%g vs oracle 256x256x200:" % (precision, rho_ref), errs)
    assert worst(errs) <= 1e-5, errs


# fp32c: the 1e-5 target; fp32s: its measured rounding floor in u (max|du|
# about 4.6e-8 against max|u| = 3.2e-3 after 2000 steps), rho and T 1e-5
BOUND_4096 = {"fp32c": {"rho": 1e-5, "u": 1e-5, "T": 1e-5},
              "fp32l": {"rho": 1e-5, "u": 1e-5, "T": 1e-5},
              "fp32s": {"rho": 1e-5, "u": 5e-5, "T": 1e-5}}


def test_fp32_vs_fp64_gpu_4096_2000_steps():
    lx, ly, steps = 4096, 4096, 2000
    f = workload.rt_fields(lx, ly, seed=workload.config_seed(3))[:4]
    lb64 = LB(lx, ly, *f, precision="fp64")
    lb64.step(steps)
    m64 = [host(t) for t in lb64.moments()]
    del lb64
    torch.cuda.empty_cache()
    results = {}
    for precision in ("fp32c", "fp32l", "fp32s"):
        lb32 = LB(lx, ly, *f, precision=precision)
        lb32.step(steps)
        results[precision] = field_errors([host(t) for t in lb32.moments()], m64)
        del lb32
        torch.cuda.empty_cache()
        print("%s vs fp64 GPU 4096x4096x2000:" % precision, results[precision])
    for precision, errs in results.items():
        b = BOUND_4096[precision]
        assert max(errs["rho_max"], errs["rho_rms"]) <= b["rho"], (precision, errs)
        assert max(errs["T_max"], errs["T_rms"]) <= b["T"], (precision, errs)
        assert max(errs["u_max"], errs["u_rms"]) <= b["u"], (precision, errs)


def _invariants(lb):
    """Total mass, momentum and energy (sum rho (|u|^2 + 2 T), D = 2) of the
    current state, summed exactly (math.fsum) from the FP64 moments."""
    import math
    rho, ux, uy, T = [host(t).astype(np.float64) for t in lb.moments()]
    return np.array([math.fsum(rho.ravel()), math.fsum((rho * ux).ravel()),
                     math.fsum((rho * uy).ravel()),
                     math.fsum((rho * (ux * ux + uy * uy + 2.0 * T)).ravel())])


# drift bounds of the invariants over 500 periodic steps, relative to the
# total mass (energy: to the total energy); measured 1.9e-14 (FP64), 7.7e-12
# (fp32c), 1.6e-11 (fp32l), 1.5e-9 (fp32s)
CONSERVATION_BOUND = {"fp64": 1e-13, "fp32c": 1e-10, "fp32l": 1e-10, "fp32s": 1e-8}


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32l", "fp32s"])
def test_collision_invariants_conserved(precision):
    """Periodic in x and y, no gravity: propagate and collide conserve mass,
    momentum and energy, so over 500 steps the totals move only by rounding.
    The FP32 collision's FP64 invariant sums and conservation correction keep
    it at the level of the FP64-collision form on the same storage; the
    shifted form, whose stored values are rounded relative to f itself, moves
    more."""
    lx, ly, n = 128, 96, 500
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=9)
    lb = LB(lx, ly, rho, ux, uy, T, precision=precision, ybc="periodic", g=(0.0, 0.0))
    a = _invariants(lb)
    lb.step(n)
    b = _invariants(lb)
    scale = np.array([a[0], a[0], a[0], a[3]])
    drift = np.abs(b - a) / scale
    print("%s invariant drift over %d steps (mass, jx, jy, energy): %s" % (precision, n, drift))
    assert drift.max() <= CONSERVATION_BOUND[precision], drift
