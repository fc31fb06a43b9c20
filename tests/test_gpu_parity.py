"""GPU (gfx950) kernels against the CPU oracle, through the C ABI.

Per-kernel parity at small sizes spanning several tiles and a ragged tail
(propagate bit-exact; bc and collide to 1e-13 of the value scale), then whole
steps on the Rayleigh-Taylor workload (every field within 1e-12 after 50
steps), both kernels paths and both memory layouts.  Inputs come from the
seeded generator shared by both sides.
"""

import numpy as np
import pytest

import oracle
from helpers import field_errors, gpu_available, worst
from paper_1703_00186_amd import workload

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1703_00186_amd import lb as lbmod


def oparams(**kw):
    base = dict(tau=0.7, gx=0.0, gy=-1e-4, t_bottom=1.5, t_top=0.5, regularize=1, ybc=0)
    base.update(kw)
    return oracle.Params(**base)


def make(lx, ly, seed=170301, mode="sinusoid", **kw):
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=seed, mode=mode)
    lb = lbmod.LB(lx, ly, rho, ux, uy, T, **kw)
    return lb, (rho, ux, uy, T)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("layout", ["soa", "column"])
@pytest.mark.parametrize("shape", [(37, 70), (256, 128), (6, 6)])
def test_init_and_moments(layout, shape):
    lx, ly = shape
    lb, fields = make(lx, ly, layout=layout)
    f_ref = oracle.init_feq(*fields)
    f_gpu = host(lb.populations())
    assert np.abs(f_gpu - f_ref).max() <= 1e-15 * 4
    m_gpu = [host(t) for t in lb.moments()]
    m_ref = oracle.moments(f_ref)
    errs = field_errors(m_gpu, m_ref)
    # the initial fluid is at rest (max |u| = 0, so the error relative to the
    # flow speed is undefined): u is checked against the thermal speed
    assert max(errs["rho_max"], errs["T_max"], errs["rho_rms"], errs["T_rms"]) < 1e-14, errs
    assert errs["info_u_thermal"] < 1e-14, errs


@pytest.mark.parametrize("layout", ["soa", "column"])
@pytest.mark.parametrize("ybc", ["walls", "periodic"])
def test_propagate_bit_exact(layout, ybc):
    lx, ly = 45, 300  # several tiles in y plus a ragged tail, odd lx
    lb, fields = make(lx, ly, layout=layout, ybc=ybc)
    rng = np.random.default_rng(11)
    f0 = rng.standard_normal((37, lx, ly))
    lb.set_state(torch.from_numpy(f0))
    lb.propagate()
    got = host(lb.get_scratch())
    ref = oracle.propagate(f0, ybc=1 if ybc == "periodic" else 0)
    known = ~np.isnan(ref)
    assert np.array_equal(got[known], ref[known])
    if ybc == "periodic":
        assert known.all()


@pytest.mark.parametrize("layout", ["soa", "column"])
def test_bc(layout):
    lx, ly = 70, 40
    lb, fields = make(lx, ly, layout=layout)
    f = oracle.run(oracle.init_feq(*fields), oparams(), 2)
    ft = oracle.propagate(f, ybc=0)
    lb.set_scratch(torch.from_numpy(np.nan_to_num(ft, nan=0.0)))
    lb.bc()
    got = host(lb.get_scratch())
    ref = oracle.bc(ft, 1.5, 0.5)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("regularize", [1, 0])
@pytest.mark.parametrize("layout", ["soa", "column"])
def test_collide(layout, regularize):
    lx, ly = 33, 200
    lb, fields = make(lx, ly, layout=layout, regularize=regularize, g=(2e-3, -1e-3))
    P = oparams(regularize=regularize, gx=2e-3, gy=-1e-3)
    f = oracle.run(oracle.init_feq(*fields), P, 3)
    ft = oracle.bc(oracle.propagate(f, ybc=0), 1.5, 0.5)
    lb.set_scratch(torch.from_numpy(ft))
    lb.collide()
    got = host(lb.get_state())
    ref = oracle.collide(ft, P)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.fixture(scope="module")
def extended_256x128_50():
    """The parity lattice after 50 steps in the oracle's extended-precision
    run (long double, model constants rounded from the binary128 solve): the
    reference against which FP64 rounding is measured.  Also the FP64
    oracle's populations and its own error against that reference."""
    lx, ly = 256, 128
    fields = workload.rt_fields(lx, ly, seed=170301)[:4]
    f0 = oracle.init_feq(*fields)
    ext = oracle.run_moments_extended(f0, oparams(), 50)
    f64 = oracle.run(f0, oparams(), 50)
    return ext, f64, field_errors(oracle.moments(f64), ext)


@pytest.mark.parametrize("kernel", ["fused", "split"])
@pytest.mark.parametrize("layout", ["soa", "column"])
def test_rt_256x128_50_steps(kernel, layout, extended_256x128_50):
    """256 x 128 Rayleigh-Taylor, 50 steps: every field (u as max|du| / max|u|,
    max and rms) within 1e-12 of the extended-precision oracle run; the
    populations within 1e-12 of the FP64 oracle's.  (The FP64 oracle's own
    distance from the extended run is printed: its f^eq polynomial and BGK
    sums carry more rounding than the GPU's Hermite-space collision.)"""
    lx, ly = 256, 128
    ext, f_ref, oracle_own = extended_256x128_50
    lb, fields = make(lx, ly, kernel=kernel, layout=layout)
    lb.step(50)
    m_gpu = [host(t) for t in lb.moments()]
    errs = field_errors(m_gpu, ext)
    print("GPU vs extended oracle:", errs)
    print("FP64 oracle vs extended oracle:", oracle_own)
    assert worst(errs) <= 1e-12, errs
    f_gpu = host(lb.populations())
    assert np.abs(f_gpu - f_ref).max() <= 1e-12 * np.abs(f_ref).max()


def test_rt_uniform_density_init():
    lx, ly = 256, 128
    lb, fields = make(lx, ly, mode="uniform")
    lb.step(50)
    ext = oracle.run_moments_extended(oracle.init_feq(*fields), oparams(), 50)
    errs = field_errors([host(t) for t in lb.moments()], ext)
    print("uniform init, GPU vs extended oracle:", errs)
    assert worst(errs) <= 1e-12, errs


@pytest.mark.parametrize("shape", [(6, 6), (7, 65), (130, 257)])
@pytest.mark.parametrize("kernel", ["fused", "split"])
def test_ragged_and_minimum_sizes(shape, kernel):
    lx, ly = shape
    lb, fields = make(lx, ly, kernel=kernel)
    lb.step(7)
    f_ref = oracle.run(oracle.init_feq(*fields), oparams(), 7)
    f_gpu = host(lb.populations())
    assert np.abs(f_gpu - f_ref).max() <= 1e-13 * np.abs(f_ref).max()


@pytest.mark.parametrize("kernel", ["fused", "split"])
def test_periodic_y_and_bgk(kernel):
    lx, ly = 64, 48
    lb, fields = make(lx, ly, kernel=kernel, ybc="periodic", regularize=0, g=(1e-3, -2e-3))
    lb.step(20)
    P = oparams(ybc=1, regularize=0, gx=1e-3, gy=-2e-3)
    f_ref = oracle.run(oracle.init_feq(*fields), P, 20)
    f_gpu = host(lb.populations())
    assert np.abs(f_gpu - f_ref).max() <= 1e-12 * np.abs(f_ref).max()


def test_fused_writes_every_site():
    """NaN-poison the destination: one fused step must overwrite all of it."""
    lx, ly = 50, 90
    lb, fields = make(lx, ly)
    lb.set_scratch(torch.full((37, lx, ly), float("nan"), dtype=torch.float64))
    lb.step(1)
    assert np.isfinite(host(lb.get_state())).all()


def test_deterministic():
    lx, ly = 96, 80
    a, _ = make(lx, ly)
    b, _ = make(lx, ly)
    a.step(10)
    b.step(10)
    assert torch.equal(a.get_state(), b.get_state())


def test_check_finite_reports_nonfinite_state():
    lx, ly = 32, 32
    lb, fields = make(lx, ly, check_finite=1)
    f = lb.get_state()
    f[5, 3, 7] = float("nan")
    lb.set_state(f)
    with pytest.raises(lbmod.LBError) as ei:
        lb.step(1)
    assert ei.value.code == -5


def _uniform_state(lb, f37):
    """The state tensor of a lattice whose every site holds the populations
    f37 (FP64 [37]), in the context's storage form: f itself (FP64),
    f - w rho_ref (shifted FP32), or deviations from a zero reference (the
    local-reference forms: packed reference word 0 means M = 0)."""
    _, _, w, _ = oracle.model()
    f = np.broadcast_to(np.asarray(f37)[:, None, None], (37, lb.lx, lb.ly))
    if lb.precision == "fp64":
        return torch.from_numpy(np.ascontiguousarray(f))
    if lb.precision in ("fp32s", "fp32s_f32sum"):
        return torch.from_numpy((f - 1.0 * w[:, None, None]).astype(np.float32))
    st = np.zeros((38, lb.lx, lb.ly), np.float32)
    st[:37] = f
    return torch.from_numpy(st)


@pytest.mark.parametrize("precision", ["fp64", "fp32s", "fp32c", "fp32l"])
@pytest.mark.parametrize("case", ["rho", "T"])
def test_check_finite_reports_unphysical_finite_state(precision, case):
    """check_finite's rho <= 0 and T <= 0 branches: a uniform, finite state
    with negative density (f = -w), or with positive density and negative
    temperature (rest population 1, the four nearest -0.01 each), is its own
    collision fixed point on a periodic lattice without gravity; the scan
    after one step must report it while every population is finite."""
    cx, cy, w, _ = oracle.model()
    if case == "rho":
        f37 = -w
    else:
        f37 = np.where(np.abs(cx) + np.abs(cy) == 1, -0.01, 0.0)
        f37[18] = 1.0
    lx, ly = 24, 20
    lb, _ = make(lx, ly, precision=precision, ybc="periodic", g=(0.0, 0.0), check_finite=1)
    lb.set_state(_uniform_state(lb, f37))
    with pytest.raises(lbmod.LBError) as ei:
        lb.step(1)
    assert ei.value.code == -5
    pops = host(lb.populations())
    assert np.isfinite(pops).all()
    rho, _, _, T = [host(t) for t in lb.moments()]
    if case == "rho":
        assert (rho <= 0).all()
    else:
        assert (rho > 0).all() and (T <= 0).all()


def test_resume_from_checkpoint_is_bit_identical():
    lx, ly = 64, 64
    lb, _ = make(lx, ly)
    lb.step(5)
    ck = lb.get_state().clone()
    lb.step(5)
    after = lb.get_state().clone()
    lb.set_state(ck)
    lb.step(5)
    assert torch.equal(lb.get_state(), after)


def test_zero_steps_leave_the_state_unchanged():
    lb, _ = make(40, 30)
    before = lb.get_state().clone()
    lb.step(0)
    lb.step_record(0, lb.new_tape(1))
    assert torch.equal(lb.get_state(), before)


@pytest.mark.parametrize("T_wall", [0.5, 1.0, 1.5])
@pytest.mark.parametrize("kernel", ["fused", "split"])
def test_rest_state_at_the_wall_temperature_is_a_fixed_point(kernel, T_wall):
    """rho = 1, u = 0, T = T_wall everywhere, g = 0, both walls at T_wall: the
    equilibrium gathered by propagate, completed by the walls and relaxed by
    collide is the same equilibrium, step after step, to accumulated rounding
    (the oracle itself drifts by 1.4e-14 to 3.6e-14 over these 25 steps)."""
    lx, ly = 40, 36
    ones = np.ones((lx, ly))
    lb = lbmod.LB(lx, ly, ones, 0 * ones, 0 * ones, T_wall * ones, kernel=kernel, g=(0.0, 0.0),
                  t_bottom=T_wall, t_top=T_wall)
    f0 = host(lb.populations())
    lb.step(25)
    f = host(lb.populations())
    assert np.abs(f - f0).max() <= 1e-13 * np.abs(f0).max()


def bits(t):
    """The raw bits of a state tensor (the packed FP16 references of the
    local-reference form need not be valid FP32 numbers)."""
    return t.view(torch.int64 if t.dtype == torch.float64 else torch.int32)


@pytest.mark.parametrize("precision", ["fp64", "fp32s", "fp32c", "fp32l"])
def test_checkpoint_file_round_trip(tmp_path, precision):
    """save_checkpoint / load_checkpoint: the resumed run is bit-identical."""
    lb, fields = make(48, 40, precision=precision)
    lb.step(7)
    path = str(tmp_path / "ck.npz")
    lb.save_checkpoint(path)
    lb.step(9)
    after = lb.get_state().clone()
    other, _ = make(48, 40, precision=precision, seed=99)
    meta = other.load_checkpoint(path)
    assert meta["precision"] == precision
    other.step(9)
    assert torch.equal(bits(other.get_state()), bits(after))
    wrong, _ = make(40, 48, precision=precision)
    with pytest.raises(ValueError):
        wrong.load_checkpoint(path)


def test_state_arguments_are_checked():
    lb, _ = make(20, 16)
    with pytest.raises(ValueError):
        lb.set_state(torch.zeros((37, 20, 15), dtype=torch.float64))
    with pytest.raises(ValueError):
        lb.set_state(torch.zeros((37, 20, 16), dtype=torch.float32))
    with pytest.raises(ValueError):
        lb.get_state(out=torch.empty((37, 20, 16), dtype=torch.float64))  # host tensor
    with pytest.raises(ValueError):
        lb.step_record(2, torch.empty((2, 4, 20, 16), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        lb.adjoint_step(torch.empty((4, 20, 15), dtype=torch.float64, device="cuda"),
                        lb.new_lambda(), lb.new_lambda())
