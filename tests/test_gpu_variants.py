"""The alternative split-stage kernels (kernel = "split_lds", "split_wide",
"split_mfma") against the CPU oracle, through the C ABI: propagate staged
through LDS or with 16-byte accesses bit-exact, the FP64 collide on the
matrix cores within 1e-13 of the value scale, and whole Rayleigh-Taylor steps
within the FP64 tolerance of the extended-precision oracle.  Sizes span
several tiles with ragged tails, and the minimum lattice."""

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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def make(lx, ly, **kw):
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=170301)
    return lbmod.LB(lx, ly, rho, ux, uy, T, **kw), (rho, ux, uy, T)


@pytest.mark.parametrize("shape", [(45, 300), (7, 1031), (6, 6)])
@pytest.mark.parametrize("ybc", ["walls", "periodic"])
@pytest.mark.parametrize("layout", ["soa", "column"])
@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
@pytest.mark.parametrize("kernel", ["split_lds", "split_wide"])
def test_propagate_variants_bit_exact(kernel, precision, layout, ybc, shape):
    """Random stored values (FP64, or FP32 for the shifted form) moved by the
    alternative propagate: every slot with a source inside the lattice equals
    the oracle's propagate exactly (the LDS tiles are 256 rows, the 16-byte
    tiles 512 / 1024 rows: 300 and 1031 leave ragged tails)."""
    lx, ly = shape
    lb, _ = make(lx, ly, kernel=kernel, precision=precision, layout=layout, ybc=ybc)
    rng = np.random.default_rng(12)
    f0 = rng.standard_normal((37, lx, ly))
    if precision == "fp32s":
        f0 = f0.astype(np.float32)
    lb.set_state(torch.from_numpy(f0))
    lb.propagate()
    got = host(lb.get_scratch())
    ref = oracle.propagate(f0.astype(np.float64), ybc=1 if ybc == "periodic" else 0)
    known = ~np.isnan(ref)
    assert np.array_equal(got[known].astype(np.float64), ref[known])
    if ybc == "periodic":
        assert known.all()


@pytest.mark.parametrize("shape", [(33, 200), (7, 65), (6, 6)])
@pytest.mark.parametrize("layout", ["soa", "column"])
@pytest.mark.parametrize("regularize", [1, 0])
def test_collide_mfma(regularize, layout, shape):
    """The matrix-core collide of a post-bc state (3 Rayleigh-Taylor steps,
    then populations perturbed by 1e-3 of their weight so that every Hermite
    mode, the ghost modes too, is present), with gravity along x and y,
    against the oracle's collide."""
    lx, ly = shape
    lb, fields = make(lx, ly, kernel="split_mfma", layout=layout, regularize=regularize,
                      g=(2e-3, -1e-3))
    P = oparams(regularize=regularize, gx=2e-3, gy=-1e-3)
    f = oracle.run(oracle.init_feq(*fields), P, 3)
    ft = oracle.bc(oracle.propagate(f, ybc=0), 1.5, 0.5)
    _, _, w, _ = oracle.model()
    rng = np.random.default_rng(3)
    ft = ft + 1e-3 * w[:, None, None] * rng.uniform(-1.0, 1.0, ft.shape)
    lb.set_scratch(torch.from_numpy(ft))
    lb.collide()
    got = host(lb.get_state())
    ref = oracle.collide(ft, P)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("mfma collide %s reg=%d %s: %.2e" % (layout, regularize, shape, err))
    assert err <= 1e-13


@pytest.fixture(scope="module")
def extended_256x128_50():
    lx, ly = 256, 128
    fields = workload.rt_fields(lx, ly, seed=170301)[:4]
    return oracle.run_moments_extended(oracle.init_feq(*fields), oparams(), 50)


@pytest.mark.parametrize("layout", ["soa", "column"])
@pytest.mark.parametrize("kernel", ["split_lds", "split_wide", "split_mfma"])
def test_variant_steps_rt_256x128_50(kernel, layout, extended_256x128_50):
    """50 whole steps with the alternative kernel in place: every field within
    1e-12 of the extended-precision oracle (u as max|du| / max|u|); the
    propagate variants give the split path's state bit for bit."""
    lx, ly = 256, 128
    lb, _ = make(lx, ly, kernel=kernel, layout=layout)
    lb.step(50)
    errs = field_errors([host(t) for t in lb.moments()], extended_256x128_50)
    print("%s %s vs extended oracle:" % (kernel, layout), errs)
    assert worst(errs) <= 1e-12, errs
    if kernel != "split_mfma":
        ref, _ = make(lx, ly, kernel="split", layout=layout)
        ref.step(50)
        assert torch.equal(lb.get_state(), ref.get_state())


@pytest.mark.parametrize("kernel", ["split_lds", "split_wide", "split_mfma"])
def test_variant_periodic_bgk(kernel):
    lx, ly = 64, 48
    lb, fields = make(lx, ly, kernel=kernel, ybc="periodic", regularize=0, g=(1e-3, -2e-3))
    lb.step(20)
    P = oparams(ybc=1, regularize=0, gx=1e-3, gy=-2e-3)
    f_ref = oracle.run(oracle.init_feq(*fields), P, 20)
    f_gpu = host(lb.populations())
    assert np.abs(f_gpu - f_ref).max() <= 1e-12 * np.abs(f_ref).max()


def test_mfma_rejects_fp32():
    with pytest.raises(lbmod.LBError) as ei:
        make(16, 16, kernel="split_mfma", precision="fp32s")
    assert ei.value.code == -1
