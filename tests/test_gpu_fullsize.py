"""Parity at the benchmark sizes, in the benchmark's launch configuration.

The whole lattice is too large for the oracle to step, so the oracle evaluates
one step at sampled sites only (propagate from the neighbours, bc, collide),
starting from the GPU's own state; the GPU's next state must agree at those
sites.  Samples: random sites, every wall row next to the periodic edges, and
the rows on both sides of the 256-row tile boundaries.
"""

import numpy as np
import pytest

import oracle
from helpers import gpu_available
from paper_1703_00186_amd import workload

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1703_00186_amd.lb import LB


def sample_sites(lx, ly, n_random=4096, seed=0):
    rng = np.random.default_rng(seed)
    xs = list(rng.integers(0, lx, n_random))
    ys = list(rng.integers(0, ly, n_random))
    for x in (0, 1, 2, 3, lx // 2, lx - 4, lx - 3, lx - 2, lx - 1):
        for y in (0, 1, 2, 3, ly - 4, ly - 3, ly - 2, ly - 1):
            xs.append(x)
            ys.append(y)
    for y in range(255, ly, 256):
        for x in (0, lx // 3, lx - 1):
            xs += [x, x]
            ys += [y, min(y + 1, ly - 1)]
    return np.array(xs, np.int32), np.array(ys, np.int32)


def oparams():
    return oracle.Params(tau=0.7, gx=0.0, gy=-1e-4, t_bottom=1.5, t_top=0.5)


@pytest.mark.parametrize("lx,ly,precision,mode,warm", [
    (1920, 2048, "fp64", "sinusoid", 50),
    (1920, 2048, "fp32c", "sinusoid", 50),
    (4096, 4096, "fp32s", "sinusoid", 20),
    (4096, 4096, "fp32c", "sinusoid", 20),
    (8192, 4096, "fp64", "multimode", 10),
    (8192, 4096, "fp32s", "multimode", 10),
    (8192, 4096, "fp32c", "multimode", 10),
    (8192, 4096, "fp32l", "multimode", 10),
])
def test_one_step_at_sampled_sites(lx, ly, precision, mode, warm):
    seed = workload.config_seed({2048: 2, 4096: 3 if lx == 4096 else 5}[ly])
    f = workload.rt_fields(lx, ly, seed=seed, mode=mode)[:4]
    lb = LB(lx, ly, *f, precision=precision)
    lb.step(warm)
    state = lb.populations().cpu().numpy()  # true populations, FP64
    lb.step(1)
    torch.cuda.synchronize()
    nxt = lb.populations().cpu().numpy()
    xs, ys = sample_sites(lx, ly)
    ref = oracle.step_sites(state, oparams(), xs, ys)
    got = nxt[:, xs, ys].T
    # FP64: rounding of one step (1e-13 of the scale); FP32 storage: one
    # rounding of each stored population (2^-24) plus the input's own
    # rounding; the FP32 collision adds its FP32 sums of the deviation from
    # the rest Maxwellian (a few 1e-7 of the largest population)
    tol = {"fp64": 1e-13, "fp32s": 3e-7, "fp32c": 1e-7, "fp32l": 1e-7}[precision]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("%s %dx%d one step at %d sampled sites: %.2e" % (precision, lx, ly, len(xs), err))
    assert err <= tol
    del lb
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kernel,precision", [
    ("split", "fp64"), ("split_lds", "fp64"), ("split_wide", "fp64"), ("split_mfma", "fp64"),
    ("split", "fp32s"), ("split_lds", "fp32s"), ("split_wide", "fp32s")])
def test_split_stage_kernels_at_sampled_sites(kernel, precision):
    """The split path and its alternative stage kernels on the 1920 x 2048
    lattice that `bench.py --variants` times: one step at sampled sites
    against the oracle."""
    lx, ly = 1920, 2048
    f = workload.rt_fields(lx, ly, seed=workload.config_seed(2))[:4]
    lb = LB(lx, ly, *f, precision=precision, kernel=kernel)
    lb.step(20)
    state = lb.populations().cpu().numpy()
    lb.step(1)
    torch.cuda.synchronize()
    nxt = lb.populations().cpu().numpy()
    xs, ys = sample_sites(lx, ly)
    ref = oracle.step_sites(state, oparams(), xs, ys)
    got = nxt[:, xs, ys].T
    tol = {"fp64": 1e-13, "fp32s": 3e-7}[precision]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("%s %s 1920x2048 one step at %d sampled sites: %.2e" % (kernel, precision, len(xs), err))
    assert err <= tol
    del lb
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", ["fp32c", "fp32l"])
def test_local_reference_form_at_maximum_column_height(precision):
    """A 6 x 4,194,304 lattice: a column of the local-reference form (38
    planes of 4,194,432 padded rows) is too tall for the 32-bit byte range of
    the buffer resources the column-layout kernel addresses through, so the
    step runs the globally addressed kernel; one step at sampled sites (the
    lattice's ends, every tile boundary of the first and last 64 tiles,
    random sites) against the oracle.  Uniform initial density (the
    hydrostatic one would span 1e-218 .. 1e72 over 4 million rows)."""
    lx, ly = 6, 1 << 22
    f = workload.rt_fields(lx, ly, seed=workload.config_seed(2), mode="uniform")[:4]
    lb = LB(lx, ly, *f, precision=precision)
    lb.step(3)
    state = lb.populations().cpu().numpy()
    lb.step(1)
    torch.cuda.synchronize()
    nxt = lb.populations().cpu().numpy()
    del lb
    torch.cuda.empty_cache()
    rng = np.random.default_rng(4)
    ys = list(rng.integers(0, ly, 4096)) + list(range(0, 8)) + list(range(ly - 8, ly))
    for y in list(range(255, 64 * 256, 256)) + list(range(ly - 64 * 256 + 255, ly, 256)):
        ys += [y, min(y + 1, ly - 1)]
    xs = np.array([i % lx for i in range(len(ys))], np.int32)
    ys = np.array(ys, np.int32)
    ref = oracle.step_sites(state, oparams(), xs, ys)
    got = nxt[:, xs, ys].T
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("%s %dx%d one step at %d sampled sites: %.2e" % (precision, lx, ly, len(xs), err))
    assert err <= 1e-7


@pytest.mark.parametrize("precision,layout,regularize", [
    ("fp64", "soa", 1), ("fp32c", "soa", 1), ("fp32l", "soa", 1),
    ("fp64", "column", 0), ("fp32c", "column", 0), ("fp32l", "column", 0)])
def test_layouts_and_bgk_at_sampled_sites(precision, layout, regularize):
    """The paper's SoA layout (the local-reference forms then run their
    globally addressed kernel) and plain BGK on the 1920 x 2048 lattice: one
    step at sampled sites against the oracle."""
    lx, ly = 1920, 2048
    f = workload.rt_fields(lx, ly, seed=workload.config_seed(2))[:4]
    lb = LB(lx, ly, *f, precision=precision, layout=layout, regularize=regularize)
    lb.step(20)
    state = lb.populations().cpu().numpy()
    lb.step(1)
    torch.cuda.synchronize()
    nxt = lb.populations().cpu().numpy()
    del lb
    torch.cuda.empty_cache()
    xs, ys = sample_sites(lx, ly)
    P = oracle.Params(tau=0.7, gx=0.0, gy=-1e-4, t_bottom=1.5, t_top=0.5, regularize=regularize)
    ref = oracle.step_sites(state, P, xs, ys)
    got = nxt[:, xs, ys].T
    tol = {"fp64": 1e-13, "fp32c": 1e-7, "fp32l": 1e-7}[precision]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("%s %s regularize=%d 1920x2048 one step at %d sampled sites: %.2e" % (
        precision, layout, regularize, len(xs), err))
    assert err <= tol
