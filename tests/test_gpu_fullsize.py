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
