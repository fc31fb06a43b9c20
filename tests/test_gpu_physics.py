"""Hydrodynamics of the GPU step itself, at sizes the oracle is not run at.

The continuum limit of Eq. (1) fixes two numbers: a transverse wave
u_y = U0 sin(k x) decays as exp(-nu k^2 t) with nu = (tau - 1/2) T, and a
longitudinal wave travels at the adiabatic sound speed sqrt(2 T) (gamma = 2
for the perfect gas p = rho T, D = 2).  Speeds and T are in the units of
c_l = r e_l, so in sites per step they are divided by r (nu by r^2).  These
hold at any lattice size; here they are checked on the GPU path directly,
on lattices 4-8 times longer than the oracle's, in FP64 and in the FP32
shifted form.  Walls are replaced by periodic y.
"""

import numpy as np
import pytest

import oracle
from helpers import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1703_00186_amd.lb import LB


@pytest.fixture(scope="module")
def r():
    return oracle.model()[3]


def wave(lx, ly, T, precision, tau, ux=None, uy=None):
    one = np.ones((lx, ly))
    return LB(lx, ly, one, one * 0 if ux is None else ux, one * 0 if uy is None else uy, T * one,
              precision=precision, ybc="periodic", g=(0.0, 0.0), tau=tau)


def mode_amplitude(lb, comp, k):
    torch.cuda.synchronize()
    u = lb.moments()[comp].mean(dim=1).cpu().numpy()
    return 2 * np.mean(u * np.sin(k * np.arange(lb.lx)))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-3), ("fp32s", 5e-3), ("fp32c", 1e-3), ("fp32l", 1e-3)])
@pytest.mark.parametrize("lx,T", [(256, 1.0), (512, 0.6)])
def test_shear_wave_viscosity(r, lx, T, precision, tol):
    ly, tau, U0 = 8, 0.7, 1e-3
    k = 2 * np.pi / lx
    x = np.arange(lx)[:, None] * np.ones((1, ly))
    lb = wave(lx, ly, T, precision, tau, uy=U0 * np.sin(k * x))
    nu_theory = (tau - 0.5) * T / r ** 2
    lb.step(200)
    a1 = mode_amplitude(lb, 2, k)
    n = int(0.5 / (nu_theory * k * k))
    lb.step(n)
    a2 = mode_amplitude(lb, 2, k)
    nu = np.log(a1 / a2) / n / k ** 2
    print("%s lx=%d T=%.1f: nu %.6f, theory %.6f" % (precision, lx, T, nu, nu_theory))
    assert abs(nu / nu_theory - 1) < tol, (nu, nu_theory)


@pytest.mark.parametrize("T", [0.6, 1.4])
def test_adiabatic_sound_speed(r, T):
    lx, ly, tau, U0 = 256, 8, 0.7, 1e-4
    k = 2 * np.pi / lx
    x = np.arange(lx)[:, None] * np.ones((1, ly))
    lb = wave(lx, ly, T, "fp64", tau, ux=U0 * np.sin(k * x))
    cs_theory = np.sqrt(2 * T) / r
    amps = []
    for _ in range(int(2.2 * 2 * np.pi / (cs_theory * k))):
        amps.append(mode_amplitude(lb, 1, k))
        lb.step(1)
    a = np.array(amps)
    zeros = [i + a[i] / (a[i] - a[i + 1]) for i in range(len(a) - 1) if a[i] * a[i + 1] < 0]
    assert len(zeros) >= 3
    cs = 2 * np.pi / (2 * np.mean(np.diff(zeros)) * k)
    print("T=%.1f: c_s %.6f, theory %.6f" % (T, cs, cs_theory))
    assert abs(cs / cs_theory - 1) < 2e-4, (cs, cs_theory)
