"""Hydrodynamic pins of the oracle: a shear wave and a sound wave.

Both are closed-form results of the continuum limit of Eq. (1): a transverse
wave u_y = U0 sin(k x) decays as exp(-nu k^2 t) with nu = (tau - 1/2) T, and a
longitudinal wave oscillates at the adiabatic sound speed c_s = sqrt(gamma T)
with gamma = (D + 2) / D = 2 for the perfect gas p = rho T of Sec. 2.  Speeds
and T are in the units of the velocities c_l = r e_l, so in sites per step
they are divided by r (and nu by r^2).  Walls are replaced by periodic y.
"""

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def r():
    return oracle.model()[3]


def _wave_init(lx, ly, T, ux=None, uy=None):
    one = np.ones((lx, ly))
    return oracle.init_feq(one, one * 0 if ux is None else ux, one * 0 if uy is None else uy, T * one)


@pytest.mark.parametrize("T", [0.6, 1.0, 1.4])
def test_shear_wave_viscosity(r, T):
    lx, ly, tau, U0 = 64, 4, 0.7, 1e-3
    k = 2 * np.pi / lx
    x = np.arange(lx)[:, None] * np.ones((1, ly))
    f = _wave_init(lx, ly, T, uy=U0 * np.sin(k * x))
    P = oracle.Params(tau=tau, gx=0, gy=0, ybc=1, regularize=1)
    nu_theory = (tau - 0.5) * T / r ** 2
    s = np.sin(k * np.arange(lx))

    def amp(f):
        return 2 * np.mean(oracle.moments(f)[2].mean(axis=1) * s)

    n1 = 100
    n2 = n1 + int(0.5 / (nu_theory * k * k))
    f1 = oracle.run(f, P, n1)
    f2 = oracle.run(f1, P, n2 - n1)
    nu = np.log(amp(f1) / amp(f2)) / (n2 - n1) / k ** 2
    assert abs(nu / nu_theory - 1) < 5e-3, (nu, nu_theory)


@pytest.mark.parametrize("T", [0.6, 1.0, 1.4])
def test_adiabatic_sound_speed(r, T):
    lx, ly, tau, U0 = 64, 4, 0.7, 1e-4
    k = 2 * np.pi / lx
    x = np.arange(lx)[:, None] * np.ones((1, ly))
    f = _wave_init(lx, ly, T, ux=U0 * np.sin(k * x))
    P = oracle.Params(tau=tau, gx=0, gy=0, ybc=1, regularize=1)
    cs_theory = np.sqrt(2 * T) / r
    s = np.sin(k * np.arange(lx))
    amps = []
    for _ in range(int(2.2 * 2 * np.pi / (cs_theory * k))):
        amps.append(2 * np.mean(oracle.moments(f)[1].mean(axis=1) * s))
        f = oracle.run(f, P, 1)
    a = np.array(amps)
    zeros = [i + a[i] / (a[i] - a[i + 1]) for i in range(len(a) - 1) if a[i] * a[i + 1] < 0]
    assert len(zeros) >= 3
    cs = 2 * np.pi / (2 * np.mean(np.diff(zeros)) * k)
    assert abs(cs / cs_theory - 1) < 2e-3, (cs, cs_theory)
