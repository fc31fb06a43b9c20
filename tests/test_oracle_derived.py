"""Pins for the oracle routines that the GPU tests lean on beyond the single
site step: the lattice-wide collide, the per-site step used for sampled
full-size parity, the kinetic energy, and the complex-arithmetic versions
used for exact linearisations (complex step).

Each is pinned by mathematics the paper fixes, not by re-running itself:
conservation and the forcing increments of the collision, the fixed point of
the whole step, Eq. (2) moments of the equilibrium (rho u and
sum |c|^2 f^eq = rho |u|^2 + 2 rho T for any input), the closed-form
derivative of KE = |j|^2 / (2 rho), and central finite differences of the
real-arithmetic routines.
"""

import numpy as np
import pytest

import oracle
from paper_1703_00186_amd import workload

H = 1e-30  # complex step


def params(**kw):
    base = dict(tau=0.7, gx=0.0, gy=-1e-4, t_bottom=1.5, t_top=0.5, regularize=1, ybc=0)
    base.update(kw)
    return oracle.Params(**base)


def velocities():
    cx, cy, _, r = oracle.model()
    return r * cx[:, None, None], r * cy[:, None, None]


def pre_collision(lx=14, ly=12, seed=3):
    """A propagated, wall-completed state away from equilibrium."""
    f = workload.rt_fields(lx, ly, seed=seed)[:4]
    f = oracle.run(oracle.init_feq(*f), params(gx=2e-3, gy=-3e-3), 3)
    return oracle.bc(oracle.propagate(f, ybc=0), 1.5, 0.5)


def site_moments(f):
    c_x, c_y = velocities()
    return f.sum(0), (c_x * f).sum(0), (c_y * f).sum(0), ((c_x ** 2 + c_y ** 2) * f).sum(0)


@pytest.mark.parametrize("regularize", [1, 0])
def test_lattice_collide_conserves_and_forces_per_site(regularize):
    ft = pre_collision()
    rho, jx, jy, e = site_moments(ft)
    for gx, gy in ((0.0, 0.0), (2e-3, -3e-3)):
        out = oracle.collide(ft, params(gx=gx, gy=gy, regularize=regularize))
        rho2, jx2, jy2, e2 = site_moments(out)
        ux, uy = jx / rho, jy / rho
        assert np.abs(rho2 - rho).max() <= 1e-14
        assert np.abs(jx2 - (jx + rho * gx)).max() <= 1e-14
        assert np.abs(jy2 - (jy + rho * gy)).max() <= 1e-14
        de = rho * (2 * (ux * gx + uy * gy) + gx * gx + gy * gy)
        assert np.abs(e2 - (e + de)).max() <= 1e-13


def test_lattice_collide_is_the_site_collision_everywhere():
    ft = pre_collision()
    P = params(gx=1e-3)
    out = oracle.collide(ft, P)
    for x, y in ((0, 0), (5, 2), (13, 11), (7, 6)):
        assert np.array_equal(out[:, x, y], oracle.collide_site(ft[:, x, y], P))


def test_step_sites_fixed_point_and_agreement_with_the_step():
    lx, ly = 14, 12
    ones = np.ones((lx, ly))
    P = params(gy=0.0, t_bottom=1.5, t_top=1.5)
    f0 = oracle.init_feq(ones, 0 * ones, 0 * ones, 1.5 * ones)
    xs = np.array([0, 1, 13, 6, 2, 12])
    ys = np.array([0, 2, 11, 6, 9, 3])
    rest = oracle.step_sites(f0, P, xs, ys)
    assert np.abs(rest - f0[:, xs, ys].T).max() <= 1e-15
    f = oracle.run(oracle.init_feq(*workload.rt_fields(lx, ly, seed=4)[:4]), params(), 2)
    got = oracle.step_sites(f, params(gx=1e-3), xs, ys)
    ref = oracle.run(f, params(gx=1e-3), 1)[:, xs, ys].T
    assert np.array_equal(got, ref)


def test_kinetic_energy_of_an_equilibrium():
    rho, ux, uy, T, _ = workload.rt_fields(10, 9, seed=5)
    rng = np.random.default_rng(5)
    ux = ux + 0.05 * rng.standard_normal(ux.shape)
    uy = uy + 0.05 * rng.standard_normal(uy.shape)
    ke = oracle.kinetic_energy(oracle.init_feq(rho, ux, uy, T))
    ref = 0.5 * np.sum(rho * (ux ** 2 + uy ** 2))
    assert abs(ke - ref) <= 1e-13 * ref


def test_complex_routines_reduce_to_the_real_ones():
    rho, ux, uy, T, _ = workload.rt_fields(12, 10, seed=6)
    f = oracle.init_feq(rho, ux, uy, T)
    fc = oracle.init_feq_complex(rho, ux, uy, T)
    assert np.abs(fc.imag).max() == 0.0
    assert np.abs(fc.real - f).max() <= 1e-15 * np.abs(f).max()
    P = params(gx=1e-3)
    r = oracle.run(f, P, 4)
    rc = oracle.run_complex(f, P, 4)
    assert np.abs(rc.imag).max() == 0.0
    assert np.abs(rc.real - r).max() <= 1e-14 * np.abs(r).max()
    assert abs(oracle.kinetic_energy_complex(r).real - oracle.kinetic_energy(r)) <= \
        1e-14 * oracle.kinetic_energy(r)
    ke = oracle.ke_after_steps_complex(P, rho, ux, uy, T, 4)
    assert ke.imag == 0.0
    assert abs(ke.real - oracle.kinetic_energy(r)) <= 1e-14 * oracle.kinetic_energy(r)


def test_complex_step_of_the_equilibrium_matches_its_moments():
    """d/du_x sum c_x f^eq = rho, d/dT sum |c|^2 f^eq = 2 rho, d/drho f^eq = f^eq / rho."""
    rho, ux, uy, T, _ = workload.rt_fields(9, 8, seed=7)
    ux = ux + 0.03
    uy = uy - 0.02
    c_x, c_y = velocities()
    f = oracle.init_feq(rho, ux, uy, T)
    d_ux = oracle.init_feq_complex(rho, ux + 1j * H, uy, T).imag / H
    assert np.abs((c_x * d_ux).sum(0) - rho).max() <= 1e-13
    d_T = oracle.init_feq_complex(rho, ux, uy, T + 1j * H).imag / H
    assert np.abs(((c_x ** 2 + c_y ** 2) * d_T).sum(0) - 2 * rho).max() <= 1e-13
    d_rho = oracle.init_feq_complex(rho + 1j * H, ux, uy, T).imag / H
    assert np.abs(d_rho - f / rho).max() <= 1e-14


def test_complex_step_of_the_kinetic_energy_is_c_dot_u_minus_half_u2():
    f = oracle.run(oracle.init_feq(*workload.rt_fields(10, 8, seed=8)[:4]), params(gx=2e-3), 5)
    v = np.random.default_rng(8).standard_normal(f.shape)
    d = oracle.kinetic_energy_complex(f + 1j * H * v).imag / H
    rho, jx, jy, _ = site_moments(f)
    ux, uy = jx / rho, jy / rho
    c_x, c_y = velocities()
    grad = c_x * ux + c_y * uy - 0.5 * (ux ** 2 + uy ** 2)
    ref = np.sum(grad * v)
    assert abs(d - ref) <= 1e-12 * np.abs(grad * v).sum()


@pytest.mark.parametrize("ybc,regularize", [(0, 1), (1, 0)])
def test_complex_step_of_the_run_matches_central_differences(ybc, regularize):
    lx, ly, n = 12, 10, 3
    P = params(gx=1e-3, ybc=ybc, regularize=regularize)
    f = oracle.run(oracle.init_feq(*workload.rt_fields(lx, ly, seed=9)[:4]), P, 2)
    v = np.random.default_rng(9).standard_normal(f.shape)
    jv = oracle.run_complex(f + 1j * H * v, P, n).imag / H
    h = 1e-6  # truncation ~5e-10, rounding ~1e-10 of max |J v| here
    fd = (oracle.run(f + h * v, P, n) - oracle.run(f - h * v, P, n)) / (2 * h)
    assert np.abs(jv - fd).max() <= 1e-8 * np.abs(jv).max()


def test_complex_step_of_ke_after_steps_matches_central_differences():
    lx, ly, n = 12, 10, 6
    P = params()
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=10)
    dT = np.random.default_rng(10).standard_normal(T.shape) * 1e-2
    d = oracle.ke_after_steps_complex(P, rho, ux, uy, T + 1j * H * dT, n).imag / H
    h = 1e-3  # measured |CS - FD| / |CS|: 1.5e-10

    def ke(Tp):
        return oracle.kinetic_energy(oracle.run(oracle.init_feq(rho, ux, uy, Tp), P, n))

    fd = (ke(T + h * dT) - ke(T - h * dT)) / (2 * h)
    assert abs(d - fd) <= 1e-8 * abs(d)
