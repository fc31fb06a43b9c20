"""Pins of the oracle's propagate and bc (Sec. 2; Sec. 4, Fig. 4)."""

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def model():
    return oracle.model()


def test_propagate_moves_each_population_by_its_hop(model):
    cx, cy, _, _ = model
    lx, ly = 11, 9
    for l in range(37):
        f = np.zeros((37, lx, ly))
        f[l, 2, 4] = 1.0
        ft = oracle.propagate(f, ybc=1)
        dest = np.argwhere(ft[l] == 1.0)
        assert dest.tolist() == [[(2 + cx[l]) % lx, (4 + cy[l]) % ly]]
        assert ft.sum() == 1.0


def test_propagate_is_a_permutation_bitwise():
    rng = np.random.default_rng(0)
    f = rng.standard_normal((37, 13, 10))
    ft = oracle.propagate(f, ybc=1)
    for l in range(37):
        assert np.array_equal(np.sort(ft[l].ravel()), np.sort(f[l].ravel()))


def test_propagate_there_and_back_is_identity():
    """Hop by +c, swap l <-> 36-l, hop again, swap back: the original bits."""
    rng = np.random.default_rng(1)
    f = rng.standard_normal((37, 8, 7))
    back = oracle.propagate(oracle.propagate(f, ybc=1)[::-1], ybc=1)[::-1]
    assert np.array_equal(back, f)


def test_walls_leave_15_8_3_unknowns(model):
    f = np.ones((37, 6, 12))
    ft = oracle.propagate(f, ybc=0)
    nan = np.isnan(ft).sum(axis=0)
    assert nan[:, 0].tolist() == [15] * 6 and nan[:, 1].tolist() == [8] * 6
    assert nan[:, 2].tolist() == [3] * 6 and nan[:, 3:9].sum() == 0
    assert nan[:, -1].tolist() == [15] * 6 and nan[:, -2].tolist() == [8] * 6
    assert nan[:, -3].tolist() == [3] * 6


def test_rest_state_at_wall_temperature_is_fixed_point():
    lx, ly = 8, 12
    T = 0.8
    one = np.ones((lx, ly))
    f = oracle.init_feq(1.3 * one, 0 * one, 0 * one, T * one)
    ft = oracle.bc(oracle.propagate(f, ybc=0), T, T)
    assert np.allclose(ft, f, rtol=0, atol=1e-15)
    P = oracle.Params(tau=0.7, gx=0, gy=0, t_bottom=T, t_top=T)
    assert np.allclose(oracle.run(f, P, 5), f, rtol=0, atol=1e-14)


def test_bc_emits_scaled_wall_maxwellian(model):
    """Unknown populations are rho_w f^eq(1, 0, T_wall) with the arriving mass kept."""
    rng = np.random.default_rng(2)
    lx, ly = 7, 10
    f = 1 + 0.1 * rng.standard_normal((37, lx, ly))
    ft = oracle.propagate(f, ybc=0)
    unknown = np.isnan(ft)
    out = oracle.bc(ft, 1.5, 0.5)
    assert np.isfinite(out).all()
    assert np.array_equal(out[~unknown], ft[~unknown])
    for y, Tw in [(0, 1.5), (1, 1.5), (2, 1.5), (ly - 1, 0.5), (ly - 2, 0.5), (ly - 3, 0.5)]:
        v = oracle.equilibrium(1.0, 0.0, 0.0, Tw)
        for x in range(lx):
            U = unknown[:, x, y]
            K = ~U
            rho_w = out[U, x, y] / v[U]
            assert np.allclose(rho_w, rho_w[0], rtol=1e-14)
            assert abs(ft[K, x, y].sum() - rho_w[0] * v[K].sum()) < 1e-13


def test_wall_maxwellians_and_bc_denominators(model):
    """Consequences of the units reading (velocities c_l = r e_l, T = 1 the
    quadrature's temperature) for the walls of the workloads (T_bottom 1.5,
    T_top 0.5): the cold wall's Maxwellian f^eq(1, 0, 0.5) has 12 negative
    entries (min v/w = -0.228: the 4th-order expansion far from T = 1), yet
    the denominators sum_K v of the bc, over the populations known at each
    wall row, stay at 0.70 or more; a change of units or wall temperatures
    that brought one near zero would make rho_w ill-conditioned."""
    cx, cy, w, _ = model
    ly = 12
    for T_wall, neg in ((1.5, 0), (0.5, 12)):
        v = oracle.equilibrium(1.0, 0.0, 0.0, T_wall)
        assert int((v < 0).sum()) == neg
        for y in (0, 1, 2, ly - 3, ly - 2, ly - 1):
            known = (y - cy >= 0) & (y - cy < ly)
            assert v[known].sum() >= 0.5, (T_wall, y, v[known].sum())
    v = oracle.equilibrium(1.0, 0.0, 0.0, 0.5)
    assert abs((v / w).min() - (-0.228)) < 1e-3
