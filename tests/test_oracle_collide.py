"""Pins of the oracle's equilibrium and collision (Sec. 2, Eqs. (1)-(2)).

The checks come from the mathematics the model must satisfy, not from the
oracle's own formulas: Gaussian raw moments, conservation laws, the fixed
point of the relaxation, the exact momentum/energy input of the forcing, and
the removal of a mode orthogonal to the Hermite basis.
"""

import numpy as np
import pytest
from numpy.polynomial import hermite_e as H

import oracle


@pytest.fixture(scope="module")
def model():
    return oracle.model()


def raw_gauss(n, mu, var):
    """E[X^n] for X ~ N(mu, var), n <= 4."""
    return [1.0, mu, mu * mu + var, mu ** 3 + 3 * mu * var,
            mu ** 4 + 6 * mu * mu * var + 3 * var * var][n]


def conserved(f, model):
    cx, cy, _, r = model
    c_x, c_y = r * cx, r * cy
    return np.array([f.sum(), (c_x * f).sum(), (c_y * f).sum(), ((c_x ** 2 + c_y ** 2) * f).sum()])


def test_equilibrium_reference_state(model):
    """At rest and T = 1 the equilibrium is exactly the weight times rho."""
    _, _, w, _ = model
    for rho in (0.5, 1.0, 2.25):
        assert np.array_equal(oracle.equilibrium(rho, 0.0, 0.0, 1.0), w * rho)


@pytest.mark.parametrize("state", [(1.0, 0.0, 0.0, 0.5), (0.8, 0.05, -0.03, 1.5),
                                   (2.0, -0.1, 0.2, 0.7), (1.3, 0.3, 0.1, 1.2)])
def test_equilibrium_gaussian_moments(model, state):
    """Moments of order <= 4 are those of rho N(u, T I) (degree-9 rule, order-4 f^eq)."""
    cx, cy, _, r = model
    rho, ux, uy, T = state
    feq = oracle.equilibrium(rho, ux, uy, T)
    c_x, c_y = r * cx, r * cy
    for p in range(5):
        for q in range(5 - p):
            got = np.sum(feq * c_x ** p * c_y ** q)
            want = rho * raw_gauss(p, ux, T) * raw_gauss(q, uy, T)
            assert abs(got - want) < 1e-13 * max(1.0, abs(want)), (p, q)


def test_macroscopic_of_equilibrium(model):
    """Eq. (2) applied to f^eq(rho, u, T) returns (rho, u, T)."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        st = np.array([rng.uniform(0.5, 2), rng.uniform(-.2, .2), rng.uniform(-.2, .2),
                       rng.uniform(0.5, 1.5)])
        got = oracle.macroscopic(oracle.equilibrium(*st))
        assert np.allclose(got, st, rtol=1e-14, atol=1e-15)


def perturbed_state(rng, model, amp=0.02):
    rho, ux, uy, T = rng.uniform(0.7, 1.5), rng.uniform(-.1, .1), rng.uniform(-.1, .1), rng.uniform(.6, 1.4)
    feq = oracle.equilibrium(rho, ux, uy, T)
    return feq * (1 + amp * rng.standard_normal(37))


@pytest.mark.parametrize("regularize", [0, 1])
def test_collision_conserves_mass_momentum_energy(model, regularize):
    rng = np.random.default_rng(2)
    P = oracle.Params(tau=0.7, gx=0.0, gy=0.0, regularize=regularize)
    for _ in range(20):
        f = perturbed_state(rng, model)
        out = oracle.collide_site(f, P)
        a, b = conserved(f, model), conserved(out, model)
        assert np.allclose(a, b, rtol=0, atol=2e-15 * 10), (a - b)
        assert not np.allclose(f, out)  # something did relax


@pytest.mark.parametrize("regularize", [0, 1])
def test_equilibrium_is_fixed_point(model, regularize):
    rng = np.random.default_rng(3)
    P = oracle.Params(tau=0.83, gx=0.0, gy=0.0, regularize=regularize)
    for _ in range(10):
        st = (rng.uniform(0.5, 2), rng.uniform(-.2, .2), rng.uniform(-.2, .2), rng.uniform(.5, 1.5))
        feq = oracle.equilibrium(*st)
        assert np.allclose(oracle.collide_site(feq, P), feq, rtol=0, atol=1e-15)


@pytest.mark.parametrize("regularize", [0, 1])
def test_forcing_increments(model, regularize):
    """One collision adds rho g to momentum and rho (2 u.g + |g|^2) to sum |c|^2 f."""
    rng = np.random.default_rng(4)
    g = np.array([0.013, -0.021])
    P = oracle.Params(tau=0.7, gx=g[0], gy=g[1], regularize=regularize)
    for _ in range(10):
        f = perturbed_state(rng, model)
        a, b = conserved(f, model), conserved(oracle.collide_site(f, P), model)
        rho, ux, uy, _ = oracle.macroscopic(f)
        u = np.array([ux, uy])
        d = b - a
        assert abs(d[0]) < 1e-14
        assert np.allclose(d[1:3], rho * g, rtol=1e-12, atol=1e-16)
        assert abs(d[3] - rho * (2 * u @ g + g @ g)) < 1e-13


def test_regularization_removes_non_hermite_mode(model):
    """A mode w He_5(c_x) is orthogonal to orders <= 4: projected away."""
    cx, cy, w, r = model
    rng = np.random.default_rng(5)
    ghost = w * H.hermeval(r * cx, [0, 0, 0, 0, 0, 1.0])
    Preg = oracle.Params(tau=0.7, gx=0, gy=-1e-3, regularize=1)
    Pbgk = oracle.Params(tau=0.7, gx=0, gy=-1e-3, regularize=0)
    f = perturbed_state(rng, model, amp=0.0)
    a = oracle.collide_site(f, Preg)
    b = oracle.collide_site(f + 0.01 * ghost, Preg)
    assert np.allclose(a, b, rtol=0, atol=1e-15)
    c = oracle.collide_site(f + 0.01 * ghost, Pbgk)
    assert np.abs(c - a).max() > 1e-4


def test_regularized_equals_bgk_inside_hermite_span(model):
    """For f in the order-<=4 span the projection is the identity (normalisation p! q!)."""
    rng = np.random.default_rng(6)
    for _ in range(10):
        f = oracle.equilibrium(rng.uniform(.6, 1.8), rng.uniform(-.2, .2), rng.uniform(-.2, .2),
                               rng.uniform(.5, 1.5))
        Preg = oracle.Params(tau=0.62, gx=1e-3, gy=-2e-3, regularize=1)
        Pbgk = oracle.Params(tau=0.62, gx=1e-3, gy=-2e-3, regularize=0)
        assert np.allclose(oracle.collide_site(f, Preg), oracle.collide_site(f, Pbgk),
                           rtol=0, atol=2e-15)


def test_bgk_relaxation_rate(model):
    """Eq. (1): with regularize = 0 and g = 0 the non-equilibrium part shrinks by (1 - 1/tau)."""
    rng = np.random.default_rng(7)
    tau = 0.9
    P = oracle.Params(tau=tau, gx=0, gy=0, regularize=0)
    f = perturbed_state(rng, model)
    feq = oracle.equilibrium(*oracle.macroscopic(f))
    out = oracle.collide_site(f, P)
    assert np.allclose(out - feq, (1 - 1 / tau) * (f - feq), rtol=0, atol=1e-16)
