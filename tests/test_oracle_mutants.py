"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle source (a dropped term,
a wrong sign, index or factor, a transposed operand, an off-by-one), builds it,
and runs the pin suite against that build in a subprocess: at least one pin
must fail.  The real oracle is never modified.
"""

import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "d2q37_oracle.cpp")
PINS = ["tests/test_oracle_model.py", "tests/test_oracle_collide.py",
        "tests/test_oracle_stream.py", "tests/test_oracle_physics.py",
        "tests/test_oracle_derived.py", "tests/test_oracle_extended.py"]

MUTANTS = {
    "equilibrium_drops_theta_squared": (
        "3.0 * th * th * (x2 * x2 - 8.0 * x2 + 8.0)", "0.0 * th * th * (x2 * x2 - 8.0 * x2 + 8.0)"),
    "equilibrium_third_order_sign": (
        "xu * (xu * xu - 3.0 * U2 + 3.0 * th", "xu * (xu * xu + 3.0 * U2 + 3.0 * th"),
    "equilibrium_reference_temperature": ("const S th = T - 1.0;", "const S th = T - 0.99;"),
    "forcing_without_tau": ("const S uxs = ux + tau * P.gx;", "const S uxs = ux + P.gx;"),
    "forcing_temperature_sign": ("tau * (1.0 - tau) * (P.gx", "tau * (1.0 + tau) * (P.gx"),
    "projection_factorial_index": (
        "/ (factorial(p) * factorial(q))", "/ (factorial(p) * factorial(p))"),
    "projection_transposed_hermite": (
        "a += h[m] * Consts<S>::H(m, p, q);", "a += h[m] * Consts<S>::H(m, q, p);"),
    "hermite_2_missing_constant": ("case 2: return x * x - 1;", "case 2: return x * x;"),
    "temperature_wrong_dimension": (
        "T = (e - rho * (ux * ux + uy * uy)) / (2.0 * rho);",
        "T = (e - rho * (ux * ux + uy * uy)) / (3.0 * rho);"),
    "propagate_wrong_direction": (
        "const int xs = wrap(x - M.cx[l], lx);", "const int xs = wrap(x + M.cx[l], lx);"),
    "bc_walls_swapped": ("const S* v = (y < 3) ? vb : vt;", "const S* v = (y < 3) ? vt : vb;"),
    "bc_off_by_one_unknown": (
        "unknown[l] = (ys < 0 || ys >= ly);", "unknown[l] = (ys < 0 || ys > ly);"),
    "bgk_rate_inverted": ("const S omega = S(1.0) / S(tau);", "const S omega = S(tau);"),
    "kinetic_energy_drops_half": (
        "ke += 0.5 * rho * (ux * ux + uy * uy);", "ke += rho * (ux * ux + uy * uy);"),
    "step_sites_reversed_gather": (
        "const int xs_ = wrap(x - M.cx[l], lx);", "const int xs_ = wrap(x + M.cx[l], lx);"),
    "extended_run_fp64_weights": (
        "static long double w(int l) { return model().wx[l]; }",
        "static long double w(int l) { return model().w[l]; }"),
    "bgk_weights_not_summing_to_one": (
        "const S keep = S(1.0) - omega;", "const S keep = S(1.0 - 1.0 / 0.7000000000000001);"),
    "quadrature_redundant_condition": (
        "{4, 2}, {8, 0}, {6, 2}, {4, 4}};", "{4, 2}, {8, 0}, {6, 2}, {2, 6}};"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation target not unique: " + old
    src = tmp_path / "mutant.cpp"
    src.write_text(text.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    oracle.compile_library(str(src), lib)
    env = dict(os.environ, ORACLE_LIBRARY=lib, OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
                         + PINS, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, "no pin failed for mutant " + name + "\n" + res.stdout[-2000:]
