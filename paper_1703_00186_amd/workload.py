"""Seeded synthetic Rayleigh-Taylor initial conditions.

Shared by the tests, the benchmark and the smoke check, and by both sides of a
parity comparison (the GPU library and the CPU oracle receive the same
arrays).  This module holds no lattice-Boltzmann arithmetic: it only builds
the initial macroscopic fields (rho0, u0, T0) on an Lx x Ly lattice, x-major
``[Lx, Ly]`` float64 (or complex128 when amplitudes are complex, for
complex-step differentiation of the initial condition).

Recipe (lattice units throughout):
  * interface height  y_i(x) = (Ly - 1)/2 + delta(x), with either
      delta(x) = 2 sin(2 pi x / Lx)                          ("sinusoid"), or
      delta(x) = sum_{k=1..16} a_k cos(2 pi k x / Lx + phi_k)  ("multimode"),
    a_k ~ U[-0.25, 0.25], phi_k ~ U[0, 2 pi);
  * background temperature, hot below and cold above,
      Tbar = T_top + (T_bottom - T_top) / (1 + exp(y - y_i))
    (a tanh profile of width 2 sites);
  * T = Tbar + eta, eta ~ U[-1e-3, 1e-3] drawn in C order over (x, y);
  * u = 0;
  * rho = p / Tbar with p hydrostatic under gravity g along -y,
      p(x, y) = exp(-G_SCALE g int_{y_i(x)}^{y} dy' / Tbar(x, y')),
    evaluated in closed form, so p = 1 and rho = 1 on the interface
    ("uniform" mode keeps rho = 1 everywhere instead).  T and g are in the
    model's velocity units, in which a hop of one site per step has speed
    about 1.19698; G_SCALE converts the pressure gradient to one per site.
All draws come from numpy's PCG64 generator with the given seed: first the 16
amplitudes, then the 16 phases (multimode only), then eta.
"""

from __future__ import annotations

import numpy as np

N_MODES = 16
G_SCALE = 1.19698  # model velocity units per (lattice site / time step)


def config_seed(k: int) -> int:
    """Seed 170300 + k of workload k: 1 parity 256 x 128, 2 speed 1920 x 2048,
    3 FP32 precision 4096 x 4096, 4 adjoint 512 x 512, 5 production
    8192 x 4096."""
    return 170300 + int(k)


def draw_modes(seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(-0.25, 0.25, N_MODES)
    phi = rng.uniform(0.0, 2.0 * np.pi, N_MODES)
    return a, phi, rng


def _log_tb_plus_tt_exp(z, t_bottom, t_top):
    """log(T_b + T_t e^z), evaluated without overflow for real or complex z."""
    z = np.asarray(z)
    pos = np.real(z) > 0
    out = np.empty(z.shape, dtype=np.result_type(z, np.float64))
    zp = z[pos]
    out[pos] = zp + np.log(t_top + t_bottom * np.exp(-zp))
    zn = z[~pos]
    out[~pos] = np.log(t_bottom + t_top * np.exp(zn))
    return out


def _inv_one_plus_exp(z):
    """1 / (1 + e^z) without overflow, for real or complex z."""
    z = np.asarray(z)
    pos = np.real(z) > 0
    out = np.empty(z.shape, dtype=np.result_type(z, np.float64))
    e = np.exp(-z[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(z[~pos]))
    return out


def _hydrostatic_integral(z, t_bottom, t_top):
    """F(z) with F'(z) = 1 / Tbar(z), Tbar(z) = T_t + (T_b - T_t)/(1 + e^z)."""
    return z / t_bottom + (1.0 / t_top - 1.0 / t_bottom) * _log_tb_plus_tt_exp(z, t_bottom, t_top)


def rt_fields(lx: int, ly: int, *, seed: int, mode: str = "sinusoid",
              t_bottom: float = 1.5, t_top: float = 0.5, g: float = 1e-4,
              noise: float = 1e-3, amplitudes=None):
    """Returns (rho0, ux0, uy0, T0, info) for a Rayleigh-Taylor lattice.

    ``amplitudes`` overrides the 16 drawn a_k (multimode); it may be complex.
    ``info`` holds the amplitudes and phases that were used.
    """
    if mode not in ("sinusoid", "multimode", "uniform"):
        raise ValueError("mode must be sinusoid, multimode or uniform")
    a, phi, rng = draw_modes(seed)
    if mode != "multimode":
        rng = np.random.Generator(np.random.PCG64(seed))
    eta = rng.uniform(-noise, noise, (lx, ly)) if noise > 0 else np.zeros((lx, ly))
    x = np.arange(lx, dtype=np.float64)[:, None]
    y = np.arange(ly, dtype=np.float64)[None, :]
    if mode == "multimode":
        amp = a if amplitudes is None else np.asarray(amplitudes)
        k = np.arange(1, N_MODES + 1, dtype=np.float64)
        delta = (amp[None, :] * np.cos(2 * np.pi * k[None, :] * x / lx + phi[None, :])).sum(axis=1)
        delta = delta[:, None]
    else:
        amp = None
        delta = 2.0 * np.sin(2 * np.pi * x / lx)
    yi = (ly - 1) / 2.0 + delta
    z = y - yi
    tbar = t_top + (t_bottom - t_top) * _inv_one_plus_exp(z)
    if mode == "uniform":
        rho = np.ones_like(tbar)
    else:
        F0 = _hydrostatic_integral(np.zeros(1), t_bottom, t_top)[0]
        p = np.exp(-G_SCALE * g * (_hydrostatic_integral(z, t_bottom, t_top) - F0))
        rho = p / tbar
    T = tbar + eta
    ux = np.zeros_like(rho)
    uy = np.zeros_like(rho)
    info = {"amplitudes": amp, "phases": phi if mode == "multimode" else None,
            "seed": seed, "mode": mode}
    return (np.ascontiguousarray(rho), np.ascontiguousarray(ux),
            np.ascontiguousarray(uy), np.ascontiguousarray(T), info)


def amplitude_gradient(lx: int, ly: int, grad_rho, grad_T, *, seed: int,
                       t_bottom: float = 1.5, t_top: float = 0.5, g: float = 1e-4,
                       noise: float = 1e-3, h: float = 1e-30) -> np.ndarray:
    """Chains dL/d(rho0, T0) to dL/da_k for the 16 multimode amplitudes.

    d(rho0, T0)/da_k is taken by complex step on the initial condition itself
    (exact to rounding); u0 does not depend on a_k.
    """
    a, _, _ = draw_modes(seed)
    out = np.zeros(N_MODES)
    for k in range(N_MODES):
        ak = a.astype(np.complex128)
        ak[k] += 1j * h
        rho, _, _, T, _ = rt_fields(lx, ly, seed=seed, mode="multimode", t_bottom=t_bottom,
                                    t_top=t_top, g=g, noise=noise, amplitudes=ak)
        out[k] = (np.sum(grad_rho * rho.imag) + np.sum(grad_T * T.imag)) / h
    return out
