"""CPU oracle for the D2Q37 thermal lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may load this package; the product path never does.

The arithmetic lives in ``d2q37_oracle.cpp`` (plain loops, FP64, no code shared
with the GPU library).  This module builds it with g++ and wraps it for NumPy.
Array conventions: populations ``f[37, Lx, Ly]`` (C order, y fastest), fields
``[Lx, Ly]``, all float64.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "d2q37_oracle.cpp")
_LIB = os.environ.get("ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle_d2q37.so")

Q = 37


def compile_library(src: str, out: str) -> str:
    """g++ -O2, no FMA contraction, no fast-math, OpenMP."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", src, "-o", tmp, "-lquadmath"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_library(force: bool = True) -> str:
    """Compile the oracle (ORACLE_LIBRARY overrides the library path to load)."""
    if force or not os.path.exists(_LIB):
        compile_library(_SRC, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("gx", ctypes.c_double),
                ("gy", ctypes.c_double), ("t_bottom", ctypes.c_double),
                ("t_top", ctypes.c_double), ("regularize", ctypes.c_int32),
                ("ybc", ctypes.c_int32)]


@dataclass
class Params:
    """Model parameters (u, T, g in the units of the scaled velocities c_l = r e_l;
    ybc: 0 = thermal walls, 1 = periodic)."""
    tau: float = 0.7
    gx: float = 0.0
    gy: float = -1e-4
    t_bottom: float = 1.5
    t_top: float = 0.5
    regularize: int = 1
    ybc: int = 0

    def c(self) -> _Params:
        return _Params(self.tau, self.gx, self.gy, self.t_bottom, self.t_top,
                       int(self.regularize), int(self.ybc))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_library(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        pp = ctypes.POINTER(_Params)
        i = ctypes.c_int
        d = ctypes.c_double
        L.oracle_model.argtypes = [ip, ip, dp, dp]
        L.oracle_model.restype = i
        L.oracle_set_threads.argtypes = [i]
        L.oracle_set_threads.restype = None
        L.oracle_get_threads.argtypes = []
        L.oracle_get_threads.restype = i
        L.oracle_equilibrium.argtypes = [d, d, d, d, dp]
        L.oracle_equilibrium.restype = None
        L.oracle_macroscopic.argtypes = [dp, dp]
        L.oracle_macroscopic.restype = None
        L.oracle_collide_site.argtypes = [pp, dp, dp]
        L.oracle_collide_site.restype = None
        L.oracle_init_feq.argtypes = [i, i, dp, dp, dp, dp, dp]
        L.oracle_init_feq.restype = None
        L.oracle_propagate.argtypes = [i, i, i, dp, dp]
        L.oracle_propagate.restype = None
        L.oracle_bc.argtypes = [i, i, d, d, dp]
        L.oracle_bc.restype = None
        L.oracle_collide.argtypes = [i, i, pp, dp, dp]
        L.oracle_collide.restype = None
        L.oracle_run.argtypes = [i, i, pp, dp, i]
        L.oracle_run.restype = None
        L.oracle_moments.argtypes = [i, i, dp, dp, dp, dp, dp]
        L.oracle_moments.restype = None
        L.oracle_kinetic_energy.argtypes = [i, i, dp]
        L.oracle_kinetic_energy.restype = d
        L.oracle_step_sites.argtypes = [i, i, pp, dp, i, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32), dp]
        L.oracle_step_sites.restype = None
        L.oracle_run_moments_ld.argtypes = [i, i, pp, dp, i, dp, dp, dp, dp, dp]
        L.oracle_run_moments_ld.restype = None
        L.oracle_run_complex.argtypes = [i, i, pp, dp, i]
        L.oracle_run_complex.restype = None
        L.oracle_init_feq_complex.argtypes = [i, i, dp, dp, dp, dp, dp]
        L.oracle_init_feq_complex.restype = None
        L.oracle_kinetic_energy_complex.argtypes = [i, i, dp, dp]
        L.oracle_kinetic_energy_complex.restype = None
        L.oracle_ke_after_steps_complex.argtypes = [i, i, pp, dp, dp, dp, dp, i, dp]
        L.oracle_ke_after_steps_complex.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def model():
    """(cx, cy, w, r) of the velocity set derived by the oracle's own solve."""
    cx = np.zeros(Q, np.int32)
    cy = np.zeros(Q, np.int32)
    w = np.zeros(Q)
    r = np.zeros(1)
    rc = lib().oracle_model(cx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            cy.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            _p(w), _p(r))
    if rc != 0:
        raise RuntimeError("oracle quadrature solve failed")
    return cx, cy, w, float(r[0])


def equilibrium(rho: float, ux: float, uy: float, T: float) -> np.ndarray:
    out = np.zeros(Q)
    lib().oracle_equilibrium(rho, ux, uy, T, _p(out))
    return out


def macroscopic(f37) -> np.ndarray:
    """(rho, ux, uy, T) of one site's populations (Eq. (2))."""
    f = _f64(f37)
    out = np.zeros(4)
    lib().oracle_macroscopic(_p(f), _p(out))
    return out


def collide_site(f37, params: Params) -> np.ndarray:
    f = _f64(f37)
    out = np.zeros(Q)
    P = params.c()
    lib().oracle_collide_site(ctypes.byref(P), _p(f), _p(out))
    return out


def init_feq(rho, ux, uy, T) -> np.ndarray:
    rho, ux, uy, T = (_f64(a) for a in (rho, ux, uy, T))
    lx, ly = rho.shape
    f = np.zeros((Q, lx, ly))
    lib().oracle_init_feq(lx, ly, _p(rho), _p(ux), _p(uy), _p(T), _p(f))
    return f


def propagate(f, ybc: int = 0) -> np.ndarray:
    f = _f64(f)
    _, lx, ly = f.shape
    out = np.empty_like(f)
    lib().oracle_propagate(lx, ly, int(ybc), _p(f), _p(out))
    return out


def bc(ft, t_bottom: float, t_top: float) -> np.ndarray:
    out = _f64(ft).copy()
    _, lx, ly = out.shape
    lib().oracle_bc(lx, ly, float(t_bottom), float(t_top), _p(out))
    return out


def collide(ft, params: Params) -> np.ndarray:
    ft = _f64(ft)
    _, lx, ly = ft.shape
    out = np.empty_like(ft)
    P = params.c()
    lib().oracle_collide(lx, ly, ctypes.byref(P), _p(ft), _p(out))
    return out


def run(f, params: Params, nsteps: int) -> np.ndarray:
    """Returns f advanced by nsteps full steps (propagate, bc, collide)."""
    out = _f64(f).copy()
    _, lx, ly = out.shape
    P = params.c()
    lib().oracle_run(lx, ly, ctypes.byref(P), _p(out), int(nsteps))
    return out


def step_sites(f, params: Params, xs, ys) -> np.ndarray:
    """Post-step populations [n, 37] at sites (xs[i], ys[i]) of the state f."""
    f = _f64(f)
    _, lx, ly = f.shape
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    out = np.zeros((len(xs), Q))
    P = params.c()
    ip = ctypes.POINTER(ctypes.c_int32)
    lib().oracle_step_sites(lx, ly, ctypes.byref(P), _p(f), len(xs), xs.ctypes.data_as(ip),
                            ys.ctypes.data_as(ip), _p(out))
    return out


def moments(f):
    f = _f64(f)
    _, lx, ly = f.shape
    rho, ux, uy, T = (np.zeros((lx, ly)) for _ in range(4))
    lib().oracle_moments(lx, ly, _p(f), _p(rho), _p(ux), _p(uy), _p(T))
    return rho, ux, uy, T


def run_moments_extended(f, params: Params, nsteps: int, with_populations: bool = False):
    """nsteps full steps from f in long double (x87, 64-bit significand) and
    the Eq. (2) moments of the result, rounded to FP64: (rho, ux, uy, T), plus
    the populations when asked.  The reference against which the rounding
    of FP64 runs (this oracle's and the GPU's) is measured."""
    f = _f64(f)
    _, lx, ly = f.shape
    rho, ux, uy, T = (np.zeros((lx, ly)) for _ in range(4))
    out = np.zeros_like(f) if with_populations else None
    P = params.c()
    lib().oracle_run_moments_ld(lx, ly, ctypes.byref(P), _p(f), int(nsteps), _p(rho), _p(ux),
                                _p(uy), _p(T), _p(out) if out is not None else None)
    return (rho, ux, uy, T, out) if with_populations else (rho, ux, uy, T)


def kinetic_energy(f) -> float:
    f = _f64(f)
    _, lx, ly = f.shape
    return float(lib().oracle_kinetic_energy(lx, ly, _p(f)))


def ke_after_steps_complex(params: Params, rho0, ux0, uy0, T0, nsteps: int) -> complex:
    """KE after nsteps from f = f^eq(rho0, u0, T0), all in complex arithmetic."""
    arrs = [np.ascontiguousarray(a, dtype=np.complex128) for a in (rho0, ux0, uy0, T0)]
    lx, ly = arrs[0].shape
    ke = np.zeros(2)
    P = params.c()
    dp = ctypes.POINTER(ctypes.c_double)
    lib().oracle_ke_after_steps_complex(
        lx, ly, ctypes.byref(P), *[a.ctypes.data_as(dp) for a in arrs], int(nsteps), _p(ke))
    return complex(ke[0], ke[1])


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _cp(a: np.ndarray):
    assert a.flags.c_contiguous and a.dtype == np.complex128
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def run_complex(f, params: Params, nsteps: int) -> np.ndarray:
    """nsteps full steps in complex arithmetic (complex-step linearisation)."""
    out = _c128(f).copy()
    _, lx, ly = out.shape
    P = params.c()
    lib().oracle_run_complex(lx, ly, ctypes.byref(P), _cp(out), int(nsteps))
    return out


def init_feq_complex(rho, ux, uy, T) -> np.ndarray:
    rho, ux, uy, T = (_c128(a) for a in (rho, ux, uy, T))
    lx, ly = rho.shape
    f = np.zeros((Q, lx, ly), dtype=np.complex128)
    lib().oracle_init_feq_complex(lx, ly, _cp(rho), _cp(ux), _cp(uy), _cp(T), _cp(f))
    return f


def kinetic_energy_complex(f) -> complex:
    f = _c128(f)
    _, lx, ly = f.shape
    ke = np.zeros(2)
    lib().oracle_kinetic_energy_complex(lx, ly, _cp(f), _p(ke))
    return complex(ke[0], ke[1])
