"""Optimised multicore CPU implementation of the D2Q37 step (comparison only).

A second, vectorised CPU implementation of the same step as the GPU library,
used by the benchmark as a stronger CPU reference than the plain oracle.  It
is never called by the GPU binding.  Built twice (AVX2 and AVX-512 targets);
the AVX-512 build is loaded when the host CPU has it.
Arrays: populations f[37, Lx, Ly] float64, as in the oracle.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "d2q37_cpu.cpp")
TARGETS = {"v3": "x86-64-v3", "v4": "x86-64-v4"}


def _lib_path(tag: str) -> str:
    return os.path.join(_HERE, "libd2q37_cpu_%s.so" % tag)


def build(force: bool = True) -> None:
    for tag, march in TARGETS.items():
        out = _lib_path(tag)
        if force or not os.path.exists(out):
            tmp = out + ".tmp%d" % os.getpid()
            subprocess.run(["g++", "-std=c++17", "-O3", "-march=" + march, "-Wno-psabi", "-fopenmp", "-fPIC",
                            "-shared", _SRC, "-o", tmp], check=True)
            os.replace(tmp, out)


def host_has_avx512() -> bool:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("flags"):
                return " avx512f " in line + " "
    except OSError:
        pass
    return False


class _Params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("gx", ctypes.c_double), ("gy", ctypes.c_double),
                ("t_bottom", ctypes.c_double), ("t_top", ctypes.c_double),
                ("regularize", ctypes.c_int32), ("ybc", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        tag = "v4" if host_has_avx512() else "v3"
        path = _lib_path(tag)
        if not os.path.exists(path):
            build(force=False)
        L = ctypes.CDLL(path)
        vp, dp, i = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        L.cpu_create.argtypes = [i, i, ctypes.POINTER(_Params)]
        L.cpu_create.restype = vp
        L.cpu_free.argtypes = [vp]
        L.cpu_free.restype = None
        L.cpu_set_populations.argtypes = [vp, dp]
        L.cpu_set_populations.restype = None
        L.cpu_get_populations.argtypes = [vp, dp]
        L.cpu_get_populations.restype = None
        L.cpu_step.argtypes = [vp, i]
        L.cpu_step.restype = None
        L.cpu_set_threads.argtypes = [i]
        L.cpu_set_threads.restype = None
        _lib = L
    return _lib


class CpuLattice:
    def __init__(self, lx: int, ly: int, f0, *, tau=0.7, gx=0.0, gy=-1e-4, t_bottom=1.5,
                 t_top=0.5, regularize=1, ybc=0):
        self.lx, self.ly = int(lx), int(ly)
        P = _Params(tau, gx, gy, t_bottom, t_top, int(regularize), int(ybc))
        self.h = lib().cpu_create(self.lx, self.ly, ctypes.byref(P))
        if not self.h:
            raise ValueError("cpu_create failed")
        self.set(f0)

    def set(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        lib().cpu_set_populations(self.h, f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))

    def get(self) -> np.ndarray:
        out = np.empty((37, self.lx, self.ly))
        lib().cpu_get_populations(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return out

    def step(self, n: int = 1):
        lib().cpu_step(self.h, int(n))

    def __del__(self):
        if getattr(self, "h", None):
            lib().cpu_free(self.h)
            self.h = None


def set_threads(n: int) -> None:
    lib().cpu_set_threads(int(n))
