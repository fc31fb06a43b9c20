"""Host-side checks of the C ABI library (no GPU work is launched).

The shared library must load and export every entry point include/lb.h
declares; argument validation and workspace sizing are pure host code.
"""

import ctypes
import os
import re

import pytest

from paper_1703_00186_amd import lb as lbmod

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lb.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int)\s+(lb_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbmod.library_path()):
        from paper_1703_00186_amd import build
        build.build()
    return lbmod.load_library()


def test_header_declares_the_binding_surface():
    assert declared_symbols() == sorted(lbmod.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_workspace_bytes(lib):
    lat = lbmod.make_lattice(1920, 2048)
    par = lbmod.make_params()
    n = ctypes.c_size_t(0)
    assert lib.lb_workspace_bytes(ctypes.byref(lat), ctypes.byref(par), ctypes.byref(n)) == 0
    # two padded FP64 buffers: 37 x (1920 + 6) x (2048 + 64) doubles each
    assert n.value >= 2 * 37 * 1926 * 2112 * 8
    assert n.value < 2 * 37 * 1926 * 2112 * 8 + (16 << 20)  # + reduction scratch
    lat32 = lbmod.make_lattice(1920, 2048, precision="fp32s")
    n32 = ctypes.c_size_t(0)
    assert lib.lb_workspace_bytes(ctypes.byref(lat32), ctypes.byref(par), ctypes.byref(n32)) == 0
    assert n32.value < 0.55 * n.value


@pytest.mark.parametrize("bad", [dict(lx=5), dict(ly=3), dict(precision=7), dict(ybc=2),
                                 dict(layout=9), dict(reserved=1), dict(lx=(1 << 22) + 1),
                                 dict(ly=(1 << 24) + 1), dict(lx=1 << 16, ly=(1 << 14) + 1)])
def test_lattice_validation(lib, bad):
    lat = lbmod.make_lattice(64, 64)
    for k, v in bad.items():
        setattr(lat, k, v)
    n = ctypes.c_size_t(0)
    par = lbmod.make_params()
    assert lib.lb_workspace_bytes(ctypes.byref(lat), ctypes.byref(par), ctypes.byref(n)) == -1
    assert lib.lb_last_error().decode()


@pytest.mark.parametrize("bad", [dict(tau=0.5), dict(tau=float("nan")), dict(t_top=0.0),
                                 dict(regularize=2), dict(kernel=5), dict(kernel=-1),
                                 dict(check_finite=-1)])
def test_params_validation(lib, bad):
    lat = lbmod.make_lattice(64, 64)
    par = lbmod.make_params()
    for k, v in bad.items():
        setattr(par, k, v)
    n = ctypes.c_size_t(0)
    assert lib.lb_workspace_bytes(ctypes.byref(lat), ctypes.byref(par), ctypes.byref(n)) == -1


def test_init_rejects_null_and_small_workspace(lib):
    lat = lbmod.make_lattice(64, 64)
    par = lbmod.make_params()
    ctx = ctypes.c_void_p(0)
    rc = lib.lb_init(ctypes.byref(lat), ctypes.byref(par), None, 0, None, None, None, None, None,
                     ctypes.byref(ctx))
    assert rc == -1 and not ctx.value
    rc = lib.lb_init(ctypes.byref(lat), ctypes.byref(par), ctypes.c_void_p(256), 16, None,
                     ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256),
                     ctypes.c_void_p(256), ctypes.byref(ctx))
    assert rc == -2 and not ctx.value


def test_null_context_is_an_argument_error(lib):
    assert lib.lb_step(None, 1) == -1
    assert lib.lb_moments(None, None, None, None, None) == -1


def test_bench_accounting_reproduces_table1():
    """592 B/site and sites/us reproduce the paper's Table 1 (K40, CUDA)."""
    import bench
    vals = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "table1_k40_cuda.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    sites = int(vals["lattice_x"] * vals["lattice_y"])
    gbs = bench.bytes_per_site("fp64") * sites / (vals["t_prop_ms"] * 1e-3) / 1e9
    assert abs(gbs - vals["prop_gbs"]) < 0.5
    assert abs(bench.mlups(sites, vals["t_collide_ms"] * 1e-3) - vals["collide_mlups"]) < 0.5
    assert abs(bench.mlups(sites, vals["t_wc_ms"] * 1e-3) - vals["wc_mlups"]) < 0.5


def test_largest_lattice_is_accepted(lib):
    lat = lbmod.make_lattice(1 << 16, 1 << 14)
    n = ctypes.c_size_t(0)
    assert lib.lb_workspace_bytes(ctypes.byref(lat), ctypes.byref(lbmod.make_params()),
                                  ctypes.byref(n)) == 0
    assert n.value > 2 * 37 * 8 * (1 << 30)


def test_version(lib):
    assert lib.lb_version() == 5


def test_binding_refuses_to_run_without_the_hip_library(monkeypatch, tmp_path):
    """No CPU fallback: with the library missing, the binding raises."""
    monkeypatch.setattr(lbmod, "_lib", None)
    monkeypatch.setattr(lbmod, "library_path", lambda: str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        lbmod.load_library()
