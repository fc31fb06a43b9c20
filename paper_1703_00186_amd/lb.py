"""Python binding of the D2Q37 C ABI (include/lb.h).

Argument marshalling only: every step of the lattice Boltzmann path runs in
the gfx950 kernels of libd2q37_lb.so.  PyTorch supplies device memory (the
workspace and all field / population tensors) and the stream.  There is no
CPU fallback: if the library is missing, loading fails with an error.
"""

from __future__ import annotations

import ctypes
import functools
import json
import os

import numpy as np
import torch

from . import build as _build

Q = 37

LB_FP64, LB_FP32_SHIFTED, LB_FP32_SHIFTED_F32SUM, LB_FP32_COLLIDE, LB_FP32_LOCAL = 0, 1, 2, 3, 4
# precision names: FP64; shifted FP32 storage with the FP64 collision, or with
# FP32 Hermite sums (ablation); FP32 storage relative to the local rest
# Maxwellian with the FP32 collision ("fp32c") or the FP64 collision ("fp32l")
PRECISIONS = {"fp64": LB_FP64, "fp32s": LB_FP32_SHIFTED, "fp32s_f32sum": LB_FP32_SHIFTED_F32SUM,
              "fp32c": LB_FP32_COLLIDE, "fp32l": LB_FP32_LOCAL}
LOCAL_FORMS = ("fp32c", "fp32l")
LB_Y_WALLS, LB_Y_PERIODIC = 0, 1
LB_LAYOUT_SOA, LB_LAYOUT_COLUMN = 0, 1
LB_KERNEL_FUSED, LB_KERNEL_SPLIT = 0, 1
LB_KERNEL_SPLIT_LDS, LB_KERNEL_SPLIT_WIDE, LB_KERNEL_SPLIT_MFMA = 2, 3, 4
KERNELS = {"fused": LB_KERNEL_FUSED, "split": LB_KERNEL_SPLIT, "split_lds": LB_KERNEL_SPLIT_LDS,
           "split_wide": LB_KERNEL_SPLIT_WIDE, "split_mfma": LB_KERNEL_SPLIT_MFMA}

ERRORS = {-1: "LB_E_ARG", -2: "LB_E_WORKSPACE", -3: "LB_E_HIP", -4: "LB_E_STATE",
          -5: "LB_E_NONFINITE"}

EXPORTS = [
    "lb_last_error", "lb_version", "lb_workspace_bytes", "lb_init", "lb_free", "lb_set_stream",
    "lb_set_params", "lb_step", "lb_moments", "lb_get_state", "lb_set_state",
    "lb_get_populations", "lb_halo", "lb_propagate", "lb_bc", "lb_collide", "lb_get_scratch",
    "lb_set_scratch", "lb_observables", "lb_run_observed", "lb_step_record", "lb_loss_ke",
    "lb_adjoint_step", "lb_adjoint_workspace_bytes", "lb_adjoint_run", "lb_adjoint_run_static",
    "lb_init_adjoint",
]

N_PROFILES = 6  # rho, u_x, u_y, T, rho |u|^2 / 2, rho T (row averages)
N_SCALARS = 4   # mass, kinetic energy, sum rho T, mixing-layer width


class LBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class Lattice(ctypes.Structure):
    _fields_ = [("lx", ctypes.c_int32), ("ly", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("ybc", ctypes.c_int32), ("layout", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("gx", ctypes.c_double), ("gy", ctypes.c_double),
                ("t_bottom", ctypes.c_double), ("t_top", ctypes.c_double),
                ("rho_ref", ctypes.c_double), ("regularize", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("check_finite", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None


def library_path() -> str:
    return _build.LIB


def load_library():
    """Loads libd2q37_lb.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError("libd2q37_lb.so is not built; run `python -m paper_1703_00186_amd.build`")
    L = ctypes.CDLL(path)
    vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    Lp, Pp = ctypes.POINTER(Lattice), ctypes.POINTER(Params)
    sig = {
        "lb_last_error": ([], ctypes.c_char_p),
        "lb_version": ([], i),
        "lb_workspace_bytes": ([Lp, Pp, ctypes.POINTER(sz)], i),
        "lb_init": ([Lp, Pp, vp, sz, vp, vp, vp, vp, vp, ctypes.POINTER(vp)], i),
        "lb_free": ([vp], i),
        "lb_set_stream": ([vp, vp], i),
        "lb_set_params": ([vp, Pp], i),
        "lb_step": ([vp, i], i),
        "lb_moments": ([vp, vp, vp, vp, vp], i),
        "lb_get_state": ([vp, vp], i),
        "lb_set_state": ([vp, vp], i),
        "lb_get_populations": ([vp, vp], i),
        "lb_halo": ([vp], i),
        "lb_propagate": ([vp], i),
        "lb_bc": ([vp], i),
        "lb_collide": ([vp], i),
        "lb_get_scratch": ([vp, vp], i),
        "lb_set_scratch": ([vp, vp], i),
        "lb_observables": ([vp, vp, vp], i),
        "lb_run_observed": ([vp, i, i, vp], i),
        "lb_step_record": ([vp, i, vp], i),
        "lb_loss_ke": ([vp, vp, vp], i),
        "lb_adjoint_step": ([vp, vp, vp, vp], i),
        "lb_adjoint_workspace_bytes": ([vp, ctypes.POINTER(sz)], i),
        "lb_adjoint_run": ([vp, i, vp, vp, vp, sz], i),
        "lb_adjoint_run_static": ([vp, i, vp, vp], i),
        "lb_init_adjoint": ([vp, vp, vp, vp, vp, vp, vp, vp, vp, vp], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise LBError(rc, load_library().lb_last_error().decode())


def _ptr(t) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def make_params(tau=0.7, g=(0.0, -1e-4), t_bottom=1.5, t_top=0.5, rho_ref=1.0, regularize=1,
                kernel="fused", check_finite=0) -> Params:
    k = KERNELS[kernel]
    return Params(float(tau), float(g[0]), float(g[1]), float(t_bottom), float(t_top),
                  float(rho_ref), int(regularize), k, int(check_finite), 0)


def make_lattice(lx, ly, precision="fp64", ybc="walls", layout="column") -> Lattice:
    p = PRECISIONS[precision]
    y = {"walls": LB_Y_WALLS, "periodic": LB_Y_PERIODIC}[ybc]
    lay = {"soa": LB_LAYOUT_SOA, "column": LB_LAYOUT_COLUMN}[layout]
    return Lattice(int(lx), int(ly), p, y, lay, 0)


def _on_device(method):
    """Runs a library call with the lattice's device current (the C ABI
    refuses calls on a context from another device)."""
    @functools.wraps(method)
    def wrapper(self, *args, **kwargs):
        with torch.cuda.device(self.device):
            return method(self, *args, **kwargs)
    return wrapper


class LB:
    """One D2Q37 lattice on one GPU.

    Initial fields rho0, ux0, uy0, T0 are [lx, ly] float64 (numpy or torch);
    they are copied to the device and the state starts at f^eq(rho0, u0, T0).
    precision: one of PRECISIONS ("fp64", "fp32c", "fp32l", "fp32s",
    "fp32s_f32sum"); params: those of make_params (tau, g, t_bottom, t_top,
    rho_ref, regularize, kernel, check_finite), kernel one of KERNELS
    ("fused"; "split"; "split_lds", "split_wide", "split_mfma": the split
    stages with an alternative propagate or collide kernel).
    """

    def __init__(self, lx, ly, rho0, ux0, uy0, T0, *, precision="fp64", ybc="walls",
                 layout="column", device="cuda:0", **params):
        self.lib = load_library()
        self.device = torch.device(device)
        self.lx, self.ly = int(lx), int(ly)
        self.precision = precision
        self.layout = layout
        self.lat = make_lattice(lx, ly, precision, ybc, layout)
        self.params = dict(params)
        self.par = make_params(**self.params)
        nbytes = ctypes.c_size_t(0)
        _check(self.lib.lb_workspace_bytes(ctypes.byref(self.lat), ctypes.byref(self.par),
                                           ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        fields = [self.field(a) for a in (rho0, ux0, uy0, T0)]
        self.ctx = ctypes.c_void_p(0)
        with torch.cuda.device(self.device):
            _check(self.lib.lb_init(ctypes.byref(self.lat), ctypes.byref(self.par),
                                    _ptr(self.workspace), nbytes.value, self._stream(),
                                    *[_ptr(f) for f in fields], ctypes.byref(self.ctx)))
        torch.cuda.current_stream(self.device).synchronize()

    # -- helpers -----------------------------------------------------------
    def _stream(self) -> ctypes.c_void_p:
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _sync_stream(self):
        _check(self.lib.lb_set_stream(self.ctx, self._stream()))

    def field(self, a) -> torch.Tensor:
        """An [lx, ly] field as a contiguous FP64 device tensor."""
        t = torch.as_tensor(a, dtype=torch.float64)
        if tuple(t.shape) != (self.lx, self.ly):
            raise ValueError("field must be [lx, ly]")
        return t.to(self.device).contiguous()

    @property
    def state_dtype(self):
        """torch dtype of the stored state: float64, or float32 for the FP32 forms."""
        return torch.float64 if self.precision == "fp64" else torch.float32

    @property
    def state_planes(self) -> int:
        """Planes of the compact state: 37 populations, plus the packed
        reference (two FP16 numbers per site) in the local-reference FP32
        forms ("fp32c", "fp32l")."""
        return Q + 1 if self.precision in LOCAL_FORMS else Q

    @property
    def state_shape(self):
        return (self.state_planes, self.lx, self.ly)

    def new_populations(self, dtype=None) -> torch.Tensor:
        """An uninitialised [37, lx, ly] device tensor (state dtype by default)."""
        return torch.empty((Q, self.lx, self.ly), dtype=dtype or self.state_dtype,
                           device=self.device)

    def new_state(self) -> torch.Tensor:
        """An uninitialised device tensor of the compact state's shape and dtype."""
        return torch.empty(self.state_shape, dtype=self.state_dtype, device=self.device)

    # adjoint populations are stored in the lattice's layout: [lx, 37, ly]
    # (column) or [37, lx, ly] (SoA); lambda_view gives the [37, lx, ly] view
    @property
    def lambda_shape(self):
        """Shape of an adjoint array in this lattice's layout."""
        return (self.lx, Q, self.ly) if self.layout == "column" else (Q, self.lx, self.ly)

    def new_lambda(self) -> torch.Tensor:
        """An uninitialised FP64 adjoint array in this lattice's layout."""
        return torch.empty(self.lambda_shape, dtype=torch.float64, device=self.device)

    def lambda_view(self, lam: torch.Tensor) -> torch.Tensor:
        """[37, lx, ly] view of an adjoint array (no copy)."""
        self._check_lambda(lam)
        return lam.permute(1, 0, 2) if self.layout == "column" else lam

    def lambda_from(self, lam_std) -> torch.Tensor:
        """Copy of a [37, lx, ly] array in the adjoint layout, on the device."""
        t = torch.as_tensor(lam_std, dtype=torch.float64).to(self.device)
        if tuple(t.shape) != (Q, self.lx, self.ly):
            raise ValueError("expected [37, lx, ly]")
        return (t.permute(1, 0, 2) if self.layout == "column" else t).contiguous()

    def _check_lambda(self, lam: torch.Tensor):
        self._expect(lam, self.lambda_shape, torch.float64, "adjoint array")

    # -- the step ------------------------------------------------------------
    @_on_device
    def set_params(self, **params):
        """Updates the given parameters; the others keep their values."""
        new = dict(self.params, **params)
        par = make_params(**new)
        _check(self.lib.lb_set_params(self.ctx, ctypes.byref(par)))
        self.params, self.par = new, par

    @_on_device
    def reinit(self, rho0, ux0, uy0, T0):
        """Restarts from f = f^eq(rho0, u0, T0) on the same workspace."""
        fields = [self.field(a) for a in (rho0, ux0, uy0, T0)]
        self.close()
        nbytes = self.workspace.numel()
        with torch.cuda.device(self.device):
            _check(self.lib.lb_init(ctypes.byref(self.lat), ctypes.byref(self.par),
                                    _ptr(self.workspace), nbytes, self._stream(),
                                    *[_ptr(f) for f in fields], ctypes.byref(self.ctx)))

    @_on_device
    def step(self, n: int = 1):
        """Advances the state by n steps on the current stream (asynchronous)."""
        self._sync_stream()
        _check(self.lib.lb_step(self.ctx, int(n)))

    @_on_device
    def capture(self, n: int = 2, pool=None):
        """Records n (even) fused steps into a CUDA/HIP graph on a side
        stream; graph.replay() then advances this lattice by n steps.

        Two ordinary steps run first (the lattice advances by 2), so that the
        halos are valid and the buffer roles settled when recording starts.
        The buffers swap once per step, so an even n returns the state to the
        buffer it started in, which is what lets the same graph run again.
        Only the fused path without check_finite is capturable.
        """
        if n <= 0 or n % 2:
            raise ValueError("n must be a positive even number")
        if self.params.get("check_finite", 0) or self.params.get("kernel", "fused") != "fused":
            raise ValueError("capture needs kernel='fused' and check_finite=0")
        self.step(2)  # halos valid, buffers settled before capture
        torch.cuda.synchronize(self.device)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, pool=pool):
            self.step(n)
        torch.cuda.synchronize(self.device)
        self._sync_stream()
        return graph

    @_on_device
    def moments(self):
        """(rho, ux, uy, T) of the current state, Eq. (2), FP64 [lx, ly] each."""
        self._sync_stream()
        out = [torch.empty((self.lx, self.ly), dtype=torch.float64, device=self.device)
               for _ in range(4)]
        _check(self.lib.lb_moments(self.ctx, *[_ptr(t) for t in out]))
        return tuple(out)

    # -- argument checks: the library trusts the sizes of the buffers it gets --
    def _expect(self, t, shape, dtype, what: str):
        if (not isinstance(t, torch.Tensor) or tuple(t.shape) != tuple(shape)
                or t.dtype != dtype or t.device != self.device or not t.is_contiguous()):
            raise ValueError("%s must be a contiguous %s tensor of shape %s on %s"
                             % (what, dtype, tuple(shape), self.device))

    def _state_arg(self, f, what: str, shape=None) -> torch.Tensor:
        """An array of the compact state's shape and dtype (FP64, the shifted
        FP32 values, or the local-reference form's deviations and packed
        references), moved to the device; no dtype conversion."""
        shape = tuple(shape or self.state_shape)
        t = torch.as_tensor(f)
        if tuple(t.shape) != shape or t.dtype != self.state_dtype:
            raise ValueError("%s must be %s of shape %s" % (what, self.state_dtype, shape))
        return t.to(self.device).contiguous()

    @_on_device
    def get_state(self, out=None) -> torch.Tensor:
        """The state in compact form, in the state dtype: [37, lx, ly] (FP64, or
        the shifted FP32 values f - w rho_ref), or [38, lx, ly] FP32 in the
        local-reference form (deviations, then the packed references); `out`
        may be given to reuse a tensor."""
        self._sync_stream()
        if out is None:
            out = self.new_state()
        else:
            self._expect(out, self.state_shape, self.state_dtype, "out")
        _check(self.lib.lb_get_state(self.ctx, _ptr(out)))
        return out

    @_on_device
    def set_state(self, f: torch.Tensor):
        """Replaces the state by f (same form and dtype as get_state returns)."""
        self._sync_stream()
        f = self._state_arg(f, "state")
        _check(self.lib.lb_set_state(self.ctx, _ptr(f)))

    @_on_device
    def populations(self) -> torch.Tensor:
        """The populations f as FP64 [37, lx, ly], in every precision form."""
        self._sync_stream()
        out = self.new_populations(torch.float64)
        _check(self.lib.lb_get_populations(self.ctx, _ptr(out)))
        return out

    # -- split stages ----------------------------------------------------------
    @_on_device
    def halo(self):
        """Refreshes the periodic halos of the state (split path)."""
        self._sync_stream()
        _check(self.lib.lb_halo(self.ctx))

    @_on_device
    def propagate(self):
        """Split path: scratch = propagate(state) (needs valid halos)."""
        self._sync_stream()
        _check(self.lib.lb_propagate(self.ctx))

    @_on_device
    def bc(self):
        """Split path: the thermal walls applied to the scratch buffer."""
        self._sync_stream()
        _check(self.lib.lb_bc(self.ctx))

    @_on_device
    def collide(self):
        """Split path: state = collide(scratch)."""
        self._sync_stream()
        _check(self.lib.lb_collide(self.ctx))

    @_on_device
    def get_scratch(self) -> torch.Tensor:
        """The scratch buffer in compact [37, lx, ly] form (state dtype)."""
        self._sync_stream()
        out = self.new_populations()
        _check(self.lib.lb_get_scratch(self.ctx, _ptr(out)))
        return out

    @_on_device
    def set_scratch(self, f: torch.Tensor):
        """Replaces the scratch buffer by f (compact form, state dtype)."""
        self._sync_stream()
        f = self._state_arg(f, "scratch", (Q, self.lx, self.ly))
        _check(self.lib.lb_set_scratch(self.ctx, _ptr(f)))

    # -- in-situ observables ------------------------------------------------
    @_on_device
    def observables(self):
        """(profiles [6, ly], scalars [4]) of the current state, on the device."""
        self._sync_stream()
        prof = torch.empty((N_PROFILES, self.ly), dtype=torch.float64, device=self.device)
        sc = torch.empty(N_SCALARS, dtype=torch.float64, device=self.device)
        _check(self.lib.lb_observables(self.ctx, _ptr(prof), _ptr(sc)))
        return prof, sc

    @_on_device
    def run_observed(self, n: int, every: int) -> torch.Tensor:
        """n steps; the 4 scalars after every `every` steps, [n // every, 4]."""
        if int(every) <= 0 or int(n) < 0:
            raise ValueError("need n >= 0 and every > 0")
        self._sync_stream()
        series = torch.empty((max(n // every, 1), N_SCALARS), dtype=torch.float64,
                             device=self.device)
        _check(self.lib.lb_run_observed(self.ctx, int(n), int(every), _ptr(series)))
        return series[: n // every]

    # -- adjoint -------------------------------------------------------------
    def new_tape(self, n: int) -> torch.Tensor:
        """An uninitialised tape for n steps: FP64 [n, 4, lx, ly]."""
        return torch.empty((n, 4, self.lx, self.ly), dtype=torch.float64, device=self.device)

    @_on_device
    def step_record(self, n: int, tape: torch.Tensor):
        """n fused steps, writing the pre-collision moments (rho, j_x, j_y,
        sum |c|^2 f) of step j to tape[j] (FP64 lattices only)."""
        self._sync_stream()
        if (not isinstance(tape, torch.Tensor) or tape.dim() != 4 or tape.shape[0] < n
                or tuple(tape.shape[1:]) != (4, self.lx, self.ly)):
            raise ValueError("tape must be [>=n, 4, lx, ly]")
        self._expect(tape, tape.shape, torch.float64, "tape")
        _check(self.lib.lb_step_record(self.ctx, int(n), _ptr(tape)))

    @_on_device
    def loss_ke(self, with_lambda: bool = True):
        """(KE [1], dKE/df or None) of the current state on the device; dKE/df
        is an adjoint array in this lattice's layout."""
        self._sync_stream()
        ke = torch.empty(1, dtype=torch.float64, device=self.device)
        lam = self.new_lambda() if with_lambda else None
        _check(self.lib.lb_loss_ke(self.ctx, _ptr(ke), _ptr(lam)))
        return ke, lam

    @_on_device
    def adjoint_step(self, tape_j: torch.Tensor, lam_in: torch.Tensor, lam_out: torch.Tensor):
        """One transposed step: lam_out = J_j^T lam_in for the step whose
        moments are tape_j (scatter form, lb_adjoint_step)."""
        self._expect(tape_j, (4, self.lx, self.ly), torch.float64, "tape_j")
        self._check_lambda(lam_in)
        self._check_lambda(lam_out)
        self._sync_stream()
        _check(self.lib.lb_adjoint_step(self.ctx, _ptr(tape_j), _ptr(lam_in), _ptr(lam_out)))

    @_on_device
    def adjoint_run(self, tape: torch.Tensor, lam: torch.Tensor, n: int = None):
        """n transposed steps (default: all of the tape), lambda^n -> lambda^0
        in place in `lam`, in the gather form (lb_adjoint_run); the padded
        adjoint buffers are allocated on first use and kept."""
        n = tape.shape[0] if n is None else int(n)
        if (not isinstance(tape, torch.Tensor) or tape.dim() != 4 or tape.shape[0] < n
                or tuple(tape.shape[1:]) != (4, self.lx, self.ly)):
            raise ValueError("tape must be [>=n, 4, lx, ly]")
        self._expect(tape, tape.shape, torch.float64, "tape")
        self._check_lambda(lam)
        self._sync_stream()
        if getattr(self, "_adj_ws", None) is None:
            nbytes = ctypes.c_size_t(0)
            _check(self.lib.lb_adjoint_workspace_bytes(self.ctx, ctypes.byref(nbytes)))
            self._adj_ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        _check(self.lib.lb_adjoint_run(self.ctx, n, _ptr(tape), _ptr(lam), _ptr(self._adj_ws),
                                       self._adj_ws.numel()))
        return lam

    @_on_device
    def adjoint_run_static(self, tape: torch.Tensor, lam: torch.Tensor, n: int = None):
        """As adjoint_run, through lb_adjoint_run_static: no workspace, the
        library's per-GPU 64 MiB scratch (small lattices only; calls that
        overlap on one GPU race)."""
        n = tape.shape[0] if n is None else int(n)
        if (not isinstance(tape, torch.Tensor) or tape.dim() != 4 or tape.shape[0] < n
                or tuple(tape.shape[1:]) != (4, self.lx, self.ly)):
            raise ValueError("tape must be [>=n, 4, lx, ly]")
        self._expect(tape, tape.shape, torch.float64, "tape")
        self._check_lambda(lam)
        self._sync_stream()
        _check(self.lib.lb_adjoint_run_static(self.ctx, n, _ptr(tape), _ptr(lam)))
        return lam

    @_on_device
    def init_adjoint(self, rho0, ux0, uy0, T0, lam0: torch.Tensor):
        """dL/d(rho0, ux0, uy0, T0) of f^0 = f^eq(rho0, u0, T0) given lam0 = dL/df^0;
        four FP64 [lx, ly] tensors."""
        self._check_lambda(lam0)
        self._sync_stream()
        fields = [self.field(a) for a in (rho0, ux0, uy0, T0)]
        out = [torch.empty((self.lx, self.ly), dtype=torch.float64, device=self.device)
               for _ in range(4)]
        _check(self.lib.lb_init_adjoint(self.ctx, *[_ptr(f) for f in fields], _ptr(lam0),
                                        *[_ptr(t) for t in out]))
        return tuple(out)

    # -- checkpoints on disk --------------------------------------------------
    def save_checkpoint(self, path: str) -> None:
        """Writes the state (compact [37, lx, ly] in the context's precision)
        and the lattice and parameters to an .npz file of plain arrays."""
        meta = {"lx": self.lx, "ly": self.ly, "precision": self.precision,
                "layout": self.layout, "ybc": int(self.lat.ybc), "params": self.params}
        state = self.get_state()
        torch.cuda.synchronize(self.device)
        np.savez(path, state=state.cpu().numpy(), meta=np.array(json.dumps(meta)))

    def load_checkpoint(self, path: str) -> dict:
        """Restores a state written by save_checkpoint into this context (same
        lattice size, precision and y boundary); returns the saved metadata.
        The parameters of this context are left as they are."""
        with np.load(path, allow_pickle=False) as z:
            meta = json.loads(str(z["meta"]))
            state = z["state"]
        if (meta["lx"], meta["ly"], meta["precision"], meta["ybc"]) != (
                self.lx, self.ly, self.precision, int(self.lat.ybc)):
            raise ValueError("checkpoint is for %dx%d %s ybc=%d" % (
                meta["lx"], meta["ly"], meta["precision"], meta["ybc"]))
        self.set_state(torch.from_numpy(state))
        return meta

    def close(self):
        """Frees the host-side context (the device workspace stays with this
        object until it is dropped)."""
        if getattr(self, "ctx", None) and self.ctx.value:
            self.lib.lb_free(self.ctx)
            self.ctx = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
