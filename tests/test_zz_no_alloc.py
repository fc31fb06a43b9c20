"""lb_adjoint_run_static: the adjoint run without a workspace argument.

Called through the C ABI (ctypes) and checked bit for bit against
lb_adjoint_run with a caller workspace, on consecutive calls whose lattices
shrink (the second call reuses the library's static scratch with the first
call's contents still in it), walls and periodic y; lattices beyond the
scratch are rejected before anything is launched.
"""

import ctypes

import numpy as np
import pytest

from helpers import gpu_available
from paper_1703_00186_amd import workload

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1703_00186_amd.lb import LB


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _static_vs_workspace(lx, ly, n, ybc):
    f = workload.rt_fields(lx, ly, seed=workload.config_seed(4), mode="multimode")[:4]
    lb = LB(lx, ly, *f, ybc=ybc)
    lb.step(3)
    tape = lb.new_tape(n)
    lb.step_record(n, tape)
    _, lam = lb.loss_ke(with_lambda=True)
    lam_ws, lam_static = lam.clone(), lam.clone()
    lb.adjoint_run(tape, lam_ws, n)
    torch.cuda.synchronize()
    print("lb_adjoint_run_static %dx%d n=%d %s" % (lx, ly, n, ybc), flush=True)
    rc = lb.lib.lb_adjoint_run_static(lb.ctx, n, _ptr(tape), _ptr(lam_static))
    assert rc == 0, lb.lib.lb_last_error().decode()
    torch.cuda.synchronize()
    assert torch.isfinite(lam_static).all()
    assert torch.equal(lam_static, lam_ws)
    return float(lam_static.abs().max())


def test_static_adjoint_matches_workspace_adjoint_on_shrinking_calls():
    a = _static_vs_workspace(96, 80, 6, "walls")
    b = _static_vs_workspace(40, 30, 4, "walls")
    c = _static_vs_workspace(32, 24, 3, "periodic")
    assert a > 0 and b > 0 and c > 0


def test_static_adjoint_rejects_large_lattice():
    from paper_1703_00186_amd.lb import LBError
    lx, ly = 400, 300  # two padded FP64 buffers: 2 x 37 x 406 x 384 x 8 B > 64 MiB
    f = workload.rt_fields(lx, ly, seed=1)[:4]
    lb = LB(lx, ly, *f)
    tape = lb.new_tape(1)
    lam = lb.new_lambda().zero_()
    with pytest.raises(LBError) as e:
        lb.adjoint_run_static(tape, lam, 1)
    assert e.value.code == -2
    assert "64 MiB" in str(e.value)
