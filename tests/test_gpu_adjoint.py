"""The hand-written adjoint on the GPU against independent linearisations.

* transposition: <J v, lam> = <v, J^T lam> for one step (propagate, walls,
  collide with gravity) and for the initial equilibrium, where J v comes from
  the CPU oracle run in complex arithmetic (complex step: exact to rounding)
  and J^T lam from the GPU adjoint kernels;
* dKE/df from lb_loss_ke against the oracle's complex-step KE;
* the gradient of KE after 200 steps with respect to the 16 interface
  amplitudes: against the oracle's complex-step gradient on 64 x 64, and, on
  the 512 x 512 lattice, against central finite differences (h = 1e-6) of the
  GPU forward run, with the adjoint costing at most 3 forward runs.
"""

import time

import numpy as np
import pytest

import oracle
from helpers import gpu_available
from paper_1703_00186_amd import workload

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1703_00186_amd import adjoint
    from paper_1703_00186_amd.lb import LB

H = 1e-30  # complex step


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def setup(lx, ly, ybc="walls", regularize=1, g=(1e-3, -2e-3), steps=3, seed=5, layout="column"):
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=seed)
    P = oracle.Params(tau=0.7, gx=g[0], gy=g[1], t_bottom=1.5, t_top=0.5,
                      regularize=regularize, ybc=1 if ybc == "periodic" else 0)
    f = oracle.run(oracle.init_feq(rho, ux, uy, T), P, steps)
    lb = LB(lx, ly, rho, ux, uy, T, ybc=ybc, regularize=regularize, g=g, layout=layout)
    return lb, P, f, (rho, ux, uy, T)


@pytest.mark.parametrize("ybc,regularize,layout", [
    ("walls", 1, "column"), ("walls", 0, "column"), ("periodic", 1, "column"),
    ("periodic", 0, "column"), ("walls", 1, "soa"), ("periodic", 0, "soa")])
def test_step_transpose(ybc, regularize, layout):
    _transpose_check(24, 20, ybc, regularize, layout)


@pytest.mark.parametrize("shape", [(6, 6), (7, 9)])
def test_step_transpose_minimum_sizes(shape):
    """Every column is an edge column and every row a wall row or next to one."""
    _transpose_check(*shape, "walls", 1, "column")


def _transpose_check(lx, ly, ybc, regularize, layout):
    lb, P, f, _ = setup(lx, ly, ybc, regularize, layout=layout)
    lb.set_state(torch.from_numpy(f))
    tape = lb.new_tape(1)
    lb.step_record(1, tape)
    rng = np.random.default_rng(7)
    for trial in range(3):
        lam = rng.standard_normal((37, lx, ly))
        v = rng.standard_normal((37, lx, ly))
        if trial == 1:  # weight the wall rows
            lam[:, :, 3:-3] *= 1e-3
            v[:, :, 3:-3] *= 1e-3
        out = lb.new_lambda()
        lb.adjoint_step(tape[0], lb.lambda_from(lam), out)
        jt_lam = host(lb.lambda_view(out))
        jv = oracle.run_complex(f + 1j * H * v, P, 1).imag / H
        a, b = np.sum(jv * lam), np.sum(v * jt_lam)
        assert abs(a - b) <= 1e-12 * (np.abs(jv * lam).sum()), (a, b)


@pytest.mark.parametrize("ybc,regularize,layout", [
    ("walls", 1, "column"), ("walls", 0, "soa"), ("periodic", 1, "column"),
    ("periodic", 0, "soa")])
@pytest.mark.parametrize("shape,n", [((6, 6), 4), ((7, 65), 3), ((37, 70), 1), ((37, 70), 7),
                                     ((130, 300), 3), ((400, 400), 2), ((400, 400), 3)])
def test_adjoint_run_equals_single_steps(ybc, regularize, layout, shape, n):
    """lb_adjoint_run gives lb_adjoint_step's result bit for bit: the gather
    form over padded buffers (ragged tiles of both tile shapes) and, at
    400 x 400, the in-cache scatter form with an even and an odd step count."""
    lx, ly = shape
    lb, P, f, _ = setup(lx, ly, ybc, regularize, layout=layout)
    lb.set_state(torch.from_numpy(f))
    tape = lb.new_tape(n)
    lb.step_record(n, tape)
    lam0 = lb.lambda_from(np.random.default_rng(n).standard_normal((37, lx, ly)))
    ref, spare = lam0.clone(), lb.new_lambda()
    for j in range(n - 1, -1, -1):
        lb.adjoint_step(tape[j], ref, spare)
        ref, spare = spare, ref
    got = lam0.clone()
    lb.adjoint_run(tape, got, n)
    torch.cuda.synchronize()
    assert torch.equal(got, ref), float((got - ref).abs().max())
    again = lam0.clone()
    lb.adjoint_run(tape, again, 0)
    assert torch.equal(again, lam0)


def test_adjoint_run_equals_single_steps_production_size():
    """The production lattice, 8192 x 4096 (gather form over two 10 GB padded
    buffers): lb_adjoint_run over 3 recorded steps of the multimode RT run
    equals 3 lb_adjoint_step calls bit for bit, starting from the kinetic
    energy's lambda."""
    lx, ly, n = 8192, 4096, 3
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=workload.config_seed(5),
                                           mode="multimode")
    lb = LB(lx, ly, rho, ux, uy, T)
    lb.step(5)
    tape = lb.new_tape(n)
    lb.step_record(n, tape)
    _, lam0 = lb.loss_ke(with_lambda=True)
    ref, spare = lam0.clone(), lb.new_lambda()
    for j in range(n - 1, -1, -1):
        lb.adjoint_step(tape[j], ref, spare)
        ref, spare = spare, ref
    del spare
    got = lam0.clone()
    del lam0
    lb.adjoint_run(tape, got, n)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(got).all())
    assert torch.equal(got, ref), float((got - ref).abs().max())


def test_tape_holds_pre_collision_moments():
    lx, ly = 24, 20
    lb, P, f, _ = setup(lx, ly)
    lb.set_state(torch.from_numpy(f))
    tape = lb.new_tape(1)
    lb.step_record(1, tape)
    ft = oracle.bc(oracle.propagate(f, ybc=0), P.t_bottom, P.t_top)
    cx, cy, _, r = oracle.model()
    c_x, c_y = r * cx[:, None, None], r * cy[:, None, None]
    ref = np.stack([ft.sum(0), (c_x * ft).sum(0), (c_y * ft).sum(0),
                    ((c_x ** 2 + c_y ** 2) * ft).sum(0)])
    assert np.allclose(host(tape[0]), ref, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("layout", ["column", "soa"])
def test_init_transpose(layout):
    lx, ly = 20, 16
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=9)
    ux = ux + 0.01
    uy = uy - 0.02
    lb = LB(lx, ly, rho, ux, uy, T, layout=layout)
    rng = np.random.default_rng(3)
    lam = rng.standard_normal((37, lx, ly))
    d = [host(t) for t in lb.init_adjoint(rho, ux, uy, T, lb.lambda_from(lam))]
    dv = [rng.standard_normal((lx, ly)) for _ in range(4)]
    fc = oracle.init_feq_complex(*[a + 1j * H * b for a, b in zip((rho, ux, uy, T), dv)])
    a = np.sum(fc.imag / H * lam)
    b = sum(np.sum(x * y) for x, y in zip(dv, d))
    assert abs(a - b) <= 1e-12 * np.abs(fc.imag / H * lam).sum()


@pytest.mark.parametrize("layout", ["column", "soa"])
def test_loss_gradient(layout):
    lx, ly = 20, 16
    lb, P, f, _ = setup(lx, ly, layout=layout)
    lb.set_state(torch.from_numpy(f))
    ke, lam = lb.loss_ke(with_lambda=True)
    assert abs(host(ke)[0] - oracle.kinetic_energy(f)) <= 1e-13 * oracle.kinetic_energy(f)
    v = np.random.default_rng(1).standard_normal((37, lx, ly))
    d = oracle.kinetic_energy_complex(f + 1j * H * v).imag / H
    lam = host(lb.lambda_view(lam))
    assert abs(np.sum(lam * v) - d) <= 1e-12 * np.abs(lam * v).sum()


def amplitude_grad_gpu(lb, lx, ly, seed, nsteps, every):
    """(KE, dKE/da_k, forward seconds, backward seconds) via the GPU adjoint."""
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=seed, mode="multimode")
    fields = [torch.from_numpy(a).cuda().requires_grad_(True) for a in (rho, ux, uy, T)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ke = adjoint.kinetic_energy(lb, *fields, nsteps=nsteps, checkpoint_every=every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ke.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g_rho, g_T = host(fields[0].grad), host(fields[3].grad)
    grad = workload.amplitude_gradient(lx, ly, g_rho, g_T, seed=seed)
    return float(ke.detach().cpu()), grad, t1 - t0, t2 - t1


@pytest.mark.parametrize("every", [20, 0])
def test_gradient_matches_oracle_complex_step_64(every):
    """Checkpoints every 20 steps, and the full tape (every = 0)."""
    lx, ly, nsteps = 64, 64, 200
    seed = workload.config_seed(4)
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=seed, mode="multimode")
    lb = LB(lx, ly, rho, ux, uy, T)
    ke, g_gpu, _, _ = amplitude_grad_gpu(lb, lx, ly, seed, nsteps, every)
    a0, _, _ = workload.draw_modes(seed)
    P = oracle.Params(tau=0.7, gx=0.0, gy=-1e-4, t_bottom=1.5, t_top=0.5)
    g_cs = np.zeros(16)
    for k in range(16):
        amp = a0.astype(np.complex128)
        amp[k] += 1j * H
        f = workload.rt_fields(lx, ly, seed=seed, mode="multimode", amplitudes=amp)[:4]
        g_cs[k] = oracle.ke_after_steps_complex(P, *f, nsteps).imag / H
    err = np.abs(g_gpu - g_cs).max() / np.abs(g_cs).max()
    assert err <= 1e-10, (err, g_gpu, g_cs)


@pytest.mark.parametrize("nsteps", [0, 1, 37])
def test_full_tape_equals_checkpointed(nsteps):
    """Both modes apply the same transposed steps to the same recorded
    moments; checkpoint intervals that do not divide the run included."""
    lx, ly = 48, 40
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=8, mode="multimode")
    lb = LB(lx, ly, rho, ux, uy, T)
    grads = []
    for every in (0, 5, 64):
        fields = [torch.from_numpy(a).cuda().requires_grad_(True) for a in (rho, ux, uy, T)]
        adjoint.kinetic_energy(lb, *fields, nsteps=nsteps, checkpoint_every=every).backward()
        grads.append(np.stack([host(f.grad) for f in fields]))
    scale = np.abs(grads[0]).max()
    for g in grads[1:]:
        assert np.abs(g - grads[0]).max() <= 1e-13 * scale


def test_full_tape_cost():
    """Without recomputation the backward pass is one adjoint launch per
    step: at most 1.5 forward runs (624 against 592 bytes per site)."""
    lx, ly, nsteps = 512, 512, 200
    seed = workload.config_seed(4)
    rho, ux, uy, T, _ = workload.rt_fields(lx, ly, seed=seed, mode="multimode")
    lb = LB(lx, ly, rho, ux, uy, T)
    amplitude_grad_gpu(lb, lx, ly, seed, 40, 0)  # warm-up
    _, g_tape, t_fwd_tape, t_bwd = amplitude_grad_gpu(lb, lx, ly, seed, nsteps, 0)
    _, g_ckpt, _, _ = amplitude_grad_gpu(lb, lx, ly, seed, nsteps, 20)
    assert np.abs(g_tape - g_ckpt).max() <= 1e-12 * np.abs(g_ckpt).max()
    fields = [lb.field(a) for a in (rho, ux, uy, T)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb.reinit(*fields)
    lb.step(nsteps)
    lb.loss_ke(with_lambda=False)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    print("full tape 512x512x200: forward %.4f s (recording %.4f s), backward %.4f s, ratio %.2f"
          % (t_fwd, t_fwd_tape, t_bwd, t_bwd / t_fwd))
    assert t_bwd <= 1.5 * t_fwd, (t_bwd, t_fwd)


def test_gradient_512_vs_finite_differences_and_cost():
    lx, ly, nsteps, every = 512, 512, 200, 20
    seed = workload.config_seed(4)
    rho, ux, uy, T, info = workload.rt_fields(lx, ly, seed=seed, mode="multimode")
    lb = LB(lx, ly, rho, ux, uy, T)
    amplitude_grad_gpu(lb, lx, ly, seed, 40, every)  # warm-up
    ke, g_adj, t_fwd_ckpt, t_bwd = amplitude_grad_gpu(lb, lx, ly, seed, nsteps, every)

    def ke_of(amp):
        f = workload.rt_fields(lx, ly, seed=seed, mode="multimode", amplitudes=amp)[:4]
        lb.reinit(*f)
        lb.step(nsteps)
        return float(host(lb.loss_ke(with_lambda=False)[0])[0])

    a0 = info["amplitudes"]
    fields = [lb.field(a) for a in (rho, ux, uy, T)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb.reinit(*fields)
    lb.step(nsteps)
    ke_fwd = float(host(lb.loss_ke(with_lambda=False)[0])[0])
    t_fwd = time.perf_counter() - t0
    assert abs(ke_fwd - ke) <= 1e-14 * ke
    # Central differences carry the rounding noise of KE divided by h.  That
    # noise is measured: KE at nine points of a line a0 + t d (d a seeded
    # unit vector, |t| <= 4e-9) minus its least-squares quadratic leaves the
    # rounding alone (the cubic term is ~1e-25 of KE); its rms sigma gives a
    # central difference an error of sigma / (sqrt(2) h) per component.
    # h = 1e-6 is checked against 1e-6 or five times that measured noise
    # (the largest of 16 components), h = 1e-5 (noise and truncation both
    # ~1e-7) against 1e-6.
    d = np.random.default_rng(7).standard_normal(16)
    d /= np.linalg.norm(d)
    ts = np.arange(-4, 5) * 1e-9
    kes = np.array([ke_of(a0 + t * d) for t in ts])
    dke = kes - kes[4]  # exact (Sterbenz); the fit then works on ~1e-10 values
    resid = dke - np.polyval(np.polyfit(ts / 1e-9, dke, 2), ts / 1e-9)
    sigma = np.sqrt(np.sum(resid ** 2) / (len(ts) - 3))
    errs = {}
    for h in (1e-6, 1e-5):
        g_fd = np.zeros(16)
        for k in range(16):
            e = np.zeros(16)
            e[k] = h
            g_fd[k] = (ke_of(a0 + e) - ke_of(a0 - e)) / (2 * h)
        errs[h] = np.abs(g_adj - g_fd).max() / np.abs(g_fd).max()
    noise_floor = 5 * sigma / (np.sqrt(2) * 1e-6) / np.abs(g_adj).max()
    print("adjoint 512x512: KE %.6e (rounding noise %.1e = %.1f ulp), max|g| %.3e, adjoint vs FD "
          "max rel %.2e (h=1e-6, measured noise floor %.1e), %.2e (h=1e-5); forward %.4f s (with "
          "checkpoints %.4f s), backward %.4f s, ratio %.2f"
          % (ke, sigma, sigma / np.spacing(ke), np.abs(g_adj).max(), errs[1e-6], noise_floor,
             errs[1e-5], t_fwd, t_fwd_ckpt, t_bwd, t_bwd / t_fwd))
    assert errs[1e-6] <= max(1e-6, noise_floor), errs
    assert errs[1e-5] <= 1e-6, errs
    assert t_bwd <= 3.0 * t_fwd, (t_bwd, t_fwd)
