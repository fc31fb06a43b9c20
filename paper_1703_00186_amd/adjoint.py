"""Differentiable D2Q37 runs: a hand-written adjoint behind torch.autograd.

``kinetic_energy(lb, rho0, ux0, uy0, T0, nsteps, checkpoint_every)`` returns
the total kinetic energy KE = (1/2) sum rho |u|^2 after ``nsteps`` steps from
f^0 = f^eq(rho0, u0, T0), as a differentiable scalar of the four initial
fields.  Forward runs the fused step and keeps the state every
``checkpoint_every`` steps; the last segment is run with lb_step_record so
that its tape (the four pre-collision moments of every site and step) is
ready when the backward pass starts.  Backward walks the segments last to
first: it restores the segment's checkpoint, recomputes the segment while
recording its tape (not needed for the last one) and applies the segment's
transposed steps from its end to its start in one lb_adjoint_run call; finally
it maps dL/df^0 to dL/d(rho0, u0, T0) (lb_init_adjoint).
With ``checkpoint_every=0`` the forward pass records the moments of every
step instead (memory: 32 bytes per site and step, e.g. 1.7 GB for 200 steps of
512 x 512, 107 GB for 100 steps of 8192 x 4096) and the backward pass only
applies the transposed steps: no recomputation.  The adjoint needs nothing of
the forward state but these moments, so both modes give the same gradient.
All arithmetic is in the gfx950 kernels; this module only sequences calls.
"""

from __future__ import annotations

import torch

from .lb import LB


class _KineticEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, ux0, uy0, T0, lb: LB, nsteps: int, every: int):
        if lb.precision != "fp64":
            raise ValueError("the adjoint needs an FP64 lattice")
        lb.reinit(rho0, ux0, uy0, T0)
        ctx.save_for_backward(rho0, ux0, uy0, T0)
        ctx.lb, ctx.nsteps = lb, nsteps
        if every <= 0:  # full tape: record every step, keep dKE/df of the end state
            ctx.tape = lb.new_tape(max(nsteps, 1))
            if nsteps:
                lb.step_record(nsteps, ctx.tape)
            ke, ctx.lam = lb.loss_ke(with_lambda=True)
            ctx.ckpts = None
            return ke[0].clone()
        # checkpoints at the start of every segment but the last, whose tape
        # is recorded right away (the backward pass starts there, so it needs
        # no recomputation); dKE/df of the end state is kept too
        ctx.tape = None
        ckpts = []
        done = 0
        while done < nsteps:
            n = min(every, nsteps - done)
            if done + n < nsteps:
                ckpts.append((lb.get_state(), n))
                lb.step(n)
            else:
                ctx.last = (lb.new_tape(n), n)
                lb.step_record(n, ctx.last[0])
            done += n
        ke, ctx.lam = lb.loss_ke(with_lambda=True)
        ctx.ckpts = ckpts
        return ke[0].clone()

    @staticmethod
    def backward(ctx, grad):
        lb: LB = ctx.lb
        rho0, ux0, uy0, T0 = ctx.saved_tensors
        if ctx.tape is not None:
            lam = ctx.lam.mul_(grad)
            lb.adjoint_run(ctx.tape, lam, ctx.nsteps)
            d = lb.init_adjoint(rho0, ux0, uy0, T0, lam)
            ctx.lb = ctx.tape = ctx.lam = None
            return d[0], d[1], d[2], d[3], None, None, None
        lam = ctx.lam.mul_(grad)
        if ctx.nsteps > 0:
            last_tape, n_last = ctx.last
            lb.adjoint_run(last_tape, lam, n_last)
            tape = last_tape
            for state, n in reversed(ctx.ckpts):
                if tape.shape[0] < n:  # the last segment may be the shorter one
                    tape = lb.new_tape(n)
                lb.set_state(state)
                lb.step_record(n, tape)
                lb.adjoint_run(tape, lam, n)
        d = lb.init_adjoint(rho0, ux0, uy0, T0, lam)
        ctx.lb = ctx.ckpts = ctx.last = ctx.lam = None
        return d[0], d[1], d[2], d[3], None, None, None


def kinetic_energy(lb: LB, rho0, ux0, uy0, T0, nsteps: int, checkpoint_every: int = 20):
    """Differentiable KE after nsteps from f^eq(rho0, u0, T0).

    checkpoint_every > 0: state checkpoints every that many steps, segments
    recomputed in the backward pass; 0: full tape, no recomputation.

    The fields may be numpy arrays or tensors (gradients flow to tensors that
    require them); they are moved to the lattice's device as FP64 [lx, ly].
    """
    fields = [torch.as_tensor(a, dtype=torch.float64).to(lb.device).contiguous()
              for a in (rho0, ux0, uy0, T0)]
    return _KineticEnergy.apply(*fields, lb, int(nsteps), int(checkpoint_every))
