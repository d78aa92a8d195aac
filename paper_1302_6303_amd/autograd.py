"""torch.autograd wrapper: dJ/dz of the time-integrated radiation energy.

RadDiffEvolve.apply(z, hier, E0, T0, dt, nsteps, ckpt_every) runs nsteps
backward-Euler implicit steps of the library state from (E0, T0) with the
material field z (all compact float64 CUDA tensors) and returns E at the
final time.  Its backward pass calls the library's checkpointed discrete
adjoint (transpose-Jacobian FGMRES per step, state checkpoints every
ckpt_every steps), which returns grad_z = (dE_N/dz)^T grad_E.

The hierarchy must have been created with bdf_max_order = 1 and at least
ceil(nsteps / ckpt_every) + ckpt_every + 3 adjoint slots.
"""
from __future__ import annotations

import torch


class RadDiffEvolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z, hier, E0, T0, dt, nsteps, ckpt_every):
        if hier.opt.bdf_max_order != 1:
            # the adjoint differentiates backward-Euler steps: a BDF2 forward
            # trajectory would get the gradient of another trajectory
            raise ValueError("RadDiffEvolve needs a hierarchy created with "
                             "bdf_max_order = 1")
        z = z.detach().contiguous()
        hier.set_fields(E0, T0, z)
        for _ in range(nsteps):
            hier.implicit_step([float(dt)] * hier.nprob)
        E, _ = hier.get_fields()
        ctx.hier = hier
        ctx.args = (E0, T0, float(dt), int(nsteps), int(ckpt_every))
        ctx.save_for_backward(z)
        return E

    @staticmethod
    def backward(ctx, grad_E):
        (z,) = ctx.saved_tensors
        E0, T0, dt, nsteps, every = ctx.args
        hier = ctx.hier
        hier.set_fields(E0, T0, z)
        gz = hier.adjoint_run([dt] * hier.nprob, nsteps, every,
                              grad_E.detach().to(torch.float64).contiguous())
        return gz.view_as(z), None, None, None, None, None, None
