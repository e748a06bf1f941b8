"""Differentiable modelling: d = S(v) src as a torch.autograd.Function.

The forward pass runs ``esi_forward_ckpt`` (modelling that keeps two time
levels of the wavefield every ``ckpt_every`` steps); the backward pass runs
``esi_gradient`` in SEED_REUSE mode: the adjoint field of dL/dd is propagated
backward while each K-step segment of the forward wavefield is recomputed
from its checkpoint and correlated with it (the adjoint-state gradient of
eq. (gradient), with the storage remedy the paper cites in Sec. 5.1).  The
gradient with respect to m = 1/v^2 is turned into one with respect to v by
``esi_grad_velocity``.  All arithmetic runs in the HIP library.
"""
from __future__ import annotations

import torch

from . import esi


class Propagate(torch.autograd.Function):
    """vel [phys] (m/s), src [nshots, nt] (point) or [nshots, nt, *phys] (dense)
    -> data [nt * nrec of the shots] on the plan's acquisition."""

    @staticmethod
    def forward(ctx, vel, src, plan, kind=esi.SRC_POINT, shot0=0, nshots=None, ckpt_every=50):
        vel_c = vel.detach().contiguous()
        src_c = src.detach().contiguous()
        plan.set_model(vel_c)
        shot0, nshots = plan._range(shot0, nshots)
        d = plan.forward_ckpt(src_c, ckpt_every, kind, shot0, nshots)
        ctx.save_for_backward(vel_c, src_c)
        ctx.plan, ctx.kind, ctx.shot0, ctx.nshots, ctx.ckpt = plan, kind, shot0, nshots, ckpt_every
        return d

    @staticmethod
    def backward(ctx, G):
        vel, src = ctx.saved_tensors
        plan = ctx.plan
        grad_src = torch.zeros_like(src) if ctx.needs_input_grad[1] else None
        # the plan still holds the model and checkpoints of this forward pass
        # unless another differentiable call ran in between: then redo it
        try:
            grad_m = plan.gradient(esi.GRAD_SEED_REUSE, src, G.contiguous(), kind=ctx.kind,
                                   shot0=ctx.shot0, nshots=ctx.nshots, grad_src=grad_src,
                                   ckpt_every=ctx.ckpt)
        except esi.EsiError:
            plan.set_model(vel)
            grad_m = plan.gradient(esi.GRAD_SEED, src, G.contiguous(), kind=ctx.kind,
                                   shot0=ctx.shot0, nshots=ctx.nshots, grad_src=grad_src,
                                   ckpt_every=ctx.ckpt)
        grad_v = plan.grad_velocity(vel, grad_m) if ctx.needs_input_grad[0] else None
        return grad_v, grad_src, None, None, None, None, None


def propagate(vel, src, plan, kind=esi.SRC_POINT, shot0=0, nshots=None, ckpt_every=50):
    """Differentiable forward modelling (see :class:`Propagate`)."""
    return Propagate.apply(vel, src, plan, kind, shot0, nshots, ckpt_every)
