"""torch.autograd wrappers of the plan API (differentiable synthesis and adjoint).

``synth(plan, alm, theta, phi)`` returns the map of ``plan.synth(alm)`` and lets
gradients flow to ``alm`` and to the point positions; ``adjoint(plan, maps)``
returns ``plan.adjoint(maps)`` with gradients to ``maps``.  All arithmetic runs in
the library (``gsht_plan_synth_vjp``, ``gsht_plan_adjoint_vjp``); these classes only
route tensors.

The positions of a plan are fixed when it is created (they are bin-sorted then), so
``theta`` and ``phi`` must hold the values the plan was created with; they are
passed only so that autograd can attach their gradients.  Gradients with respect
to complex tensors follow torch's convention dL/dRe + i dL/dIm.
"""
from __future__ import annotations

import torch


class _Synth(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alm, theta, phi, plan):
        ctx.plan = plan
        ctx.save_for_backward(alm)
        return plan.synth(alm.detach().contiguous())

    @staticmethod
    def backward(ctx, gmap):
        (alm,) = ctx.saved_tensors
        want_a, want_t, want_p = ctx.needs_input_grad[:3]
        galm, gth, gph = ctx.plan.synth_vjp(alm.detach().contiguous(), gmap.contiguous(),
                                            want_a, want_t, want_p)
        return galm, gth, gph, None


class _Adjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, maps, plan):
        ctx.plan = plan
        return plan.adjoint(maps.detach().contiguous())

    @staticmethod
    def backward(ctx, galm):
        if not ctx.needs_input_grad[0]:
            return None, None
        return ctx.plan.adjoint_vjp(galm.contiguous()), None


def synth(plan, alm, theta=None, phi=None):
    """Differentiable synthesis on the plan's points; theta/phi (the plan's own
    positions, FP64) are optional and only needed for position gradients."""
    if theta is None:
        theta = torch.zeros(plan.npts, dtype=torch.float64, device=plan.device)
    if phi is None:
        phi = torch.zeros(plan.npts, dtype=torch.float64, device=plan.device)
    return _Synth.apply(alm, theta, phi, plan)


def adjoint(plan, maps):
    """Differentiable adjoint synthesis on the plan's points."""
    return _Adjoint.apply(maps, plan)
