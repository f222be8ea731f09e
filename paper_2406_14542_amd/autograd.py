"""Differentiable synthesis: gradients with respect to the coefficients and the point positions.

``synthesis(plan, alm, theta=None, phi=None)`` returns the maps of Eq. (3) and supports
torch autograd with respect to the coefficients and, when ``theta`` / ``phi`` are given as
tensors that require grad (the plan's point coordinates, e.g. lensing deflections), with
respect to the point positions.  Forward and backward only call the library:
* forward: ``nusht_synthesis`` or, if a position gradient is needed,
  ``nusht_synthesis_deriv`` (map and its theta/phi derivatives from one fine grid);
* backward: ``nusht_vjp_alm`` (the adjoint kernel path, Eq. 2, with the complex-gradient
  convention dL/dRe a + i dL/dIm a: 2 Y^H g for m > 0, Re Y^H g for m = 0) and
  ``nusht_vjp_points`` (sum over maps of g * dmap/dtheta, g * dmap/dphi).
The plan's points are fixed; ``theta`` / ``phi`` only carry the gradient back to the caller,
and must hold the coordinates the plan was built on (checked: ValueError otherwise).
``synthesis_spin(plan, spin, alm)`` is the spin-weighted synthesis with its coefficient
gradient (``nusht_vjp_alm_spin``).
"""
from __future__ import annotations

import torch


class SynthesisFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alm, theta, phi, plan):
        need_pos = bool(ctx.needs_input_grad[1] or ctx.needs_input_grad[2])
        a = alm.detach()
        if need_pos:
            f, dth, dph = plan.synthesis_deriv(a)
            ctx.save_for_backward(dth, dph)
        else:
            f = plan.synthesis(a)
        ctx.plan = plan
        ctx.need_pos = need_pos
        ctx.squeeze = alm.dim() == 1
        return f[0] if ctx.squeeze else f

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        g2 = g.reshape(-1, plan.npts).contiguous()
        grad_alm = grad_th = grad_ph = None
        if ctx.needs_input_grad[0]:
            grad_alm = plan.vjp_alm(g2)
            if ctx.squeeze:
                grad_alm = grad_alm[0]
        if ctx.need_pos:
            dth, dph = ctx.saved_tensors
            gt, gp = plan.vjp_points(g2, dth, dph, ctx.needs_input_grad[1],
                                     ctx.needs_input_grad[2])
            grad_th = gt if ctx.needs_input_grad[1] else None
            grad_ph = gp if ctx.needs_input_grad[2] else None
        return grad_alm, grad_th, grad_ph, None


class SpinSynthesisFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alm, plan, spin):
        ctx.plan = plan
        ctx.spin = spin
        ctx.squeeze = alm.dim() == 2
        f = plan.synthesis_spin(spin, alm.detach())
        return f[0] if ctx.squeeze else f

    @staticmethod
    def backward(ctx, g):
        grad = ctx.plan.vjp_alm_spin(ctx.spin, g.reshape(-1, 2, ctx.plan.npts).contiguous())
        return (grad[0] if ctx.squeeze else grad), None, None


def synthesis_spin(plan, spin, alm):
    """Differentiable spin-weighted synthesis (gradient/curl coefficients [F, 2, nalm] ->
    (Q, U) maps [F, 2, npts]) with respect to the coefficients; the backward pass is
    ``nusht_vjp_alm_spin``."""
    return SpinSynthesisFn.apply(alm, plan, spin)


def synthesis(plan, alm, theta=None, phi=None):
    """Differentiable type-2 transform on the plan's points."""
    if theta is not None or phi is not None:
        plan.check_points(theta, phi)
    if theta is None:
        theta = torch.zeros(plan.npts, dtype=torch.float64, device=alm.device)
    if phi is None:
        phi = torch.zeros(plan.npts, dtype=torch.float64, device=alm.device)
    return SynthesisFn.apply(alm, theta, phi, plan)
