"""Differentiable random batch Ewald forces for PyTorch.

``rbe_forces(ctx, pos, q)`` returns the forces of the active mode sample
(Fourier part of eq. 3.6 plus the real-space part of eq. 2.11 and the
shifted LJ of eq. 4.1, as selected by ``parts``) as a tensor that carries a
gradient: the backward pass calls the library's hand-written adjoint
``rbe_forces_vjp`` (vector-Jacobian product with respect to positions and
charges at the same mode sample).  Both directions run in the HIP kernels of
librbe; this module only allocates outputs and passes pointers.

``force_matching_loss`` is the loss of a force-matching fit: the mean over
all 3N components of (F - F_ref)^2 with a constant reference F_ref.
"""
from __future__ import annotations

import torch

from . import rbe as R


class RBEForces(torch.autograd.Function):
    """F(pos, q) at the context's active modes; backward through the adjoint."""

    @staticmethod
    def forward(fctx, pos, q, ctx, parts):
        pos = pos.detach().contiguous()
        q = q.detach().contiguous()
        F = torch.zeros_like(pos)
        if parts & R.RBE_PART_KSPACE:
            R.rbe_kspace_forces(ctx, pos, q, F)
        if parts & R.RBE_PART_REAL:
            R.rbe_real_forces(ctx, pos, q, F, accumulate=bool(parts & R.RBE_PART_KSPACE))
        fctx.save_for_backward(pos, q)
        fctx.rbe_ctx = ctx
        fctx.parts = parts
        return F

    @staticmethod
    def backward(fctx, grad_force):
        pos, q = fctx.saved_tensors
        gF = grad_force.contiguous()
        gpos = torch.empty_like(pos)
        gq = torch.empty_like(q)
        R.rbe_forces_vjp(fctx.rbe_ctx, pos, q, gF, gpos, gq, fctx.parts)
        need_pos, need_q = fctx.needs_input_grad[0], fctx.needs_input_grad[1]
        return (gpos if need_pos else None), (gq if need_q else None), None, None


def rbe_forces(ctx, pos, q, parts=R.RBE_PART_ALL):
    """Forces [3, N] of the active mode sample, differentiable in pos and q."""
    return RBEForces.apply(pos, q, ctx, parts)


def force_matching_loss(ctx, pos, q, F_ref, parts=R.RBE_PART_ALL):
    """Mean over all 3N components of (F(pos, q) - F_ref)^2; F_ref is constant."""
    F = rbe_forces(ctx, pos, q, parts)
    return ((F - F_ref.detach()) ** 2).mean()
