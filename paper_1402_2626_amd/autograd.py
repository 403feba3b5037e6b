"""``torch.autograd.Function`` for F(x) with the adjoint J^H v as backward.

Forward runs ``pe_eval`` with J = NULL (F only).  Backward runs
``pe_eval_adjoint``, which never forms J: with the incoming gradient g (the
re and im planes of grad_F read as a complex vector), the gradient with
respect to the re and im planes of x is the complex vector J(x)^H g.  For a
real loss of a holomorphic F this is the exact real gradient: for
l = 1/2 |F|^2, g = F and the result is the Gauss-Newton gradient J^H F.

Limbs: at level L > 1 the incoming gradient's limbs are read as a level-L
expansion (their sum) and the returned gradient is a level-L expansion in the
limbs of x's layout.  At L = 1 this is plain real-valued autograd.
"""
from __future__ import annotations

import torch


class PolyEval(torch.autograd.Function):
    """``F = PolyEval.apply(x, system)`` for x[P, 2, L, n] float64 on the GPU."""

    @staticmethod
    def forward(ctx, x, system):
        F, _ = system.eval(x.contiguous(), want_J=False)
        ctx.save_for_backward(x)
        ctx.system = system
        return F

    @staticmethod
    def backward(ctx, grad_F):
        (x,) = ctx.saved_tensors
        g = ctx.system.adjoint(x.contiguous(), grad_F.contiguous())
        return g, None


def poly_eval(x, system):
    return PolyEval.apply(x, system)
