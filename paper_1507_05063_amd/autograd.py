"""Differentiable EXCMG solve: a torch.autograd.Function whose backward is the adjoint solve.

Forward: u = EXCMG(f, g) (interior: the compact-scheme solution; boundary: g).
Backward, for an upstream gradient G = dL/du: solve M lambda = G_I with the same symmetric operator M = -A_h (by the
same cascade), then dL/df = -R^T lambda and dL/dg = A_IB^T lambda + G on the boundary (excmg_adjoint).  The gradient
is that of the exact discrete solution map; the forward solve's dependence on its tolerance is not differentiated.
"""
from __future__ import annotations

import torch


class ExcmgSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, g, solver):
        u, _, _ = solver.solve(f.detach().contiguous(), g.detach().contiguous())
        ctx.solver = solver
        return u

    @staticmethod
    def backward(ctx, grad_u):
        dLdf, dLdg, _, _ = ctx.solver.adjoint(grad_u.detach().contiguous())
        return dLdf, dLdg, None


def solve(f, g, solver):
    """u = EXCMG(f, g) with gradients to f and g."""
    return ExcmgSolve.apply(f, g, solver)
