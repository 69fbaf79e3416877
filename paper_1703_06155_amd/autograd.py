"""Differentiable solve: x = A(chi)^-1 b through the H^2 factorization.

The forward pass is ``h2_solve``; the backward pass is the conjugate-transpose
sweep over the same factors (``h2_solve_adjoint``), which gives the gradient
with respect to the right-hand side, and ``h2_contrast_gradient``, which turns
it into the gradient with respect to the per-cell contrast (column j of A is
chi_j (k^2 h^3 G e_j + c e_j) + e_j, so dA/dchi_j = (A e_j - e_j) / chi_j).
Both passes can be refined against the H^2 matrix to a relative residual.
"""
from __future__ import annotations

import numpy as np
import torch

from . import H2


class H2Solve(torch.autograd.Function):
    """x = H2Solve.apply(b, chi, solver, tol, max_iter).

    ``b``: complex128 CUDA tensor (N or N x nrhs); ``chi``: float64 tensor of
    the contrast the solver was factored with (the tensor the gradient flows
    to); ``solver``: a factored :class:`H2`; ``tol`` > 0 refines both the
    solve and the adjoint solve to that relative residual.
    """

    @staticmethod
    def forward(ctx, b, chi, solver: H2, tol: float = 0.0, max_iter: int = 20):
        if chi.numel() != solver.n or not np.array_equal(chi.detach().cpu().numpy(), solver.chi):
            raise ValueError("chi differs from the contrast the solver was built or set with")
        x = solver.solve(b, tol=tol, max_iter=max_iter)
        ctx.solver, ctx.tol, ctx.max_iter = solver, tol, max_iter
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        gx = gx.to(torch.complex128).contiguous()
        lam = ctx.solver.solve_adjoint(gx, tol=ctx.tol, max_iter=ctx.max_iter)
        gb = lam if ctx.needs_input_grad[0] else None
        gchi = ctx.solver.contrast_gradient(x, gx, lam) if ctx.needs_input_grad[1] else None
        return gb, gchi, None, None, None


def h2_solve(b, chi, solver: H2, tol: float = 0.0, max_iter: int = 20):
    """Differentiable x = A(chi)^-1 b (see :class:`H2Solve`)."""
    return H2Solve.apply(b, chi, solver, tol, max_iter)
