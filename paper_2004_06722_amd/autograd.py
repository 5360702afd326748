"""Differentiable variable-coefficient Poisson solve on the HIP path.

u = A(kappa)^{-1} b, where A(kappa) is the masked stiffness matrix with the
coefficient kappa at the quadrature points (section 4, eq. (hm1)/(ip1) with
mu = kappa; section 5, eq. (bk5x) with kappa_q G_q). A is symmetric, so the
backward pass solves A lambda = dL/du with the same operator (adjoint CG) and
returns

    dL/dkappa_q = - sum_c (D lambda_c)_q^T G_q (D u_c)_q   (bp_grad_kappa)
    dL/db       = lambda.

The misfit L = 1/2 sum_c (u - u_t)_c^T M (u - u_t)_c and its gradient M (u - u_t)
come from bp_mass_misfit. Both solves, the gradient kernel and the misfit run
in libbp.so; torch only holds the tensors, records the graph and scales the
returned gradients by the incoming one (the chain rule).
"""
from __future__ import annotations

import torch

from .bp import Operator


class PoissonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa: torch.Tensor, b: torch.Tensor, op: Operator, rtol: float,
                maxit: int):
        op.set_coeff(kappa.detach().contiguous())
        u, st = op.pcg_solve(b.detach().contiguous(), rtol=rtol, maxit=maxit)
        if not st["converged"]:
            raise RuntimeError(f"forward solve did not reach rtol={rtol}: {st}")
        ctx.op, ctx.rtol, ctx.maxit = op, rtol, maxit
        ctx.save_for_backward(kappa, u)
        return u

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        kappa, u = ctx.saved_tensors
        op = ctx.op
        op.set_coeff(kappa.detach().contiguous())
        lam, st = op.pcg_solve(grad_u.detach().contiguous(), rtol=ctx.rtol, maxit=ctx.maxit)
        if not st["converged"]:
            raise RuntimeError(f"adjoint solve did not reach rtol={ctx.rtol}: {st}")
        g_kappa = op.grad_kappa(lam, u) if ctx.needs_input_grad[0] else None
        g_b = lam if ctx.needs_input_grad[1] else None
        return g_kappa, g_b, None, None, None


class MassNormLoss(torch.autograd.Function):
    """L = 1/2 sum_c d_c^T M d_c with d = u - u_target and M the operator's own
    (unmasked) mass matrix; dL/du = M d since M is symmetric."""

    @staticmethod
    def forward(ctx, u: torch.Tensor, u_target: torch.Tensor, op: Operator):
        # the library forms d, M d and the sum (bp_mass_misfit)
        loss, Md = op.mass_misfit(u.detach().contiguous(), u_target.detach().contiguous())
        ctx.save_for_backward(Md)
        return torch.tensor(loss, dtype=torch.float64, device=u.device)

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (Md,) = ctx.saved_tensors
        return g * Md, -g * Md, None


def poisson_solve(op: Operator, kappa: torch.Tensor, b: torch.Tensor, rtol: float = 1e-12,
                  maxit: int = 100000) -> torch.Tensor:
    return PoissonSolve.apply(kappa, b, op, rtol, maxit)


def mass_norm_loss(op: Operator, u: torch.Tensor, u_target: torch.Tensor) -> torch.Tensor:
    return MassNormLoss.apply(u, u_target, op)
