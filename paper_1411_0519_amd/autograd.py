"""Differentiable heat-equation solve: u = L^{-1} F(f, u0) with a hand-written
adjoint (backward-in-time multigrid on L^T) for the backward pass.

forward:  F = rhs(f, u0) (load vector of Sec. 1), u = solve(L, F)
backward: lam = solve(L^T, dJ/du), dJ/df = rhs^T(lam)_f, dJ/du0 = rhs^T(lam)_u0
"""
import torch


class HeatSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, u0, solver, rtol, maxit):
        F = solver.rhs(f.contiguous(), u0.contiguous() if u0 is not None else None)
        u, _, _ = solver.solve(F, rtol=rtol, maxit=maxit)
        ctx.solver, ctx.rtol, ctx.maxit = solver, rtol, maxit
        ctx.has_u0 = u0 is not None
        return u

    @staticmethod
    def backward(ctx, grad_u):
        lam, gf, gu0, _, _ = ctx.solver.adjoint(grad_u.contiguous(), rtol=ctx.rtol, maxit=ctx.maxit)
        return gf, (gu0 if ctx.has_u0 else None), None, None, None


def heat_solve(f, u0, solver, rtol=1e-12, maxit=100):
    """u(f, u0) on the solver's grid; differentiable in f and u0."""
    return HeatSolve.apply(f, u0, solver, rtol, maxit)
