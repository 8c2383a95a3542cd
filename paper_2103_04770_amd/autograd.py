"""torch.autograd wrappers of the two solves of the staggered scheme.

The forward passes call helmholtz_solve / fftg_solve; the backward passes call
the library's adjoint entry points (implicit differentiation at the converged
state: nothing of the Krylov iterations is kept).  Every tensor is a CUDA
float64 tensor on the solver's device, in numpy axis order.

    abar = helmholtz(solver, alpha, ell2)          d/d alpha and d/d ell2
    eps  = mechanics(solver, D, phase, table, nfields, state_n, target)
                                                   d/d D (frozen damage)
"""
from __future__ import annotations

import torch


class _Helmholtz(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha, ell2, solver, tol, maxit):
        abar = torch.zeros_like(alpha)
        solver.helmholtz_solve(alpha.contiguous(), ell2.contiguous(), abar, tol=tol, maxit=maxit)
        ctx.save_for_backward(ell2, abar)
        ctx.solver, ctx.tol, ctx.maxit = solver, tol, maxit
        return abar

    @staticmethod
    def backward(ctx, gbar):
        ell2, abar = ctx.saved_tensors
        dalpha = torch.zeros_like(abar)
        dell2 = torch.empty_like(abar)
        ctx.solver.helmholtz_adjoint(ell2, abar, gbar.contiguous(), dalpha, dell2, tol=ctx.tol,
                                     maxit=ctx.maxit)
        return dalpha, dell2, None, None, None


def helmholtz(solver, alpha, ell2, tol=1e-10, maxit=2000):
    """abar = L(ell2)^-1 alpha (Algorithm 2), differentiable in alpha and ell2."""
    return _Helmholtz.apply(alpha, ell2, solver, tol, maxit)


class _Mechanics(torch.autograd.Function):
    @staticmethod
    def forward(ctx, D, solver, phase, table, nfields, state_n, target, eps0, opts):
        eps = eps0.detach().clone().contiguous()
        sig = torch.empty_like(eps)
        st1 = torch.empty_like(state_n)
        alpha = torch.empty_like(D) if nfields else None
        solver.fftg_solve(phase, table, nfields, D.contiguous() if nfields else None, state_n,
                          target, eps, sig, st1, alpha, **opts)
        ctx.save_for_backward(D, eps)
        ctx.args = (solver, phase, table, nfields, state_n, target, opts)
        return eps

    @staticmethod
    def backward(ctx, geps):
        D, eps = ctx.saved_tensors
        solver, phase, table, nfields, state_n, target, opts = ctx.args
        mu = torch.empty_like(eps)
        dD = torch.empty_like(D)
        solver.fftg_solve_adjoint(phase, table, nfields, D.contiguous(), state_n, target, eps,
                                  geps.contiguous(), mu, dD, cg_tol=opts.get("cg_tol", 1e-8),
                                  cg_maxit=opts.get("cg_maxit", 5000))
        return dD, None, None, None, None, None, None, None, None


def mechanics(solver, D, phase, table, nfields, state_n, target, eps0=None, **opts):
    """Converged strain of the mechanics solve at frozen damage D
    (fftg_solve), differentiable in D."""
    if eps0 is None:
        eps0 = torch.zeros((solver.c,) + solver.spatial, dtype=torch.float64, device=D.device)
    return _Mechanics.apply(D, solver, phase, table, nfields, state_n, target, eps0, opts)
