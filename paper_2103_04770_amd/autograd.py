"""torch.autograd wrappers around the library's solves and their adjoints.

Forward passes call the library (helmholtz_solve, fftg_solve, fftg_damage,
fftg_ell2); backward passes call its adjoint entry points (helmholtz_adjoint,
fftg_solve_adjoint, fftg_damage_adjoint, fftg_phase_sums).  The solves are
differentiated implicitly at the converged state: nothing of the Krylov
iterations is kept.  Tensors are CUDA float64 in numpy axis order.

    ell2     = ell2_field(solver, ell, phase, table)     d/d ell (per phase)
    abar     = helmholtz(solver, alpha, ell2)            d/d alpha, d/d ell2
    D        = damage(solver, abar, phase, table)        d/d abar
    eps, sig = mechanics(solver, D, phase, table, nfields, state_n, target)
                                                         d/d D (frozen damage)

staggered_increment() differentiates a whole converged increment of the
staggered scheme (the damage feeding back into the local sources through the
mechanics) in the per-phase lengths, through fftg_staggered_adjoint.
staggered_path() differentiates a whole load path of such increments (every
increment's plastic history carried into the next), walking them backwards
with fftg_increment_adjoint (path_gradient).

one_pass() chains them for one field: the per-voxel local source alpha (e.g.
the local equivalent plastic strain) and the per-phase lengths give abar, the
damage, and the strain and stress of the mechanics at that damage, so that
torch.autograd.grad of <sigma_11> or <D> with respect to alpha and the
lengths runs entirely through the adjoints.
"""
from __future__ import annotations

import numpy as np
import torch


def _with_lengths(table, ell, field):
    tab = []
    for q, t in enumerate(table):
        t = dict(t)
        e = list(t["ell"]) + [0.0] * (field + 1 - len(t["ell"]))
        e[field] = float(ell[q])
        t["ell"] = e
        tab.append(t)
    return tab


class _Ell2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ell, solver, phase, table, field):
        tab = _with_lengths(table, ell.detach().cpu().numpy(), field)
        out = torch.empty(solver.spatial, dtype=torch.float64, device="cuda")
        solver.fftg_ell2(phase, tab, field, out)
        ctx.save_for_backward(ell)
        ctx.args = (solver, phase, len(table))
        return out

    @staticmethod
    def backward(ctx, g):
        (ell,) = ctx.saved_tensors
        solver, phase, nphase = ctx.args
        sums = solver.fftg_phase_sums(phase, nphase, g.contiguous())
        return (2.0 * ell * torch.from_numpy(sums).to(ell), None, None, None, None)


def ell2_field(solver, ell, phase, table, field=0):
    """ell2(x) = ell_q^2 on phase q, differentiable in the per-phase lengths ell."""
    return _Ell2.apply(ell, solver, phase, table, field)


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


class _Damage(torch.autograd.Function):
    @staticmethod
    def forward(ctx, abar, solver, phase, table, hist):
        D = torch.empty_like(abar)
        solver.fftg_damage(phase, table, abar.shape[0], abar.contiguous(), hist, D)
        ctx.save_for_backward(abar)
        ctx.args = (solver, phase, table, hist)
        return D

    @staticmethod
    def backward(ctx, gD):
        (abar,) = ctx.saved_tensors
        solver, phase, table, hist = ctx.args
        ga = torch.empty_like(abar)
        solver.fftg_damage_adjoint(phase, table, abar.shape[0], abar, hist, gD.contiguous(), ga)
        return ga, None, None, None, None


def damage(solver, abar, phase, table, hist=None):
    """Damage fields [J][N] from the non-local fields abar [J][N] (the law of
    the staggered step), differentiable in abar."""
    if hist is None:
        hist = torch.zeros_like(abar)
    return _Damage.apply(abar, solver, phase, table, hist)


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
        return eps, sig

    @staticmethod
    def backward(ctx, geps, gsig):
        D, eps = ctx.saved_tensors
        solver, phase, table, nfields, state_n, target, opts = ctx.args
        mu = torch.empty_like(eps)
        dD = torch.empty_like(D)
        geps = torch.zeros_like(eps) if geps is None else geps.contiguous()
        solver.fftg_solve_adjoint(phase, table, nfields, D.contiguous(), state_n, target, eps,
                                  geps, mu, dD, cg_tol=opts.get("cg_tol", 1e-8),
                                  cg_maxit=opts.get("cg_maxit", 5000),
                                  gsig=None if gsig is None else gsig.contiguous())
        return dD, None, None, None, None, None, None, None, None


def mechanics(solver, D, phase, table, nfields, state_n, target, eps0=None, **opts):
    """(eps, sigma) of the mechanics solve at frozen damage D (fftg_solve),
    differentiable in D."""
    if eps0 is None:
        eps0 = torch.zeros((solver.c,) + solver.spatial, dtype=torch.float64, device=D.device)
    return _Mechanics.apply(D, solver, phase, table, nfields, state_n, target, eps0, opts)


def one_pass(solver, alpha, ell, phase, table, target, field=0, helm_tol=1e-10, **opts):
    """alpha (local source of `field`, [N]) and per-phase lengths ell ->
    abar, D, eps, sigma: one pass of the staggered scheme (mechanics at the
    damage of the non-local field), differentiable in alpha and ell.  The
    table must have one non-local field (nfields = 1)."""
    ell2 = ell2_field(solver, ell, phase, table, field)
    abar = helmholtz(solver, alpha, ell2, tol=helm_tol)
    D = damage(solver, abar.unsqueeze(0), phase, table)
    state_n = torch.zeros((7,) + solver.spatial, dtype=torch.float64, device=alpha.device)
    eps, sig = mechanics(solver, D, phase, table, 1, state_n, target, **opts)
    return abar, D, eps, sig


class _StaggeredIncrement(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ell, solver, phase, table, nfields, state_n, target, field, opts):
        tab = _with_lengths(table, ell.detach().cpu().numpy(), field)
        state = state_n.detach().clone().contiguous()
        sig = torch.empty((solver.c,) + solver.spatial, dtype=torch.float64, device="cuda")
        d = solver.staggered_step(phase, tab, nfields, state, target, sig, **opts)
        if not d["converged"]:
            raise RuntimeError("staggered increment did not converge: %s" % d)
        c = solver.c
        abar = state[c + 7 + nfields:].clone()
        ctx.save_for_backward(ell, state_n, state)
        ctx.args = (solver, phase, tab, nfields, target, field, opts, len(table))
        return sig, abar

    @staticmethod
    def backward(ctx, gsig, gabar):
        ell, state_n, state = ctx.saved_tensors
        solver, phase, tab, nfields, target, field, opts, nphase = ctx.args
        dell2 = torch.empty((nfields,) + solver.spatial, dtype=torch.float64, device="cuda")
        tol = min(opts.get("stagger_tol", 1e-6), 1e-8)
        d = solver.fftg_staggered_adjoint(
            phase, tab, nfields, state_n.contiguous(), state, target, dell2,
            g_sig=None if gsig is None else gsig.contiguous(),
            g_abar=None if gabar is None else gabar.contiguous(),
            cg_tol=opts.get("cg_tol", 1e-8), pcg_tol=opts.get("pcg_tol", 1e-8), tol=tol,
            maxit=opts.get("max_stagger", 20) * 10)
        if not d["converged"]:
            raise RuntimeError("staggered adjoint did not converge: %s" % d)
        sums = solver.fftg_phase_sums(phase, nphase, dell2[field].contiguous())
        return (2.0 * ell * torch.from_numpy(sums).to(ell), None, None, None, None, None, None,
                None, None)


def staggered_increment(solver, ell, phase, table, nfields, state_n, target, field=0, **opts):
    """One converged staggered increment from the packed state_n (returns the
    stress field and the non-local fields at t_{n+1}), differentiable in the
    per-phase lengths `ell` of `field` (the total derivative at the fixed
    point).  Sources covered by the adjoint: the J2 damage matrix."""
    return _StaggeredIncrement.apply(ell, solver, phase, table, nfields, state_n, target, field,
                                     opts)


def path_gradient(solver, phase, table, nfields, states, targets, g_sig, cg_tol=1e-10,
                  pcg_tol=1e-10, tol=1e-10, maxit=200):
    """dJ/dell2_j(x) (nfields, *S) of J = g_sig . sigma after the last
    increment of a converged load path: states[k] is the packed state before
    increment k (states[-1] after the last), targets[k] its macro target.
    The increments are walked last to first; each fftg_increment_adjoint call
    returns the cotangents of the history (plastic state, damage history) its
    increment started from, which the call for the increment before receives.
    Returns (dell2, stats of every call, last first)."""
    S = solver.spatial
    f64 = dict(dtype=torch.float64, device="cuda")
    total = torch.zeros((nfields,) + S, **f64)
    dl = torch.empty((nfields,) + S, **f64)
    cur = None                                     # (g_epsp, g_kappa, g_hist) coming in
    nxt = (torch.empty((6,) + S, **f64), torch.empty(S, **f64),
           torch.empty((nfields,) + S, **f64))
    log = []
    for k in range(len(targets) - 1, -1, -1):
        d = solver.fftg_increment_adjoint(
            phase, table, nfields, states[k], states[k + 1], targets[k], dl, *nxt,
            g_sig=g_sig if k == len(targets) - 1 else None,
            g_epsp=None if cur is None else cur[0], g_kappa=None if cur is None else cur[1],
            g_hist=None if cur is None else cur[2], cg_tol=cg_tol, pcg_tol=pcg_tol, tol=tol,
            maxit=maxit)
        if not d["converged"]:
            raise RuntimeError("increment adjoint %d did not converge: %s" % (k, d))
        log.append(d)
        total += dl
        if cur is None:
            cur = tuple(torch.empty_like(t) for t in nxt)
        cur, nxt = nxt, cur
    return total, log


class _StaggeredPath(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ell, solver, phase, table, nfields, state_0, targets, field, opts):
        tab = _with_lengths(table, ell.detach().cpu().numpy(), field)
        state = state_0.detach().clone().contiguous()
        sig = torch.empty((solver.c,) + solver.spatial, dtype=torch.float64, device="cuda")
        states = [state.clone()]
        for k, tgt in enumerate(targets):
            d = solver.staggered_step(phase, tab, nfields, state, tgt, sig, **opts)
            if not d["converged"]:
                raise RuntimeError("increment %d did not converge: %s" % (k, d))
            states.append(state.clone())
        ctx.save_for_backward(ell)
        ctx.args = (solver, phase, tab, nfields, states, targets, field, opts, len(table))
        return sig

    @staticmethod
    def backward(ctx, gsig):
        (ell,) = ctx.saved_tensors
        solver, phase, tab, nfields, states, targets, field, opts, nphase = ctx.args
        dell2, _ = path_gradient(solver, phase, tab, nfields, states, targets, gsig.contiguous(),
                                 cg_tol=opts.get("cg_tol", 1e-8), pcg_tol=opts.get("pcg_tol", 1e-8),
                                 tol=min(opts.get("stagger_tol", 1e-6), 1e-8),
                                 maxit=opts.get("max_stagger", 20) * 10)
        sums = solver.fftg_phase_sums(phase, nphase, dell2[field].contiguous())
        return (2.0 * ell * torch.from_numpy(sums).to(ell), None, None, None, None, None, None,
                None, None)


def staggered_path(solver, ell, phase, table, nfields, state_0, targets, field=0, **opts):
    """The stress field after a load path of converged staggered increments
    (macro targets `targets`, from the packed state_0), differentiable in the
    per-phase lengths `ell` of `field` through the whole path.  Keeps every
    increment's packed state on the device.  Phases covered: J2 damage
    (linear hardening), elastic and cracking."""
    return _StaggeredPath.apply(ell, solver, phase, table, nfields, state_0, list(targets), field,
                                opts)
