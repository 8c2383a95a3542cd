"""Gradients of the two solves of the staggered scheme by implicit
differentiation at the converged state (adjoint method).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Helmholtz (Sec. 3.2.3, Algorithm 2).  In real space the operator is
    L(ell2) u = u + sum_j G_j^T ( ell2 * G_j u ),   G_j = F^-1 diag(i q~_j) F,
symmetric positive definite (G_j^T = -G_j).  For abar = L^-1 alpha and a
scalar J(abar) with gbar = dJ/dabar:
    lam        = L^-1 gbar                        (same PCG: L is symmetric)
    dJ/dalpha  = lam
    dJ/dell2(x) = - sum_j (G_j lam)(x) (G_j abar)(x)
since dJ = lam . (dalpha - dL abar) and dL = sum_j G_j^T diag(dell2) G_j.

Mechanics at frozen damage (Sec. 3.2.2).  The converged strain solves
G*(sigma(eps, D) - Sigma_bar) = 0 with eps - (macro part) compatible; with
sigma = (1 - D) sigma_eff(eps) in a damaging phase, d sigma / dD = -sigma_eff.
Linearising, G*(K : deps) = G*(sigma_eff dD) on the admissible space V
(compatible fluctuations plus means on the stress-controlled components),
where A = G* K is symmetric positive definite.  For J(eps, sigma) with
geps = dJ/deps and gsig = dJ/dsigma (partial derivatives), the strain
cotangent is g = geps + K gsig (K symmetric), and
    mu = A^-1 G*(g)  (plain CG, as the Newton correction)
    dJ/dD_j(x) = (mu(x) - gsig(x)) : sigma_eff(x)   for a voxel whose phase
                 is driven by field j (0 elsewhere),
since dJ = g . deps - gsig . sigma_eff dD, g . deps = (G* g) . deps =
mu . G*(sigma_eff dD), and mu lies in V.  K is the consistent tangent at the
converged strain, recomputed from the state (Krylov iterates are never
stored).
"""
from __future__ import annotations

import numpy as np

from . import galerkin, helmholtz, material, spectral


def grad_fields(u, qt):
    """Real gradient components G_j u (j in physical order) of a real field."""
    uh = np.fft.fftn(u)
    return [np.real(np.fft.ifftn(1j * qj * uh)) for qj in qt]


def helmholtz_adjoint(abar, gbar, ell2, h=1.0, scheme=spectral.ROTATED, ell2_ref=-1.0,
                      tol=1e-8, maxit=1000):
    """Returns dict(dalpha, dell2, iters) for J(abar), gbar = dJ/dabar."""
    S = abar.shape
    r = helmholtz.helmholtz_solve(gbar, ell2, h=h, scheme=scheme, ell2_ref=ell2_ref, tol=tol,
                                  maxit=maxit)
    lam = r["abar"]
    _, qt = spectral.symbols(S, h, scheme)
    qt = [np.broadcast_to(v, S) for v in qt]
    gl, ga = grad_fields(lam, qt), grad_fields(abar, qt)
    dell2 = -sum(a * b for a, b in zip(gl, ga))
    return dict(dalpha=lam, dell2=dell2, iters=r["iters"])


def phase_length_gradient(dell2, phase, table, j):
    """dJ/d ell_q of field j for every phase q, from dJ/dell2(x)
    (ell2(x) = ell_q^2 on phase q)."""
    return np.array([2.0 * float(table[q]["ell"][j]) * float(dell2[phase == q].sum())
                     for q in range(len(table))])


def damage_adjoint(phase, table, abar, hist, gD):
    """gabar = gD dD/dabar for the linear damage law of material.
    damage_from_nonlocal: slope 1/(dR - dC) where dC < abar < dR below the
    cap and abar (not the cracking history) drives D; 0 elsewhere (one-sided
    at the kinks)."""
    g = np.zeros(abar.shape)
    for p, ph in enumerate(table):
        j = ph["dfield"]
        if ph["model"] == "gtn":
            raise NotImplementedError("adjoint of the Gurson porosity update")
        if j < 0 or ph["model"] == "elastic":
            continue
        sel = phase == p
        a = abar[j][sel]
        by_abar = np.ones(a.shape, bool) if ph["model"] != "elastic_cracking" else \
            ~(hist[j][sel] > a)
        d = (a - ph["dC"]) / (ph["dR"] - ph["dC"])
        inside = by_abar & (d > 0.0) & (d < ph["dmax"])
        g[j][sel] = np.where(inside, gD[j][sel] / (ph["dR"] - ph["dC"]), 0.0)
    return g


def mechanics_adjoint(phase, table, D, epsp_n, kappa_n, target, eps, gbar, nfields, h=1.0,
                      scheme=spectral.ROTATED, cg_tol=1e-8, cg_maxit=5000, gsig=None):
    """Returns dict(mu, dD, cg_iters) for J(eps, sigma) with gbar = dJ/deps and
    gsig = dJ/dsigma (c, *S; None = 0), at the converged strain eps of
    galerkin.fftg_solve with the same inputs."""
    mask = np.asarray(target[0])
    S = phase.shape
    q = spectral.projection_symbol(S, h, scheme)
    st = material.constitutive(eps, epsp_n, kappa_n, D, phase, table, nfields)
    C = st["C"]
    g = gbar if gsig is None else gbar + material.apply_tangent(C, gsig)
    b = galerkin.project(g, q, mask)
    mu, it, _, _ = galerkin.cg(lambda p: galerkin.project(material.apply_tangent(C, p), q, mask),
                               b, cg_tol, cg_maxit)
    sig = st["sigma"]
    dD = np.zeros((nfields,) + S)
    for p, ph in enumerate(table):
        j = ph["dfield"]
        if ph["model"] == "gtn":
            raise NotImplementedError("adjoint of the Gurson return at frozen porosity")
        if j < 0 or ph["model"] == "elastic":
            continue
        sel = phase == p
        w = 1.0 - D[j][sel]
        seff = sig[:, sel] / w[None]
        m = mu[:, sel] if gsig is None else mu[:, sel] - gsig[:, sel]
        dD[j][sel] = (m * seff).sum(axis=0)
    return dict(mu=mu, dD=dD, cg_iters=it)
