"""One load increment of the iterated staggered scheme (Sec. 3.2, Algorithm 1).

Per increment n -> n+1, with macro targets (mask, E, S) at t_{n+1}:
  initial guess: eps^(0) = eps_n with the strain-controlled means moved to
                 E_{n+1}; abar^(0) = abar_n
  repeat (k = 0, 1, ...):
    (i)   mechanics with the non-local fields frozen at abar^(k):
          D^(k) = D(abar^(k)), Newton + CG (galerkin.fftg_solve) from eps^(k)
          -> eps^(k+1), eps_p, eps_p(eq), local sources alpha_j
    (ii)  for every field j: Helmholtz PCG (helmholtz.helmholtz_solve) with
          source alpha_j, lengths ell_j(x) of the phase table, started from
          abar_j^(k) -> abar_j^(k+1)
    (iii) ERR = max( max_x ||eps^(k+1) - eps^(k)||_F / ||<eps^(k+1)>||_F ,
                     ||abar_j^(k+1) - abar_j^(k)||_2 / ||abar_j^(k+1)||_2 )
  while ERR > TOL and k < max_iters.  (The paper's loop test reads
  "ERR < TOL"; iterating while the error is above the tolerance is the
  meaning used.)  The field error is taken as 0 when the field did not
  change, and its denominator is floored at 1e-12 sqrt(N).
  commit: the state at t_{n+1} is the last iterate; the cracking history is
  hist <- max(hist, abar), and a Gurson phase stores its porosity f_{n+1}
  of the final non-local fields in its first history slot.
With max_iters = 1 this is the "simple staggered" variant (one pass).
"""
from __future__ import annotations

import numpy as np

from . import galerkin, helmholtz, material, spectral


def ell2_field(phase, table, j):
    tab = np.array([float(ph["ell"][j]) ** 2 for ph in table])
    return tab[phase]


def staggered_step(phase, table, nfields, state, target, h=1.0,
                   scheme=spectral.ROTATED, cg_tol=1e-8, cg_maxit=5000,
                   pcg_tol=1e-8, pcg_maxit=2000, newton_tol=1e-8,
                   newton_maxit=50, stagger_tol=1e-6, max_stagger=20,
                   newton_div=0, abort_on_mech_failure=False):
    """state: dict(eps (c,*S), epsp (6,*S), kappa S, hist (J,*S), abar (J,*S)).
    newton_div: see galerkin.fftg_solve.  abort_on_mech_failure: leave the
    loop as soon as a mechanics solve does not converge (the increment is then
    reported as not converged; the adaptive load driver cuts it back).
    Returns (new_state, sigma, homog dict(sigma=<sigma>, eps=<eps>), stats);
    stats["mech_converged"] tells whether the last mechanics solve converged,
    stats["inner_converged"] whether every inner solve of the last pass (the
    Newton iteration and each Helmholtz PCG) met its stop test."""
    mask, Emac, Smac = target
    S = phase.shape
    N = int(np.prod(S))
    J = nfields
    epsp_n, kappa_n = state["epsp"], state["kappa"]
    hist_n = state["hist"]
    eps_k = galerkin.set_strain_means(state["eps"], np.asarray(mask), Emac)
    abar_k = state["abar"].copy()
    ell2 = [ell2_field(phase, table, j) for j in range(J)]
    stats = dict(stagger_iters=0, newton_iters=0, cg_iters=0, pcg_iters=0, err=np.inf,
                 converged=False, mech_converged=False, inner_converged=False)
    mech = None
    for k in range(max_stagger):
        D = material.damage_from_nonlocal(phase, table, abar_k, hist_n, state["abar"])
        mech = galerkin.fftg_solve(phase, table, D, epsp_n, kappa_n, target, eps_k,
                                   h=h, scheme=scheme, cg_tol=cg_tol, cg_maxit=cg_maxit,
                                   newton_tol=newton_tol, newton_maxit=newton_maxit,
                                   nfields=J, newton_div=newton_div)
        stats["newton_iters"] += mech["newton_iters"]
        stats["cg_iters"] += mech["cg_iters"]
        stats["mech_converged"] = mech["converged"]
        stats["inner_converged"] = False
        if abort_on_mech_failure and not mech["converged"]:
            stats["stagger_iters"] = k + 1
            eps_k = mech["eps"]
            break
        abar_new = np.empty_like(abar_k)
        inner_ok = bool(mech["converged"])
        for j in range(J):
            hs = helmholtz.helmholtz_solve(mech["alpha"][j], ell2[j], h=h, scheme=scheme,
                                           x0=abar_k[j], tol=pcg_tol, maxit=pcg_maxit)
            abar_new[j] = hs["abar"]
            stats["pcg_iters"] += hs["iters"]
            inner_ok = inner_ok and bool(hs["converged"])
        stats["inner_converged"] = inner_ok
        eps_new = mech["eps"]
        de = eps_new - eps_k
        mean_norm = np.sqrt(sum(float(eps_new[i].mean()) ** 2 for i in range(eps_new.shape[0])))
        err = float(np.sqrt((de * de).sum(axis=0)).max()) / (mean_norm if mean_norm > 0 else 1.0)
        for j in range(J):
            da = abar_new[j] - abar_k[j]
            nd = float(np.sqrt((da * da).sum()))
            if nd > 0.0:
                na = float(np.sqrt((abar_new[j] * abar_new[j]).sum()))
                err = max(err, nd / max(na, 1e-12 * np.sqrt(N)))
        eps_k, abar_k = eps_new, abar_new
        stats["stagger_iters"] = k + 1
        stats["err"] = err
        if err <= stagger_tol:
            stats["converged"] = True
            break
    new_state = dict(eps=eps_k, epsp=mech["epsp"], kappa=mech["kappa"],
                     hist=material.commit_history(phase, table, abar_k, hist_n, state["abar"]),
                     abar=abar_k)
    sig = mech["sigma"]
    c = sig.shape[0]
    homog = dict(sigma=np.array([sig[i].mean() for i in range(c)]),
                 eps=np.array([eps_k[i].mean() for i in range(c)]))
    return new_state, sig, homog, stats


def initial_state(shape, ndim, nfields):
    c = 3 if ndim == 2 else 6
    return dict(eps=np.zeros((c,) + tuple(shape)), epsp=np.zeros((6,) + tuple(shape)),
                kappa=np.zeros(tuple(shape)), hist=np.zeros((nfields,) + tuple(shape)),
                abar=np.zeros((nfields,) + tuple(shape)))
