"""FFT-Galerkin mechanical solver with mixed macroscopic control (Sec. 3.2.2).

Projection G* (eq. weakeq / eqdiscrete2).  For a frequency xi != 0 with
|q|^2 > 0 the projector is the orthogonal projection (in the Frobenius
product) of a symmetric tensor tau_hat onto the compatible tensors
sym(u (x) q):
    t = tau_hat q,   P tau_hat = (t(x)q + q(x)t)/|q|^2 - (q(x)q)(q.t)/|q|^4 .
Where |q|^2 = 0 at xi != 0 (rotated scheme, two or more Nyquist components)
no compatible field exists and P = 0.  At xi = 0 the projector keeps exactly
the stress-controlled Mandel components: G*(0) = diag(mask).  This is the
reading used for the paper's "modified zero frequency" of the mixed-control
projector: the test space is {compatible fluctuation + constant tensor on
the stress-controlled components}, and testing the residual with a constant
tensor enforces <sigma>_HK = Sigma_HK, while the strain-controlled means
<eps>_hk = E_hk are never changed by a correction in that space.

Newton + CG (eq. lin_stress and the linear system after it): at each Newton
iterate the stress and consistent tangent are evaluated, the residual is
b = -G*(sigma - Sigma_bar) (Sigma_bar = imposed stress on the controlled
components), and G*(K : d_eps) = b is solved by plain conjugate gradients in
the real-space Mandel dot product, from d_eps = 0, until ||r|| <= tol ||b||.
Stopping: ||b||_2 <= newton_tol * max(||sigma||_2, s_ref sqrt(N)) after at
least one correction; s_ref = largest yield stress of the table (1 MPa when
no phase yields).
"""
from __future__ import annotations

import numpy as np

from . import mandel, material, spectral


def _axes(ndim):
    return tuple(range(1, ndim + 1))


def project(tau, q, mask):
    """Apply G* to a real Mandel field tau (c, *S); q from spectral.symbols.

    Uses the full complex spectrum (numpy.fft.fftn / ifftn)."""
    c = tau.shape[0]
    S = tau.shape[1:]
    ndim = len(S)
    ax = _axes(ndim)
    th = spectral.fftn(tau, axes=ax)
    T = mandel.to_tensor(th)                          # (d, d, *S)
    qv = np.stack([np.broadcast_to(qj, S) for qj in q])  # (d, *S)
    q2 = (qv * qv).sum(axis=0)
    inv = np.where(q2 > 0, 1.0 / np.where(q2 > 0, q2, 1.0), 0.0)
    t = np.einsum("ab...,b...->a...", T, qv)
    s = (qv * t).sum(axis=0)
    P = (np.einsum("a...,b...->ab...", t, qv) + np.einsum("a...,b...->ab...", qv, t)) * inv \
        - np.einsum("a...,b...->ab...", qv, qv) * (s * inv * inv)
    out = mandel.from_tensor(P)
    zero = (slice(None),) + (0,) * ndim
    out[zero] = np.asarray(mask, dtype=np.float64) * th[zero]
    return np.real(spectral.ifftn(out, axes=ax))


def cg(apply_A, b, tol, maxit):
    """Plain conjugate gradients from x = 0 in the real-space dot product.

    Returns (x, iterations, ||r||/||b||, converged)."""
    x = np.zeros_like(b)
    nb = np.sqrt(np.vdot(b, b).real)
    if nb == 0.0:
        return x, 0, 0.0, True
    r = b.copy()
    p = r.copy()
    rr = np.vdot(r, r).real
    it = 0
    while it < maxit:
        Ap = apply_A(p)
        pAp = np.vdot(p, Ap).real
        if pAp <= 0.0:
            break
        a = rr / pAp
        x = x + a * p
        r = r - a * Ap
        rr_new = np.vdot(r, r).real
        it += 1
        if np.sqrt(rr_new) <= tol * nb:
            return x, it, np.sqrt(rr_new) / nb, True
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, it, np.sqrt(rr) / nb, False


def sigma_ref(table):
    s = max([float(ph["sy"]) for ph in table] + [0.0])
    return s if s > 0 else 1.0


def set_strain_means(eps, mask, Emac):
    """Shift the strain-controlled components so that <eps>_hk = E_hk."""
    out = eps.copy()
    ndim = eps.ndim - 1
    for k in range(eps.shape[0]):
        if not mask[k]:
            out[k] += Emac[k] - eps[k].mean()
    return out


def fftg_solve(phase, table, D, epsp_n, kappa_n, target, eps0, h=1.0,
               scheme=spectral.ROTATED, cg_tol=1e-8, cg_maxit=5000,
               newton_tol=1e-8, newton_maxit=50, nfields=None, newton_div=0):
    """Mechanics at frozen damage (Algorithm 1, step (i)).

    target = (mask, E, S) Mandel; eps0 (c, *S) initial guess.
    newton_div > 0: give up (not converged) once the Newton residual has grown
    in newton_div consecutive corrections (used by the adaptive load driver,
    where a diverging increment is cut back instead of iterated to the end).
    Returns dict(eps, sigma, epsp, kappa, alpha, newton_iters, cg_iters,
    relres, converged)."""
    mask, Emac, Smac = target
    mask = np.asarray(mask)
    S = phase.shape
    c = eps0.shape[0]
    N = int(np.prod(S))
    J = D.shape[0] if nfields is None else nfields
    q = spectral.projection_symbol(S, h, scheme)
    Sbar = np.where(mask.astype(bool), np.asarray(Smac, dtype=np.float64), 0.0)
    Sbar_f = Sbar.reshape((c,) + (1,) * len(S))
    eps = set_strain_means(eps0, mask, Emac)
    sref = sigma_ref(table)
    cg_total = 0
    converged = False
    relres = np.inf
    grown = 0
    r = 0
    while True:
        st = material.constitutive(eps, epsp_n, kappa_n, D, phase, table, J)
        b = -project(st["sigma"] - Sbar_f, q, mask)
        nb = np.sqrt((b * b).sum())
        ns = np.sqrt((st["sigma"] * st["sigma"]).sum())
        prev = relres
        relres = nb / max(ns, sref * np.sqrt(N))
        grown = grown + 1 if (r >= 1 and relres > prev) else 0
        if r >= 1 and relres <= newton_tol:
            converged = True
            break
        if newton_div > 0 and grown >= newton_div:
            break
        if r >= newton_maxit:
            break
        C = st["C"]
        d, it, _, _ = cg(lambda p: project(material.apply_tangent(C, p), q, mask),
                         b, cg_tol, cg_maxit)
        cg_total += it
        eps = eps + d
        r += 1
    return dict(eps=eps, sigma=st["sigma"], epsp=st["epsp"], kappa=st["kappa"],
                alpha=st["alpha"], newton_iters=r, cg_iters=cg_total,
                relres=relres, converged=converged)
