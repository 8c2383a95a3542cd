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

from . import galerkin, helmholtz, mandel, material, spectral


def grad_fields(u, qt):
    """Real gradient components G_j u (j in physical order) of a real field."""
    uh = spectral.fftn(u)
    return [np.real(spectral.ifftn(1j * qj * uh)) for qj in qt]


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


def source_derivative(eps, epsp_n, kappa_n, phase, table, nfields):
    """d alpha_j / d eps per voxel, (J, c, *S).

    j2_damage phase driven by field j: the source is eps_p(eq) = kappa_n + dk
    with dk = (sqrt(3/2) ||s_tr|| - sy - H kappa_n)/(3 mu + H) where plastic,
    so d alpha / d eps = sqrt(3/2) 2 mu n / (3 mu + H), n the unit deviatoric
    trial direction (0 where elastic).
    elastic_cracking phase: the source is the Mazars equivalent strain
    alpha = ||<eps>_+|| (positive part of the strain tensor), whose gradient
    is <eps>_+ / alpha (alpha^2 / 2 has gradient <eps>_+); 0 where alpha = 0.
    The positive part comes from numpy's symmetric eigen-solver."""
    c = eps.shape[0]
    S = eps.shape[1:]
    e6 = mandel.expand_plane(eps) if c == 3 else eps
    I = mandel.identity(6).reshape((6,) + (1,) * len(S))
    out = np.zeros((nfields, 6) + S)
    for p, ph in enumerate(table):
        j = ph["dfield"]
        if ph["model"] == "elastic_cracking" and j >= 0:
            sel = phase == p
            T = mandel.to_tensor(e6[:, sel])                     # (3, 3, m)
            w, V = np.linalg.eigh(np.moveaxis(T, -1, 0))       # (m, 3), (m, 3, 3)
            wp = np.maximum(w, 0.0)
            pos = np.einsum("mik,mk,mjk->ijm", V, wp, V)         # <eps>_+ (3, 3, m)
            a = np.sqrt((wp * wp).sum(axis=1))
            g = mandel.from_tensor(pos) / np.where(a > 0, a, 1.0)[None]
            out[j][:, sel] += np.where(a > 0, 1.0, 0.0)[None] * g
            continue
        if ph["model"] != "j2_damage" or j < 0:
            continue
        K, mu = material.lame(ph["E"], ph["nu"])
        ee = e6 - epsp_n
        tr = ee[0] + ee[1] + ee[2]
        s = 2.0 * mu * (ee - tr / 3.0 * I)
        ns = np.sqrt((s * s).sum(axis=0))
        plastic = (phase == p) & (np.sqrt(1.5) * ns - (ph["sy"] + ph["H"] * kappa_n) > 0.0)
        g = np.where(plastic, np.sqrt(1.5) * 2.0 * mu / (3.0 * mu + ph["H"])
                     / np.where(ns > 0, ns, 1.0), 0.0)
        out[j] += g[None] * s
    if c == 3:
        out = out[:, mandel.PLANE_IDX]
    return out


def staggered_adjoint(phase, table, nfields, state_n, eps, abar, target, g_eps=None,
                      g_sig=None, g_abar=None, g_D=None, h=1.0, scheme=spectral.ROTATED,
                      cg_tol=1e-12, pcg_tol=1e-12, tol=1e-12, maxit=200):
    """Gradient of J(eps, sigma, abar, D) at a converged staggered increment
    (Algorithm 1 at its fixed point: mechanics at D(abar), Helmholtz with the
    sources alpha(eps)) with respect to the squared lengths ell2_j(x).

    Linearising both equations, a change of ell2 moves abar by
    dabar = -(I - T)^-1 L^-1 dL abar, with the staggered map
    T = L^-1 alpha' A^-1 G* sigma_eff D' (A = G* K).  Hence
        dJ/dell2_j(x) = -sum_i (G_i lam_j)(x) (G_i abar_j)(x),  lam = L^-1 z,
    where z solves the transposed staggered fixed point
        z = hv + T^T z,   T^T z = D' (sigma_eff : A^-1 G*(alpha'^T L^-1 z)),
        hv = D' ((mu0 - g_sig) : sigma_eff + g_D) + g_abar,
        mu0 = A^-1 G*(g_eps + K g_sig)
    (the damage term is mechanics_adjoint's dD, the damage-law slope D' is
    damage_adjoint's).  Iterated like the forward scheme until
    ||z_new - z|| <= tol ||z_new||.  Returns dict(dell2 (J, *S), lam, z, iters,
    mu (the total mechanics adjoint), D, zeta (the total damage cotangent dJ/dD))."""
    S = phase.shape
    c = eps.shape[0]
    J = nfields
    zf = np.zeros((c,) + S)
    g_eps = zf if g_eps is None else g_eps
    D = material.damage_from_nonlocal(phase, table, abar, state_n["hist"], state_n["abar"])
    ell2 = [np.array([float(t["ell"][j]) ** 2 for t in table])[phase] for j in range(J)]
    m0 = mechanics_adjoint(phase, table, D, state_n["epsp"], state_n["kappa"], target, eps, g_eps,
                           J, h=h, scheme=scheme, cg_tol=cg_tol, gsig=g_sig)
    gD = m0["dD"] if g_D is None else m0["dD"] + g_D
    hv = damage_adjoint(phase, table, abar, state_n["hist"], gD)
    if g_abar is not None:
        hv = hv + g_abar
    dadx = source_derivative(eps, state_n["epsp"], state_n["kappa"], phase, table, J)
    z = hv.copy()
    lam = np.zeros((J,) + S)
    it = 0
    for it in range(1, maxit + 1):
        for j in range(J):
            lam[j] = helmholtz.helmholtz_solve(z[j], ell2[j], h=h, scheme=scheme, x0=lam[j],
                                               tol=pcg_tol, maxit=5000)["abar"]
        rhs = (lam[:, None] * dadx).sum(axis=0)
        m = mechanics_adjoint(phase, table, D, state_n["epsp"], state_n["kappa"], target, eps,
                              rhs, J, h=h, scheme=scheme, cg_tol=cg_tol)
        z_new = hv + damage_adjoint(phase, table, abar, state_n["hist"], m["dD"])
        dz = float(np.sqrt(((z_new - z) ** 2).sum()))
        nz = float(np.sqrt((z_new ** 2).sum()))
        z = z_new
        if dz <= tol * max(nz, 1e-300):
            break
    for j in range(J):
        lam[j] = helmholtz.helmholtz_solve(z[j], ell2[j], h=h, scheme=scheme, x0=lam[j],
                                           tol=pcg_tol, maxit=5000)["abar"]
    _, qt = spectral.symbols(S, h, scheme)
    qt = [np.broadcast_to(v, S) for v in qt]
    dell2 = np.stack([-sum(a * b for a, b in zip(grad_fields(lam[j], qt), grad_fields(abar[j], qt)))
                      for j in range(J)])
    # total mechanics adjoint: mu = A^-1 G*(g_eps + K g_sig + alpha'^T lam), and
    # the total damage cotangent zeta = dJ/dD at the fixed point
    rhs = g_eps + (lam[:, None] * dadx).sum(axis=0)
    mt = mechanics_adjoint(phase, table, D, state_n["epsp"], state_n["kappa"], target, eps, rhs, J,
                           h=h, scheme=scheme, cg_tol=cg_tol, gsig=g_sig)
    zeta = mt["dD"] if g_D is None else mt["dD"] + g_D
    return dict(dell2=dell2, lam=lam, z=z, iters=it, mu=mt["mu"], D=D, zeta=zeta)


def history_partials(eps, epsp_n, kappa_n, phase, table):
    """Partial derivatives of the J2 return (linear hardening) of every voxel
    with respect to its strain and its history, in 6-component Mandel form:
      dk_de   (6, M)    d kappa_{n+1} / d eps   = sqrt(3/2) 2 mu n / (3 mu + H)
      dk_dkn  (M,)      d kappa_{n+1} / d kappa_n = 3 mu / (3 mu + H)
      dep_de  (6, 6, M) d eps_p,{n+1} / d eps
                        = 3 mu/(3 mu + H) n(x)n + sqrt(3/2) dk 2 mu/||s|| (I_dev - n(x)n)
      dep_dkn (6, M)    d eps_p,{n+1} / d kappa_n = -sqrt(3/2) H/(3 mu + H) n
      ds_dkn  (6, M)    d sigma_eff / d kappa_n = 2 mu sqrt(3/2) H/(3 mu + H) n
    where plastic (n the unit deviatoric trial direction, dk the increment);
    elastic voxels and other phases keep their history (dk_dkn = 1, rest 0).
    Since the return depends on eps - eps_p,n, the derivatives in eps_p,n are
    minus those in eps (and d sigma_eff / d eps_p,n = -C_tangent)."""
    M = eps.shape[1]
    I6 = mandel.identity(6)
    Idev = np.eye(6) - np.outer(I6, I6) / 3.0
    out = dict(dk_de=np.zeros((6, M)), dk_dkn=np.ones(M), dep_de=np.zeros((6, 6, M)),
               dep_dkn=np.zeros((6, M)), ds_dkn=np.zeros((6, M)))
    for p, ph in enumerate(table):
        if ph["model"] != "j2_damage":
            continue
        sel = np.nonzero(phase == p)[0]
        K, mu = material.lame(ph["E"], ph["nu"])
        H = ph["H"]
        ee = eps[:, sel] - epsp_n[:, sel]
        tr = ee[0] + ee[1] + ee[2]
        s = 2.0 * mu * (ee - tr / 3.0 * I6[:, None])
        ns = np.sqrt((s * s).sum(axis=0))
        f = np.sqrt(1.5) * ns - (ph["sy"] + H * kappa_n[sel])
        pl = f > 0.0
        idx = sel[pl]
        n = s[:, pl] / ns[pl]
        dk = f[pl] / (3.0 * mu + H)
        a = 3.0 * mu / (3.0 * mu + H)
        out["dk_de"][:, idx] = np.sqrt(1.5) * 2.0 * mu / (3.0 * mu + H) * n
        out["dk_dkn"][idx] = a
        nn = np.einsum("im,jm->ijm", n, n)
        out["dep_de"][:, :, idx] = a * nn + (np.sqrt(1.5) * dk * 2.0 * mu / ns[pl])[None, None] * (
            Idev[:, :, None] - nn)
        out["dep_dkn"][:, idx] = -np.sqrt(1.5) * H / (3.0 * mu + H) * n
        out["ds_dkn"][:, idx] = 2.0 * mu * np.sqrt(1.5) * H / (3.0 * mu + H) * n
    return out


def increment_adjoint(phase, table, nfields, state_n, state_np1, target, g_sig=None,
                      g_epsp=None, g_kappa=None, g_hist=None, **kw):
    """Adjoint of one converged staggered increment with respect to the
    squared lengths and to the plastic history it started from.

    J depends on this increment through sigma (g_sig, c comps) and through the
    committed plastic state eps_p,{n+1}, kappa_{n+1} (cotangents g_epsp (6),
    g_kappa, coming from later increments).  The committed-state cotangents
    become a strain cotangent g_eps = dep_de^T g_epsp + dk_de g_kappa; the
    coupled adjoint (staggered_adjoint) then gives mu and lam, and the history
    cotangents are (sigma = (1 - D) sigma_eff, alpha = kappa_{n+1} on the
    phase's field)
      dJ/d eps_p,n = (1 - D) C_eff^T (mu - g_sig) - lam dk_de
                     + (I - dep_de)^T g_epsp - dk_de g_kappa   (J2 voxels; an elastic
                     voxel passes g_epsp through: its stress ignores eps_p,n)
      dJ/d kappa_n = (1 - D) ds_dkn . (g_sig - mu) + lam dk_dkn
                     + dep_dkn . g_epsp + dk_dkn g_kappa
    (a parameter theta entering sigma at fixed strain contributes
    (g_sig - mu) . d sigma/d theta, one entering the source lam d alpha/d theta).

    The damage history hist_{n+1} = max(hist_n, abar) (cotangent g_hist, J
    fields) is read back only by the cracking law D = D(max(hist_n, abar)).
    Where abar is the max (abar >= hist_n, the damage law's own convention at
    the tie) g_hist joins the abar cotangent of the fixed point; where hist_n
    is, it passes to hist_n, and so does the total damage cotangent zeta of
    a cracking voxel whose history drives D inside the slope band:
      dJ/d hist_n = g_hist [hist_n > abar] + zeta / (dR - dC) [cracking, hist_n > abar,
                    0 < (hist_n - dC)/(dR - dC) < dmax]
    Returns dict(dell2, g_epsp_n (6, *S), g_kappa_n (*S), g_hist_n (J, *S), iters)."""
    S = phase.shape
    M = phase.size
    eps = state_np1["eps"]
    c = eps.shape[0]
    for ph in table:
        if ph["model"] not in ("elastic", "j2_damage", "elastic_cracking"):
            raise NotImplementedError("history adjoint: J2 damage, elastic and cracking phases only")
    e6 = (mandel.expand_plane(eps) if c == 3 else eps).reshape(6, M)
    ep_n = state_n["epsp"].reshape(6, M)
    k_n = state_n["kappa"].reshape(M)
    hp = history_partials(e6, ep_n, k_n, phase.reshape(M), table)
    cidx = mandel.PLANE_IDX if c == 3 else list(range(6))
    ge = np.zeros((6, M))
    if g_epsp is not None:
        ge += np.einsum("ijm,im->jm", hp["dep_de"], g_epsp.reshape(6, M))
    if g_kappa is not None:
        ge += hp["dk_de"] * g_kappa.reshape(M)[None]
    g_eps = ge[cidx].reshape((c,) + S)
    abar = state_np1["abar"]
    by_hist = state_n["hist"] > abar              # the history, not abar, is the max
    g_abar = None if g_hist is None else np.where(by_hist, 0.0, g_hist)
    r = staggered_adjoint(phase, table, nfields, state_n, eps, abar, target,
                          g_eps=g_eps, g_sig=g_sig, g_abar=g_abar, **kw)
    mu = r["mu"].reshape(c, M)
    gs = np.zeros((c, M)) if g_sig is None else g_sig.reshape(c, M)
    w6 = np.zeros((6, M))
    w6[cidx] = mu - gs                                # mu - g_sig, zero off-plane in 2D
    # (1 - D) C_eff of the J2 phases; an elastic phase's stress does not
    # depend on eps_p,n (it acts on the total strain), its history only passes
    # through
    C6 = np.zeros((6, 6, M))
    for p, ph in enumerate(table):
        sel = np.nonzero(phase.reshape(M) == p)[0]
        if ph["model"] == "j2_damage":
            C6[:, :, sel] = material.j2_return_map(e6[:, sel], ep_n[:, sel], k_n[sel], ph["E"],
                                                   ph["nu"], ph["sy"], ph["H"])[3]
    w1 = np.ones(M)
    lam_v = np.zeros(M)
    for p, ph in enumerate(table):
        sel = phase.reshape(M) == p
        j = ph["dfield"]
        if ph["model"] == "j2_damage" and j >= 0:
            w1[sel] = 1.0 - r["D"][j].reshape(M)[sel]
            lam_v[sel] = r["lam"][j].reshape(M)[sel]
    gep = w1[None] * np.einsum("ijm,im->jm", C6, w6) - lam_v[None] * hp["dk_de"]
    gk = -w1 * (hp["ds_dkn"] * w6).sum(axis=0) + lam_v * hp["dk_dkn"]
    if g_epsp is not None:
        gp = g_epsp.reshape(6, M)
        gep += gp - np.einsum("ijm,im->jm", hp["dep_de"], gp)
        gk += (hp["dep_dkn"] * gp).sum(axis=0)
    if g_kappa is not None:
        gkap = g_kappa.reshape(M)
        gep -= hp["dk_de"] * gkap[None]
        gk += hp["dk_dkn"] * gkap
    gh = np.zeros(abar.shape) if g_hist is None else np.where(by_hist, g_hist, 0.0)
    for p, ph in enumerate(table):
        j = ph["dfield"]
        if ph["model"] != "elastic_cracking" or j < 0:
            continue
        sel = phase == p
        d = (state_n["hist"][j][sel] - ph["dC"]) / (ph["dR"] - ph["dC"])
        inside = by_hist[j][sel] & (d > 0.0) & (d < ph["dmax"])
        gh[j][sel] += np.where(inside, r["zeta"][j][sel] / (ph["dR"] - ph["dC"]), 0.0)
    return dict(dell2=r["dell2"], g_epsp_n=gep.reshape((6,) + S), g_kappa_n=gk.reshape(S),
                g_hist_n=gh, iters=r["iters"])


def path_gradient(phase, table, nfields, states, targets, g_sig, **kw):
    """dJ/d ell2_j(x) of J = g_sig . sigma after the last of a sequence of
    converged staggered increments, through the whole path: states[k] is the
    state before increment k (states[-1] after the last), targets[k] its
    macro target.  Walks the increments backwards, passing the history
    cotangents (plastic state and damage history) from each increment to the
    one before (increment_adjoint)."""
    n = len(targets)
    ge = gk = gh = None
    dell2 = 0.0
    for k in range(n - 1, -1, -1):
        r = increment_adjoint(phase, table, nfields, states[k], states[k + 1], targets[k],
                              g_sig=g_sig if k == n - 1 else None, g_epsp=ge, g_kappa=gk,
                              g_hist=gh, **kw)
        dell2 = dell2 + r["dell2"]
        ge, gk, gh = r["g_epsp_n"], r["g_kappa_n"], r["g_hist_n"]
    return dell2
