"""Per-voxel constitutive update with frozen damage (Sec. 2.1.2, Sec. 2.2.3,
appendix A.2, and step (i) of Algorithm 1).

Matrix ('j2_damage'): the Lemaitre-type model.  Undamaged effective stress
from isotropic elasticity on eps - eps_p (Sec. 2.1.2), J2 yield function
||dev sigma_eff|| - sqrt(2/3) sigma_0(eps_p) <= 0 with linear hardening
sigma_0 = sy + H eps_p (Sec. 4), associative flow
d eps_p = lambda dev/||dev||, d eps_p(eq) = sqrt(2/3) lambda, integrated by
backward Euler (Sec. 3.1, appendix A.2).  The appendix's sqrt(3/2) factors
are read as the main text's sqrt(2/3) and the total form
sigma = (1 - D) sigma_eff (eq. effective_stress) is used.  For linear
hardening the backward-Euler update is the closed-form radial return; its
consistent tangent is the textbook one for that return (Simo & Hughes 1998,
Box 3.2).  D is frozen within the mechanical solve (Algorithm 1 (i)), so the
mechanical tangent is (1 - D) times the effective one.

Damage laws (eq. non-local_damage_lemaitre with the cap D <= 0.99 of Sec. 4):
  j2_damage        D = clip((abar - dC)/(dR - dC), 0, dmax)
  elastic_cracking D = clip((max(hist, abar) - dC)/(dR - dC), 0, dmax)
The cracking phase (an elastic phase with an equivalent-strain damage driven
by its own non-local field) is not part of the paper: its local source is the
Mazars equivalent strain sqrt(sum <e_i>_+^2) of the principal strains e_i.

Gurson-Tvergaard-Needleman matrix ('gtn', module gtn): two non-local
fields, j = dfield (matrix plastic strain e0) and j + 1 (trace of eps_p); the
frozen "damage" of field j is the porosity f, which enters the yield function
instead of a stiffness factor (sigma is not scaled by 1 - f).  The scalar
state slot holds e0 and hist_j holds the committed porosity f_n.

Local sources alpha_j (Sec. 2.2.1: alpha_q = 0 outside the phase that owns it):
  j2_damage phase with dfield = j  -> alpha_j = eps_p (equivalent plastic strain)
  cracking phase with dfield = j   -> alpha_j = Mazars equivalent strain
  gtn phase with dfield = j        -> alpha_j = e0, alpha_{j+1} = tr(eps_p)
  everything else                  -> 0
"""
from __future__ import annotations

import numpy as np

from . import gtn
from .mandel import identity, expand_plane, PLANE_IDX

SQ32 = np.sqrt(1.5)


def lame(E, nu):
    mu = E / (2.0 * (1.0 + nu))
    K = E / (3.0 * (1.0 - 2.0 * nu))
    return K, mu


def _tr(x):
    return x[0] + x[1] + x[2]


def _dev(x):
    I = identity(6).reshape((6,) + (1,) * (x.ndim - 1))
    return x - _tr(x) / 3.0 * I


def elastic_tangent(K, mu):
    """6x6 Mandel isotropic stiffness K I(x)I + 2 mu I_dev."""
    I = identity(6)
    Idev = np.eye(6) - np.outer(I, I) / 3.0
    return K * np.outer(I, I) + 2.0 * mu * Idev


def j2_return_map(eps, epsp_n, kappa_n, E, nu, sy, H):
    """Backward-Euler J2 update on the effective (undamaged) stress.

    eps, epsp_n: (6, M) Mandel; kappa_n: (M,).  Returns
    sig_eff (6, M), epsp (6, M), kappa (M,), C (6, 6, M) consistent tangent.
    """
    K, mu = lame(E, nu)
    I = identity(6)
    Idev = np.eye(6) - np.outer(I, I) / 3.0
    ee = eps - epsp_n
    sig_tr = K * _tr(ee)[None] * I[:, None] + 2.0 * mu * _dev(ee)
    s_tr = _dev(sig_tr)
    ns = np.sqrt((s_tr * s_tr).sum(axis=0))
    q_tr = SQ32 * ns
    f = q_tr - (sy + H * kappa_n)
    plastic = f > 0.0
    M = eps.shape[1]
    dk = np.where(plastic, f / (3.0 * mu + H), 0.0)
    n = np.where(plastic[None], s_tr / np.where(ns > 0, ns, 1.0)[None], 0.0)
    epsp = epsp_n + SQ32 * dk[None] * n
    kappa = kappa_n + dk
    sig = sig_tr - 2.0 * mu * SQ32 * dk[None] * n
    C = np.empty((6, 6, M))
    C[:] = (K * np.outer(I, I) + 2.0 * mu * Idev)[:, :, None]
    if plastic.any():
        idx = np.nonzero(plastic)[0]
        theta = 1.0 - 2.0 * mu * SQ32 * dk[idx] / ns[idx]
        thetab = 1.0 / (1.0 + H / (3.0 * mu)) - (1.0 - theta)
        nn = np.einsum("im,jm->ijm", n[:, idx], n[:, idx])
        C[:, :, idx] = (K * np.outer(I, I)[:, :, None]
                        + 2.0 * mu * theta[None, None] * Idev[:, :, None]
                        - 2.0 * mu * thetab[None, None] * nn)
    return sig, epsp, kappa, C


def mazars_equivalent(eps6):
    """sqrt(sum of squared positive principal strains); eps6 (6, M) Mandel.
    Principal strains from numpy's symmetric eigen-solver."""
    r2 = np.sqrt(2.0)
    M = eps6.shape[1]
    T = np.empty((M, 3, 3))
    T[:, 0, 0], T[:, 1, 1], T[:, 2, 2] = eps6[0], eps6[1], eps6[2]
    T[:, 1, 2] = T[:, 2, 1] = eps6[3] / r2
    T[:, 0, 2] = T[:, 2, 0] = eps6[4] / r2
    T[:, 0, 1] = T[:, 1, 0] = eps6[5] / r2
    w = np.linalg.eigvalsh(T)
    wp = np.maximum(w, 0.0)
    return np.sqrt((wp * wp).sum(axis=1))


def damage_from_nonlocal(phase, table, abar, hist, abar_n=None):
    """Frozen damage fields D_j(x) from the non-local fields abar_j.

    abar, hist: (J, *S).  D_j is nonzero only in voxels of a damaging phase
    whose driving field is j; returns (J, *S).  A gtn phase takes the
    porosity update from the committed fields abar_n and porosity hist_j."""
    D = np.zeros(abar.shape)
    for p, ph in enumerate(table):
        j = ph["dfield"]
        if j < 0 or ph["model"] == "elastic":
            continue
        sel = phase == p
        if ph["model"] == "gtn":
            an = np.zeros(abar.shape) if abar_n is None else abar_n
            D[j][sel] = gtn.porosity_update(hist[j][sel], abar[j][sel], an[j][sel],
                                            abar[j + 1][sel], an[j + 1][sel], ph)
            continue
        a = abar[j][sel]
        if ph["model"] == "elastic_cracking":
            a = np.maximum(hist[j][sel], a)
        D[j][sel] = np.clip((a - ph["dC"]) / (ph["dR"] - ph["dC"]), 0.0, ph["dmax"])
    return D


def commit_history(phase, table, abar, hist_n, abar_n):
    """History fields at the end of an increment: max(hist, abar) (the
    cracking law's irreversibility), except the porosity slot of a gtn phase,
    which takes the porosity f_{n+1} of the final non-local fields."""
    hist = np.maximum(hist_n, abar)
    for p, ph in enumerate(table):
        if ph["model"] == "gtn":
            j = ph["dfield"]
            sel = phase == p
            hist[j][sel] = gtn.porosity_update(hist_n[j][sel], abar[j][sel], abar_n[j][sel],
                                               abar[j + 1][sel], abar_n[j + 1][sel], ph)
    return hist


def constitutive(eps, epsp_n, kappa_n, D, phase, table, nfields):
    """Evaluate stress, tangent, trial state and local sources on the grid.

    eps: (c, *S) with c = 6 (3D) or 3 (2D plane strain); epsp_n: (6, *S);
    kappa_n: S; D: (J, *S) frozen damage per field (a voxel takes the field
    its phase names, none for an undamaged phase); phase: S uint8.
    Returns dict with
      sigma (c, *S), C (c, c, *S), epsp (6, *S), kappa S, alpha (J, *S).
    """
    c = eps.shape[0]
    S = eps.shape[1:]
    M = int(np.prod(S))
    e6 = (expand_plane(eps) if c == 3 else eps).reshape(6, M)
    ep_n = epsp_n.reshape(6, M)
    k_n = kappa_n.reshape(M)
    Dj = D.reshape(D.shape[0], M) if nfields > 0 else np.zeros((0, M))
    ph = phase.reshape(M)
    sig6 = np.zeros((6, M))
    C6 = np.zeros((6, 6, M))
    epsp = ep_n.copy()
    kappa = k_n.copy()
    alpha = np.zeros((nfields, M))
    for p, mat in enumerate(table):
        sel = np.nonzero(ph == p)[0]
        if sel.size == 0:
            continue
        if mat["model"] == "j2_damage":
            s, ep, k, C = j2_return_map(e6[:, sel], ep_n[:, sel], k_n[sel],
                                        mat["E"], mat["nu"], mat["sy"], mat["H"])
            epsp[:, sel] = ep
            kappa[sel] = k
            if mat["dfield"] >= 0:
                alpha[mat["dfield"], sel] = k
        elif mat["model"] == "gtn":
            j = mat["dfield"]
            s, ep, k, Cg, _ = gtn.return_map(e6[:, sel], ep_n[:, sel], k_n[sel], Dj[j, sel], mat)
            C = 0.5 * (Cg + np.swapaxes(Cg, 0, 1))
            epsp[:, sel] = ep
            kappa[sel] = k
            alpha[j, sel] = k
            alpha[j + 1, sel] = ep[0] + ep[1] + ep[2]
        else:
            K, mu = lame(mat["E"], mat["nu"])
            Ce = elastic_tangent(K, mu)
            s = Ce @ e6[:, sel]
            C = np.broadcast_to(Ce[:, :, None], (6, 6, sel.size))
            if mat["model"] == "elastic_cracking" and mat["dfield"] >= 0:
                alpha[mat["dfield"], sel] = mazars_equivalent(e6[:, sel])
        j = mat["dfield"]
        w = 1.0 - Dj[j, sel] if (j >= 0 and mat["model"] not in ("elastic", "gtn")) \
            else np.ones(sel.size)
        sig6[:, sel] = w[None] * s
        C6[:, :, sel] = w[None, None] * C
    if c == 3:
        sig = sig6[PLANE_IDX]
        Cc = C6[np.ix_(PLANE_IDX, PLANE_IDX)]
    else:
        sig, Cc = sig6, C6
    return dict(sigma=sig.reshape((c,) + S), C=Cc.reshape((c, c) + S),
                epsp=epsp.reshape((6,) + S), kappa=kappa.reshape(S),
                alpha=alpha.reshape((nfields,) + S))


def apply_tangent(C, p):
    """(C : p)(x) for a per-voxel Mandel matrix C (c, c, *S) and field p (c, *S)."""
    return np.einsum("ij...,j...->i...", C, p)
