"""Non-local Gurson-Tvergaard-Needleman matrix at frozen porosity
(Sec. 2.1.1, Sec. 2.3 non-local Gurson extension, appendix A.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model.  Yield function (eq. yield_gurson), with the Mises stress q and the
mean stress sm = tr(sigma)/3 (the paper's pressure is p = -sm; cosh is even):
    phi = (q/s0)^2 + 2 q1 f* cosh(3 q2 sm / (2 s0)) - (1 + q3 f*^2)
Isotropic elasticity on eps - eps_p (eq. elasticity_gurson, integrated to the
total form for constant moduli), normality d eps_p = dlam dphi/dsigma
(eq. flow_rule_gurson), matrix plastic strain from the plastic work
sigma : d eps_p = (1 - f) s0 d e0 (eq. micro-macro), hardening of Aravas type
s0/sy = (s0/sy + 3 mu e0 / sy)^n (eq. aravas), effective porosity f*(f)
(eq. effective_porosity) with the cap f* <= fu of Sec. 4.

Frozen porosity.  In the non-local model the porosity rate is driven by the
two non-local fields (eq. non-local_porosity_gurson): field j carries the
matrix plastic strain e0 and field j + 1 the trace of eps_p.  Within the
mechanics of one staggered iteration (Algorithm 1 (i)) these are frozen, so
f and f* are fixed per voxel and the local update is a plain plasticity
return with a pressure-sensitive yield surface.  The backward-Euler update
of appendix A.1 then reads, with the plastic strain increment split as
d eps_p = u N + v I/3 (N = 3 s/(2 q), so u = dlam dphi/dq, v = dlam dphi/dsm):
    q  = q_tr - 3 mu u,    sm = sm_tr - K v,    e0 = e0_n + w,  s0 = s0(e0)
    F1 = u dphi/dsm - v dphi/dq = 0     (one multiplier for both parts)
    F2 = phi(q, sm, s0, f*) = 0          (consistency)
    F3 = (1 - f) s0 w - (q u + sm v) = 0 (plastic work; sigma : N = q)
solved per voxel by nested bracketed root finding (return_map).

Porosity update (backward Euler of eq. non-local_porosity_gurson, appendix
A.1, nucleation of eq. nucleation at the end-of-step non-local e0):
    f_{n+1} = (f_n + A_N(ebar_{n+1}) d ebar + d trbar) / (1 + d trbar)
clamped at 0 from below (a reading: the paper does not say what happens
under plastic compaction).

Tangent.  The consistent tangent of the return comes from linearising
F = 0 in (q_tr, sm_tr).  The Newton systems of the mechanics are solved with
conjugate gradients (Sec. 3.2.2), which needs a symmetric operator; this
tangent comes out symmetric at frozen porosity (pinned against its transpose
and a central difference of the return), and the mechanics takes its
symmetric part so that rounding cannot break that.

Readings (the paper is silent): the plastic strain increment is split
into its Mises and volumetric parts as above (Aravas 1987); the return is
computed by nested bracketed root finding, which needs no starting guess
and reaches the unique solution for any trial state.
"""
from __future__ import annotations

import numpy as np

from .mandel import identity

SQ32 = np.sqrt(1.5)


def lame(E, nu):
    return E / (3.0 * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def flow_stress(e0, sy, mu, n, tol=1e-15, maxit=100):
    """s0(e0) and ds0/de0 for the Aravas law s0/sy = (s0/sy + 3 mu e0/sy)^n.

    y = s0/sy solves g(y) = y - (y + c e0)^n = 0, c = 3 mu / sy; g is
    increasing and convex for y + c e0 >= 1 and positive at y = 1 + c e0,
    so Newton from there decreases monotonically to the root."""
    e0 = np.asarray(e0, dtype=np.float64)
    c = 3.0 * mu / sy
    y = 1.0 + c * e0
    for _ in range(maxit):
        z = y + c * e0
        g = y - z ** n
        dg = 1.0 - n * z ** (n - 1.0)
        step = g / dg
        y = y - step
        if np.all(np.abs(step) <= tol * y):
            break
    z = y + c * e0
    zn1 = n * z ** (n - 1.0)
    dy = zn1 * c / (1.0 - zn1)
    return sy * y, sy * dy


def fstar(f, mat):
    """Effective porosity (eq. effective_porosity), capped at fu."""
    q1, q3, fC, fF = mat["q1"], mat["q3"], mat["fC"], mat["fF"]
    fV = (q1 + np.sqrt(q1 * q1 - q3)) / q3
    fs = np.where(f < fC, f, np.where(f < fF, fC + (fV - fC) / (fF - fC) * (f - fC), fV))
    return np.minimum(fs, mat["fu"])


def nucleation_rate(e, mat):
    """A_N of eq. nucleation (Chu and Needleman)."""
    fN, eN, sN = mat["fN"], mat["eN"], mat["sN"]
    return fN / (sN * np.sqrt(2.0 * np.pi)) * np.exp(-0.5 * ((e - eN) / sN) ** 2)


def porosity_update(f_n, ebar, ebar_n, trbar, trbar_n, mat):
    """f_{n+1} from the non-local fields at n and n+1 (backward Euler)."""
    de = ebar - ebar_n
    dt = trbar - trbar_n
    f = (f_n + nucleation_rate(ebar, mat) * de + dt) / (1.0 + dt)
    return np.maximum(f, 0.0)


def _yield(q, sm, s0, fs, mat):
    t = 1.5 * mat["q2"] * sm / s0
    return (q / s0) ** 2 + 2.0 * mat["q1"] * fs * np.cosh(t) - (1.0 + mat["q3"] * fs * fs)


def _residual_and_jacobian(x, q_tr, sm_tr, e0_n, f, fs, mat, K, mu):
    """F (3, M) and dF/d(u, v, w) (3, 3, M), dF/d(q_tr, sm_tr) (3, 2, M)."""
    u, v, w = x
    q1, q2 = mat["q1"], mat["q2"]
    q = q_tr - 3.0 * mu * u
    sm = sm_tr - K * v
    s0, h = flow_stress(e0_n + w, mat["sy"], mu, mat["n"])
    t = 1.5 * q2 * sm / s0
    tm = 1.5 * q2 / s0                       # dt/dsm
    sh, ch = np.sinh(t), np.cosh(t)
    A = 3.0 * q1 * q2 * fs                   # s0 dphi/dsm = A sinh(t)
    F1 = A * u * sh - 2.0 * v * q / s0       # s0 (u dphi/dsm - v dphi/dq)
    F2 = (q / s0) ** 2 + 2.0 * q1 * fs * ch - (1.0 + mat["q3"] * fs * fs)
    F3 = (1.0 - f) * w - (q * u + sm * v) / s0   # plastic work / s0
    # partial derivatives in (u, v, w) direct, q, sm, s0
    d1 = dict(u=A * sh, v=-2.0 * q / s0, w=0.0, q=-2.0 * v / s0, sm=A * u * ch * tm,
              s0=-A * u * ch * t / s0 + 2.0 * v * q / s0 ** 2)
    d2 = dict(u=0.0, v=0.0, w=0.0, q=2.0 * q / s0 ** 2, sm=2.0 * q1 * fs * sh * tm,
              s0=-2.0 * q * q / s0 ** 3 - 2.0 * q1 * fs * sh * t / s0)
    d3 = dict(u=-q / s0, v=-sm / s0, w=1.0 - f, q=-u / s0, sm=-v / s0,
              s0=(q * u + sm * v) / s0 ** 2)
    M = q_tr.shape[0]
    Jx = np.empty((3, 3, M))
    Jt = np.empty((3, 2, M))
    for i, d in enumerate((d1, d2, d3)):
        Jx[i, 0] = d["u"] - 3.0 * mu * d["q"]
        Jx[i, 1] = d["v"] - K * d["sm"]
        Jx[i, 2] = d["w"] + h * d["s0"]
        Jt[i, 0] = d["q"]
        Jt[i, 1] = d["sm"]
    return np.stack([F1, F2, F3]), Jx, Jt


def _solve3(Jx, b):
    """Solve Jx y = b for each voxel (Jx (3, 3, M), b (3, M)); y = 0 where Jx
    is singular or not finite (states far outside any converged solution,
    e.g. inside a diverging Newton iteration)."""
    A = np.moveaxis(Jx, -1, 0)
    det = np.linalg.det(A)
    ok = np.isfinite(det) & (det != 0.0) & np.isfinite(b).all(axis=0)
    y = np.zeros(b.shape)
    if ok.any():
        y[:, ok] = np.linalg.solve(A[ok], np.moveaxis(b[:, ok], -1, 0)[..., None])[..., 0].T
    return y


def illinois(fun, a, b, fa, fb, maxit=200):
    """Vectorised bracketed root of fun on [a, b] with fa fb <= 0: the
    Illinois variant of regula falsi (Dowell and Jarratt 1971), with a
    bisection step whenever the secant point leaves the bracket.  Stops when
    the bracket is a few ulps wide or fun is exactly 0."""
    a, b, fa, fb = (np.array(v, dtype=np.float64) for v in (a, b, fa, fb))
    side = np.zeros(a.shape, dtype=np.int8)
    done = (fa == 0.0) | (fb == 0.0) | (a == b)
    root = np.where(fb == 0.0, b, a)
    for _ in range(maxit):
        act = ~done
        if not act.any():
            break
        den = fb - fa
        c = np.where(den != 0.0, b - fb * (b - a) / np.where(den != 0.0, den, 1.0), 0.5 * (a + b))
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        c = np.where((c > lo) & (c < hi), c, 0.5 * (a + b))
        fc = np.where(act, fun(c), 0.0)
        same = np.sign(fc) == np.sign(fb)
        # c replaces b; if b's side was kept twice in a row, halve f(a)
        fa = np.where(act & same & (side == -1), 0.5 * fa, fa)
        a = np.where(act & ~same, b, a)
        fa = np.where(act & ~same, fb, fa)
        side = np.where(act, np.where(same, -1, 1), side).astype(np.int8)
        b = np.where(act, c, b)
        fb = np.where(act, fc, fb)
        width = np.abs(b - a)
        newly = act & ((fc == 0.0) | (width <= 4.0 * np.finfo(float).eps * np.maximum(np.abs(b), 1e-300)))
        root = np.where(newly, b, root)
        done |= newly
    return np.where(done, root, b)


def _surface_q(sm, s0, fs, mat):
    """Mises stress on the yield surface at mean stress sm (phi = 0)."""
    g = 1.0 + mat["q3"] * fs * fs - 2.0 * mat["q1"] * fs * np.cosh(1.5 * mat["q2"] * sm / s0)
    return s0 * np.sqrt(np.maximum(g, 0.0))


def _apex(s0, fs, mat):
    """Largest |sm| on the yield surface (q = 0); inf without porosity."""
    q1, q2, q3 = mat["q1"], mat["q2"], mat["q3"]
    b = 2.0 * q1 * fs
    ratio = np.where(b > 0.0, (1.0 + q3 * fs * fs) / np.where(b > 0.0, b, 1.0), np.inf)
    return np.where(b > 0.0, 2.0 * s0 / (3.0 * q2) * np.arccosh(np.maximum(ratio, 1.0)), np.inf)


def _project(q_tr, sm_tr, s0, fs, mat, K, mu):
    """Return onto the yield surface for fixed s0 (no hardening in this
    step): the point (q(sm), sm) of the surface where the plastic strain
    increment u N + v I/3, u = (q_tr - q)/(3 mu), v = (sm_tr - sm)/K, is
    normal to it (F1 = 0).  For a trial point outside the surface the root
    lies between sm = 0 and sm_tr (clamped to the apex), where the normality
    residual changes sign."""
    q1, q2 = mat["q1"], mat["q2"]
    kap = 1.5 * q2 / s0

    def g(sm):
        q = _surface_q(sm, s0, fs, mat)
        u = (q_tr - q) / (3.0 * mu)
        v = (sm_tr - sm) / K
        return u * 2.0 * q1 * fs * kap * np.sinh(kap * sm) - v * 2.0 * q / s0 ** 2

    apex = _apex(s0, fs, mat)
    clamped = np.abs(sm_tr) >= apex
    end = np.clip(sm_tr, -apex, apex)
    zero = np.zeros_like(end)
    # at the apex q = 0 exactly (the square root there only sees rounding)
    g_apex = q_tr / (3.0 * mu) * 2.0 * q1 * fs * kap * np.sinh(kap * end)
    sm = illinois(g, zero, end, g(zero), np.where(clamped, g_apex, g(end)))
    q = np.where(clamped & (sm == end), 0.0, _surface_q(sm, s0, fs, mat))
    # a surface that contains the trial point returns the trial point
    inside = _yield(q_tr, sm_tr, s0, fs, mat) <= 0.0
    q = np.where(inside, q_tr, q)
    sm = np.where(inside, sm_tr, sm)
    return q, sm, (q_tr - q) / (3.0 * mu), (sm_tr - sm) / K


def return_map(eps, epsp_n, e0_n, f, mat):
    """Backward-Euler GTN update at frozen porosity f.

    eps, epsp_n: (6, M) Mandel; e0_n, f: (M,).  Returns
    sigma (6, M), epsp (6, M), e0 (M,), C (6, 6, M) consistent tangent, and
    the increments (u, v, w) (3, M).

    Nested bracketed roots: for a trial increment w of e0 the stress is the
    normal return onto the surface of s0(e0_n + w) (_project); the plastic
    work F3(w) = (1 - f) s0 w - (q u + sm v) is negative at w = 0 and
    non-negative at w_hi = (q u + sm v)|_{w=0} / ((1 - f) s0(e0_n)), since a
    larger flow stress only shrinks the return."""
    K, mu = lame(mat["E"], mat["nu"])
    I = identity(6)
    M = eps.shape[1]
    ee = eps - epsp_n
    tr = ee[0] + ee[1] + ee[2]
    dev = ee - (tr / 3.0)[None] * I[:, None]
    s_tr = 2.0 * mu * dev
    q_tr = SQ32 * np.sqrt((s_tr * s_tr).sum(axis=0))
    sm_tr = K * tr
    fs = fstar(f, mat)
    s0_n, _ = flow_stress(e0_n, mat["sy"], mu, mat["n"])
    plastic = _yield(q_tr, sm_tr, s0_n, fs, mat) > 0.0
    x = np.zeros((3, M))
    Ce = K * np.outer(I, I) + 2.0 * mu * (np.eye(6) - np.outer(I, I) / 3.0)
    C = np.repeat(Ce[:, :, None], M, axis=2)
    Nd = np.zeros((6, M))
    pos = q_tr > 0.0
    Nd[:, pos] = 1.5 * s_tr[:, pos] / q_tr[pos]
    idx = np.nonzero(plastic)[0]
    if idx.size:
        qt, st, en, fi, fsi = q_tr[idx], sm_tr[idx], e0_n[idx], f[idx], fs[idx]

        def work(w):
            s0, _ = flow_stress(en + w, mat["sy"], mu, mat["n"])
            q, sm, u, v = _project(qt, st, s0, fsi, mat, K, mu)
            return (1.0 - fi) * s0 * w - (q * u + sm * v)

        f0 = work(np.zeros(idx.size))
        w_hi = -f0 / ((1.0 - fi) * s0_n[idx])
        w = illinois(work, np.zeros(idx.size), w_hi, f0, work(w_hi))
        s0, _ = flow_stress(en + w, mat["sy"], mu, mat["n"])
        q, sm, u, v = _project(qt, st, s0, fsi, mat, K, mu)
        xi = np.stack([u, v, w])
        x[:, idx] = xi
        _, Jx, Jt = _residual_and_jacobian(xi, qt, st, en, fi, fsi, mat, K, mu)
        # d(u, v, w) / d(q_tr, sm_tr) from the linearised local system
        dxd = np.stack([-_solve3(Jx, Jt[:, k]) for k in range(2)], axis=1)  # (3, 2, m)
        Aq, Bq = dxd[0, 0], dxd[0, 1]
        Av, Bv = dxd[1, 0], dxd[1, 1]
        th = np.where(qt > 0.0, q / np.where(qt > 0.0, qt, 1.0), 1.0)
        Ni = Nd[:, idx]
        NN = np.einsum("im,jm->ijm", Ni, Ni)
        NI = np.einsum("im,j->ijm", Ni, I)
        IN = np.einsum("i,jm->ijm", I, Ni)
        Idev = np.eye(6) - np.outer(I, I) / 3.0
        C[:, :, idx] = (2.0 * mu * th[None, None] * Idev[:, :, None]
                        + (K * (1.0 - K * Bv))[None, None] * np.outer(I, I)[:, :, None]
                        + (4.0 * mu / 3.0 * (1.0 - 3.0 * mu * Aq - th))[None, None] * NN
                        - (2.0 * mu * K * Av)[None, None] * IN
                        - (2.0 * mu * K * Bq)[None, None] * NI)
    u, v, w = x
    dep = u[None] * Nd + (v / 3.0)[None] * I[:, None]
    epsp = epsp_n + dep
    sig = s_tr - 2.0 * mu * u[None] * Nd + (sm_tr - K * v)[None] * I[:, None]
    return sig, epsp, e0_n + w, C, x
