"""Generalised Helmholtz equation abar - div(ell^2(x) grad abar) = alpha in
Fourier space, solved by preconditioned CG (Sec. 3.2.3, eq. LhelmFourier,
eq. preconditioner, Algorithm 2).

Operator, with the derivative symbol q_tilde (see spectral):
    L u_hat = u_hat - i sum_j q~_j F( ell^2 F^-1( i q~_j u_hat ) )
which is the paper's u_hat + xi . F(ell^2 F^-1(xi u_hat)) with xi -> q~,
written with the factors i so that every intermediate field is real; ell^2
multiplies at the voxel centres.
Preconditioner: M r_hat = r_hat / (1 + ell_ref^2 |q~|^2), where
ell_ref^2 = <ell^2> (volume mean) unless given.
ConjGrad(A, M, b, TOL): returns x with ||A x - b|| < TOL ||b||.

Everything runs on the full complex spectrum (numpy fftn / ifftn) with the
Hermitian inner product Re(sum a conj(b)).
"""
from __future__ import annotations

import numpy as np

from . import spectral


def operator(u_hat, ell2, qt):
    S = u_hat.shape
    out = u_hat.copy()
    for qj in qt:
        g = spectral.ifftn(1j * qj * u_hat)      # i q~_j u_hat -> real gradient field
        hh = spectral.fftn(ell2 * np.real(g))
        out = out - 1j * qj * hh
    return out


def pcg(apply_A, apply_M, b, x0, tol, maxit):
    """Preconditioned CG in the Hermitian inner product.
    Returns (x, iterations, ||r||/||b||, converged)."""
    dot = lambda a, c: np.vdot(c, a).real  # Re(sum a conj(c))
    nb = np.sqrt(dot(b, b))
    if nb == 0.0:
        return np.zeros_like(b), 0, 0.0, True
    x = x0.copy()
    r = b - apply_A(x)
    nr = np.sqrt(dot(r, r))
    if nr <= tol * nb:
        return x, 0, nr / nb, True
    z = apply_M(r)
    p = z.copy()
    rz = dot(r, z)
    it = 0
    while it < maxit:
        Ap = apply_A(p)
        pAp = dot(p, Ap)
        if pAp <= 0.0:
            break
        a = rz / pAp
        x = x + a * p
        r = r - a * Ap
        it += 1
        nr = np.sqrt(dot(r, r))
        if nr <= tol * nb:
            return x, it, nr / nb, True
        z = apply_M(r)
        rz_new = dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, nr / nb, False


def helmholtz_solve(alpha, ell2, h=1.0, scheme=spectral.ROTATED, ell2_ref=-1.0,
                    x0=None, tol=1e-8, maxit=1000):
    """Algorithm 2 for one field.  alpha, ell2: real arrays with the grid
    shape; x0: initial guess in real space (default 0).
    Returns dict(abar, iters, relres, converged)."""
    S = alpha.shape
    _, qt = spectral.symbols(S, h, scheme)
    qt = [np.broadcast_to(v, S) for v in qt]
    if ell2_ref is None or ell2_ref <= 0:
        ell2_ref = float(np.mean(ell2))
    q2 = sum(v * v for v in qt)
    Minv = 1.0 / (1.0 + ell2_ref * q2)
    b = spectral.fftn(alpha)
    xh0 = spectral.fftn(x0) if x0 is not None else np.zeros_like(b)
    x, it, rel, ok = pcg(lambda u: operator(u, ell2, qt), lambda r: Minv * r,
                         b, xh0, tol, maxit)
    return dict(abar=np.real(spectral.ifftn(x)), iters=it, relres=rel, converged=ok)
