"""Pins of the checker's Helmholtz PCG (Sec. 3.2.3, Algorithm 2)."""
import numpy as np
import pytest

from oracle import helmholtz, spectral
from tests._pins import dense_helmholtz as _dense_L


@pytest.mark.parametrize("shape", [(6, 8), (4, 4, 6), (3, 4, 6)])
def test_matches_dense_real_space_solve(shape):
    h = 0.8
    rng = np.random.default_rng(0)
    phase = (rng.uniform(size=shape) < 0.4)
    ell2 = np.where(phase, 0.3 ** 2, 2.0 ** 2)
    alpha = np.abs(rng.standard_normal(shape))
    r = helmholtz.helmholtz_solve(alpha, ell2, h=h, tol=1e-14, maxit=500)
    ref = np.linalg.solve(_dense_L(shape, ell2, h), alpha.reshape(-1)).reshape(shape)
    assert r["converged"]
    assert np.abs(r["abar"] - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("shape", [(16, 16), (8, 12, 16)])
def test_constant_length_closed_form_one_iteration(shape):
    """Uniform ell: the preconditioner is the exact inverse, so PCG stops
    after one iteration with abar_hat = alpha_hat / (1 + ell^2 |q~|^2)."""
    rng = np.random.default_rng(1)
    alpha = rng.standard_normal(shape)
    ell = 2.5
    r = helmholtz.helmholtz_solve(alpha, np.full(shape, ell * ell), tol=1e-12)
    _, qt = spectral.symbols(shape)
    q2 = sum(np.broadcast_to(v, shape) ** 2 for v in qt)
    ref = np.real(np.fft.ifftn(np.fft.fftn(alpha) / (1 + ell * ell * q2)))
    assert r["iters"] == 1
    assert np.abs(r["abar"] - ref).max() <= 1e-14 * np.abs(alpha).max()


def test_mean_preserved_and_zero_length_identity():
    shape = (8, 8, 8)
    rng = np.random.default_rng(2)
    alpha = np.abs(rng.standard_normal(shape))
    ell2 = np.where(rng.uniform(size=shape) < 0.3, 0.01, 4.0)
    r = helmholtz.helmholtz_solve(alpha, ell2, tol=1e-13)
    assert abs(r["abar"].mean() - alpha.mean()) <= 1e-14 * alpha.mean()
    r0 = helmholtz.helmholtz_solve(alpha, np.zeros(shape), tol=1e-13)
    assert np.abs(r0["abar"] - alpha).max() <= 1e-15 * alpha.max()


def test_operator_symmetric_positive():
    shape = (6, 8, 10)
    rng = np.random.default_rng(3)
    ell2 = rng.uniform(0.01, 3.0, size=shape)
    _, qt = spectral.symbols(shape)
    qt = [np.broadcast_to(v, shape) for v in qt]
    x = np.fft.fftn(rng.standard_normal(shape))
    y = np.fft.fftn(rng.standard_normal(shape))
    Lx = helmholtz.operator(x, ell2, qt)
    Ly = helmholtz.operator(y, ell2, qt)
    a = np.vdot(y, Lx).real
    b = np.vdot(Ly, x).real
    assert abs(a - b) <= 1e-12 * abs(a)
    assert np.vdot(x, Lx).real >= np.vdot(x, x).real * (1 - 1e-14)
    # Hermitian input -> Hermitian output (the field stays real)
    assert np.abs(np.fft.ifftn(Lx).imag).max() <= 1e-12 * np.abs(np.fft.ifftn(Lx).real).max()


def test_interface_contrast_limits_leakage():
    """Sec. 2.2.1 remark: a small length in the non-host phase keeps the
    non-local field from spreading into it; leakage falls as the ratio grows."""
    n = 64
    shape = (4, n)
    x = np.arange(n)
    host = (x >= 16) & (x < 48)
    alpha = np.broadcast_to(np.where(host, 1.0, 0.0), shape).copy()
    leak = []
    for ratio in (1.0, 5.0, 50.0):
        ell2 = np.broadcast_to(np.where(host, 4.0 ** 2, (4.0 / ratio) ** 2), shape).copy()
        r = helmholtz.helmholtz_solve(alpha, ell2, tol=1e-12, maxit=5000)
        leak.append(r["abar"][:, ~host].sum() / r["abar"].sum())
    assert leak[0] > leak[1] > leak[2]


@pytest.mark.parametrize("shape", [(8, 6), (6, 8, 10)])
def test_energy_form_of_the_operator(shape):
    """p . L p = sum |p|^2 + sum ell^2 |grad p|^2 over the voxels, for the
    gradient the operator itself uses (i q~_j); the spectral side is the
    weighted half-spectrum sum.  The GPU's PCG forms p . L p from these two
    real-space and spectral pieces instead of from L p."""
    rng = np.random.default_rng(5)
    N = int(np.prod(shape))
    p = rng.standard_normal(shape)
    ell2 = rng.uniform(0.05, 4.0, size=shape)
    _, qt = spectral.symbols(shape)
    qt = [np.broadcast_to(v, shape) for v in qt]
    P = spectral.fftn(p)
    LP = helmholtz.operator(P, ell2, qt)
    spectral_sum = float(np.vdot(P, LP).real) / N
    grads = [np.real(spectral.ifftn(1j * qj * P)) for qj in qt]
    energy = float((p * p).sum()) + float(sum((ell2 * g * g).sum() for g in grads))
    assert abs(spectral_sum - energy) <= 1e-12 * energy
    # the half spectrum with Hermitian weights gives the same first term
    n1 = shape[-1]
    Ph = np.fft.rfftn(p, axes=tuple(range(len(shape))))
    wt = np.full(Ph.shape[-1], 2.0)
    wt[0] = 1.0
    if n1 % 2 == 0:
        wt[-1] = 1.0
    assert abs(float((wt * np.abs(Ph) ** 2).sum()) / N - float((p * p).sum())) <= 1e-12 * N
