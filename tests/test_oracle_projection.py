"""Pins of the checker's Galerkin projection with mixed control (Sec. 3.2.2)."""
import numpy as np
import pytest

from oracle import galerkin, mandel, spectral
from tests._pins import rotated_strain

CASES = [((6, 8), 3), ((4, 6, 8), 6), ((6, 6, 6), 6)]


def _rand(shape, c, seed):
    return np.random.default_rng(seed).standard_normal((c,) + shape)


def _dot(a, b):
    return float((a * b).sum())


@pytest.mark.parametrize("shape,c", CASES)
@pytest.mark.parametrize("scheme", [spectral.ROTATED, spectral.SPECTRAL])
def test_idempotent_selfadjoint_contractive(shape, c, scheme):
    q, qt = spectral.symbols(shape, 1.0, scheme)
    qq = q if scheme == spectral.ROTATED else qt
    mask = np.array([0, 1, 1, 0, 1, 0][:c])
    a, b = _rand(shape, c, 1), _rand(shape, c, 2)
    Pa = galerkin.project(a, qq, mask)
    Pb = galerkin.project(b, qq, mask)
    scale = _dot(a, a)
    assert np.abs(galerkin.project(Pa, qq, mask) - Pa).max() <= 1e-13 * np.abs(a).max()
    assert abs(_dot(Pa, b) - _dot(a, Pb)) <= 1e-12 * scale
    assert _dot(Pa, Pa) <= _dot(a, a) * (1 + 1e-14)


@pytest.mark.parametrize("shape,c", CASES)
def test_compatible_fields_are_fixed(shape, c):
    """A rotated-stencil symmetric gradient of any corner displacement
    field (built in real space, no FFT) is left unchanged."""
    d = len(shape)
    U = np.random.default_rng(3).standard_normal((d,) + shape)
    eps = rotated_strain(U, 1.0)
    assert np.abs(eps.reshape(c, -1).mean(axis=1)).max() < 1e-13
    q, _ = spectral.symbols(shape, 1.0, spectral.ROTATED)
    for mask in (np.zeros(c, int), np.ones(c, int)):
        Pe = galerkin.project(eps, q, mask)
        assert np.abs(Pe - eps).max() <= 1e-13 * np.abs(eps).max()


@pytest.mark.parametrize("shape,c", CASES)
def test_range_is_compatible(shape, c):
    """Projected fields satisfy the discrete compatibility (inc eps = 0):
    q x eps_hat x q = 0 at every frequency."""
    q, _ = spectral.symbols(shape, 1.0, spectral.ROTATED)
    e = galerkin.project(_rand(shape, c, 4), q, np.zeros(c, int))
    d = len(shape)
    E = mandel.to_tensor(np.fft.fftn(e, axes=tuple(range(1, d + 1))))
    qv = [np.broadcast_to(v, shape) for v in q]
    scale = np.abs(E).max() * max(np.abs(v).max() for v in qv) ** 2
    if d == 2:
        inc = qv[1] ** 2 * E[0, 0] + qv[0] ** 2 * E[1, 1] - 2 * qv[0] * qv[1] * E[0, 1]
        assert np.abs(inc).max() <= 1e-12 * scale
    else:
        eps3 = np.zeros((3, 3, 3))
        for i, j, k in [(0, 1, 2), (1, 2, 0), (2, 0, 1)]:
            eps3[i, j, k], eps3[j, i, k] = 1, -1
        # inc(E)_ab = e_aik e_bjl q_i q_j E_kl
        inc = np.einsum("aik,bjl,i...,j...,kl...->ab...", eps3, eps3,
                        np.stack(qv), np.stack(qv), E)
        assert np.abs(inc).max() <= 1e-12 * scale


@pytest.mark.parametrize("shape,c", CASES)
def test_equilibrated_fields_are_annihilated(shape, c):
    """tau_hat with tau_hat q = 0 at every xi != 0 and zero mean on the
    stress-controlled components is in the kernel of G*."""
    d = len(shape)
    q, _ = spectral.symbols(shape, 1.0, spectral.ROTATED)
    ax = tuple(range(1, d + 1))
    A = mandel.to_tensor(np.fft.fftn(_rand(shape, c, 5), axes=ax))
    qv = np.stack([np.broadcast_to(v, shape) for v in q])
    q2 = (qv * qv).sum(0)
    inv = np.where(q2 > 0, 1 / np.where(q2 > 0, q2, 1), 0)
    Pi = np.eye(d).reshape(d, d, *([1] * d)) - np.einsum("a...,b...->ab...", qv, qv) * inv
    T = np.einsum("ab...,bc...,cd...->ad...", Pi, A, Pi)
    tau = np.real(np.fft.ifftn(mandel.from_tensor(T), axes=ax))
    mask = np.array([0, 1, 1, 0, 1, 1][:c])
    tau[mask.astype(bool)] -= tau[mask.astype(bool)].reshape(int(mask.sum()), -1).mean(1).reshape(
        (-1,) + (1,) * d)
    out = galerkin.project(tau, q, mask)
    assert np.abs(out).max() <= 1e-13 * np.abs(tau).max()


@pytest.mark.parametrize("shape,c", CASES)
def test_zero_frequency_keeps_stress_controlled_means(shape, c):
    q, _ = spectral.symbols(shape, 1.0, spectral.ROTATED)
    tau = _rand(shape, c, 6) + np.arange(1, c + 1).reshape((c,) + (1,) * len(shape))
    mask = np.array([1, 0, 1, 1, 0, 1][:c])
    out = galerkin.project(tau, q, mask)
    m_in = tau.reshape(c, -1).mean(1)
    m_out = out.reshape(c, -1).mean(1)
    assert np.allclose(m_out, mask * m_in, atol=1e-13)


@pytest.mark.parametrize("shape,c", CASES)
def test_krylov_dot_in_real_space(shape, c):
    """The CG's p.Ap where p lies in the range of the projection: with A p =
    G*(K:p) and G* an orthogonal projection, p . G*(K:p) = p . (K:p), which
    Parseval's identity turns into a sum over voxels (the GPU's x pass forms
    p.Ap that way instead of on the spectrum).  Checked here with a random
    symmetric positive definite Mandel tangent per voxel and the mixed-control
    mask, against the half-spectrum sum with Hermitian weights."""
    rng = np.random.default_rng(11)
    q, _ = spectral.symbols(shape)
    mask = np.array([0, 1, 1, 0, 1, 0][:c])
    p = galerkin.project(rng.standard_normal((c,) + shape), q, mask)
    B = rng.standard_normal((c, c) + shape) * 0.3
    C = np.einsum("ik...,jk...->ij...", B, B) + 2.0 * np.eye(c).reshape((c, c) + (1,) * len(shape))
    Kp = np.einsum("ij...,j...->i...", C, p)
    real_sum = float((p * Kp).sum())
    assert abs(float((p * galerkin.project(Kp, q, mask)).sum()) - real_sum) <= 1e-12 * abs(real_sum)
    # the same number from the half spectra (weights 2 off the kx = 0 and
    # Nyquist planes), divided by the voxel count
    N = int(np.prod(shape))
    ax = tuple(range(1, len(shape) + 1))
    P = np.fft.rfftn(p, axes=ax)  # the last axis is halved
    W = np.fft.rfftn(Kp, axes=ax)
    n1 = shape[-1]
    wt = np.full(P.shape[-1], 2.0)
    wt[0] = 1.0
    if n1 % 2 == 0:
        wt[-1] = 1.0
    half = float((wt * (P.real * W.real + P.imag * W.imag)).sum()) / N
    assert abs(half - real_sum) <= 1e-12 * abs(real_sum)
