"""Pins of the checker's transform convention and derivative symbols."""
import numpy as np
import pytest

from oracle import spectral
from tests._pins import naive_dft, rotated_gradient


@pytest.mark.parametrize("shape", [(6, 10), (8, 8, 8), (4, 6, 12), (12, 12, 12)])
def test_library_fft_is_the_naive_dft(shape):
    x = np.random.default_rng(0).standard_normal(shape)
    X = spectral.fftn(x)
    ref = naive_dft(x)
    assert np.abs(X - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.allclose(spectral.ifftn(X).real, x, rtol=0, atol=1e-14 * np.abs(x).max())
    # over a subset of the axes (the Galerkin projection transforms the
    # spatial axes of a component-major array)
    X2 = spectral.fftn(np.stack([x, 2 * x]), axes=tuple(range(1, x.ndim + 1)))
    assert np.abs(X2[1] - 2 * ref).max() <= 2e-13 * np.abs(ref).max()
    # Parseval
    assert abs((np.abs(X) ** 2).sum() / x.size - (x * x).sum()) <= 1e-12 * (x * x).sum()


def test_frequencies_are_the_centred_set():
    # Sec. 3.2.1: xi = 2 pi / L (n - N/2), n in [0, N)  (even N)
    for n in (8, 12, 32):
        th, m = spectral.theta_1d(n)
        centred = np.sort(2 * np.pi * (np.arange(n) - n // 2) / n)
        assert np.allclose(np.sort(th), centred, atol=0)


@pytest.mark.parametrize("shape", [(6, 8), (4, 6, 8)])
def test_rotated_symbol_is_the_corner_stencil(shape):
    """The rotated-scheme symbol times i exp(i sum theta/2) must equal the DFT
    eigenvalue of the real-space rotated stencil (corner values -> centre
    derivative), computed by applying the stencil to plane waves."""
    h = 0.7
    q, qt = spectral.symbols(shape, h, spectral.ROTATED)
    ndim = len(shape)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(shape)
    grads = rotated_gradient(u, h)
    U = np.fft.fftn(u)
    thetas = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(n) for n in shape], indexing="ij")
    phase = np.exp(1j * sum(thetas) / 2.0)
    for j in range(ndim):
        G = np.fft.fftn(grads[j])
        sym = 1j * q[j] * phase
        assert np.abs(G - sym * U).max() <= 1e-12 * np.abs(U).max()


def test_q_tilde_vanishes_on_nyquist_and_is_odd_elsewhere():
    shape = (6, 8, 10)
    q, qt = spectral.symbols(shape, 1.0, spectral.ROTATED)
    for j in range(3):
        ax = 2 - j
        n = shape[ax]
        sl = [slice(None)] * 3
        sl[ax] = n // 2
        assert np.all(qt[j][tuple(sl)] == 0)
        # odd under xi -> -xi away from Nyquist planes
        idx = [(-np.arange(s)) % s for s in shape]
        flipped = qt[j][np.ix_(*idx)]
        assert np.allclose(flipped, -qt[j], atol=1e-15)
    # |q|^2 = 0 exactly where two or more components are at Nyquist
    q2 = sum(v * v for v in q)
    assert q2[3, 4, 0] == 0 and q2[3, 0, 5] == 0 and q2[0, 0, 0] == 0
    # zero set: xi = 0, plus the three lines with two Nyquist components
    # (the all-Nyquist corner belongs to all three lines)
    assert np.count_nonzero(q2 == 0) == 1 + (6 + 8 + 10 - 2)


def test_spectral_symbol():
    q, qt = spectral.symbols((4, 8), 2.0, spectral.SPECTRAL)
    th, _ = spectral.theta_1d(8)
    assert np.allclose(q[0][0], th / 2.0)
