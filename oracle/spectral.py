"""Discrete frequencies and derivative symbols (Sec. 3.2.1, discretization).

Fields live at voxel centres x_i = (n_i + 1/2) h of an N_1 x N_2 (x N_3)
periodic grid, stored as numpy arrays with axes (z, y, x) -- physical axis 1
(x) is the last numpy axis.  The discrete frequencies are the centred set
xi_i = 2 pi m_i / L_i, m_i in {-N_i/2, ..., N_i/2 - 1} (N_i even), which is
the same set as numpy's standard FFT order; theta_i = xi_i h = 2 pi m_i / N_i.

Derivative symbols (the paper names Willot's rotated finite-difference scheme
and does not print it; this is the reading used here):
  ROTATED : q_j = (2/h) sin(theta_j/2) prod_{m != j} cos(theta_m/2)
            i.e. Willot's rotated-scheme frequency with its common phase
            factor exp(i sum theta / 2) removed (it cancels in the projector);
  SPECTRAL: q_j = theta_j / h  (plain spectral derivative, test option).
q_tilde is q with q_tilde_j = 0 on the Nyquist plane m_j = -N_j/2 of axis j
(even N_j): a first-order symbol must be odd under xi -> -xi for the
derivative of a real field to stay real, and the Nyquist plane is its own
mirror image.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft

ROTATED = "rotated"
SPECTRAL = "spectral"

# Threads of the library FFT (scipy.fft): every core this process may run on,
# for arrays large enough to pay for them (starting the threads costs about
# 0.6 ms, 20x a small grid's whole transform).  The threads share out whole
# 1D transforms, so the result is the same bit for bit either way.
WORKERS = len(os.sched_getaffinity(0))
THREADED_MIN = 1 << 16


def _workers(x):
    return WORKERS if x.size >= THREADED_MIN else 1


def fftn(x, axes=None):
    """Unnormalised DFT X[k] = sum_n x[n] exp(-2 pi i k.n / N) over `axes`
    (all by default), the library primitive of every transform here."""
    return scipy.fft.fftn(x, axes=axes, workers=_workers(x))


def ifftn(X, axes=None):
    """Inverse of fftn, normalised by 1/N."""
    return scipy.fft.ifftn(X, axes=axes, workers=_workers(X))


def theta_1d(n):
    """theta = 2 pi m / n with m in standard FFT order."""
    m = np.fft.fftfreq(n) * n
    return 2.0 * np.pi * m / n, m


def _axis_view(v, ndim, j):
    """Reshape a 1D array along physical axis j (0 = x) for broadcasting on
    arrays with numpy axes (z, y, x)."""
    shp = [1] * ndim
    shp[ndim - 1 - j] = v.shape[0]
    return v.reshape(shp)


def symbols(shape, h=1.0, scheme=ROTATED):
    """Return (q, q_tilde): lists of ndim arrays (physical axis order x, y, z),
    each broadcastable to `shape` (numpy order)."""
    ndim = len(shape)
    thetas, nyq = [], []
    for j in range(ndim):
        n = shape[ndim - 1 - j]
        th, m = theta_1d(n)
        thetas.append(_axis_view(th, ndim, j))
        isnyq = (n % 2 == 0) & (m == -n // 2)
        nyq.append(_axis_view(isnyq, ndim, j))
    # cos(theta/2) is exactly zero on a Nyquist plane (theta = -pi); the
    # floating-point cos(-pi/2) is 6e-17, which would leave |q|^2 ~ 1e-32
    # instead of 0 where two Nyquist components meet.
    halfcos = [np.where(nyq[m], 0.0, np.cos(thetas[m] / 2.0)) for m in range(ndim)]
    q = []
    for j in range(ndim):
        if scheme == ROTATED:
            v = (2.0 / h) * np.sin(thetas[j] / 2.0)
            for m in range(ndim):
                if m != j:
                    v = v * halfcos[m]
        elif scheme == SPECTRAL:
            v = thetas[j] / h + 0.0 * sum(thetas)
        else:
            raise ValueError(scheme)
        q.append(np.broadcast_to(v, shape).copy())
    qt = [np.where(np.broadcast_to(nyq[j], shape), 0.0, q[j]) for j in range(ndim)]
    return q, qt


def projection_symbol(shape, h=1.0, scheme=ROTATED):
    """Symbol used by the Galerkin projection.  ROTATED: q itself (the
    projector depends on q (x) q only, which is even on the Nyquist planes).
    SPECTRAL: q_tilde, since theta_j/h is not odd on its own Nyquist plane
    and the projected field would not stay real."""
    q, qt = symbols(shape, h, scheme)
    return q if scheme == ROTATED else qt
