"""Mandel representation of symmetric second-order tensors.

3D: (T11, T22, T33, sqrt2 T23, sqrt2 T13, sqrt2 T12); 2D: (T11, T22, sqrt2 T12).
With this scaling the tensor double contraction A:B is the plain dot product
of the Mandel vectors.
"""
from __future__ import annotations

import numpy as np

R2 = np.sqrt(2.0)
# (row, col) of each Mandel slot, 0-based
PAIRS3 = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
PAIRS2 = [(0, 0), (1, 1), (0, 1)]


def pairs(c):
    return PAIRS3 if c == 6 else PAIRS2


def to_tensor(m):
    """Mandel (c, ...) -> full tensor (d, d, ...)."""
    c = m.shape[0]
    d = 3 if c == 6 else 2
    T = np.zeros((d, d) + m.shape[1:], dtype=m.dtype)
    for k, (a, b) in enumerate(pairs(c)):
        if a == b:
            T[a, a] = m[k]
        else:
            T[a, b] = m[k] / R2
            T[b, a] = m[k] / R2
    return T


def from_tensor(T):
    """Full (symmetric) tensor (d, d, ...) -> Mandel (c, ...)."""
    d = T.shape[0]
    c = 6 if d == 3 else 3
    m = np.zeros((c,) + T.shape[2:], dtype=T.dtype)
    for k, (a, b) in enumerate(pairs(c)):
        if a == b:
            m[k] = T[a, a]
        else:
            m[k] = R2 * 0.5 * (T[a, b] + T[b, a])
    return m


def identity(c=6):
    v = np.zeros(c)
    v[:3 if c == 6 else 2] = 1.0
    return v


def expand_plane(m3):
    """2D plane-strain Mandel (3, ...) -> 3D Mandel (6, ...) with the
    out-of-plane strain components zero."""
    out = np.zeros((6,) + m3.shape[1:], dtype=m3.dtype)
    out[0], out[1], out[5] = m3[0], m3[1], m3[2]
    return out


def reduce_plane(m6):
    """3D Mandel (6, ...) -> in-plane Mandel (3, ...)."""
    return np.stack([m6[0], m6[1], m6[5]])


PLANE_IDX = [0, 1, 5]
