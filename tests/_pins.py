"""Independent constructions used to pin the CPU checker (test helpers).

Nothing here is shared with the GPU library: these are textbook definitions
written directly (a naive DFT, the rotated finite-difference stencil in real
space, circulant matrices from trigonometric sums).
"""
import numpy as np


def naive_dft(x):
    """O(N^2) multi-dimensional DFT, X[k] = sum_n x[n] exp(-2 pi i k.n / N)."""
    out = np.asarray(x, dtype=np.complex128)
    for ax in range(out.ndim):
        n = out.shape[ax]
        k = np.arange(n)
        W = np.exp(-2j * np.pi * np.outer(k, k) / n)
        out = np.moveaxis(np.tensordot(W, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
    return out


def rotated_gradient(u, h=1.0):
    """Willot's rotated finite-difference gradient of a periodic scalar field
    given at voxel corners: the derivative along axis j at voxel n is the
    average over the 2^(d-1) voxel edges parallel to j of the forward
    difference u(n + e_j + b) - u(n + b), b in the other axes' {0,1}.
    u: numpy array (z, y, x) of corner values (corner n at position n h).
    Returns list over physical axes (x, y, z) of arrays (z, y, x)."""
    d = u.ndim
    grads = []
    for j in range(d):
        ax = d - 1 - j
        diff = np.roll(u, -1, axis=ax) - u
        others = [a for a in range(d) if a != ax]
        acc = np.zeros_like(u)
        for bits in range(2 ** len(others)):
            v = diff
            for t, a in enumerate(others):
                if (bits >> t) & 1:
                    v = np.roll(v, -1, axis=a)
            acc = acc + v
        grads.append(acc / (2 ** len(others)) / h)
    return grads


def rotated_strain(U, h=1.0):
    """Mandel strain sym(grad U) at voxel centres from a corner displacement
    field U (d, *S) with the rotated stencil."""
    d = U.shape[0]
    G = [rotated_gradient(U[i], h) for i in range(d)]  # G[i][j] = d u_i / d x_j
    r2 = np.sqrt(2.0)
    if d == 3:
        return np.stack([G[0][0], G[1][1], G[2][2],
                         r2 * 0.5 * (G[1][2] + G[2][1]),
                         r2 * 0.5 * (G[0][2] + G[2][0]),
                         r2 * 0.5 * (G[0][1] + G[1][0])])
    return np.stack([G[0][0], G[1][1], r2 * 0.5 * (G[0][1] + G[1][0])])


def _circulants(n, h):
    """Real circulant matrices of F^-1 diag(i s) F and F^-1 diag(c) F for
    s = (2/h) sin(theta/2), c = cos(theta/2) (both zero on the Nyquist
    frequency), built from trigonometric sums (no FFT)."""
    m = np.fft.fftfreq(n) * n
    th = 2 * np.pi * m / n
    nyq = (n % 2 == 0) & (m == -n // 2)
    s = np.where(nyq, 0.0, (2 / h) * np.sin(th / 2))
    c = np.where(nyq, 0.0, np.cos(th / 2))
    d = np.subtract.outer(np.arange(n), np.arange(n))
    ang = np.multiply.outer(d, th)
    Smat = -(np.sin(ang) * s).sum(-1) / n
    Cmat = (np.cos(ang) * c).sum(-1) / n
    return Smat, Cmat


def dense_gradients(shape, h):
    """Dense real matrices Q_j (physical axis j) of the rotated first-order
    derivative with zeroed Nyquist planes, acting on flattened (z, y, x)
    fields."""
    ndim = len(shape)
    mats = [_circulants(shape[ndim - 1 - j], h) for j in range(ndim)]  # physical order
    out = []
    for j in range(ndim):
        Q = np.ones((1, 1))
        for ax in range(ndim):            # numpy axis order z, y, x
            pj = ndim - 1 - ax
            Q = np.kron(Q, mats[pj][0] if pj == j else mats[pj][1])
        out.append(Q)
    return out


def dense_helmholtz(shape, ell2, h):
    N = int(np.prod(shape))
    L = np.eye(N)
    for Q in dense_gradients(shape, h):
        L += Q.T @ np.diag(ell2.reshape(-1)) @ Q
    return L
