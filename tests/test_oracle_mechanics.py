"""Pins of the checker's FFT-Galerkin mechanics with mixed control
(Sec. 3.2.2) against closed forms and an independent real-space assembly."""
import numpy as np
import pytest
from scipy import optimize

from oracle import galerkin, mandel, material, spectral
from tests._pins import rotated_strain

EM, NUM, SY, H = 70000.0, 0.3, 300.0, 500.0
EP, NUP = 400000.0, 0.2


def el(E, nu, ell=1.0):
    return dict(model="elastic", E=E, nu=nu, sy=0.0, H=0.0, dfield=-1, dC=0, dR=1, dmax=0,
                ell=[ell])


def j2(ell=2.0):
    return dict(model="j2_damage", E=EM, nu=NUM, sy=SY, H=H, dfield=0, dC=0.03, dR=0.2,
                dmax=0.99, ell=[ell])


def solve(phase, table, target, c, tol=1e-13, ntol=1e-12, eps0=None):
    S = phase.shape
    eps0 = np.zeros((c,) + S) if eps0 is None else eps0
    return galerkin.fftg_solve(phase, table, np.zeros((1,) + S), np.zeros((6,) + S),
                               np.zeros(S), target, eps0, cg_tol=tol, newton_tol=ntol)


def test_homogeneous_strain_control_is_uniform():
    S = (4, 6, 8)
    phase = np.zeros(S, np.uint8)
    Emac = np.array([1e-3, -2e-4, 3e-4, 1e-4, -5e-5, 2e-4])
    r = solve(phase, [el(EM, NUM)], (np.zeros(6, np.uint8), Emac, np.zeros(6)), 6)
    assert np.abs(r["eps"] - Emac.reshape(6, 1, 1, 1)).max() <= 1e-16


def test_homogeneous_j2_uniaxial_closed_form():
    """Homogeneous J2 under 3D uniaxial mixed control: Sigma11 on the
    bilinear curve sy + E_t (E11 - eps_Y), E_t = E H/(E + H)."""
    S = (4, 4, 4)
    phase = np.zeros(S, np.uint8)
    e11 = 5e-3
    mask = np.array([0, 1, 1, 1, 1, 1], np.uint8)
    Emac = np.array([e11, 0, 0, 0, 0, 0.0])
    r = solve(phase, [j2()], (mask, Emac, np.zeros(6)), 6, ntol=1e-13)
    Et = EM * H / (EM + H)
    s11 = SY + Et * (e11 - SY / EM)
    kap = e11 - s11 / EM
    e22 = -NUM * s11 / EM - kap / 2
    sig = r["sigma"].reshape(6, -1)
    eps = r["eps"].reshape(6, -1)
    assert np.abs(sig[0] - s11).max() <= 1e-9 * s11
    assert np.abs(sig[1:]).max() <= 1e-8
    assert np.abs(eps[1] - e22).max() <= 1e-12 and np.abs(eps[2] - e22).max() <= 1e-12
    assert abs(s11 - 300.3546099290780) < 1e-9


def test_plane_strain_homogeneous_matches_point_driver():
    """2D plane strain, homogeneous J2, uniaxial mixed control: equals a
    single material point with e11 given and sigma22 = sigma12 = 0 solved by
    scipy root-finding."""
    S = (4, 6)
    phase = np.zeros(S, np.uint8)
    e11 = 4e-3
    mask = np.array([0, 1, 1], np.uint8)
    r = solve(phase, [j2()], (mask, np.array([e11, 0, 0.0]), np.zeros(3)), 3, ntol=1e-13)

    def resid(x):
        e = mandel.expand_plane(np.array([[e11], [x[0]], [x[1]]]))
        s = material.j2_return_map(e, np.zeros((6, 1)), np.zeros(1), EM, NUM, SY, H)[0]
        return [s[1, 0] / SY, s[5, 0] / SY]

    sol = optimize.root(resid, [-1e-3, 0.0], tol=1e-15)
    e = mandel.expand_plane(np.array([[e11], [sol.x[0]], [sol.x[1]]]))
    s = material.j2_return_map(e, np.zeros((6, 1)), np.zeros(1), EM, NUM, SY, H)[0]
    assert np.abs(r["eps"][1] - sol.x[0]).max() <= 1e-11
    assert np.abs(r["sigma"][0] - s[0, 0]).max() <= 1e-9 * abs(s[0, 0])


@pytest.mark.parametrize("fb", [0.25, 0.5])
def test_laminate_voigt_reuss(fb):
    """Layers normal to x1: strain-controlled normal strain and transverse
    shear give the Reuss averages, in-plane shear and uniaxial stress along
    the layers (equal nu) the Voigt averages -- all exact for laminates."""
    S = (4, 4, 8)
    phase = np.zeros(S, np.uint8)
    nb = int(fb * 8)
    phase[:, :, :nb] = 1
    A = el(70000.0, 0.25)
    B = el(210000.0, 0.25)
    tab = [A, B]
    f = np.array([1 - fb, fb])
    K, mu = zip(*[material.lame(m["E"], m["nu"]) for m in tab])
    K, mu = np.array(K), np.array(mu)
    Pmod = K + 4 * mu / 3
    z6 = np.zeros(6, np.uint8)
    # normal strain e11
    r = solve(phase, tab, (z6, np.array([1e-3, 0, 0, 0, 0, 0.0]), np.zeros(6)), 6)
    s11 = 1e-3 / (f / Pmod).sum()
    assert np.abs(r["sigma"][0] - s11).max() <= 1e-10 * s11
    # transverse shear (Mandel slot 5 = sqrt2 e12)
    r = solve(phase, tab, (z6, np.array([0, 0, 0, 0, 0, 1e-3]), np.zeros(6)), 6)
    mu_r = 1 / (f / mu).sum()
    assert abs(r["sigma"][5].mean() - 2 * mu_r * 1e-3) <= 1e-10 * 2 * mu_r * 1e-3
    assert np.abs(r["sigma"][5] - 2 * mu_r * 1e-3).max() <= 1e-9 * 2 * mu_r * 1e-3
    # in-plane shear (slot 3 = sqrt2 e23): Voigt, strain uniform
    r = solve(phase, tab, (z6, np.array([0, 0, 0, 1e-3, 0, 0]), np.zeros(6)), 6)
    assert abs(r["sigma"][3].mean() - 2 * (f * mu).sum() * 1e-3) <= 1e-10 * 2 * mu.max() * 1e-3
    assert np.abs(r["eps"][3] - 1e-3).max() <= 1e-14
    # uniaxial stress along x2 (mixed control), equal nu: Voigt on E
    mask = np.array([1, 0, 1, 1, 1, 1], np.uint8)
    r = solve(phase, tab, (mask, np.array([0, 1e-3, 0, 0, 0, 0]), np.zeros(6)), 6)
    Ev = (f * np.array([A["E"], B["E"]])).sum()
    assert abs(r["sigma"][1].mean() - Ev * 1e-3) <= 1e-10 * Ev * 1e-3
    means = r["sigma"].reshape(6, -1).mean(1)
    assert np.abs(means[mask.astype(bool)]).max() <= 1e-8 * Ev * 1e-3


def _assemble_B(S, c):
    d = len(S)
    N = int(np.prod(S))
    B = np.zeros((c * N, d * N))
    for col in range(d * N):
        U = np.zeros(d * N)
        U[col] = 1.0
        B[:, col] = rotated_strain(U.reshape((d,) + S)).reshape(-1)
    return B


@pytest.mark.parametrize("S", [(4, 4), (6, 4), (4, 4, 4)])
def test_matches_real_space_rotated_fd_assembly(S):
    """Heterogeneous elastic, strain control: the Galerkin strain equals the
    energy minimiser over corner displacements with the rotated stencil,
    assembled and solved densely (no FFT)."""
    d = len(S)
    c = 6 if d == 3 else 3
    N = int(np.prod(S))
    rng = np.random.default_rng(7)
    phase = (rng.uniform(size=S) < 0.4).astype(np.uint8)
    tab = [el(EM, NUM), el(EP, NUP)]
    Emac = np.array([1e-3, -3e-4, 2e-4, 1e-4, -2e-4, 3e-4])[:c] if d == 3 else \
        np.array([1e-3, -3e-4, 2e-4])
    r = solve(phase, tab, (np.zeros(c, np.uint8), Emac, np.zeros(c)), c)
    # block-diagonal stiffness in the (comp, voxel) ordering of the flattened fields
    Cs = []
    for m in tab:
        K, mu = material.lame(m["E"], m["nu"])
        C6 = material.elastic_tangent(K, mu)
        Cs.append(C6 if c == 6 else C6[np.ix_([0, 1, 5], [0, 1, 5])])
    ph = phase.reshape(-1)
    Cbig = np.zeros((c * N, c * N))
    for x in range(N):
        idx = np.arange(c) * N + x
        Cbig[np.ix_(idx, idx)] = Cs[ph[x]]
    B = _assemble_B(S, c)
    Ef = np.repeat(Emac, N)
    u, *_ = np.linalg.lstsq(B.T @ Cbig @ B, -B.T @ Cbig @ Ef, rcond=1e-12)
    eps_fd = (Ef + B @ u).reshape((c,) + S)
    assert np.abs(r["eps"] - eps_fd).max() <= 1e-10 * np.abs(Emac).max()


def test_mixed_control_constraints_and_equilibrium():
    S = (8, 8, 8)
    rng = np.random.default_rng(8)
    phase = (rng.uniform(size=S) < 0.3).astype(np.uint8)
    tab = [j2(), el(EP, NUP)]
    mask = np.array([0, 1, 1, 0, 1, 1], np.uint8)
    Emac = np.array([4e-3, 0, 0, 1e-4, 0, 0])
    Smac = np.array([0, 20.0, -10.0, 0, 5.0, 0])
    r = solve(phase, tab, (mask, Emac, Smac), 6, tol=1e-12, ntol=1e-11)
    assert r["converged"]
    m_eps = r["eps"].reshape(6, -1).mean(1)
    m_sig = r["sigma"].reshape(6, -1).mean(1)
    assert np.allclose(m_eps[~mask.astype(bool)], Emac[~mask.astype(bool)], atol=1e-15)
    assert np.abs(m_sig - Smac)[mask.astype(bool)].max() <= 1e-7
    q, _ = spectral.symbols(S)
    T = mandel.to_tensor(np.fft.fftn(r["sigma"], axes=(1, 2, 3)))
    div = np.einsum("ab...,b...->a...", T, np.stack(q))
    assert np.abs(div).max() <= 1e-8 * np.abs(T).max()
    assert (r["kappa"] > 0).any()
