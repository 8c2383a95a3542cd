"""Pins of the checker's constitutive update (Sec. 2.1.2, appendix A.2)."""
import numpy as np
import pytest

from oracle import material, mandel

E, NU, SY, H = 70000.0, 0.3, 300.0, 500.0


def _rand_strain(M, scale, seed):
    return scale * np.random.default_rng(seed).standard_normal((6, M))


def test_elastic_below_yield():
    eps = _rand_strain(50, 1e-4, 0)
    s, ep, k, C = material.j2_return_map(eps, np.zeros((6, 50)), np.zeros(50), E, NU, SY, H)
    K, mu = material.lame(E, NU)
    lam = K - 2 * mu / 3
    T = mandel.to_tensor(eps)
    tr = T[0, 0] + T[1, 1] + T[2, 2]
    sig = lam * tr * np.eye(3)[:, :, None] + 2 * mu * T      # Hooke's law, tensor form
    assert np.allclose(s, mandel.from_tensor(sig), rtol=1e-13, atol=1e-10)
    assert np.all(k == 0) and np.all(ep == 0)


def test_uniaxial_closed_form_point():
    """Radial return of a uniaxial-stress strain state lands on the
    hardening curve sigma = sy + H eps_p with eps_p = e11 - sigma/E."""
    e11 = 5e-3
    s11 = (E * SY + E * H * e11) / (E + H)
    kap = e11 - s11 / E
    e22 = -NU * s11 / E - kap / 2
    eps = np.array([[e11], [e22], [e22], [0], [0], [0]])
    s, ep, k, C = material.j2_return_map(eps, np.zeros((6, 1)), np.zeros(1), E, NU, SY, H)
    assert abs(s[0, 0] - s11) <= 1e-10 * s11
    assert np.abs(s[1:, 0]).max() <= 1e-9 * s11
    assert abs(k[0] - kap) <= 1e-12
    assert abs(s11 - 300.354609929078) < 1e-9


def test_consistency_and_incompressibility():
    M = 200
    eps = _rand_strain(M, 3e-3, 1)
    epn = _rand_strain(M, 1e-3, 2)
    epn -= (epn[0] + epn[1] + epn[2]) / 3 * mandel.identity(6)[:, None]
    kn = np.abs(np.random.default_rng(3).standard_normal(M)) * 1e-2
    s, ep, k, C = material.j2_return_map(eps, epn, kn, E, NU, SY, H)
    dev = s - (s[0] + s[1] + s[2]) / 3 * mandel.identity(6)[:, None]
    q = np.sqrt(1.5 * (dev * dev).sum(0))
    pl = k > kn
    assert pl.sum() > 20 and (~pl).sum() > 5
    assert np.allclose(q[pl], SY + H * k[pl], rtol=1e-12)
    assert np.all(q[~pl] <= SY + H * kn[~pl] + 1e-9)
    assert np.abs(ep[0] + ep[1] + ep[2]).max() < 1e-15


def test_tangent_matches_central_differences():
    M = 60
    eps = _rand_strain(M, 3e-3, 4)
    epn = np.zeros((6, M))
    kn = np.zeros(M)
    s0, _, k0, C = material.j2_return_map(eps, epn, kn, E, NU, SY, H)
    assert (k0 > 0).sum() > 30
    hstep = 1e-7
    for a in range(6):
        dp = eps.copy(); dp[a] += hstep
        dm = eps.copy(); dm[a] -= hstep
        sp = material.j2_return_map(dp, epn, kn, E, NU, SY, H)[0]
        sm = material.j2_return_map(dm, epn, kn, E, NU, SY, H)[0]
        fd = (sp - sm) / (2 * hstep)
        assert np.abs(fd - C[:, a, :]).max() <= 1e-6 * np.abs(C).max()
    # symmetric
    assert np.abs(C - C.transpose(1, 0, 2)).max() <= 1e-10 * np.abs(C).max()


def test_damage_law_piecewise():
    table = [dict(model="j2_damage", dfield=0, dC=0.03, dR=0.2, dmax=0.99),
             dict(model="elastic_cracking", dfield=1, dC=1e-3, dR=1e-2, dmax=0.99),
             dict(model="elastic", dfield=-1, dC=0, dR=1, dmax=0)]
    phase = np.array([0, 0, 0, 0, 1, 1, 1, 2], dtype=np.uint8)
    abar = np.zeros((2, 8))
    abar[0, :4] = [0.01, 0.03, 0.115, 0.5]
    abar[1, 4:7] = [5e-4, 5.5e-3, 0.0]
    hist = np.zeros((2, 8))
    hist[1, 6] = 2e-2
    abar[0, 7] = 1.0
    D = material.damage_from_nonlocal(phase, table, abar, hist)
    assert np.allclose(D[0, :4], [0.0, 0.0, 0.5, 0.99], atol=1e-15)
    assert np.allclose(D[1, 4:7], [0.0, 0.5, 0.99], atol=1e-15)
    assert D[0, 7] == 0 and D[1, 7] == 0 and np.all(D[1, :4] == 0) and np.all(D[0, 4:] == 0)


def test_mazars_equivalent_strain():
    rng = np.random.default_rng(5)
    w = rng.standard_normal((3, 40)) * 1e-3
    ref = np.sqrt((np.maximum(w, 0) ** 2).sum(0))
    # rotate the diagonal tensors by random rotations
    out = np.empty((6, 40))
    for m in range(40):
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        T = Q @ np.diag(w[:, m]) @ Q.T
        out[:, m] = mandel.from_tensor(T[:, :, None])[:, 0]
    assert np.allclose(material.mazars_equivalent(out), ref, atol=1e-15)


def test_plane_strain_restriction_and_damage_scaling():
    shape = (4, 5)
    phase = np.zeros(shape, np.uint8)
    phase[0, 0] = 1
    table = [dict(model="j2_damage", E=E, nu=NU, sy=SY, H=H, dfield=0, dC=0.03, dR=0.2,
                  dmax=0.99, ell=[1.0]),
             dict(model="elastic", E=4e5, nu=0.2, sy=0, H=0, dfield=-1, dC=0, dR=1, dmax=0,
                  ell=[0.1])]
    eps = np.random.default_rng(6).standard_normal((3,) + shape) * 3e-3
    D = np.full((1,) + shape, 0.25)
    st = material.constitutive(eps, np.zeros((6,) + shape), np.zeros(shape), D, phase, table, 1)
    st0 = material.constitutive(eps, np.zeros((6,) + shape), np.zeros(shape), 0 * D, phase,
                                table, 1)
    m = phase == 0
    assert np.allclose(st["sigma"][:, m], 0.75 * st0["sigma"][:, m], rtol=1e-14)
    assert np.allclose(st["sigma"][:, ~m], st0["sigma"][:, ~m], rtol=1e-14)
    # the 3x3 in-plane tangent is the restriction of the 6x6 one
    e6 = mandel.expand_plane(eps.reshape(3, -1))
    s6, _, k6, C6 = material.j2_return_map(e6, np.zeros_like(e6), np.zeros(e6.shape[1]),
                                           E, NU, SY, H)
    idx = np.nonzero(m.reshape(-1))[0]
    C3 = st0["C"].reshape(3, 3, -1)[:, :, idx]
    assert np.allclose(C3, C6[np.ix_([0, 1, 5], [0, 1, 5])][:, :, idx], rtol=1e-14)
    assert np.allclose(st0["alpha"][0].reshape(-1)[idx], k6[idx], rtol=1e-14)
    assert np.all(st0["alpha"][0][~m] == 0)
