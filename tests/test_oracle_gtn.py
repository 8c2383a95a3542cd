"""Pins of the checker's Gurson-Tvergaard-Needleman matrix (Sec. 2.1.1, the
non-local Gurson extension, appendix A.1) against closed forms, scalar root
finds of reduced problems, invariants and central differences."""
import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.special import erf

from oracle import galerkin, gtn, staggered
from paper_2103_04770_amd import microstructure as ms

I6 = np.array([1.0, 1, 1, 0, 0, 0])


def _mat(**kw):
    return ms.matrix_gtn(ell=[2.0, 2.0], **kw)


def _q_sm(sig):
    sm = (sig[0] + sig[1] + sig[2]) / 3.0
    dev = sig - sm[None] * I6[:, None]
    return np.sqrt(1.5 * (dev * dev).sum(axis=0)), sm


def _states(rng, M, scale, frange):
    eps = rng.normal(scale=scale, size=(6, M))
    eps[:3] += rng.normal(scale=scale, size=M)
    epn = rng.normal(scale=scale / 3, size=(6, M))
    epn[:3] -= epn[:3].mean(axis=0)
    e0n = np.abs(rng.normal(scale=0.05, size=M))
    f = rng.uniform(*frange, size=M)
    return eps, epn, e0n, f


def test_aravas_flow_stress():
    m = _mat()
    K, mu = gtn.lame(m["E"], m["nu"])
    e = np.concatenate([[0.0], np.logspace(-6, 0, 40)])
    s0, h = gtn.flow_stress(e, m["sy"], mu, m["n"])
    y = s0 / m["sy"]
    # the implicit law itself holds, starting at the yield stress
    assert np.abs(y - (y + 3 * mu * e / m["sy"]) ** m["n"]).max() <= 1e-14
    assert s0[0] == pytest.approx(m["sy"], rel=1e-15)
    # initial slope from the law at e0 = 0: y' = n (y' + c) -> 3 mu n / (1 - n)
    assert h[0] == pytest.approx(3 * mu * m["n"] / (1 - m["n"]), rel=1e-13)
    d = 1e-6 * np.maximum(e, 1e-3)
    fd = (gtn.flow_stress(e + d, m["sy"], mu, m["n"])[0]
          - gtn.flow_stress(np.maximum(e - d, 0), m["sy"], mu, m["n"])[0]) / (e + d - np.maximum(e - d, 0))
    assert np.allclose(h, fd, rtol=1e-6)
    assert np.all(np.diff(s0) > 0)


def test_effective_porosity_branches():
    m = _mat()
    fV = (m["q1"] + np.sqrt(m["q1"] ** 2 - m["q3"])) / m["q3"]
    # f_V* is where the surface shrinks to the origin: phi(0) = 0
    assert gtn._yield(0.0, 0.0, 1.0, fV, m) == pytest.approx(0.0, abs=1e-15)
    assert fV == pytest.approx(2.0 / 3.0, rel=1e-15)
    f = np.array([0.0, 0.1, 0.15, 0.2, 0.25, 0.3])
    fs = gtn.fstar(f, dict(m, fu=1.0))
    assert np.allclose(fs, [0.0, 0.1, 0.15, 0.15 + (fV - 0.15) * 0.5, fV, fV], rtol=1e-15)
    assert np.allclose(gtn.fstar(f, m), np.minimum(fs, 0.6))
    # continuity at fC and fF
    eps = 1e-12
    for a in (m["fC"], m["fF"]):
        lo, hi = gtn.fstar(np.array([a - eps, a + eps]), dict(m, fu=1.0))
        assert abs(hi - lo) < 1e-10


def test_porosity_update_converges_to_exact_integrals():
    m = _mat(fN=0.04, eN=0.1, sN=0.05)
    # nucleation only: f = fN/2 [erf((e - eN)/(sqrt2 sN)) - erf(-eN/(sqrt2 sN))]
    e = np.linspace(0.0, 0.3, 30001)
    f = 0.0
    for k in range(1, e.size):
        f = gtn.porosity_update(f, e[k], e[k - 1], 0.0, 0.0, m)
    r2 = np.sqrt(2.0)
    exact = 0.5 * m["fN"] * (erf((0.3 - m["eN"]) / (r2 * m["sN"])) - erf(-m["eN"] / (r2 * m["sN"])))
    assert f == pytest.approx(exact, rel=1e-4)
    # growth only: df = (1 - f) dtr  ->  1 - f = (1 - f0) exp(-tr)
    m0 = _mat(fN=0.0)
    t = np.linspace(0.0, 0.2, 20001)
    f = 0.01
    for k in range(1, t.size):
        f = gtn.porosity_update(f, 0.0, 0.0, t[k], t[k - 1], m0)
    assert f == pytest.approx(1.0 - 0.99 * np.exp(-0.2), rel=1e-5)


def test_return_map_without_porosity_is_j2_with_aravas_hardening():
    """f = 0: the mean stress does not enter the yield function, the flow is
    deviatoric and the return is the J2 radial return with the nonlinear
    flow stress: 3 mu dq = q_tr - s0(e0_n + dq), solved here by brentq."""
    m = _mat()
    K, mu = gtn.lame(m["E"], m["nu"])
    rng = np.random.default_rng(11)
    eps, epn, e0n, _ = _states(rng, 24, 5e-3, (0, 0))
    f = np.zeros(24)
    sig, ep, e0, C, x = gtn.return_map(eps, epn, e0n, f, m)
    ee = eps - epn
    tr = ee[:3].sum(axis=0)
    s_tr = 2 * mu * (ee - tr / 3 * I6[:, None])
    q_tr = np.sqrt(1.5 * (s_tr * s_tr).sum(axis=0))
    for i in range(24):
        s0n = gtn.flow_stress(e0n[i], m["sy"], mu, m["n"])[0]
        if q_tr[i] <= s0n:
            dq = 0.0
        else:
            dq = brentq(lambda d: q_tr[i] - 3 * mu * d - gtn.flow_stress(e0n[i] + d, m["sy"], mu,
                                                                         m["n"])[0],
                        0.0, q_tr[i] / (3 * mu), xtol=1e-300, rtol=1e-15)
        Nd = 1.5 * s_tr[:, i] / q_tr[i]
        ref = s_tr[:, i] - 2 * mu * dq * Nd + K * tr[i] * I6
        assert np.abs(sig[:, i] - ref).max() <= 1e-11 * np.abs(ref).max()
        assert e0[i] == pytest.approx(e0n[i] + dq, rel=1e-11, abs=1e-15)
        assert np.abs(ep[:, i] - (epn[:, i] + dq * Nd)).max() <= 1e-11 * max(dq, 1e-12)


def test_return_map_hydrostatic_closed_form():
    """Pure dilatation (q_tr = 0) with porosity: the return goes to the apex,
    sm = 2 s0/(3 q2) arccosh((1 + q3 f*^2)/(2 q1 f*)), and the plastic work
    (1 - f) s0 de0 = sm dv fixes e0 (a scalar brentq)."""
    m = _mat()
    K, mu = gtn.lame(m["E"], m["nu"])
    for f, tr in ((0.05, 6e-3), (0.2, 3e-3), (0.02, -2e-2)):
        fs = float(gtn.fstar(np.array(f), m))
        eps = np.array([[tr / 3], [tr / 3], [tr / 3], [0.0], [0.0], [0.0]])
        sig, ep, e0, C, x = gtn.return_map(eps, np.zeros((6, 1)), np.zeros(1), np.array([f]), m)
        sm_tr = K * tr
        acs = np.arccosh((1 + m["q3"] * fs * fs) / (2 * m["q1"] * fs))

        def apex(w):
            return np.sign(sm_tr) * 2 * gtn.flow_stress(w, m["sy"], mu, m["n"])[0] / (3 * m["q2"]) * acs

        def work(w):
            s0 = gtn.flow_stress(w, m["sy"], mu, m["n"])[0]
            sm = apex(w)
            return (1 - f) * s0 * w - sm * (sm_tr - sm) / K

        w = brentq(work, 0.0, 1.0, xtol=1e-300, rtol=1e-15)
        assert sig[0, 0] == pytest.approx(apex(w), rel=1e-12)
        assert np.abs(sig[3:, 0]).max() == 0.0
        assert e0[0] == pytest.approx(w, rel=1e-11)
        assert ep[:3, 0].sum() == pytest.approx((sm_tr - apex(w)) / K, rel=1e-11)


@pytest.mark.parametrize("scale,frange", [(2e-3, (0.0, 0.05)), (1e-2, (0.0, 0.5)),
                                          (3e-2, (0.2, 0.3))])
def test_return_map_invariants(scale, frange):
    """Consistency phi = 0, normality of d eps_p to the yield surface (the
    gradient of phi by central differences in the stress), the plastic-work
    identity and the elastic law, on random states that reach the
    coalescence branch and the cap of f*."""
    m = _mat()
    K, mu = gtn.lame(m["E"], m["nu"])
    rng = np.random.default_rng(int(scale * 1e4))
    M = 200
    eps, epn, e0n, f = _states(rng, M, scale, frange)
    sig, ep, e0, C, x = gtn.return_map(eps, epn, e0n, f, m)
    fs = gtn.fstar(f, m)
    q, sm = _q_sm(sig)
    s0 = gtn.flow_stress(e0, m["sy"], mu, m["n"])[0]
    phi = gtn._yield(q, sm, s0, fs, m)
    pl = x[0] + np.abs(x[1]) > 0
    assert pl.sum() > M // 2
    assert np.abs(phi[pl]).max() <= 1e-12
    assert np.all(phi[~pl] <= 0)
    # elastic law
    ee = eps - ep
    tr = ee[:3].sum(axis=0)
    ref = K * tr[None] * I6[:, None] + 2 * mu * (ee - tr / 3 * I6[:, None])
    assert np.abs(sig - ref).max() <= 1e-10 * np.abs(sig).max()
    # plastic work
    dep = ep - epn
    wk = (sig * dep).sum(axis=0)
    assert np.abs(wk - (1 - f) * s0 * (e0 - e0n)).max() <= 1e-12 * np.abs(wk).max()
    # normality: d eps_p parallel to dphi/dsigma
    hs = 1e-6 * np.abs(sig).max(axis=0)
    grad = np.zeros((6, M))
    for k in range(6):
        sp, sn = sig.copy(), sig.copy()
        sp[k] += hs
        sn[k] -= hs
        grad[k] = (gtn._yield(*_q_sm(sp), s0, fs, m) - gtn._yield(*_q_sm(sn), s0, fs, m)) / (2 * hs)
    g, d = grad[:, pl], dep[:, pl]
    lam = (g * d).sum(axis=0) / (g * g).sum(axis=0)
    assert np.all(lam > 0)
    resid = np.abs(d - lam[None] * g).max(axis=0) / np.abs(d).max(axis=0)
    assert resid.max() <= 1e-6


def test_tangent_is_the_derivative_and_symmetric():
    m = _mat()
    rng = np.random.default_rng(21)
    for scale, fr in ((2e-3, (0.0, 0.05)), (1e-2, (0.0, 0.5))):
        M = 30
        eps, epn, e0n, f = _states(rng, M, scale, fr)
        sig, ep, e0, C, x = gtn.return_map(eps, epn, e0n, f, m)
        h = 1e-7 * scale
        Cfd = np.zeros((6, 6, M))
        for k in range(6):
            a, b = eps.copy(), eps.copy()
            a[k] += h
            b[k] -= h
            Cfd[:, k] = (gtn.return_map(a, epn, e0n, f, m)[0] - gtn.return_map(b, epn, e0n, f, m)[0]) / (2 * h)
        nrm = np.abs(C).max(axis=(0, 1))
        assert (np.abs(Cfd - C).max(axis=(0, 1)) / nrm).max() <= 1e-5
        assert (np.abs(C - np.swapaxes(C, 0, 1)).max(axis=(0, 1)) / nrm).max() <= 1e-11


def _one_point_uniaxial(m, e11, epn, e0n, f):
    """Homogeneous uniaxial stress at frozen porosity: the lateral strains
    e22 = e33 make sigma22 = sigma33 = 0 (brentq on the return map)."""
    def s22(el):
        e = np.array([[e11], [el], [el], [0.0], [0.0], [0.0]])
        return gtn.return_map(e, epn, np.array([e0n]), np.array([f]), m)[0][1, 0]

    el = brentq(s22, -1.5 * e11, 0.5 * e11, xtol=1e-300, rtol=1e-15)
    e = np.array([[e11], [el], [el], [0.0], [0.0], [0.0]])
    sig, ep, e0, _, _ = gtn.return_map(e, epn, np.array([e0n]), np.array([f]), m)
    return sig[:, 0], el, ep, float(e0[0])


def test_homogeneous_mechanics_equals_one_point_driver():
    """Homogeneous Gurson RVE under uniaxial mixed control at frozen porosity
    (f = 0 and f = 0.1) equals the one-point uniaxial-stress driver."""
    m = _mat()
    S = (4, 4, 4)
    phase = np.zeros(S, np.uint8)
    for f in (0.0, 0.1):
        for e11 in (2e-3, 6e-3):
            D = np.zeros((2,) + S)
            D[0] = f
            out = galerkin.fftg_solve(phase, [m], D, np.zeros((6,) + S), np.zeros(S),
                                      ms.uniaxial_mixed(3, e11), np.zeros((6,) + S),
                                      cg_tol=1e-13, newton_tol=1e-12, newton_maxit=60, nfields=2)
            assert out["converged"]
            sig, el, _, e0 = _one_point_uniaxial(m, e11, np.zeros((6, 1)), 0.0, f)
            assert out["sigma"][0].mean() == pytest.approx(sig[0], rel=1e-10)
            assert out["eps"][1].mean() == pytest.approx(el, rel=1e-9)
            assert out["kappa"].mean() == pytest.approx(e0, rel=1e-9, abs=1e-14)


def test_staggered_homogeneous_equals_local_porosity_driver():
    """Homogeneous sources make the non-local fields equal the local ones
    (the Helmholtz operator maps constants to themselves), so the converged
    staggered increments of a homogeneous Gurson RVE follow the local model:
    per increment, f_{n+1} is the fixed point of the porosity update with e0
    and tr(eps_p) from the one-point driver at frozen f_{n+1} (brentq in f)."""
    m = _mat(fN=0.2, eN=0.004, sN=0.002)
    S = (4, 4, 4)
    phase = np.zeros(S, np.uint8)
    st = staggered.initial_state(S, 3, 2)
    epn, e0n, trn, fn = np.zeros((6, 1)), 0.0, 0.0, 0.0
    for e11 in (3e-3, 6e-3, 9e-3):
        st, sig, homog, stats = staggered.staggered_step(
            phase, [m], 2, st, ms.uniaxial_mixed(3, e11), cg_tol=1e-13, pcg_tol=1e-13,
            newton_tol=1e-12, newton_maxit=60, stagger_tol=1e-12, max_stagger=60)
        assert stats["converged"]

        def resid(f):
            _, _, ep, e0 = _one_point_uniaxial(m, e11, epn, e0n, f)
            return f - gtn.porosity_update(fn, e0, e0n, ep[:3].sum(), trn, m)

        f = brentq(resid, 0.0, 0.5, xtol=1e-300, rtol=1e-15)
        s, _, ep, e0 = _one_point_uniaxial(m, e11, epn, e0n, f)
        assert homog["sigma"][0] == pytest.approx(s[0], rel=1e-9)
        assert st["hist"][0].mean() == pytest.approx(f, rel=1e-8)
        assert st["kappa"].mean() == pytest.approx(e0, rel=1e-9)
        assert st["abar"][1].mean() == pytest.approx(ep[:3].sum(), rel=1e-8)
        epn, e0n, trn, fn = ep, e0, float(ep[:3].sum()), f
    assert fn > 0.01          # porosity did grow over the path


def test_homogeneous_plane_strain_equals_one_point_driver():
    """2D plane strain (eps33 = eps13 = eps23 = 0) with a frozen porosity:
    the homogeneous Gurson RVE under E11 with sigma22 = sigma12 = 0 equals a
    one-point driver solving sigma22(e22) = 0 on the 3D return map."""
    m = _mat()
    S = (4, 6)
    phase = np.zeros(S, np.uint8)
    for f, e11 in ((0.0, 4e-3), (0.12, 6e-3)):
        D = np.zeros((2,) + S)
        D[0] = f
        out = galerkin.fftg_solve(phase, [m], D, np.zeros((6,) + S), np.zeros(S),
                                  ms.uniaxial_mixed(2, e11), np.zeros((3,) + S),
                                  cg_tol=1e-13, newton_tol=1e-12, newton_maxit=60, nfields=2)
        assert out["converged"]

        def ret(e22):
            e = np.array([[e11], [e22], [0.0], [0.0], [0.0], [0.0]])
            return gtn.return_map(e, np.zeros((6, 1)), np.zeros(1), np.array([f]), m)

        e22 = brentq(lambda x: ret(x)[0][1, 0], -1.5 * e11, 0.5 * e11, xtol=1e-300, rtol=1e-15)
        sig, ep, e0, _, _ = ret(e22)
        assert out["sigma"][0].mean() == pytest.approx(sig[0, 0], rel=1e-10)
        assert out["eps"][1].mean() == pytest.approx(e22, rel=1e-9)
        assert out["kappa"].mean() == pytest.approx(e0[0], rel=1e-9, abs=1e-14)
        # the out-of-plane stress the plane-strain constraint carries
        assert sig[2, 0] != 0.0
