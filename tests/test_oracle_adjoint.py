"""Pins of the checker's adjoint gradients: the Helmholtz solve against a
dense real-space construction (no FFT), the mechanics solve against central
finite differences of the forward solve."""
import numpy as np
import pytest

from oracle import adjoint, galerkin, helmholtz
from paper_2103_04770_amd import microstructure as ms
from tests._pins import dense_gradients, dense_helmholtz


@pytest.mark.parametrize("shape", [(4, 4, 6), (6, 8)])
def test_helmholtz_adjoint_equals_dense_gradient(shape):
    rng = np.random.default_rng(0)
    alpha = rng.standard_normal(shape)
    ell2 = rng.uniform(0.0, 3.0, size=shape)
    w = rng.standard_normal(shape)                  # J = w . abar
    L = dense_helmholtz(shape, ell2, 1.0)
    abar = np.linalg.solve(L, alpha.reshape(-1))
    lam = np.linalg.solve(L, w.reshape(-1))        # L is symmetric
    Qs = dense_gradients(shape, 1.0)
    dell2 = -sum((Q @ lam) * (Q @ abar) for Q in Qs)
    fwd = helmholtz.helmholtz_solve(alpha, ell2, tol=1e-14, maxit=500)
    r = adjoint.helmholtz_adjoint(fwd["abar"], w, ell2, tol=1e-14, maxit=500)
    assert np.abs(r["dalpha"].reshape(-1) - lam).max() <= 1e-11 * np.abs(lam).max()
    assert np.abs(r["dell2"].reshape(-1) - dell2).max() <= 1e-10 * np.abs(dell2).max()


def test_helmholtz_phase_length_gradient_by_finite_differences():
    shape = (6, 6, 6)
    rng = np.random.default_rng(1)
    phase = (rng.uniform(size=shape) < 0.3).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[0.7])]
    alpha = np.abs(rng.standard_normal(shape))
    w = rng.standard_normal(shape)

    def J(ells):
        ell2 = np.array([e * e for e in ells])[phase]
        return float((w * helmholtz.helmholtz_solve(alpha, ell2, tol=1e-14,
                                                    maxit=500)["abar"]).sum())
    ell2 = np.array([4.0, 0.49])[phase]
    fwd = helmholtz.helmholtz_solve(alpha, ell2, tol=1e-14, maxit=500)
    r = adjoint.helmholtz_adjoint(fwd["abar"], w, ell2, tol=1e-14, maxit=500)
    g = adjoint.phase_length_gradient(r["dell2"], phase, table, 0)
    hh = 1e-5
    for q, base in enumerate([2.0, 0.7]):
        ep, em = [2.0, 0.7], [2.0, 0.7]
        ep[q] += hh
        em[q] -= hh
        fd = (J(ep) - J(em)) / (2 * hh)
        assert g[q] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_mechanics_adjoint_by_finite_differences():
    """J = w . eps at the converged strain, D perturbed along a random
    direction on the damaging voxels (central differences, h = 1e-6)."""
    S = (6, 6, 6)
    rng = np.random.default_rng(3)
    phase = (rng.uniform(size=S) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
    D0 = np.where(phase == 0, rng.uniform(0.1, 0.5, size=S), 0.0)[None]
    z6, z = np.zeros((6,) + S), np.zeros(S)
    tgt = ms.uniaxial_mixed(3, 6e-3)
    w = rng.standard_normal((6,) + S)
    kw = dict(cg_tol=1e-13, newton_tol=1e-13, newton_maxit=60)

    def solve(D):
        return galerkin.fftg_solve(phase, table, D, z6, z, tgt, z6.copy(), **kw)

    base = solve(D0)
    assert base["converged"]
    r = adjoint.mechanics_adjoint(phase, table, D0, z6, z, tgt, base["eps"], w, 1,
                                  cg_tol=1e-13)
    dirn = np.where(phase == 0, rng.standard_normal(S), 0.0)[None]
    hh = 1e-6
    jp = float((w * solve(D0 + hh * dirn)["eps"]).sum())
    jm = float((w * solve(D0 - hh * dirn)["eps"]).sum())
    fd = (jp - jm) / (2 * hh)
    ad = float((r["dD"] * dirn).sum())
    assert ad == pytest.approx(fd, rel=1e-5)
    # no sensitivity where no damage law acts
    assert np.all(r["dD"][0][phase == 1] == 0)


def test_mechanics_adjoint_mixed_control_by_finite_differences():
    """Same check in 2D plane strain under pure stress control of the shear."""
    S = (8, 12)
    rng = np.random.default_rng(4)
    phase = (rng.uniform(size=S) < 0.3).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_cracking(ell=[1.0], dfield=0)]
    D0 = rng.uniform(0.05, 0.4, size=S)[None]
    z6, z = np.zeros((6,) + S), np.zeros(S)
    tgt = (np.array([0, 1, 1], np.uint8), np.array([4e-3, 0.0, 0.0]), np.array([0.0, 0.0, 30.0]))
    w = rng.standard_normal((3,) + S)
    kw = dict(cg_tol=1e-13, newton_tol=1e-13, newton_maxit=60)

    def solve(D):
        return galerkin.fftg_solve(phase, table, D, z6, z, tgt, np.zeros((3,) + S), **kw)

    base = solve(D0)
    r = adjoint.mechanics_adjoint(phase, table, D0, z6, z, tgt, base["eps"], w, 1,
                                  cg_tol=1e-13)
    dirn = rng.standard_normal((1,) + S)
    hh = 1e-6
    fd = (float((w * solve(D0 + hh * dirn)["eps"]).sum()) -
          float((w * solve(D0 - hh * dirn)["eps"]).sum())) / (2 * hh)
    assert float((r["dD"] * dirn).sum()) == pytest.approx(fd, rel=1e-5)


def test_homogenised_stress_gradient_by_finite_differences():
    """J = <sigma_11> (a function of eps and D through the stress) under
    uniaxial mixed control: dJ/dD from the adjoint with the stress cotangent
    against central differences."""
    S = (6, 6, 8)
    rng = np.random.default_rng(9)
    phase = (rng.uniform(size=S) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
    D0 = np.where(phase == 0, rng.uniform(0.1, 0.5, size=S), 0.0)[None]
    z6, z = np.zeros((6,) + S), np.zeros(S)
    tgt = ms.uniaxial_mixed(3, 6e-3)
    N = phase.size
    kw = dict(cg_tol=1e-13, newton_tol=1e-13, newton_maxit=60)

    def J(D):
        r = galerkin.fftg_solve(phase, table, D, z6, z, tgt, z6.copy(), **kw)
        return float(r["sigma"][0].mean()), r

    j0, base = J(D0)
    gsig = np.zeros((6,) + S)
    gsig[0] = 1.0 / N
    r = adjoint.mechanics_adjoint(phase, table, D0, z6, z, tgt, base["eps"], np.zeros((6,) + S),
                                  1, cg_tol=1e-13, gsig=gsig)
    dirn = np.where(phase == 0, rng.standard_normal(S), 0.0)[None]
    hh = 1e-6
    fd = (J(D0 + hh * dirn)[0] - J(D0 - hh * dirn)[0]) / (2 * hh)
    assert float((r["dD"] * dirn).sum()) == pytest.approx(fd, rel=1e-5)


def _chain_case():
    S = (6, 8, 8)
    rng = np.random.default_rng(12)
    phase = (rng.uniform(size=S) < 0.3).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0], dC=0.001, dR=0.02), ms.particle_elastic(ell=[0.5])]
    # per-voxel local source: an equivalent plastic strain field concentrated
    # in the matrix, so that the non-local field crosses the damage onset
    alpha = np.where(phase == 0, rng.uniform(0.0, 0.02, size=S), 0.0)
    return S, phase, table, alpha


def _chain_forward(S, phase, table, alpha, ells):
    from oracle import material
    ell2 = np.array([e * e for e in ells])[phase]
    abar = helmholtz.helmholtz_solve(alpha, ell2, tol=1e-14, maxit=500)["abar"]
    hist = np.zeros((1,) + S)
    D = material.damage_from_nonlocal(phase, table, abar[None], hist)
    z6, z = np.zeros((6,) + S), np.zeros(S)
    tgt = ms.uniaxial_mixed(3, 4e-3)
    m = galerkin.fftg_solve(phase, table, D, z6, z, tgt, z6.copy(), cg_tol=1e-13,
                            newton_tol=1e-13, newton_maxit=60)
    return dict(ell2=ell2, abar=abar, D=D, hist=hist, eps=m["eps"], sigma=m["sigma"], tgt=tgt)


def test_one_pass_chain_gradients_by_finite_differences():
    """J1 = <sigma_11>, J2 = <D> through alpha -> abar -> D -> (eps, sigma):
    the adjoint chain's dJ/d ell_matrix and its derivative along a random
    source direction against central differences."""
    S, phase, table, alpha = _chain_case()
    ells = [2.0, 0.5]
    f = _chain_forward(S, phase, table, alpha, ells)
    N = phase.size
    z6, z = np.zeros((6,) + S), np.zeros(S)
    assert 0.05 < (f["D"] > 0).mean() < 0.95

    def grads(which):
        if which == "stress":
            gsig = np.zeros((6,) + S)
            gsig[0] = 1.0 / N
            mech = adjoint.mechanics_adjoint(phase, table, f["D"], z6, z, f["tgt"], f["eps"],
                                             np.zeros((6,) + S), 1, cg_tol=1e-13, gsig=gsig)
            gD = mech["dD"]
        else:
            gD = np.full((1,) + S, 1.0 / N)
        ga = adjoint.damage_adjoint(phase, table, f["abar"][None], f["hist"], gD)[0]
        h = adjoint.helmholtz_adjoint(f["abar"], ga, f["ell2"], tol=1e-14, maxit=500)
        return h["dalpha"], adjoint.phase_length_gradient(h["dell2"], phase,
                                                         [dict(t, ell=[e]) for t, e in
                                                          zip(table, ells)], 0)

    def J(which, a, e):
        g = _chain_forward(S, phase, table, a, e)
        return float(g["sigma"][0].mean()) if which == "stress" else float(g["D"].mean())

    rng = np.random.default_rng(13)
    dirn = np.where(phase == 0, rng.standard_normal(S), 0.0) * 1e-3
    for which in ("stress", "damage"):
        dal, dell = grads(which)
        hh = 1e-4
        fd_l = (J(which, alpha, [2.0 + hh, 0.5]) - J(which, alpha, [2.0 - hh, 0.5])) / (2 * hh)
        assert dell[0] == pytest.approx(fd_l, rel=1e-4)
        ha = 1e-3
        fd_a = (J(which, alpha + ha * dirn, ells) - J(which, alpha - ha * dirn, ells)) / (2 * ha)
        assert float((dal * dirn).sum()) == pytest.approx(fd_a, rel=1e-4)


def _stag_case():
    S = (12, 16)
    rng = np.random.default_rng(21)
    phase = (rng.uniform(size=S) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0], dC=0.0005, dR=0.02), ms.particle_elastic(ell=[0.5])]
    return S, phase, table


STAG_TOLS = dict(cg_tol=1e-13, pcg_tol=1e-13, newton_tol=1e-12, newton_maxit=60,
                 stagger_tol=1e-13, max_stagger=300)


def _stag_increment(phase, table, st_n, e11):
    from oracle import staggered
    st, sig, hom, stats = staggered.staggered_step(phase, table, 1, st_n,
                                                   ms.uniaxial_mixed(phase.ndim, e11), **STAG_TOLS)
    assert stats["converged"]
    return st, sig, hom, stats


def test_source_derivative_by_finite_differences():
    """d kappa / d eps of the J2 return (the local source of the matrix field)
    against central differences of the constitutive update."""
    from oracle import material
    S = (4, 6)
    rng = np.random.default_rng(3)
    phase = (rng.uniform(size=S) < 0.3).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[0.5])]
    eps = rng.normal(scale=4e-3, size=(3,) + S)
    epsp = rng.normal(scale=1e-3, size=(6,) + S)
    epsp[:3] -= epsp[:3].mean(axis=0)
    kap = np.abs(rng.normal(scale=2e-3, size=S))
    D = np.zeros((1,) + S)
    d = adjoint.source_derivative(eps, epsp, kap, phase, table, 1)
    h = 1e-8
    for k in range(3):
        ep, em = eps.copy(), eps.copy()
        ep[k] += h
        em[k] -= h
        fd = (material.constitutive(ep, epsp, kap, D, phase, table, 1)["alpha"]
              - material.constitutive(em, epsp, kap, D, phase, table, 1)["alpha"]) / (2 * h)
        assert np.abs(fd[0] - d[0, k]).max() <= 1e-6 * np.abs(d[0]).max()
    assert np.abs(d[0]).max() > 0


@pytest.mark.parametrize("which", ["sigma11", "mean_damage", "mean_abar"])
def test_staggered_adjoint_by_finite_differences(which):
    """Gradient of J after a converged staggered increment (damage active,
    damage feeding back into the local source through the mechanics) with
    respect to the per-phase lengths, against central differences of the
    converged increment."""
    from oracle import staggered
    S, phase, table = _stag_case()
    st0 = staggered.initial_state(S, 2, 1)
    st_n, _, _, _ = _stag_increment(phase, table, st0, 3e-3)
    e11 = 5e-3
    st, sig, hom, stats = _stag_increment(phase, table, st_n, e11)
    assert stats["stagger_iters"] > 2        # a real fixed point, not one pass
    N = phase.size
    kw = {}
    if which == "sigma11":
        g = np.zeros((3,) + S)
        g[0] = 1.0 / N
        kw["g_sig"] = g
    elif which == "mean_damage":
        kw["g_D"] = np.full((1,) + S, 1.0 / N)
    else:
        kw["g_abar"] = np.full((1,) + S, 1.0 / N)
    r = adjoint.staggered_adjoint(phase, table, 1, st_n, st["eps"], st["abar"],
                                  ms.uniaxial_mixed(2, e11), **kw)
    grad = adjoint.phase_length_gradient(r["dell2"][0], phase, table, 0)

    def J(tab):
        from oracle import material
        s2, sg, hm, _ = _stag_increment(phase, tab, st_n, e11)
        if which == "sigma11":
            return hm["sigma"][0]
        if which == "mean_damage":
            return material.damage_from_nonlocal(phase, tab, s2["abar"], st_n["hist"]).mean()
        return s2["abar"].mean()

    for q in range(2):
        hq = 1e-4 * table[q]["ell"][0]
        tp = [dict(t) for t in table]
        tm = [dict(t) for t in table]
        tp[q]["ell"] = [table[q]["ell"][0] + hq]
        tm[q]["ell"] = [table[q]["ell"][0] - hq]
        fd = (J(tp) - J(tm)) / (2 * hq)
        assert grad[q] == pytest.approx(fd, rel=2e-4, abs=1e-6 * abs(grad).max())
    assert r["iters"] > 2


def test_staggered_adjoint_3d_by_finite_differences():
    """The converged-increment adjoint in 3D (J = <sigma_11>) against central
    differences of converged increments."""
    from oracle import staggered
    S = (6, 8, 8)
    rng = np.random.default_rng(21)
    phase = (rng.uniform(size=S) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0], dC=0.0005, dR=0.02), ms.particle_elastic(ell=[0.5])]
    st_n, _, _, _ = _stag_increment(phase, table, staggered.initial_state(S, 3, 1), 3e-3)
    st, _, _, stats = _stag_increment(phase, table, st_n, 5e-3)
    assert stats["stagger_iters"] > 2
    g = np.zeros((6,) + S)
    g[0] = 1.0 / phase.size
    r = adjoint.staggered_adjoint(phase, table, 1, st_n, st["eps"], st["abar"],
                                  ms.uniaxial_mixed(3, 5e-3), g_sig=g)
    grad = adjoint.phase_length_gradient(r["dell2"][0], phase, table, 0)
    for q in range(2):
        hq = 1e-4 * table[q]["ell"][0]
        vals = []
        for sgn in (1, -1):
            tb = [dict(t) for t in table]
            tb[q]["ell"] = [table[q]["ell"][0] + sgn * hq]
            vals.append(_stag_increment(phase, tb, st_n, 5e-3)[2]["sigma"][0])
        fd = (vals[0] - vals[1]) / (2 * hq)
        assert grad[q] == pytest.approx(fd, rel=2e-4, abs=1e-6 * abs(grad).max())


def test_cracking_source_derivative_by_finite_differences():
    """d alpha / d eps of the Mazars equivalent strain (cracking phase)
    against central differences of the constitutive sources, 3D and 2D."""
    from oracle import material
    rng = np.random.default_rng(4)
    table = [ms.elastic_phase(70000.0, 0.3, ell=(1.0, 1.0)),
             ms.particle_cracking(ell=[1.0, 1.0], dfield=1)]
    for S, c in (((4, 5, 3), 6), ((5, 6), 3)):
        phase = (rng.uniform(size=S) < 0.6).astype(np.uint8)
        eps = rng.normal(scale=3e-3, size=(c,) + S)
        z6, z = np.zeros((6,) + S), np.zeros(S)
        D = np.zeros((2,) + S)
        d = adjoint.source_derivative(eps, z6, z, phase, table, 2)
        h = 1e-9
        for k in range(c):
            ep, em = eps.copy(), eps.copy()
            ep[k] += h
            em[k] -= h
            fd = (material.constitutive(ep, z6, z, D, phase, table, 2)["alpha"]
                  - material.constitutive(em, z6, z, D, phase, table, 2)["alpha"]) / (2 * h)
            assert np.abs(fd[1] - d[1, k]).max() <= 1e-5 * np.abs(d[1]).max()
        assert np.abs(d[1]).max() > 0 and np.abs(d[0]).max() == 0


def test_staggered_adjoint_two_fields_by_finite_differences():
    """The converged-increment adjoint with both sources of the benchmark
    table (J2 damage matrix on field 0, particle cracking on field 1):
    d<sigma_11>/d ell for every phase and field against central differences."""
    from oracle import staggered
    S = (10, 12)
    rng = np.random.default_rng(23)
    phase = (rng.uniform(size=S) < 0.3).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0, 0.04], dfield=0, dC=0.0005, dR=0.02),
             ms.particle_cracking(ell=[0.04, 1.0], dfield=1, k0=5e-4, kf=5e-3)]

    def inc(tab, st_n, e11):
        st, sig, hom, stats = staggered.staggered_step(phase, tab, 2, st_n,
                                                       ms.uniaxial_mixed(2, e11), **STAG_TOLS)
        assert stats["converged"]
        return st, hom

    st_n, _ = inc(table, staggered.initial_state(S, 2, 2), 2e-3)
    st, hom = inc(table, st_n, 3e-3)
    assert st["abar"][1].max() > 5e-4        # cracking field past its threshold
    g = np.zeros((3,) + S)
    g[0] = 1.0 / phase.size
    r = adjoint.staggered_adjoint(phase, table, 2, st_n, st["eps"], st["abar"],
                                  ms.uniaxial_mixed(2, 3e-3), g_sig=g)
    for j in range(2):
        grad = adjoint.phase_length_gradient(r["dell2"][j], phase, table, j)
        for q in range(2):
            e0 = table[q]["ell"][j]
            hq = 1e-4 * e0
            vals = []
            for sgn in (1, -1):
                tb = [dict(t, ell=list(t["ell"])) for t in table]
                tb[q]["ell"][j] = e0 + sgn * hq
                vals.append(inc(tb, st_n, 3e-3)[1]["sigma"][0])
            fd = (vals[0] - vals[1]) / (2 * hq)
            assert grad[q] == pytest.approx(fd, rel=5e-4, abs=1e-5 * max(abs(grad).max(), 1e-9))



def test_history_partials_by_finite_differences():
    """Derivatives of the J2 return in the strain and in the plastic history
    against central differences of the return map."""
    from oracle import material
    rng = np.random.default_rng(9)
    M = 40
    ph = ms.matrix_j2_damage(ell=[1.0])
    eps = rng.normal(scale=4e-3, size=(6, M))
    epn = rng.normal(scale=1e-3, size=(6, M))
    epn[:3] -= epn[:3].mean(axis=0)
    kn = np.abs(rng.normal(scale=2e-3, size=M))
    phase = np.zeros(M, np.uint8)
    hp = adjoint.history_partials(eps, epn, kn, phase, [ph])

    def rm(e, p, k):
        s, ep, kap, C = material.j2_return_map(e, p, k, ph["E"], ph["nu"], ph["sy"], ph["H"])
        return s, ep, kap

    h = 1e-8
    for i in range(6):
        d = np.zeros((6, 1))
        d[i] = h
        sp, epp, kp = rm(eps + d, epn, kn)
        sm, epm, km = rm(eps - d, epn, kn)
        assert np.allclose((kp - km) / (2 * h), hp["dk_de"][i], rtol=1e-5, atol=1e-6)
        assert np.allclose((epp - epm) / (2 * h), hp["dep_de"][:, i], rtol=1e-5, atol=1e-6)
        # eps_p,n enters through eps - eps_p,n only
        sp, epp, kp = rm(eps, epn + d, kn)
        sm, epm, km = rm(eps, epn - d, kn)
        assert np.allclose((kp - km) / (2 * h), -hp["dk_de"][i], rtol=1e-5, atol=1e-6)
    hk = 1e-9
    sp, epp, kp = rm(eps, epn, kn + hk)
    sm, epm, km = rm(eps, epn, kn - hk)
    assert np.allclose((kp - km) / (2 * hk), hp["dk_dkn"], rtol=1e-6)
    assert np.allclose((epp - epm) / (2 * hk), hp["dep_dkn"], rtol=1e-5, atol=1e-6)
    assert np.allclose((sp - sm) / (2 * hk), hp["ds_dkn"], rtol=1e-5, atol=1e-3)
    assert (hp["dk_dkn"] < 1).sum() > M // 4          # plastic voxels present


def _path(phase, table, e11s, ells=None):
    from oracle import staggered
    tab = [dict(t) for t in table]
    if ells is not None:
        for t, e in zip(tab, ells):
            t["ell"] = [e]
    st = staggered.initial_state(phase.shape, phase.ndim, 1)
    states, targets = [st], []
    hom = None
    for e in e11s:
        tgt = ms.uniaxial_mixed(phase.ndim, e)
        st, sig, hom, stats = staggered.staggered_step(phase, tab, 1, st, tgt, **STAG_TOLS)
        assert stats["converged"]
        states.append(st)
        targets.append(tgt)
    return states, targets, hom


def test_increment_adjoint_history_by_finite_differences():
    """Cotangents of the plastic history (eps_p,n and kappa_n) of one
    converged increment, J = <sigma_11>, against directional central
    differences of the increment."""
    from oracle import staggered
    S, phase, table = _stag_case()
    states, targets, _ = _path(phase, table, [3e-3, 5e-3])
    st_n, st = states[1], states[2]
    c = 3
    g = np.zeros((c,) + S)
    g[0] = 1.0 / phase.size
    r = adjoint.increment_adjoint(phase, table, 1, st_n, st, targets[1], g_sig=g)
    rng = np.random.default_rng(2)
    de = rng.standard_normal((6,) + S)           # every voxel, particles included
    dk = np.abs(rng.standard_normal(S))

    def J(stn):
        return staggered.staggered_step(phase, table, 1, stn, targets[1],
                                        **STAG_TOLS)[2]["sigma"][0]

    for name, pert, grad in (("epsp", de, r["g_epsp_n"]), ("kappa", dk, r["g_kappa_n"])):
        h = 1e-7
        sp = dict(st_n, **{name: st_n[name] + h * pert})
        sm = dict(st_n, **{name: st_n[name] - h * pert})
        fd = (J(sp) - J(sm)) / (2 * h)
        assert float((grad * pert).sum()) == pytest.approx(fd, rel=2e-4), name


def test_path_gradient_by_finite_differences():
    """d<sigma_11>/d ell after a three-increment path, through the history of
    every increment, against central differences of the whole path; it
    differs from the last increment's own total derivative."""
    S, phase, table = _stag_case()
    e11s = [2e-3, 4e-3, 6e-3]
    states, targets, hom = _path(phase, table, e11s)
    g = np.zeros((3,) + S)
    g[0] = 1.0 / phase.size
    dl = adjoint.path_gradient(phase, table, 1, states, targets, g)
    grad = adjoint.phase_length_gradient(dl[0], phase, table, 0)
    last = adjoint.staggered_adjoint(phase, table, 1, states[-2], states[-1]["eps"],
                                     states[-1]["abar"], targets[-1], g_sig=g)
    one = adjoint.phase_length_gradient(last["dell2"][0], phase, table, 0)
    ells = [t["ell"][0] for t in table]
    for q in range(2):
        hq = 1e-4 * ells[q]
        vals = []
        for sgn in (1, -1):
            e = list(ells)
            e[q] += sgn * hq
            vals.append(_path(phase, table, e11s, e)[2]["sigma"][0])
        fd = (vals[0] - vals[1]) / (2 * hq)
        assert grad[q] == pytest.approx(fd, rel=5e-4, abs=1e-6 * abs(grad).max())
    assert np.abs(grad - one).max() > 1e-3 * np.abs(grad).max()


def _two_field_case():
    S = (10, 12)
    rng = np.random.default_rng(23)
    phase = (rng.uniform(size=S) < 0.3).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0, 0.04], dfield=0, dC=0.0005, dR=0.02),
             ms.particle_cracking(ell=[0.04, 1.0], dfield=1, k0=5e-4, kf=5e-3)]
    return S, phase, table


def test_increment_adjoint_damage_history_by_finite_differences():
    """Cotangent of the damage history hist_n (read back by the cracking law
    through max(hist_n, abar)) of one converged two-field increment, with
    J = <sigma_11> + sum c . hist_{n+1} (so that an incoming history cotangent
    is exercised too), against directional central differences in hist_n.
    The history is raised above abar on some cracking voxels, as after an
    earlier, larger load, so that it drives their damage."""
    from oracle import staggered
    S, phase, table = _two_field_case()
    st0 = staggered.initial_state(S, 2, 2)
    st_n = staggered.staggered_step(phase, table, 2, st0, ms.uniaxial_mixed(2, 2e-3),
                                    **STAG_TOLS)[0]
    rng = np.random.default_rng(5)
    crack = phase == 1
    raise_ = crack & (rng.uniform(size=S) < 0.5)
    st_n = dict(st_n, hist=st_n["hist"].copy())
    st_n["hist"][1][raise_] = np.maximum(st_n["hist"][1][raise_], st_n["abar"][1][raise_]) + \
        rng.uniform(1e-3, 2e-3, size=int(raise_.sum()))
    tgt = ms.uniaxial_mixed(2, 3e-3)
    st = staggered.staggered_step(phase, table, 2, st_n, tgt, **STAG_TOLS)[0]
    by_hist = st_n["hist"][1] > st["abar"][1] + 1e-5
    assert (by_hist & crack).sum() >= 5 and (~by_hist & crack & (st["abar"][1] > 5e-4)).sum() >= 5
    g = np.zeros((3,) + S)
    g[0] = 1.0 / phase.size
    cw = np.zeros((2,) + S)
    cw[1] = rng.standard_normal(S) / phase.size
    r = adjoint.increment_adjoint(phase, table, 2, st_n, st, tgt, g_sig=g, g_hist=cw)
    dh = np.zeros((2,) + S)
    dh[1] = np.where(by_hist, rng.uniform(0.5, 1.0, size=S), 0.0)   # stays on its side of the max
    dh[1] += np.where(~by_hist & ~crack, rng.uniform(0.0, 1.0, size=S), 0.0)

    def J(hist):
        s2, _, hom, stats = staggered.staggered_step(phase, table, 2, dict(st_n, hist=hist), tgt,
                                                     **STAG_TOLS)
        assert stats["converged"]
        return hom["sigma"][0] + float((cw * s2["hist"]).sum())

    h = 1e-7
    fd = (J(st_n["hist"] + h * dh) - J(st_n["hist"] - h * dh)) / (2 * h)
    got = float((r["g_hist_n"] * dh).sum())
    assert got == pytest.approx(fd, rel=2e-4)
    assert abs(got) > 1e-3 * abs(float((cw * dh).sum())) + 1e-12


def test_path_gradient_with_cracking_and_unloading_by_finite_differences():
    """d<sigma_11>/d ell of both fields and both phases after a two-field
    path that loads and partly unloads (E11 2e-3, 3e-3, 2.5e-3): on unloading
    the cracking voxels' damage stays at its history, so the gradient runs
    through the damage-history cotangents too.  Against central differences of
    the whole path."""
    from oracle import staggered
    S, phase, table = _two_field_case()
    e11s = [2e-3, 3e-3, 2.5e-3]

    def path(tab):
        st = staggered.initial_state(S, 2, 2)
        states, targets = [st], []
        hom = None
        for e in e11s:
            tgt = ms.uniaxial_mixed(2, e)
            st, _, hom, stats = staggered.staggered_step(phase, tab, 2, st, tgt, **STAG_TOLS)
            assert stats["converged"]
            states.append(st)
            targets.append(tgt)
        return states, targets, hom

    states, targets, _ = path(table)
    held = (states[2]["hist"][1] > states[3]["abar"][1]) & (phase == 1) & \
        (states[2]["hist"][1] > 5e-4)
    assert held.sum() >= 5                         # damage held at its history on unloading
    g = np.zeros((3,) + S)
    g[0] = 1.0 / phase.size
    dl = adjoint.path_gradient(phase, table, 2, states, targets, g)
    for j in range(2):
        grad = adjoint.phase_length_gradient(dl[j], phase, table, j)
        for q in range(2):
            e0 = table[q]["ell"][j]
            hq = 1e-4 * e0
            vals = []
            for sgn in (1, -1):
                tb = [dict(t, ell=list(t["ell"])) for t in table]
                tb[q]["ell"][j] = e0 + sgn * hq
                vals.append(path(tb)[2]["sigma"][0])
            fd = (vals[0] - vals[1]) / (2 * hq)
            assert grad[q] == pytest.approx(fd, rel=5e-4, abs=1e-5 * max(abs(grad).max(), 1e-9)), \
                (j, q)


def test_path_gradient_spectral_scheme_and_voxel_size_by_finite_differences():
    """The path gradient with the SPECTRAL derivative symbols and a voxel
    size h = 0.5 (two increments, damage active), against central differences
    of the whole path in both per-phase lengths."""
    from oracle import spectral, staggered
    S = (12, 16)
    rng = np.random.default_rng(17)
    phase = (rng.uniform(size=S) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[1.0], dC=0.0005, dR=0.02), ms.particle_elastic(ell=[0.25])]
    tols = dict(cg_tol=1e-13, pcg_tol=1e-13, newton_tol=1e-12, stagger_tol=1e-12, max_stagger=200)
    targets = [ms.uniaxial_mixed(2, e) for e in (3e-3, 4e-3)]

    def path(tab):
        st = staggered.initial_state(S, 2, 1)
        states, hom = [st], None
        for tgt in targets:
            st, _, hom, stats = staggered.staggered_step(phase, tab, 1, st, tgt, h=0.5,
                                                         scheme=spectral.SPECTRAL, **tols)
            assert stats["converged"]
            states.append(st)
        return states, hom

    states, _ = path(table)
    assert states[-1]["abar"].max() > table[0]["dC"]
    g = np.zeros((3,) + S)
    g[0] = 1.0 / phase.size
    dl = adjoint.path_gradient(phase, table, 1, states, targets, g, h=0.5,
                               scheme=spectral.SPECTRAL, cg_tol=1e-13, pcg_tol=1e-13, tol=1e-12,
                               maxit=300)
    grad = adjoint.phase_length_gradient(dl[0], phase, table, 0)
    for q in range(2):
        e0 = table[q]["ell"][0]
        hq = 1e-4 * e0
        vals = []
        for sgn in (1, -1):
            tb = [dict(t, ell=list(t["ell"])) for t in table]
            tb[q]["ell"][0] = e0 + sgn * hq
            vals.append(path(tb)[1]["sigma"][0])
        fd = (vals[0] - vals[1]) / (2 * hq)
        assert grad[q] == pytest.approx(fd, rel=5e-4, abs=1e-6 * abs(grad).max())
