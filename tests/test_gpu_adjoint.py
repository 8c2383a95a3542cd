"""Adjoint entry points (helmholtz_adjoint, fftg_solve_adjoint) and their
torch.autograd wrappers against the oracle's adjoints."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import adjoint, galerkin, helmholtz  # noqa: E402
from paper_2103_04770_amd import microstructure as ms  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def solver(shape_np, **kw):
    from paper_2103_04770_amd import Solver
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Solver(tuple(reversed(shape_np)), **kw)


@pytest.mark.parametrize("shape", [(8, 12, 16), (12, 18)])
def test_helmholtz_adjoint_matches_oracle(shape):
    say("helmholtz adjoint", shape)
    rng = np.random.default_rng(5)
    alpha = np.abs(rng.standard_normal(shape))
    ell2 = rng.uniform(0.0, 3.0, size=shape)
    gbar = rng.standard_normal(shape)
    fwd = helmholtz.helmholtz_solve(alpha, ell2, tol=1e-13, maxit=2000)
    ref = adjoint.helmholtz_adjoint(fwd["abar"], gbar, ell2, tol=1e-13, maxit=2000)
    s = solver(shape)
    dal = torch.zeros(shape, dtype=torch.float64, device="cuda")
    dl2 = torch.empty(shape, dtype=torch.float64, device="cuda")
    d = s.helmholtz_adjoint(dev(ell2), dev(fwd["abar"]), dev(gbar), dal, dl2, tol=1e-13,
                            maxit=2000)
    assert d["converged"]
    a, l2 = dal.cpu().numpy(), dl2.cpu().numpy()
    assert np.abs(a - ref["dalpha"]).max() <= 1e-10 * np.abs(ref["dalpha"]).max()
    assert np.abs(l2 - ref["dell2"]).max() <= 1e-9 * np.abs(ref["dell2"]).max()


def _mech_case(shape, seed):
    rng = np.random.default_rng(seed)
    phase = (rng.uniform(size=shape) < 0.3).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_cracking(ell=[1.0], dfield=0)]
    D = rng.uniform(0.05, 0.45, size=shape)[None]
    c = 6 if len(shape) == 3 else 3
    tgt = ms.uniaxial_mixed(len(shape), 5e-3)
    return rng, phase, table, D, c, tgt


@pytest.mark.parametrize("shape", [(8, 12, 16), (16, 12)])
def test_mechanics_adjoint_matches_oracle(shape):
    say("mechanics adjoint", shape)
    rng, phase, table, D, c, tgt = _mech_case(shape, 6)
    z6, z = np.zeros((6,) + shape), np.zeros(shape)
    fwd = galerkin.fftg_solve(phase, table, D, z6, z, tgt, np.zeros((c,) + shape),
                              cg_tol=1e-13, newton_tol=1e-13, newton_maxit=60)
    gbar = rng.standard_normal((c,) + shape)
    ref = adjoint.mechanics_adjoint(phase, table, D, z6, z, tgt, fwd["eps"], gbar, 1,
                                    cg_tol=1e-13)
    s = solver(shape)
    mu = torch.empty((c,) + shape, dtype=torch.float64, device="cuda")
    dD = torch.empty((1,) + shape, dtype=torch.float64, device="cuda")
    d = s.fftg_solve_adjoint(dev(phase, torch.uint8), table, 1, dev(D), dev(np.zeros((7,) + shape)),
                             tgt, dev(fwd["eps"]), dev(gbar), mu, dD, cg_tol=1e-13)
    assert d["converged"]
    m, g = mu.cpu().numpy(), dD.cpu().numpy()
    assert np.abs(m - ref["mu"]).max() <= 1e-9 * np.abs(ref["mu"]).max()
    assert np.abs(g - ref["dD"]).max() <= 1e-9 * np.abs(ref["dD"]).max()


def test_autograd_helmholtz_gradients():
    """J = sum w abar through the autograd wrapper: gradients equal the
    oracle's adjoint, and a central difference of the GPU forward along a
    random ell2 direction agrees with the directional derivative."""
    from paper_2103_04770_amd import autograd as ag
    shape = (8, 8, 12)
    say("autograd helmholtz", shape)
    rng = np.random.default_rng(7)
    alpha = np.abs(rng.standard_normal(shape))
    ell2 = rng.uniform(0.5, 2.0, size=shape)
    w = rng.standard_normal(shape)
    s = solver(shape)
    a_t = dev(alpha).requires_grad_(True)
    l_t = dev(ell2).requires_grad_(True)
    abar = ag.helmholtz(s, a_t, l_t, tol=1e-13)
    J = (dev(w) * abar).sum()
    ga, gl = torch.autograd.grad(J, (a_t, l_t))
    fwd = helmholtz.helmholtz_solve(alpha, ell2, tol=1e-13, maxit=2000)
    ref = adjoint.helmholtz_adjoint(fwd["abar"], w, ell2, tol=1e-13, maxit=2000)
    assert np.abs(ga.cpu().numpy() - ref["dalpha"]).max() <= 1e-9 * np.abs(ref["dalpha"]).max()
    assert np.abs(gl.cpu().numpy() - ref["dell2"]).max() <= 1e-8 * np.abs(ref["dell2"]).max()
    dirn = rng.standard_normal(shape)
    hh = 1e-5
    with torch.no_grad():
        jp = float((dev(w) * ag.helmholtz(s, dev(alpha), dev(ell2 + hh * dirn), tol=1e-13)).sum())
        jm = float((dev(w) * ag.helmholtz(s, dev(alpha), dev(ell2 - hh * dirn), tol=1e-13)).sum())
    fd = (jp - jm) / (2 * hh)
    assert float((gl.cpu().numpy() * dirn).sum()) == pytest.approx(fd, rel=1e-6)


def test_autograd_mechanics_gradient():
    from paper_2103_04770_amd import autograd as ag
    shape = (8, 8, 12)
    say("autograd mechanics", shape)
    rng, phase, table, D, c, tgt = _mech_case(shape, 8)
    w = rng.standard_normal((c,) + shape)
    s = solver(shape)
    D_t = dev(D).requires_grad_(True)
    opts = dict(cg_tol=1e-13, newton_tol=1e-13, newton_maxit=60)
    eps, _ = ag.mechanics(s, D_t, dev(phase, torch.uint8), table, 1,
                          dev(np.zeros((7,) + shape)), tgt, **opts)
    J = (dev(w) * eps).sum()
    (gD,) = torch.autograd.grad(J, (D_t,))
    z6, z = np.zeros((6,) + shape), np.zeros(shape)
    fwd = galerkin.fftg_solve(phase, table, D, z6, z, tgt, np.zeros((c,) + shape), **opts)
    ref = adjoint.mechanics_adjoint(phase, table, D, z6, z, tgt, fwd["eps"], w, 1, cg_tol=1e-13)
    assert np.abs(gD.cpu().numpy() - ref["dD"]).max() <= 1e-8 * np.abs(ref["dD"]).max()


def test_one_pass_chain_gradients_match_oracle():
    """<sigma_11> and <D> through alpha -> abar -> D -> (eps, sigma) with the
    library's autograd chain: gradients with respect to the per-voxel source
    and the per-phase lengths against the oracle's adjoint chain."""
    from paper_2103_04770_amd import autograd as ag
    from tests.test_oracle_adjoint import _chain_case, _chain_forward
    S, phase, table, alpha = _chain_case()
    say("one-pass chain", S)
    ells = [2.0, 0.5]
    f = _chain_forward(S, phase, table, alpha, ells)
    N = phase.size
    z6, z = np.zeros((6,) + S), np.zeros(S)
    tab = [dict(t, ell=[e]) for t, e in zip(table, ells)]
    refs = {}
    for which in ("stress", "damage"):
        if which == "stress":
            gsig = np.zeros((6,) + S)
            gsig[0] = 1.0 / N
            gD = adjoint.mechanics_adjoint(phase, table, f["D"], z6, z, f["tgt"], f["eps"],
                                           np.zeros((6,) + S), 1, cg_tol=1e-13, gsig=gsig)["dD"]
        else:
            gD = np.full((1,) + S, 1.0 / N)
        ga = adjoint.damage_adjoint(phase, table, f["abar"][None], f["hist"], gD)[0]
        h = adjoint.helmholtz_adjoint(f["abar"], ga, f["ell2"], tol=1e-14, maxit=500)
        refs[which] = (h["dalpha"], adjoint.phase_length_gradient(h["dell2"], phase, tab, 0))
    s = solver(S)
    ph = dev(phase, torch.uint8)
    for which in ("stress", "damage"):
        a_t = dev(alpha).requires_grad_(True)
        e_t = torch.tensor(ells, dtype=torch.float64, device="cuda", requires_grad=True)
        abar, D, eps, sig = ag.one_pass(s, a_t, e_t, ph, table, f["tgt"], helm_tol=1e-14,
                                        cg_tol=1e-13, newton_tol=1e-13, newton_maxit=60)
        if which == "stress":
            assert np.abs(sig.detach().cpu().numpy() - f["sigma"]).max() <= 1e-9 * np.abs(
                f["sigma"]).max()
        J = sig[0].mean() if which == "stress" else D.mean()
        ga, ge = torch.autograd.grad(J, (a_t, e_t))
        ra, re = refs[which]
        say(which, "dJ/dell gpu", ge.cpu().numpy(), "oracle", re)
        assert np.abs(ga.cpu().numpy() - ra).max() <= 1e-7 * np.abs(ra).max()
        assert np.allclose(ge.cpu().numpy(), re, rtol=1e-7, atol=1e-12 * np.abs(re).max())


def _pack(st):
    return np.concatenate([st["eps"], st["epsp"], st["kappa"][None], st["hist"], st["abar"]])


@pytest.mark.parametrize("shape,which", [((12, 16), "sigma11"), ((12, 16), "mean_damage"),
                                         ((6, 8, 8), "sigma11"), ((6, 8, 8), "mean_abar")])
def test_staggered_adjoint_matches_oracle(shape, which):
    """fftg_staggered_adjoint at a converged increment (damage active, fed
    back into the source through the mechanics) against the oracle's
    transposed staggered fixed point."""
    from oracle import staggered
    from tests.test_oracle_adjoint import STAG_TOLS
    say("staggered adjoint", shape, which)
    rng = np.random.default_rng(21)
    phase = (rng.uniform(size=shape) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0], dC=0.0005, dR=0.02), ms.particle_elastic(ell=[0.5])]
    nd = len(shape)
    c = 6 if nd == 3 else 3
    st_n, _, _, _ = staggered.staggered_step(phase, table, 1, staggered.initial_state(shape, nd, 1),
                                             ms.uniaxial_mixed(nd, 3e-3), **STAG_TOLS)
    tgt = ms.uniaxial_mixed(nd, 5e-3)
    st, _, _, stats = staggered.staggered_step(phase, table, 1, st_n, tgt, **STAG_TOLS)
    assert stats["converged"] and stats["stagger_iters"] > 2
    N = phase.size
    kw, kg = {}, {}
    if which == "sigma11":
        g = np.zeros((c,) + shape)
        g[0] = 1.0 / N
        kw["g_sig"], kg["g_sig"] = g, dev(g)
    elif which == "mean_damage":
        g = np.full((1,) + shape, 1.0 / N)
        kw["g_D"], kg["g_D"] = g, dev(g)
    else:
        g = np.full((1,) + shape, 1.0 / N)
        kw["g_abar"], kg["g_abar"] = g, dev(g)
    ref = adjoint.staggered_adjoint(phase, table, 1, st_n, st["eps"], st["abar"], tgt, **kw)
    s = solver(shape)
    dl = torch.empty((1,) + shape, dtype=torch.float64, device="cuda")
    lam = torch.empty((1,) + shape, dtype=torch.float64, device="cuda")
    d = s.fftg_staggered_adjoint(dev(phase, torch.uint8), table, 1, dev(_pack(st_n)), dev(_pack(st)),
                                 tgt, dl, lam=lam, cg_tol=1e-13, pcg_tol=1e-13, tol=1e-12,
                                 maxit=300, **kg)
    say("  gpu passes", d["stagger_iters"], "cg", d["cg_iters"], "pcg", d["pcg_iters"],
        "oracle passes", ref["iters"])
    assert d["converged"]
    got = dl.cpu().numpy()
    assert np.abs(got - ref["dell2"]).max() <= 1e-8 * np.abs(ref["dell2"]).max()
    assert np.abs(lam.cpu().numpy() - ref["lam"]).max() <= 1e-8 * np.abs(ref["lam"]).max()
    gq = adjoint.phase_length_gradient(got[0], phase, table, 0)
    rq = adjoint.phase_length_gradient(ref["dell2"][0], phase, table, 0)
    assert np.allclose(gq, rq, rtol=1e-8)


def test_staggered_adjoint_rejects_uncovered_sources():
    from paper_2103_04770_amd.binding import FFTGError
    shape = (8, 8, 8)
    s = solver(shape)
    table = [ms.matrix_gtn(ell=[2.0, 2.0]), ms.particle_elastic(ell=[0.1, 0.1])]
    z = dev(np.zeros((6 + 7 + 4,) + shape))
    with pytest.raises(FFTGError, match="UNSUPPORTED"):
        s.fftg_staggered_adjoint(dev(np.zeros(shape), torch.uint8), table, 2, z, z,
                                 ms.uniaxial_mixed(3, 1e-3),
                                 torch.empty((2,) + shape, dtype=torch.float64, device="cuda"))


def test_autograd_staggered_increment_matches_oracle_gradient():
    """torch.autograd through a whole converged increment: d<sigma_11>/d ell
    (per phase) equals the oracle's adjoint of the converged increment."""
    from oracle import staggered
    from paper_2103_04770_amd import autograd as ag
    from tests.test_oracle_adjoint import STAG_TOLS
    shape = (6, 8, 8)
    say("autograd staggered increment", shape)
    rng = np.random.default_rng(21)
    phase = (rng.uniform(size=shape) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0], dC=0.0005, dR=0.02), ms.particle_elastic(ell=[0.5])]
    st_n, _, _, _ = staggered.staggered_step(phase, table, 1, staggered.initial_state(shape, 3, 1),
                                             ms.uniaxial_mixed(3, 3e-3), **STAG_TOLS)
    tgt = ms.uniaxial_mixed(3, 5e-3)
    st, _, hom, _ = staggered.staggered_step(phase, table, 1, st_n, tgt, **STAG_TOLS)
    g = np.zeros((6,) + shape)
    g[0] = 1.0 / phase.size
    ref = adjoint.staggered_adjoint(phase, table, 1, st_n, st["eps"], st["abar"], tgt, g_sig=g)
    rq = adjoint.phase_length_gradient(ref["dell2"][0], phase, table, 0)
    s = solver(shape)
    ell = torch.tensor([2.0, 0.5], dtype=torch.float64, device="cuda", requires_grad=True)
    opts = dict(cg_tol=1e-13, pcg_tol=1e-13, newton_tol=1e-12, newton_maxit=60,
                stagger_tol=1e-12, max_stagger=300)
    sig, abar = ag.staggered_increment(s, ell, dev(phase, torch.uint8), table, 1,
                                       dev(_pack(st_n)), tgt, **opts)
    J = sig[0].mean()
    assert float(J.detach()) == pytest.approx(hom["sigma"][0], rel=1e-9)
    (ge,) = torch.autograd.grad(J, (ell,))
    say("  dJ/dell gpu", ge.cpu().numpy(), "oracle", rq)
    assert np.allclose(ge.cpu().numpy(), rq, rtol=1e-7)


@pytest.mark.parametrize("shape", [(12, 16), (6, 8, 12)])
def test_staggered_adjoint_two_fields_matches_oracle(shape):
    """Both sources of the benchmark table (J2 damage matrix on field 0,
    particle cracking on field 1, cracking active): dJ/dell2 of both fields
    against the oracle's transposed fixed point."""
    from oracle import staggered
    from tests.test_oracle_adjoint import STAG_TOLS
    say("staggered adjoint two fields", shape)
    rng = np.random.default_rng(23)
    phase = (rng.uniform(size=shape) < 0.3).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0, 0.04], dfield=0, dC=0.0005, dR=0.02),
             ms.particle_cracking(ell=[0.04, 1.0], dfield=1, k0=5e-4, kf=5e-3)]
    nd = len(shape)
    c = 6 if nd == 3 else 3
    st_n, _, _, _ = staggered.staggered_step(phase, table, 2, staggered.initial_state(shape, nd, 2),
                                             ms.uniaxial_mixed(nd, 2e-3), **STAG_TOLS)
    tgt = ms.uniaxial_mixed(nd, 3e-3)
    st, _, _, stats = staggered.staggered_step(phase, table, 2, st_n, tgt, **STAG_TOLS)
    assert stats["converged"] and st["abar"][1].max() > 5e-4
    g = np.zeros((c,) + shape)
    g[0] = 1.0 / phase.size
    ref = adjoint.staggered_adjoint(phase, table, 2, st_n, st["eps"], st["abar"], tgt, g_sig=g)
    s = solver(shape)
    dl = torch.empty((2,) + shape, dtype=torch.float64, device="cuda")
    d = s.fftg_staggered_adjoint(dev(phase, torch.uint8), table, 2, dev(_pack(st_n)), dev(_pack(st)),
                                 tgt, dl, g_sig=dev(g), cg_tol=1e-13, pcg_tol=1e-13, tol=1e-12,
                                 maxit=300)
    say("  gpu passes", d["stagger_iters"], "oracle passes", ref["iters"])
    assert d["converged"]
    got = dl.cpu().numpy()
    for j in range(2):
        assert np.abs(got[j] - ref["dell2"][j]).max() <= 1e-8 * np.abs(ref["dell2"][j]).max()



@pytest.mark.parametrize("shape", [(12, 16), (6, 8, 8)])
def test_increment_adjoint_matches_oracle(shape):
    """fftg_increment_adjoint at a converged increment with history
    cotangents coming in (random g_epsp, g_kappa, J = <sigma_11>): dJ/dell2
    and the cotangents of the starting history against the oracle."""
    from oracle import staggered
    from tests.test_oracle_adjoint import STAG_TOLS
    say("increment adjoint", shape)
    rng = np.random.default_rng(21)
    phase = (rng.uniform(size=shape) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0], dC=0.0005, dR=0.02), ms.particle_elastic(ell=[0.5])]
    nd = len(shape)
    c = 6 if nd == 3 else 3
    st_n, _, _, _ = staggered.staggered_step(phase, table, 1, staggered.initial_state(shape, nd, 1),
                                             ms.uniaxial_mixed(nd, 3e-3), **STAG_TOLS)
    tgt = ms.uniaxial_mixed(nd, 5e-3)
    st, _, _, stats = staggered.staggered_step(phase, table, 1, st_n, tgt, **STAG_TOLS)
    assert stats["converged"]
    g = np.zeros((c,) + shape)
    g[0] = 1.0 / phase.size
    gp = rng.standard_normal((6,) + shape) / phase.size
    gk = rng.standard_normal(shape) / phase.size
    gh = rng.standard_normal((1,) + shape) / phase.size
    ref = adjoint.increment_adjoint(phase, table, 1, st_n, st, tgt, g_sig=g, g_epsp=gp, g_kappa=gk,
                                    g_hist=gh, cg_tol=1e-13, pcg_tol=1e-13, tol=1e-12, maxit=300)
    s = solver(shape)
    dl = torch.empty((1,) + shape, dtype=torch.float64, device="cuda")
    gpn = torch.empty((6,) + shape, dtype=torch.float64, device="cuda")
    gkn = torch.empty(shape, dtype=torch.float64, device="cuda")
    ghn = torch.empty((1,) + shape, dtype=torch.float64, device="cuda")
    d = s.fftg_increment_adjoint(dev(phase, torch.uint8), table, 1, dev(_pack(st_n)),
                                 dev(_pack(st)), tgt, dl, gpn, gkn, ghn, g_sig=dev(g),
                                 g_epsp=dev(gp), g_kappa=dev(gk), g_hist=dev(gh), cg_tol=1e-13,
                                 pcg_tol=1e-13, tol=1e-12, maxit=300)
    say("  gpu passes", d["stagger_iters"], "oracle passes", ref["iters"])
    assert d["converged"]
    # no cracking phase: the committed history is read by nothing, and where
    # hist_n stays the max its cotangent passes through bit for bit
    assert np.array_equal(ghn.cpu().numpy(), ref["g_hist_n"])
    for name, got, want in (("dell2", dl, ref["dell2"]), ("g_epsp_n", gpn, ref["g_epsp_n"]),
                            ("g_kappa_n", gkn, ref["g_kappa_n"])):
        got = got.cpu().numpy()
        err = np.abs(got - want).max() / np.abs(want).max()
        say("  ", name, "rel err %.2e" % err)
        assert err <= 1e-8, name
    # elastic particles pass the incoming plastic-history cotangents through
    part = phase == 1
    assert np.array_equal(gkn.cpu().numpy()[part], gk[part])


def test_path_gradient_matches_oracle():
    """d<sigma_11>/d ell2 after a three-increment path run on the GPU,
    chained backwards through every increment's plastic history, against the
    oracle's path gradient on its own path; the per-phase dJ/d ell through
    torch.autograd (staggered_path) agrees too."""
    from oracle import staggered
    from paper_2103_04770_amd import autograd as ag
    from tests.test_oracle_adjoint import STAG_TOLS
    shape = (12, 16)
    say("path gradient", shape)
    rng = np.random.default_rng(21)
    phase = (rng.uniform(size=shape) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0], dC=0.0005, dR=0.02), ms.particle_elastic(ell=[0.5])]
    targets = [ms.uniaxial_mixed(2, e) for e in (2e-3, 4e-3, 6e-3)]
    st = staggered.initial_state(shape, 2, 1)
    ostates = [st]
    for tgt in targets:
        st, _, hom, stats = staggered.staggered_step(phase, table, 1, st, tgt, **STAG_TOLS)
        assert stats["converged"]
        ostates.append(st)
    g = np.zeros((3,) + shape)
    g[0] = 1.0 / phase.size
    ref = adjoint.path_gradient(phase, table, 1, ostates, targets, g, cg_tol=1e-13, pcg_tol=1e-13,
                                tol=1e-12, maxit=300)
    rq = adjoint.phase_length_gradient(ref[0], phase, table, 0)
    s = solver(shape)
    ph = dev(phase, torch.uint8)
    opts = dict(cg_tol=1e-13, pcg_tol=1e-13, newton_tol=1e-12, newton_maxit=60,
                stagger_tol=1e-13, max_stagger=300)
    state = dev(np.zeros((3 + 7 + 2,) + shape))
    sig = torch.empty((3,) + shape, dtype=torch.float64, device="cuda")
    states = [state.clone()]
    for tgt in targets:
        assert s.staggered_step(ph, table, 1, state, tgt, sig, **opts)["converged"]
        states.append(state.clone())
    dl, log = ag.path_gradient(s, ph, table, 1, states, targets, dev(g), cg_tol=1e-13,
                               pcg_tol=1e-13, tol=1e-12, maxit=300)
    got = dl.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say("  passes", [d["stagger_iters"] for d in log], "rel err %.2e" % err)
    assert err <= 1e-7
    ell = torch.tensor([2.0, 0.5], dtype=torch.float64, device="cuda", requires_grad=True)
    sg = ag.staggered_path(s, ell, ph, table, 1, states[0], targets, **opts)
    J = sg[0].mean()
    assert float(J.detach()) == pytest.approx(hom["sigma"][0], rel=1e-9)
    (ge,) = torch.autograd.grad(J, (ell,))
    say("  dJ/dell gpu", ge.cpu().numpy(), "oracle", rq)
    assert np.allclose(ge.cpu().numpy(), rq, rtol=1e-7)


def test_increment_adjoint_rejects_uncovered_phases():
    from paper_2103_04770_amd.binding import FFTGError
    shape = (8, 8, 8)
    s = solver(shape)
    table = [ms.matrix_gtn(ell=[2.0, 2.0]), ms.particle_elastic(ell=[0.1, 0.1])]
    z = dev(np.zeros((6 + 7 + 4,) + shape))
    f = lambda *k: torch.empty(k + shape, dtype=torch.float64, device="cuda")  # noqa: E731
    with pytest.raises(FFTGError, match="UNSUPPORTED"):
        s.fftg_increment_adjoint(dev(np.zeros(shape), torch.uint8), table, 2, z, z,
                                 ms.uniaxial_mixed(3, 1e-3), f(2), f(6), f(), f(2))


def _two_field_case(shape):
    rng = np.random.default_rng(23)
    phase = (rng.uniform(size=shape) < 0.3).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0, 0.04], dfield=0, dC=0.0005, dR=0.02),
             ms.particle_cracking(ell=[0.04, 1.0], dfield=1, k0=5e-4, kf=5e-3)]
    return phase, table


@pytest.mark.parametrize("shape", [(12, 16), (6, 8, 12)])
def test_increment_adjoint_damage_history_matches_oracle(shape):
    """Two fields (J2 damage matrix, particle cracking) with the history
    raised above abar on some cracking voxels, so that it drives their damage,
    and random incoming history cotangents: dJ/dell2 and the cotangents of
    the plastic state and damage history against the oracle."""
    from oracle import staggered
    from tests.test_oracle_adjoint import STAG_TOLS
    say("increment adjoint, damage history", shape)
    phase, table = _two_field_case(shape)
    nd = len(shape)
    c = 6 if nd == 3 else 3
    st_n = staggered.staggered_step(phase, table, 2, staggered.initial_state(shape, nd, 2),
                                    ms.uniaxial_mixed(nd, 2e-3), **STAG_TOLS)[0]
    rng = np.random.default_rng(5)
    raise_ = (phase == 1) & (rng.uniform(size=shape) < 0.5)
    st_n = dict(st_n, hist=st_n["hist"].copy())
    st_n["hist"][1][raise_] = np.maximum(st_n["hist"][1][raise_], st_n["abar"][1][raise_]) + \
        rng.uniform(1e-3, 2e-3, size=int(raise_.sum()))
    tgt = ms.uniaxial_mixed(nd, 3e-3)
    st, _, _, stats = staggered.staggered_step(phase, table, 2, st_n, tgt, **STAG_TOLS)
    assert stats["converged"]
    g = np.zeros((c,) + shape)
    g[0] = 1.0 / phase.size
    N = phase.size
    gp = rng.standard_normal((6,) + shape) / N
    gk = rng.standard_normal(shape) / N
    gh = rng.standard_normal((2,) + shape) / N
    kw = dict(cg_tol=1e-13, pcg_tol=1e-13, tol=1e-12, maxit=300)
    ref = adjoint.increment_adjoint(phase, table, 2, st_n, st, tgt, g_sig=g, g_epsp=gp, g_kappa=gk,
                                    g_hist=gh, **kw)
    s = solver(shape)
    f = lambda *k: torch.empty(k + shape, dtype=torch.float64, device="cuda")  # noqa: E731
    dl, gpn, gkn, ghn = f(2), f(6), f(), f(2)
    d = s.fftg_increment_adjoint(dev(phase, torch.uint8), table, 2, dev(_pack(st_n)),
                                 dev(_pack(st)), tgt, dl, gpn, gkn, ghn, g_sig=dev(g),
                                 g_epsp=dev(gp), g_kappa=dev(gk), g_hist=dev(gh), **kw)
    say("  gpu passes", d["stagger_iters"], "oracle passes", ref["iters"])
    assert d["converged"]
    held = (st_n["hist"][1] > st["abar"][1]) & (phase == 1)
    assert held.sum() >= 5
    for name, got, want in (("dell2", dl, ref["dell2"]), ("g_epsp_n", gpn, ref["g_epsp_n"]),
                            ("g_kappa_n", gkn, ref["g_kappa_n"]), ("g_hist_n", ghn, ref["g_hist_n"])):
        got = got.cpu().numpy()
        for j in range(want.shape[0] if name in ("dell2", "g_hist_n") else 1):
            w = want[j] if name in ("dell2", "g_hist_n") else want
            gg = got[j] if name in ("dell2", "g_hist_n") else got
            err = np.abs(gg - w).max() / max(np.abs(w).max(), 1e-300)
            say("  ", name, j, "rel err %.2e" % err)
            assert err <= 1e-8, (name, j)


def test_path_gradient_with_cracking_and_unloading_matches_oracle():
    """A two-field path that loads and partly unloads (E11 2e-3, 3e-3,
    2.5e-3; the cracking damage is held at its history on unloading), run on
    the GPU: the path gradient of <sigma_11> for both fields against the
    oracle's on its own path."""
    from oracle import staggered
    from paper_2103_04770_amd import autograd as ag
    from tests.test_oracle_adjoint import STAG_TOLS
    shape = (12, 16)
    say("path gradient, cracking and unloading", shape)
    phase, table = _two_field_case(shape)
    targets = [ms.uniaxial_mixed(2, e) for e in (2e-3, 3e-3, 2.5e-3)]
    st = staggered.initial_state(shape, 2, 2)
    ostates = [st]
    for tgt in targets:
        st = staggered.staggered_step(phase, table, 2, st, tgt, **STAG_TOLS)[0]
        ostates.append(st)
    g = np.zeros((3,) + shape)
    g[0] = 1.0 / phase.size
    kw = dict(cg_tol=1e-13, pcg_tol=1e-13, tol=1e-12, maxit=300)
    ref = adjoint.path_gradient(phase, table, 2, ostates, targets, g, **kw)
    s = solver(shape)
    ph = dev(phase, torch.uint8)
    opts = dict(cg_tol=1e-13, pcg_tol=1e-13, newton_tol=1e-12, newton_maxit=60,
                stagger_tol=1e-13, max_stagger=300)
    state = dev(np.zeros((3 + 7 + 4,) + shape))
    sig = torch.empty((3,) + shape, dtype=torch.float64, device="cuda")
    states = [state.clone()]
    for tgt in targets:
        assert s.staggered_step(ph, table, 2, state, tgt, sig, **opts)["converged"]
        states.append(state.clone())
    dl, log = ag.path_gradient(s, ph, table, 2, states, targets, dev(g), **kw)
    got = dl.cpu().numpy()
    for j in range(2):
        err = np.abs(got[j] - ref[j]).max() / np.abs(ref[j]).max()
        say("  field", j, "passes", [x["stagger_iters"] for x in log], "rel err %.2e" % err)
        assert err <= 1e-7


def test_path_gradient_fp32_refined_matches_oracle():
    """The FP32-refined form (FP32 Krylov vectors and transforms, FP64
    reductions, return maps and history cotangents) along the same
    three-increment path at the production staggered tolerance (1e-6; the
    FP32 Helmholtz solves cannot settle the fixed point much below it):
    dJ/dell2 within 1e-4 of the FP64 oracle's path gradient.  The adjoint's
    Krylov solves run without refinement at the FP32 floor of 1e-5 relative
    residual, and the transposed fixed point (contraction ~0.7 per pass here)
    amplifies that about threefold; the 128^3 workload agrees with its FP64
    run to 4e-6."""
    from oracle import staggered
    from paper_2103_04770_amd import FP32_REFINED, autograd as ag
    from tests.test_oracle_adjoint import STAG_TOLS
    shape = (12, 16)
    say("path gradient fp32-refined", shape)
    rng = np.random.default_rng(21)
    phase = (rng.uniform(size=shape) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0], dC=0.0005, dR=0.02), ms.particle_elastic(ell=[0.5])]
    targets = [ms.uniaxial_mixed(2, e) for e in (2e-3, 4e-3, 6e-3)]
    st = staggered.initial_state(shape, 2, 1)
    ostates = [st]
    for tgt in targets:
        st, _, _, stats = staggered.staggered_step(phase, table, 1, st, tgt, **STAG_TOLS)
        ostates.append(st)
    g = np.zeros((3,) + shape)
    g[0] = 1.0 / phase.size
    ref = adjoint.path_gradient(phase, table, 1, ostates, targets, g, cg_tol=1e-13, pcg_tol=1e-13,
                                tol=1e-12, maxit=300)
    s = solver(shape, prec=FP32_REFINED)
    ph = dev(phase, torch.uint8)
    opts = dict(cg_tol=1e-10, pcg_tol=1e-10, newton_tol=1e-10, newton_maxit=60,
                stagger_tol=1e-6, max_stagger=300)
    state = dev(np.zeros((3 + 7 + 2,) + shape))
    sig = torch.empty((3,) + shape, dtype=torch.float64, device="cuda")
    states = [state.clone()]
    for tgt in targets:
        d = s.staggered_step(ph, table, 1, state, tgt, sig, **opts)
        say("  forward", d["stagger_iters"], "passes, err %.1e" % d["err"])
        assert d["converged"]
        states.append(state.clone())
    dl, log = ag.path_gradient(s, ph, table, 1, states, targets, dev(g), cg_tol=1e-10,
                               pcg_tol=1e-10, tol=1e-6, maxit=300)
    got = dl.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    gq = adjoint.phase_length_gradient(got[0], phase, table, 0)
    rq = adjoint.phase_length_gradient(ref[0], phase, table, 0)
    say("  passes", [d["stagger_iters"] for d in log], "rel err %.2e" % err, "dJ/dell", gq, rq)
    assert err <= 1e-4
    assert np.allclose(gq, rq, rtol=1e-4)


def test_increment_adjoint_error_paths():
    """Host-side failure handling of fftg_increment_adjoint: a missing output
    is INVALID; a fixed point cut at maxit = 1 returns NOT_CONVERGED (a
    warning: the outputs are written, finite)."""
    import ctypes as ct
    from oracle import staggered
    from paper_2103_04770_amd.binding import FFTGError, KrylovOpts, _macro, phase_table
    from tests.test_oracle_adjoint import STAG_TOLS
    shape = (12, 16)
    rng = np.random.default_rng(21)
    phase = (rng.uniform(size=shape) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0], dC=0.0005, dR=0.02), ms.particle_elastic(ell=[0.5])]
    st_n = staggered.staggered_step(phase, table, 1, staggered.initial_state(shape, 2, 1),
                                    ms.uniaxial_mixed(2, 3e-3), **STAG_TOLS)[0]
    tgt = ms.uniaxial_mixed(2, 5e-3)
    st = staggered.staggered_step(phase, table, 1, st_n, tgt, **STAG_TOLS)[0]
    s = solver(shape)
    f = lambda *k: torch.empty(k + shape, dtype=torch.float64, device="cuda")  # noqa: E731
    g = torch.zeros((3,) + shape, dtype=torch.float64, device="cuda")
    g[0] = 1.0 / phase.size
    args = (dev(phase, torch.uint8), table, 1, dev(_pack(st_n)), dev(_pack(st)), tgt)
    dl, gpn, gkn, ghn = f(1), f(6), f(), f(1)
    # g_hist_n missing: rejected by the library before any launch
    m = _macro(tgt)
    rc = s.lib.fftg_increment_adjoint(
        s.h, args[0].data_ptr(), phase_table(table), len(table), 1, args[3].data_ptr(),
        args[4].data_ptr(), ct.byref(m), None, None, None, None, dl.data_ptr(), gpn.data_ptr(),
        gkn.data_ptr(), None, ct.byref(KrylovOpts(1e-8, 100)), ct.byref(KrylovOpts(1e-8, 100)),
        1e-8, 10, None)
    with pytest.raises(FFTGError, match="INVALID"):
        s._check(rc)
    d = s.fftg_increment_adjoint(*args, dl, gpn, gkn, ghn, g_sig=g, cg_tol=1e-12, pcg_tol=1e-12,
                                 tol=1e-14, maxit=1)
    assert not d["converged"] and d["stagger_iters"] == 1
    for t in (dl, gpn, gkn, ghn):
        assert torch.isfinite(t).all()


def test_path_gradient_spectral_scheme_and_voxel_size():
    """The path gradient with the SPECTRAL derivative symbols and a voxel
    size h = 0.5 (lengths in the same unit), two increments with damage
    active: against the oracle's path gradient with the same scheme and h."""
    from oracle import spectral, staggered
    from paper_2103_04770_amd import SPECTRAL, autograd as ag
    shape = (12, 16)
    say("path gradient spectral h=0.5", shape)
    rng = np.random.default_rng(17)
    phase = (rng.uniform(size=shape) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[1.0], dC=0.0005, dR=0.02), ms.particle_elastic(ell=[0.25])]
    tols = dict(cg_tol=1e-13, pcg_tol=1e-13, newton_tol=1e-12, stagger_tol=1e-12, max_stagger=200)
    targets = [ms.uniaxial_mixed(2, e) for e in (3e-3, 4e-3)]
    st = staggered.initial_state(shape, 2, 1)
    ostates = [st]
    for tgt in targets:
        st, _, _, stats = staggered.staggered_step(phase, table, 1, st, tgt, h=0.5,
                                                   scheme=spectral.SPECTRAL, **tols)
        assert stats["converged"]
        ostates.append(st)
    assert st["abar"].max() > table[0]["dC"]
    g = np.zeros((3,) + shape)
    g[0] = 1.0 / phase.size
    kw = dict(cg_tol=1e-13, pcg_tol=1e-13, tol=1e-12, maxit=300)
    ref = adjoint.path_gradient(phase, table, 1, ostates, targets, g, h=0.5,
                                scheme=spectral.SPECTRAL, **kw)
    s = solver(shape, scheme=SPECTRAL, h=0.5)
    ph = dev(phase, torch.uint8)
    state = dev(np.zeros((3 + 7 + 2,) + shape))
    sig = torch.empty((3,) + shape, dtype=torch.float64, device="cuda")
    states = [state.clone()]
    for tgt in targets:
        assert s.staggered_step(ph, table, 1, state, tgt, sig, **tols)["converged"]
        states.append(state.clone())
    dl, log = ag.path_gradient(s, ph, table, 1, states, targets, dev(g), **kw)
    got = dl.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say("  passes", [x["stagger_iters"] for x in log], "rel err %.2e" % err)
    assert err <= 1e-7
