"""Pins of the checker's staggered increment (Sec. 3.2, Algorithm 1)."""
import numpy as np

from oracle import galerkin, staggered
from paper_2103_04770_amd import microstructure as ms
from tests._pins import dense_helmholtz

TOLS = dict(cg_tol=1e-12, pcg_tol=1e-12, newton_tol=1e-11)


def _setup(n=8, seed=0):
    S = (n, n, n)
    rng = np.random.default_rng(seed)
    phase = (rng.uniform(size=S) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
    return S, phase, table


def test_elastic_regime_gives_zero_nonlocal_field():
    S, phase, table = _setup()
    st = staggered.initial_state(S, 3, 1)
    tgt = ms.uniaxial_mixed(3, 1e-3)
    new, sig, hom, stats = staggered.staggered_step(phase, table, 1, st, tgt, stagger_tol=1e-10,
                                                    **TOLS)
    assert np.all(new["kappa"] == 0) and np.all(new["abar"] == 0)
    assert stats["converged"] and stats["stagger_iters"] == 2 and stats["pcg_iters"] == 0


def test_before_damage_onset_equals_mechanics_alone():
    S, phase, table = _setup()
    st = staggered.initial_state(S, 3, 1)
    tgt = ms.uniaxial_mixed(3, 6e-3)
    new, sig, hom, stats = staggered.staggered_step(phase, table, 1, st, tgt, stagger_tol=1e-10,
                                                    **TOLS)
    assert new["kappa"].max() > 0 and new["abar"].max() < 0.03
    mech = galerkin.fftg_solve(phase, table, np.zeros((1,) + S), st["epsp"], st["kappa"], tgt,
                               st["eps"], cg_tol=1e-12, newton_tol=1e-11)
    assert np.abs(mech["eps"] - new["eps"]).max() <= 1e-10 * 6e-3
    assert np.allclose(hom["sigma"], mech["sigma"].reshape(6, -1).mean(1), rtol=0, atol=1e-8)


def test_converged_increment_is_a_fixed_point():
    """After damage onset: once converged, another staggered pass from the
    converged state changes the fields by less than the tolerance."""
    S, phase, table = _setup(seed=1)
    table[0]["dC"], table[0]["dR"] = 0.001, 0.05
    st = staggered.initial_state(S, 3, 1)
    tgt = ms.uniaxial_mixed(3, 8e-3)
    new, sig, hom, stats = staggered.staggered_step(phase, table, 1, st, tgt, stagger_tol=1e-9,
                                                    **TOLS)
    assert stats["converged"] and stats["stagger_iters"] > 2
    from oracle import material
    D = material.damage_from_nonlocal(phase, table, new["abar"], st["hist"])
    assert D.max() > 0
    # one more pass, frozen at the converged non-local field
    mech = galerkin.fftg_solve(phase, table, D, st["epsp"], st["kappa"], tgt, new["eps"],
                               cg_tol=1e-12, newton_tol=1e-11)
    assert np.abs(mech["eps"] - new["eps"]).max() <= 1e-8 * 8e-3
    # and the non-local field solves the Helmholtz equation of the final
    # local source (dense real-space solve, no FFT)
    ell2 = staggered.ell2_field(phase, table, 0)
    ref = np.linalg.solve(dense_helmholtz(S, ell2, 1.0), mech["alpha"][0].reshape(-1))
    assert np.abs(new["abar"][0].reshape(-1) - ref).max() <= 1e-8 * ref.max()


def test_simple_staggered_is_one_pass():
    w = ms.workload("disc2d_32")
    st = staggered.initial_state(w["shape"], 2, 1)
    new, sig, hom, stats = staggered.staggered_step(w["phase"], w["table"], 1, st, w["load"][0],
                                                    max_stagger=1)
    assert stats["stagger_iters"] == 1
    assert abs(hom["eps"][0] - 5e-3) < 1e-15
    assert abs(hom["sigma"][1]) < 1e-5 * hom["sigma"][0]


# ---------------------------------------------------------------------------
# Irreversibility of the particle cracking law (reading C10: the cracking
# damage is driven by the history kappa = max over the path of the non-local
# equivalent strain; the history committed at the end of an increment is
# max(hist_n, abar_{n+1})).
#
# Closed form for a homogeneous cracking RVE under uniaxial mixed control
# (E11 prescribed, every other mean stress zero): whatever the damage, the
# strain is uniform with eps22 = eps33 = -nu E11 (uniaxial stress of an
# isotropic solid scaled by 1 - D), so the Mazars equivalent strain is
# sqrt(<eps_i>_+^2) = E11 for E11 > 0; a constant source gives abar = E11
# exactly (the Helmholtz operator maps constants to themselves); hence
# hist_{n+1} = max(hist_n, E11), D = clip((hist - k0)/(kf - k0), 0, dmax) and
# <sigma_11> = (1 - D) E E11.
# ---------------------------------------------------------------------------
_CRACK_PATH = (4e-3, 2e-3, 3e-3, 5e-3)   # load, unload, reload below the peak, past it


def _cracking_path_against_hand_values():
    """Runs the oracle along _CRACK_PATH on a homogeneous cracking RVE and
    returns the list of mismatches against the hand values (empty = pass)."""
    S = (4, 4, 4)
    phase = np.zeros(S, dtype=np.uint8)
    mat = ms.particle_cracking(ell=[1.5], dfield=0)
    table = [mat]
    E, k0, kf = mat["E"], mat["dC"], mat["dR"]
    st = staggered.initial_state(S, 3, 1)
    peak = 0.0
    bad = []
    for e11 in _CRACK_PATH:
        st, sig, hom, stats = staggered.staggered_step(phase, table, 1, st,
                                                       ms.uniaxial_mixed(3, e11),
                                                       stagger_tol=1e-12, **TOLS)
        peak = max(peak, e11)
        D = min(max((peak - k0) / (kf - k0), 0.0), mat["dmax"])
        if not stats["converged"]:
            bad.append((e11, "not converged"))
        if np.abs(st["abar"][0] - e11).max() > 1e-14:
            bad.append((e11, "abar", float(np.abs(st["abar"][0] - e11).max())))
        if np.abs(st["hist"][0] - peak).max() > 1e-14:
            bad.append((e11, "hist", float(np.abs(st["hist"][0] - peak).max())))
        s11 = (1.0 - D) * E * e11
        if np.abs(sig[0] - s11).max() > 1e-11 * s11:
            bad.append((e11, "sigma11", float(np.abs(sig[0] - s11).max()), s11))
        if abs(hom["sigma"][0] - s11) > 1e-11 * s11:
            bad.append((e11, "<sigma11>", float(hom["sigma"][0]), s11))
    return bad


def test_cracking_history_is_the_running_maximum():
    """Load, unload, reload below the previous peak, reload past it: the
    committed history is the running maximum of the non-local equivalent
    strain voxel by voxel, and the damage stays at D(history) on unloading."""
    assert _cracking_path_against_hand_values() == []


def test_cracking_history_pin_catches_wrong_commits(monkeypatch):
    """Planted mistakes in the checker's history commit (the history taken
    as the new field alone, or as the previous increment's field) fail the
    pin above."""
    from oracle import material

    def no_max(phase, table, abar, hist_n, abar_n):
        return abar.copy()

    def previous_field(phase, table, abar, hist_n, abar_n):
        return abar_n.copy()

    for wrong in (no_max, previous_field):
        monkeypatch.setattr(material, "commit_history", wrong)
        assert _cracking_path_against_hand_values() != []
    monkeypatch.undo()
    assert _cracking_path_against_hand_values() == []
