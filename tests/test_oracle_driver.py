"""Pins of the checker's adaptive load driver (variable increments with a
smallest admissible increment, Sec. 4.2)."""
import numpy as np
import pytest

from oracle import driver, galerkin, staggered
from paper_2103_04770_amd import microstructure as ms


def _mock_step(limit):
    """Stand-in increment: succeeds iff the load-factor step is <= limit; the
    'state' records the load factor reached."""
    calls = []

    def step(state, target):
        t_new = target[1][0] / 1e-2
        ok = t_new - state["t"] <= limit + 1e-12
        calls.append((state["t"], t_new, ok))
        new = dict(t=t_new)
        return new, dict(sigma=np.zeros(6), eps=np.zeros(6)), dict(
            converged=ok, mech_converged=True, stagger_iters=1, newton_iters=1, cg_iters=0,
            pcg_iters=0, err=0.0)
    return step, calls


def test_cutback_and_growth_sequence():
    """dt0 = 0.4, limit 0.15, growth 1.5: worked by hand,
    0.4 x, 0.2 x, 0.1 ok | 0.15 ok | 0.225 x, 0.1125 ok | 0.16875 x,
    0.084375 ok | 0.1265625 ok ..."""
    step, calls = _mock_step(0.15)
    out = driver.drive(None, None, 0, dict(t=0.0), ms.uniaxial_mixed(3, 1e-2), dt=0.4,
                       dt_min=1e-6, grow=1.5, step=step)
    ts = [r["t"] for r in out["records"]]
    cuts = [r["cutbacks"] for r in out["records"]]
    assert ts[:5] == pytest.approx([0.1, 0.25, 0.3625, 0.446875, 0.5734375], abs=1e-15)
    assert cuts[:5] == [2, 0, 1, 1, 0]
    assert out["reason"] == driver.REACHED and out["t"] == 1.0 and ts[-1] == 1.0
    # no accepted step is larger than the limit, and every rejected one is
    steps = np.diff([0.0] + ts)
    assert steps.max() <= 0.15 + 1e-12
    assert all((t1 - t0 > 0.15) != ok for t0, t1, ok in calls)
    assert len(calls) == len(ts) + sum(cuts)


def test_floor_stops_the_run():
    step, calls = _mock_step(-1.0)  # every attempt fails
    out = driver.drive(None, None, 0, dict(t=0.0), ms.uniaxial_mixed(3, 1e-2), dt=0.1,
                       dt_min=1e-3, step=step)
    # 0.1 / 2^7 < 1e-3 <= 0.1 / 2^6: seven failed attempts
    assert out["reason"] == driver.FLOOR and out["records"] == [] and len(calls) == 7
    assert out["t"] == 0.0 and out["dt"] == pytest.approx(0.1 / 128)


def test_record_and_attempt_limits():
    step, _ = _mock_step(0.15)
    out = driver.drive(None, None, 0, dict(t=0.0), ms.uniaxial_mixed(3, 1e-2), dt=0.1,
                       max_records=3, step=step)
    assert out["reason"] == driver.RECORDS and len(out["records"]) == 3
    step, _ = _mock_step(0.15)
    out = driver.drive(None, None, 0, dict(t=0.0), ms.uniaxial_mixed(3, 1e-2), dt=0.4,
                       max_attempts=2, step=step)
    assert out["reason"] == driver.ATTEMPTS and out["records"] == []


def test_homogeneous_elastic_path_is_linear():
    """Uniform isotropic elastic RVE under uniaxial stress: every increment is
    accepted without cutback and <sigma11> = E E11, <eps22> = -nu E11 (closed
    form)."""
    S = (4, 6, 8)
    phase = np.zeros(S, np.uint8)
    table = [ms.elastic_phase(70000.0, 0.3, ell=(1.0,))]
    st = staggered.initial_state(S, 3, 1)
    out = driver.drive(phase, table, 1, st, ms.uniaxial_mixed(3, 2e-3), dt=0.25, grow=1.5,
                       cg_tol=1e-12, pcg_tol=1e-12, newton_tol=1e-11, stagger_tol=1e-10)
    ts = [r["t"] for r in out["records"]]
    assert ts == [0.25, 0.625, 1.0] and out["reason"] == driver.REACHED
    for r in out["records"]:
        E11 = 2e-3 * r["t"]
        assert r["sigma"][0] == pytest.approx(70000.0 * E11, rel=1e-10)
        assert r["eps"][1] == pytest.approx(-0.3 * E11, rel=1e-10)
        # the first pass moves the strain off its guess, the second confirms
        assert r["cutbacks"] == 0 and r["stagger_iters"] == 2


def test_split_run_equals_single_run():
    """The position (state, t, dt) is all the driver carries: a run stopped
    half-way and resumed from it repeats the single run exactly."""
    S = (6, 6, 6)
    rng = np.random.default_rng(1)
    phase = (rng.uniform(size=S) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
    kw = dict(dt=0.3, dt_min=1e-2, cg_tol=1e-12, pcg_tol=1e-12, newton_tol=1e-11,
              stagger_tol=1e-8, max_stagger=3)
    tgt = ms.uniaxial_mixed(3, 8e-3)
    one = driver.drive(phase, table, 1, staggered.initial_state(S, 3, 1), tgt, **kw)
    half = driver.drive(phase, table, 1, staggered.initial_state(S, 3, 1), tgt, max_records=2,
                        **kw)
    kw2 = dict(kw, dt=half["dt"])
    rest = driver.drive(phase, table, 1, half["state"], tgt, t0=half["t"], **kw2)
    both = half["records"] + rest["records"]
    assert [r["t"] for r in both] == [r["t"] for r in one["records"]]
    assert all(np.array_equal(a["sigma"], b["sigma"]) for a, b in zip(both, one["records"]))
    assert np.array_equal(rest["state"]["eps"], one["state"]["eps"])
    assert rest["reason"] == one["reason"] and rest["t"] == one["t"]


def test_newton_divergence_guard():
    """With newton_tol = 0 the Newton iteration runs into its rounding floor,
    where the residual goes up and down.  The residual history is read off
    runs without the guard cut after r corrections; the guarded run must stop
    exactly after the first run of `div` consecutive increases, with the same
    iterate."""
    S = (4, 4, 6)
    rng = np.random.default_rng(2)
    phase = (rng.uniform(size=S) < 0.3).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
    D = np.zeros((1,) + S)
    z6, z = np.zeros((6,) + S), np.zeros(S)
    tgt = ms.uniaxial_mixed(3, 2e-3)
    kw = dict(cg_tol=1e-12, newton_tol=0.0)
    K = 12
    hist = [galerkin.fftg_solve(phase, table, D, z6, z, tgt, z6.copy(), newton_maxit=r,
                                **kw)["relres"] for r in range(K + 1)]
    stops = {}
    for div in (1, 2, 3):
        grown, stop = 0, None
        for r in range(1, K + 1):
            grown = grown + 1 if hist[r] > hist[r - 1] else 0
            if grown >= div:
                stop = r
                break
        stops[div] = stop
        g = galerkin.fftg_solve(phase, table, D, z6, z, tgt, z6.copy(), newton_maxit=K,
                                newton_div=div, **kw)
        ref = galerkin.fftg_solve(phase, table, D, z6, z, tgt, z6.copy(),
                                  newton_maxit=K if stop is None else stop, **kw)
        assert g["newton_iters"] == (K if stop is None else stop) and not g["converged"]
        assert np.array_equal(g["eps"], ref["eps"])
    assert stops[1] is not None, hist
