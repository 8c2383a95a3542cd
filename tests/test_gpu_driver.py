"""The adaptive load driver (fftg_drive, Sec. 4.2) against the oracle's, and
its checkpoint / resume through LoadDriver."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import driver as odriver, staggered  # noqa: E402
from paper_2103_04770_amd import microstructure as ms  # noqa: E402

TOLS = dict(cg_tol=1e-12, pcg_tol=1e-12, newton_tol=1e-11)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rve(n=8, seed=1, dC=0.001, dR=0.05):
    S = (n, n, n)
    rng = np.random.default_rng(seed)
    phase = (rng.uniform(size=S) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
    table[0]["dC"], table[0]["dR"] = dC, dR
    return S, phase, table


def _solver(S):
    from paper_2103_04770_amd import Solver
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Solver(tuple(reversed(S)))


def _gpu_drive(S, phase, table, tgt, **kw):
    s = _solver(S)
    state = torch.zeros((6 + 7 + 2,) + S, dtype=torch.float64, device="cuda")
    sig = torch.zeros((6,) + S, dtype=torch.float64, device="cuda")
    out = s.fftg_drive(torch.from_numpy(phase).cuda(), table, 1, state, tgt, sig, **kw)
    torch.cuda.synchronize()
    out["state"] = state.cpu().numpy()
    return out


def _compare(g, o, S, label):
    tg = [r["t"] for r in g["records"]]
    to = [r["t"] for r in o["records"]]
    say(label, "gpu t", tg, "reason", g["reason"], "| oracle t", to, "reason", o["reason"])
    say(label, "gpu cut", [r["cutbacks"] for r in g["records"]],
        "oracle cut", [r["cutbacks"] for r in o["records"]])
    assert tg == to
    assert [r["cutbacks"] for r in g["records"]] == [r["cutbacks"] for r in o["records"]]
    assert g["reason"] == o["reason"] and g["t"] == o["t"] and g["dt"] == o["dt"]
    for a, b in zip(g["records"], o["records"]):
        assert np.abs(a["sigma"] - b["sigma"]).max() <= 1e-9 * np.abs(b["sigma"]).max()
        assert np.abs(a["eps"] - b["eps"]).max() <= 1e-10 * np.abs(b["eps"]).max()
    eps_o = o["state"]["eps"]
    assert np.abs(g["state"][:6] - eps_o).max() <= 1e-9 * np.abs(eps_o).max()


def test_drive_cutbacks_match_oracle():
    """Damage sets in early (eps_C = 1e-3) and three staggered passes are not
    enough to converge an increment that starts it: attempts are cut back
    until the run reaches the smallest increment.  Every accept/reject
    decision has a wide margin (rejected ERR >= 7e-7, accepted <= 1e-11
    against a tolerance of 1e-8)."""
    S, phase, table = _rve()
    tgt = ms.uniaxial_mixed(3, 0.02)
    kw = dict(dt=0.3, dt_min=1e-3, max_stagger=3, stagger_tol=1e-8, **TOLS)
    say("drive cutbacks 8^3")
    g = _gpu_drive(S, phase, table, tgt, **kw)
    o = odriver.drive(phase, table, 1, staggered.initial_state(S, 3, 1), tgt, **kw)
    assert o["reason"] == odriver.FLOOR and len(o["records"]) >= 3
    assert not g["converged"]
    _compare(g, o, S, "cutbacks")


def test_drive_to_the_end_matches_oracle():
    """No damage (thresholds out of reach): the driver grows its increment and
    reaches the end of the path."""
    S, phase, table = _rve(n=12, seed=4, dC=1.0, dR=2.0)
    tgt = ms.uniaxial_mixed(3, 0.01)
    kw = dict(dt=0.2, grow=1.5, dt_max=0.3, max_stagger=4, stagger_tol=1e-9, **TOLS)
    say("drive to end 12^3")
    g = _gpu_drive(S, phase, table, tgt, **kw)
    o = odriver.drive(phase, table, 1, staggered.initial_state(S, 3, 1), tgt, **kw)
    assert o["reason"] == odriver.REACHED and g["converged"]
    _compare(g, o, S, "end")


def test_checkpoint_resume_repeats_the_run(tmp_path):
    from paper_2103_04770_amd.driver import LoadDriver
    S, phase, table = _rve(n=8, seed=2, dC=0.004, dR=0.1)
    tgt = ms.uniaxial_mixed(3, 0.012)
    opts = dict(dt_min=1e-2, max_stagger=6, stagger_tol=1e-8, **TOLS)
    ph = torch.from_numpy(phase).cuda()
    say("checkpoint/resume 8^3")
    full = LoadDriver(_solver(S), ph, table, 1, tgt, dt=0.25, **opts)
    full.run()
    ck = str(tmp_path / "drive.npz")
    part = LoadDriver(_solver(S), ph, table, 1, tgt, dt=0.25, **opts)
    part.run(chunk=2, checkpoint=ck)          # runs to the end, checkpoint after each chunk
    assert [r["t"] for r in part.records] == [r["t"] for r in full.records]
    # stop early, then resume from the file with a fresh solver
    first = LoadDriver(_solver(S), ph, table, 1, tgt, dt=0.25, **opts)
    out = first.solver.fftg_drive(ph, table, 1, first.state, first.target_end, first.sigma,
                                  t=0.0, dt=0.25, max_records=2, **opts)
    first.t, first.dt, first.records = out["t"], out["dt"], out["records"]
    first.save(ck)
    resumed = LoadDriver.resume(ck, _solver(S), ph, table, 1, tgt, **opts)
    assert resumed.t == first.t and resumed.dt == first.dt and len(resumed.records) == 2
    resumed.run()
    assert [r["t"] for r in resumed.records] == [r["t"] for r in full.records]
    assert resumed.reason == full.reason
    assert torch.equal(resumed.state, full.state) and torch.equal(resumed.sigma, full.sigma)
    say("records", len(full.records), "reason", full.reason, "t", full.t)


def test_drive_rejects_bad_options():
    from paper_2103_04770_amd import FFTGError
    S, phase, table = _rve(n=4)
    s = _solver(S)
    state = torch.zeros((15,) + S, dtype=torch.float64, device="cuda")
    sig = torch.zeros((6,) + S, dtype=torch.float64, device="cuda")
    ph = torch.from_numpy(phase).cuda()
    for bad in (dict(dt=0.0), dict(dt_min=-1.0), dict(grow=0.5), dict(newton_div=-1)):
        with pytest.raises(FFTGError) as e:
            s.fftg_drive(ph, table, 1, state, ms.uniaxial_mixed(3, 1e-3), sig, **bad)
        assert e.value.code == -1
    # nothing to do: already at the end
    out = s.fftg_drive(ph, table, 1, state, ms.uniaxial_mixed(3, 1e-3), sig, t=1.0)
    assert out["converged"] and out["records"] == [] and out["attempts"] == 0


def test_json_runner_logs_every_increment(tmp_path):
    """python -m paper_2103_04770_amd.run: one JSON line per accepted
    increment, the same responses as the driver called directly."""
    import json
    from paper_2103_04770_amd import run as runmod
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("json runner")
    cfg = runmod.RunConfig(workload="disc2d_32", e11_end=0.01, log=str(tmp_path / "r.jsonl"),
                           checkpoint=str(tmp_path / "r.npz"), chunk=2,
                           driver=dict(dt=0.25, dt_min=1e-3, grow=1.5))
    reason, n = runmod.run(cfg)
    lines = [json.loads(l) for l in open(cfg.log)]
    say("  reason", reason, "increments", n, [round(l["t"], 4) for l in lines])
    assert reason == 0 and n == len(lines) > 0
    assert lines[-1]["t"] == 1.0 and all(len(l["sigma"]) == 3 for l in lines)
    assert all(l["cg_iters"] > 0 and l["galerkin_bytes_per_iter"] > 0 for l in lines)
    # the same path through fftg_drive directly
    from paper_2103_04770_amd import Solver, microstructure as ms
    w = ms.workload("disc2d_32")
    s = Solver(tuple(reversed(w["shape"])))
    state = torch.zeros((3 + 7 + 2,) + w["shape"], dtype=torch.float64, device="cuda")
    sig = torch.zeros((3,) + w["shape"], dtype=torch.float64, device="cuda")
    out = s.fftg_drive(torch.from_numpy(w["phase"]).cuda(), w["table"], 1, state,
                       ms.uniaxial_mixed(2, 0.01), sig, dt=0.25, dt_min=1e-3, grow=1.5,
                       **cfg.tolerances)
    assert [r["t"] for r in out["records"]] == [l["t"] for l in lines]
    for r, l in zip(out["records"], lines):
        assert np.allclose(r["sigma"], l["sigma"], rtol=0, atol=0)


def test_driver_path_gradient_matches_oracle():
    """LoadDriver(keep_states=True).path_gradient(): d<sigma_11>/d ell2
    through the increments the adaptive driver accepted (the second one grown
    by the driver), against the oracle's path gradient along the same
    increments."""
    from oracle import adjoint
    from paper_2103_04770_amd.driver import LoadDriver
    shape = (12, 16)
    rng = np.random.default_rng(21)
    phase = (rng.uniform(size=shape) < 0.25).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0], dC=0.0005, dR=0.02), ms.particle_elastic(ell=[0.5])]
    tols = dict(cg_tol=1e-13, pcg_tol=1e-13, newton_tol=1e-12, stagger_tol=1e-12,
                max_stagger=300)
    s = _solver(shape)
    ph = torch.from_numpy(phase).cuda()
    drv = LoadDriver(s, ph, table, 1, ms.uniaxial_mixed(2, 6e-3), dt=0.4, dt_min=1e-3, grow=1.5,
                     keep_states=True, **tols)
    reason = drv.run(t_end=1.0)
    say("driver path gradient: t", drv.state_t, "reason", reason)
    assert reason == 0 and len(drv.states) == len(drv.records) + 1 >= 3
    dl, per = drv.path_gradient(cg_tol=1e-13, pcg_tol=1e-13, tol=1e-12, maxit=300)
    targets = drv.targets()
    st = staggered.initial_state(shape, 2, 1)
    ostates = [st]
    for tgt in targets:
        st, _, _, stats = staggered.staggered_step(phase, table, 1, st, tgt, **tols)
        assert stats["converged"]
        ostates.append(st)
    g = np.zeros((3,) + shape)
    g[0] = 1.0 / phase.size
    ref = adjoint.path_gradient(phase, table, 1, ostates, targets, g, cg_tol=1e-13,
                                pcg_tol=1e-13, tol=1e-12, maxit=300)
    got = dl.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    rq = adjoint.phase_length_gradient(ref[0], phase, table, 0)
    say("  rel err %.2e" % err, "dJ/dell", per[0], rq)
    assert err <= 1e-7
    assert np.allclose(per[0], rq, rtol=1e-7)


def test_json_runner_gradient_line(tmp_path):
    """RunConfig(gradient=True): after the increment lines, one line with
    d<sigma_11>/d ell per field and phase through the whole run, equal to
    LoadDriver.path_gradient on the same run."""
    import json
    from paper_2103_04770_amd import run as runmod
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    # E11 = 0.004 stays below the loss of stability of this disc (near 0.0057,
    # where the transposed staggered iteration no longer contracts)
    cfg = runmod.RunConfig(workload="disc2d_32", e11_end=0.004, log=str(tmp_path / "g.jsonl"),
                           gradient=True, table_overrides=[{"dC": 0.001, "dR": 0.05}],
                           driver=dict(dt=0.25, dt_min=1e-3, grow=1.5))
    reason, n = runmod.run(cfg)
    lines = [json.loads(l) for l in open(cfg.log)]
    say("json runner gradient", reason, n, lines[-1])
    assert reason == 0 and len(lines) == n + 1
    g = lines[-1]["dJ_dell_by_field"]
    assert lines[-1]["from_t"] == 0.0 and lines[-1]["to_t"] == 1.0
    assert len(g) == 1 and len(g[0]) == 2 and all(np.isfinite(g[0])) and abs(g[0][0]) > 0


def test_drive_fp32_refined_matches_fp64():
    """The adaptive driver on an FP32-refined handle: the same accepted load
    factors as on an FP64 handle (the decisions have wide margins) and
    homogenised stresses within 1e-6 of the FP64 run at every increment."""
    from paper_2103_04770_amd import FP32_REFINED, Solver
    S, phase, table = _rve(n=12, seed=4, dC=0.001, dR=0.05)
    tgt = ms.uniaxial_mixed(3, 0.012)
    kw = dict(dt=0.25, dt_min=1e-3, grow=1.5, max_attempts=40, cg_tol=1e-10, pcg_tol=1e-10,
              newton_tol=1e-9, stagger_tol=1e-6, max_stagger=40)
    res = {}
    for name, prec in (("fp64", None), ("fp32", FP32_REFINED)):
        if not torch.cuda.is_available():
            pytest.skip("no GPU")
        s = Solver(tuple(reversed(S))) if prec is None else Solver(tuple(reversed(S)), prec=prec)
        state = torch.zeros((6 + 7 + 2,) + S, dtype=torch.float64, device="cuda")
        sig = torch.zeros((6,) + S, dtype=torch.float64, device="cuda")
        res[name] = s.fftg_drive(torch.from_numpy(phase).cuda(), table, 1, state, tgt, sig, **kw)
        s.close()
    t64 = [r["t"] for r in res["fp64"]["records"]]
    t32 = [r["t"] for r in res["fp32"]["records"]]
    say("driver fp64 t", t64, res["fp64"]["reason"], "| fp32 t", t32, res["fp32"]["reason"])
    assert t64 == t32 and res["fp64"]["reason"] == res["fp32"]["reason"] == 0
    for a, b in zip(res["fp32"]["records"], res["fp64"]["records"]):
        assert np.abs(a["sigma"] - b["sigma"]).max() <= 1e-6 * np.abs(b["sigma"]).max()
