"""Lockstep classes of fftg_batch_step: RVEs of one grid advance together,
every Galerkin CG and Helmholtz PCG iteration one set of launches over the
whole class.  Each member must stay bitwise equal to its own staggered_step
(states, stresses, iteration counts, staggered errors), also when members
leave the staggered loop after different numbers of passes, carry different
macro targets, need two non-local fields, or fail validation."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2103_04770_amd import microstructure as ms  # noqa: E402

TOLS = dict(cg_tol=1e-10, pcg_tol=1e-10, newton_tol=1e-10, stagger_tol=1e-8, max_stagger=12)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _damage_rves(sizes, seed0):
    out = []
    for b, n in enumerate(sizes):
        vf = 0.08 + 0.04 * (b % 5)
        phase, _, _ = ms.rsa_spheres((n, n, n), seed0 + b, radius_range=(2.0, 4.0),
                                     volume_fraction=vf)
        table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
        table[0]["dC"], table[0]["dR"] = 0.002, 0.05
        out.append(dict(shape=(n, n, n), phase=phase, table=table, nfields=1))
    return out


def _targets(n, e11s):
    """Per-member uniaxial targets, one member with a prescribed transverse
    stress (mixed control with a non-zero stress target)."""
    out = []
    for i in range(n):
        mask, E, S = ms.uniaxial_mixed(3, e11s[i % len(e11s)])
        if i == 1:
            S = S.copy()
            S[1] = 40.0
        out.append((mask, E, S))
    return out


def _alone(r, prec, loads):
    """The increments of one RVE through staggered_step on its own."""
    from paper_2103_04770_amd import Solver
    S, J = r["shape"], r["nfields"]
    s = Solver(tuple(reversed(S)), prec=prec)
    state = torch.zeros((6 + 7 + 2 * J,) + S, dtype=torch.float64, device="cuda")
    sig = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
    ph = torch.from_numpy(r["phase"]).cuda()
    res = [s.staggered_step(ph, r["table"], J, state, tgt, sig, **TOLS) for tgt in loads]
    torch.cuda.synchronize()
    s.close()
    return res, state, sig


def _check_member(i, r, prec, loads, res_b, batch):
    res_a, state, sig = _alone(r, prec, loads)
    for k in range(len(loads)):
        a, b = res_a[k], res_b[k][i]
        for key in ("stagger_iters", "newton_iters", "cg_iters", "pcg_iters", "err", "relres",
                    "inner_converged"):
            assert a[key] == b[key], (i, k, key, a[key], b[key])
        assert np.array_equal(a["sigma_mean"], b["sigma_mean"]), (i, k)
        assert np.array_equal(a["eps_mean"], b["eps_mean"]), (i, k)
    assert torch.equal(state, batch.states[i]) and torch.equal(sig, batch.sigmas[i]), i
    return [res_b[k][i]["stagger_iters"] for k in range(len(loads))]


@pytest.mark.parametrize("form", ["fp64", "fp32_refined"])
def test_lockstep_class_equals_each_rve_alone(form):
    """Two classes (five 16^3 RVEs, three 24^3 RVEs) with per-member targets,
    two increments; every member bitwise equal to its own staggered_step."""
    from paper_2103_04770_amd import FP32_REFINED, FP64
    from paper_2103_04770_amd.batch import RVEBatch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    prec = FP64 if form == "fp64" else FP32_REFINED
    rves = _damage_rves([16, 16, 24, 16, 24, 16, 24, 16], 300)
    n = len(rves)
    say("lockstep classes", [r["shape"][0] for r in rves], form)
    batch = RVEBatch(rves, prec=prec)
    loads = [_targets(n, [3e-3, 2e-3, 4e-3]), _targets(n, [6e-3, 5e-3, 7e-3])]
    res = [batch.step(tg, nworkers=2, **TOLS) for tg in loads]
    torch.cuda.synchronize()
    passes = []
    for i, r in enumerate(rves):
        passes.append(_check_member(i, r, prec, [loads[k][i] for k in range(2)], res, batch))
    say("staggered passes per member:", passes)
    # members left the loop after different numbers of passes
    assert len({p[1] for p in passes}) > 1
    batch.close()


def test_lockstep_equals_rves_on_their_own_streams(monkeypatch):
    """The same batch with FFTG_BATCH_LOCKSTEP=0 (every RVE alone on its own
    handle and stream) gives bitwise the same states and stats."""
    from paper_2103_04770_amd.batch import RVEBatch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rves = _damage_rves([16, 16, 16, 16], 400)
    tg = _targets(len(rves), [4e-3, 6e-3])
    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("FFTG_BATCH_LOCKSTEP", mode)
        batch = RVEBatch(rves)
        res = batch.step(tg, nworkers=2, **TOLS)
        torch.cuda.synchronize()
        out[mode] = (res, [t.clone() for t in batch.states], [t.clone() for t in batch.sigmas])
        batch.close()
    for i in range(len(rves)):
        a, b = out["1"][0][i], out["0"][0][i]
        assert all(a[k] == b[k] for k in ("stagger_iters", "cg_iters", "pcg_iters", "err")), i
        assert torch.equal(out["1"][1][i], out["0"][1][i])
        assert torch.equal(out["1"][2][i], out["0"][2][i])


def test_lockstep_gurson_class():
    """A class of three 16^3 Gurson RVEs (two non-local fields each: six
    Helmholtz systems in one lockstep solve), FP64."""
    from paper_2103_04770_amd import FP64
    from paper_2103_04770_amd.batch import RVEBatch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rves = []
    for b in range(3):
        phase, _, _ = ms.rsa_spheres((16, 16, 16), 500 + b, radius_range=(2.0, 4.0),
                                     volume_fraction=0.15 + 0.05 * b)
        table = [ms.matrix_gtn(ell=[2.0, 2.0], fN=0.04, eN=0.02, sN=0.01),
                 ms.particle_elastic(ell=[0.04, 0.04])]
        rves.append(dict(shape=(16, 16, 16), phase=phase, table=table, nfields=2))
    batch = RVEBatch(rves, prec=FP64)
    loads = [_targets(3, [6e-3, 5e-3])]
    res = [batch.step(loads[0], nworkers=1, **TOLS)]
    torch.cuda.synchronize()
    for i, r in enumerate(rves):
        say("gurson member", i, _check_member(i, r, FP64, [loads[0][i]], res, batch))
    batch.close()


def test_lockstep_class_with_an_invalid_member():
    """A member whose phase array holds an id outside its table fails with
    FFTG_E_INVALID before any solve; the rest of its class is unaffected."""
    from paper_2103_04770_amd import FP64
    from paper_2103_04770_amd.batch import RVEBatch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rves = _damage_rves([16, 16, 16], 600)
    bad = rves[1]["phase"].copy()
    bad[3, 4, 5] = 7
    rves[1] = dict(rves[1], phase=bad)
    batch = RVEBatch(rves, prec=FP64)
    tg = _targets(3, [5e-3])
    res = [batch.step(tg, nworkers=1, strict=False, **TOLS)]
    torch.cuda.synchronize()
    assert res[0][1]["status"] == -1 and "phase id" in res[0][1]["error"]
    for i in (0, 2):
        _check_member(i, rves[i], FP64, [tg[i]], res, batch)
    batch.close()


def test_many_rves_on_concurrent_streams_match_lockstep(monkeypatch):
    """Sixteen FP32-refined RVEs, each alone on its own stream with eight
    worker threads (kernels of different RVEs interleave on the GPU), against
    the same RVEs as lockstep classes: no member fails, and the two runs
    agree bitwise (status, iteration counts, staggered error, states)."""
    from paper_2103_04770_amd import FP32_REFINED
    from paper_2103_04770_amd.batch import RVEBatch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rves = _damage_rves([24, 32, 24, 32] * 4, 700)
    tg = _targets(len(rves), [3e-3, 5e-3])
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("FFTG_BATCH_LOCKSTEP", mode)
        batch = RVEBatch(rves, prec=FP32_REFINED)
        res = [batch.step(tg, nworkers=8, **TOLS) for _ in range(2)]
        torch.cuda.synchronize()
        out[mode] = (res, [t.clone() for t in batch.states])
        batch.close()
    conv = 0
    for i in range(len(rves)):
        for k in range(2):
            a, b = out["0"][0][k][i], out["1"][0][k][i]
            assert a["status"] >= 0 and a["status"] == b["status"], (i, k)
            assert a["cg_iters"] == b["cg_iters"] and a["err"] == b["err"], (i, k)
            conv += a["converged"]
        assert torch.equal(out["0"][1][i], out["1"][1][i]), i
    say("converged increments:", conv, "of", 2 * len(rves))
    assert conv >= len(rves)


def test_folded_scalar_steps_agree_with_scalar_kernels(monkeypatch):
    """The Galerkin CG with its scalar steps folded into the passes
    (FFTG_GAL_FOLD=1) against the default with scalar kernels: a lockstep
    class and a lone RVE through one increment agree to rounding (the partial
    sums are added in another order)."""
    from paper_2103_04770_amd import FP64
    from paper_2103_04770_amd.batch import RVEBatch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rves = _damage_rves([16, 16, 16, 24], 800)
    tg = _targets(len(rves), [4e-3, 5e-3])
    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("FFTG_GAL_FOLD", mode)
        batch = RVEBatch(rves, prec=FP64)
        res = batch.step(tg, nworkers=2, **dict(TOLS, max_stagger=60))
        torch.cuda.synchronize()
        out[mode] = (res, [t.clone() for t in batch.states])
        batch.close()
    for i in range(len(rves)):
        a, b = out["1"][0][i], out["0"][0][i]
        assert a["converged"] and b["converged"], i
        assert abs(a["cg_iters"] - b["cg_iters"]) <= 0.05 * b["cg_iters"] + 2, i
        rel = np.abs(a["sigma_mean"] - b["sigma_mean"]).max() / np.abs(b["sigma_mean"]).max()
        assert rel <= 1e-9, (i, rel)
        e = (out["1"][1][i][:6] - out["0"][1][i][:6]).abs().max().item()
        assert e <= 1e-9 * out["0"][1][i][:6].abs().max().item(), (i, e)
