"""Batches of independent RVEs (fftg_batch_step): every RVE gets exactly the
result of staggered_step run on its own, and one member matches the
oracle."""
import ctypes as ct
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import staggered  # noqa: E402
from paper_2103_04770_amd import microstructure as ms  # noqa: E402

TOLS = dict(cg_tol=1e-10, pcg_tol=1e-10, newton_tol=1e-10, stagger_tol=1e-8, max_stagger=10)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rves():
    out = []
    for b, (n, vf) in enumerate([(12, 0.2), (16, 0.1), (24, 0.25), (32, 0.15), (48, 0.2),
                                 (16, 0.3)]):
        phase, _, _ = ms.rsa_spheres((n, n, n), 100 + b, radius_range=(2.0, 4.0),
                                     volume_fraction=vf)
        table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
        table[0]["dC"], table[0]["dR"] = 0.002, 0.05
        out.append(dict(shape=(n, n, n), phase=phase, table=table, nfields=1))
    return out


@pytest.mark.parametrize("form", ["fp64", "fp32_refined"])
def test_batch_equals_each_rve_alone(form):
    """Every member of the batch (both precision forms) is bitwise equal to
    the same increments run alone: states, stresses and iteration counts."""
    from paper_2103_04770_amd import FP32_REFINED, FP64, Solver
    from paper_2103_04770_amd.batch import RVEBatch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    prec = FP64 if form == "fp64" else FP32_REFINED
    rves = _rves()
    say("batch of", [r["shape"][0] for r in rves], form)
    batch = RVEBatch(rves, prec=prec)
    loads = [ms.uniaxial_mixed(3, 3e-3), ms.uniaxial_mixed(3, 6e-3)]
    res = [batch.step(tgt, nworkers=3, **TOLS) for tgt in loads]
    torch.cuda.synchronize()
    for i, r in enumerate(rves):
        S = r["shape"]
        s = Solver(tuple(reversed(S)), prec=prec)
        state = torch.zeros((15,) + S, dtype=torch.float64, device="cuda")
        sig = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
        ph = torch.from_numpy(r["phase"]).cuda()
        for k, tgt in enumerate(loads):
            d = s.staggered_step(ph, r["table"], 1, state, tgt, sig, **TOLS)
            assert d["cg_iters"] == res[k][i]["cg_iters"]
            assert d["pcg_iters"] == res[k][i]["pcg_iters"]
            assert np.array_equal(d["sigma_mean"], res[k][i]["sigma_mean"])
        torch.cuda.synchronize()
        assert torch.equal(state, batch.states[i]) and torch.equal(sig, batch.sigmas[i])
        say("rve", i, S, "stagger", [res[k][i]["stagger_iters"] for k in range(2)],
            "s11", res[1][i]["sigma_mean"][0])
    batch.close()


def test_batch_member_matches_oracle():
    from paper_2103_04770_amd.batch import RVEBatch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rves = _rves()[:3]
    batch = RVEBatch(rves)
    tgt = ms.uniaxial_mixed(3, 6e-3)
    tols = dict(cg_tol=1e-12, pcg_tol=1e-12, newton_tol=1e-11, stagger_tol=1e-10, max_stagger=20)
    out = batch.step(tgt, nworkers=3, **tols)
    r = rves[1]
    new, sig, hom, stats = staggered.staggered_step(r["phase"], r["table"], 1,
                                                    staggered.initial_state(r["shape"], 3, 1),
                                                    tgt, **tols)
    say("oracle stagger", stats["stagger_iters"], "gpu", out[1]["stagger_iters"])
    assert stats["converged"] and out[1]["converged"]
    assert np.abs(out[1]["sigma_mean"] - hom["sigma"]).max() <= 1e-9 * np.abs(hom["sigma"]).max()
    eps = batch.states[1][:6].cpu().numpy()
    assert np.abs(eps - new["eps"]).max() <= 1e-9 * np.abs(new["eps"]).max()
    batch.close()


def test_batch_rejects_a_shared_handle():
    from paper_2103_04770_amd import load_library
    from paper_2103_04770_amd.batch import RVEBatch
    from paper_2103_04770_amd.binding import BatchItem, KrylovOpts
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    batch = RVEBatch(_rves()[:1])
    items = (BatchItem * 2)()
    for it in items:
        it.h = batch.solvers[0].h
    lib = load_library()
    rc = lib.fftg_batch_step(items, 2, 2, ct.byref(KrylovOpts(1e-8, 10)),
                             ct.byref(KrylovOpts(1e-8, 10)), 1e-8, 5, 1e-6, 2)
    assert rc == -1
    batch.close()


def test_mixed_batch_of_gurson_and_damage_rves():
    """A batch mixing Gurson RVEs (two non-local fields) and J2-damage RVEs
    (one field): every member bitwise equal to its own staggered_step."""
    from paper_2103_04770_amd import Solver
    from paper_2103_04770_amd.batch import RVEBatch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rves = _rves()[:3]
    for b, n in enumerate((16, 24)):
        phase, _, _ = ms.rsa_spheres((n, n, n), 200 + b, radius_range=(2.0, 4.0),
                                     volume_fraction=0.2)
        table = [ms.matrix_gtn(ell=[2.0, 2.0], fN=0.04, eN=0.02, sN=0.01),
                 ms.particle_elastic(ell=[0.04, 0.04])]
        rves.append(dict(shape=(n, n, n), phase=phase, table=table, nfields=2))
    say("mixed batch", [(r["shape"][0], r["nfields"]) for r in rves])
    batch = RVEBatch(rves)
    tgt = ms.uniaxial_mixed(3, 6e-3)
    res = batch.step(tgt, nworkers=3, **TOLS)
    torch.cuda.synchronize()
    for i, r in enumerate(rves):
        S, J = r["shape"], r["nfields"]
        s = Solver(tuple(reversed(S)))
        state = torch.zeros((6 + 7 + 2 * J,) + S, dtype=torch.float64, device="cuda")
        sig = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
        d = s.staggered_step(torch.from_numpy(r["phase"]).cuda(), r["table"], J, state, tgt, sig,
                             **TOLS)
        torch.cuda.synchronize()
        assert d["cg_iters"] == res[i]["cg_iters"] and d["pcg_iters"] == res[i]["pcg_iters"]
        assert torch.equal(state, batch.states[i]) and torch.equal(sig, batch.sigmas[i])
        s.close()
    batch.close()
