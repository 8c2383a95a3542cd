"""Parity at the benchmark's full size (128^3, two non-local fields), in the
configuration bench.py times.  The oracle cannot run whole increments at this
size inside a test, so the GPU result is checked with the oracle's own
operators: macro constraints, equilibrium (the oracle's projection of the GPU
stress), the Helmholtz equation (the oracle's operator applied to the GPU
non-local fields), and the constitutive update recomputed by the oracle at
sampled voxels from the GPU strain and state.
"""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import galerkin, helmholtz, material, spectral, staggered  # noqa: E402
from paper_2103_04770_amd import microstructure as ms  # noqa: E402

TOLS = dict(cg_tol=1e-8, pcg_tol=1e-8, newton_tol=1e-8, stagger_tol=1e-6, max_stagger=20)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def run128():
    from paper_2103_04770_amd import Solver, FP64, FP32_REFINED
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = ms.workload("spheres_two_fields_128")
    shape, J = w["shape"], w["nfields"]
    out = {}
    for prec in ("fp64", "fp32"):
        s = Solver(tuple(reversed(shape)), prec=FP64 if prec == "fp64" else FP32_REFINED)
        state = torch.zeros((6 + 7 + 2 * J,) + shape, dtype=torch.float64, device="cuda")
        sig = torch.empty((6,) + shape, dtype=torch.float64, device="cuda")
        ph = torch.from_numpy(w["phase"]).cuda()
        hist = []
        prev = None
        for k in range(3):
            prev = state.detach().cpu().numpy() if k == 2 else prev
            say("128^3", prec, "increment", k)
            d = s.staggered_step(ph, w["table"], J, state, w["load"][k], sig, **TOLS)
            hist.append(d)
        torch.cuda.synchronize()
        out[prec] = dict(stats=hist, state=state.cpu().numpy(), sig=sig.cpu().numpy(),
                         prev=prev)
        s.close()
    out["w"] = w
    return out


def test_macro_constraints(run128):
    w = run128["w"]
    for prec in ("fp64", "fp32"):
        d = run128[prec]["stats"][-1]
        mask, E, S = w["load"][2]
        assert abs(d["eps_mean"][0] - E[0]) <= 1e-15
        assert np.abs(d["sigma_mean"][1:]).max() <= 1e-6 * abs(d["sigma_mean"][0])
        assert d["converged"]


def test_equilibrium_by_oracle_projection(run128):
    """||G*(sigma - Sbar)|| relative to ||sigma|| at the Newton tolerance."""
    w = run128["w"]
    sig = run128["fp64"]["sig"]
    mask, E, S = w["load"][2]
    q = spectral.projection_symbol(w["shape"])
    r = galerkin.project(sig, q, mask)
    sref = galerkin.sigma_ref(w["table"])
    rel = np.sqrt((r * r).sum()) / max(np.sqrt((sig * sig).sum()), sref * np.sqrt(sig[0].size))
    say("equilibrium residual", rel)
    assert rel <= 2e-8


def test_helmholtz_fields_by_oracle_operator(run128):
    """Each non-local field solves its Helmholtz equation with the local
    source the oracle recomputes from the GPU strain and state."""
    w = run128["w"]
    shape, J = w["shape"], w["nfields"]
    st = run128["fp64"]["state"]
    prev = run128["fp64"]["prev"]
    c = 6
    eps = st[:c]
    epsp_n, kap_n = prev[c:c + 6], prev[c + 6]
    hist_n = prev[c + 7:c + 7 + J]
    abar = st[c + 7 + J:]
    D = material.damage_from_nonlocal(w["phase"], w["table"], abar, hist_n)
    loc = material.constitutive(eps, epsp_n, kap_n, D, w["phase"], w["table"], J)
    _, qt = spectral.symbols(shape)
    qt = [np.broadcast_to(v, shape) for v in qt]
    for j in range(J):
        ell2 = staggered.ell2_field(w["phase"], w["table"], j)
        a = loc["alpha"][j]
        if np.abs(a).max() == 0:
            assert np.abs(abar[j]).max() == 0
            continue
        La = np.real(np.fft.ifftn(helmholtz.operator(np.fft.fftn(abar[j]), ell2, qt)))
        rel = np.sqrt(((La - a) ** 2).sum()) / np.sqrt((a * a).sum())
        say("field", j, "Helmholtz residual", rel)
        # the last PCG solved with exactly this source (tolerance 1e-8)
        assert rel <= 1e-7


def test_sampled_constitutive_by_oracle(run128):
    """Sampled voxels: the oracle's return map from the GPU strain, the state
    at t_n and the damage of the final non-local fields reproduces the GPU
    stress.  The GPU stress comes from the last mechanics solve, whose damage
    used the non-local fields of the previous staggered pass: voxels below the
    damage threshold (by a margin) must agree to rounding, the others to the
    staggered tolerance."""
    w = run128["w"]
    J, table = w["nfields"], w["table"]
    st, prev, sig = run128["fp64"]["state"], run128["fp64"]["prev"], run128["fp64"]["sig"]
    c = 6
    rng = np.random.default_rng(0)
    idx = rng.choice(sig[0].size, 4000, replace=False)

    def flat(a):
        return a.reshape(a.shape[0], -1)[:, idx] if a.ndim == 4 else a.reshape(-1)[idx]

    phase = w["phase"].reshape(-1)[idx]
    abar, hist_n = flat(st[c + 7 + J:]), flat(prev[c + 7:c + 7 + J])
    D = material.damage_from_nonlocal(phase, table, abar, hist_n)
    kap_n = flat(prev[c + 6])
    loc = material.constitutive(flat(st[:c]), flat(prev[c:c + 6]), kap_n, D, phase, table, J)
    ref, got = loc["sigma"], flat(sig)
    smax = np.abs(ref).max()
    # driving value of each sampled voxel's own damage field, and its margin
    # below the threshold
    below = np.ones(idx.size, bool)
    for p, ph in enumerate(table):
        sel = phase == p
        j = ph["dfield"]
        a = abar[j][sel]
        if ph["model"] == "elastic_cracking":
            a = np.maximum(hist_n[j][sel], a)
        below[sel] = a < ph["dC"] - 1e-3 * (ph["dR"] - ph["dC"])
    err_all = np.abs(got - ref).max() / smax
    err_und = np.abs(got - ref)[:, below].max() / smax
    say("sampled constitutive: undamaged", int(below.sum()), "err", err_und,
        "| all err", err_all, "| plastic", int((loc["kappa"] > kap_n).sum()))
    assert below.sum() > 1000
    assert err_und <= 1e-12
    assert err_all <= 1e-5
    kap = flat(st[c + 6])
    assert np.abs(kap - loc["kappa"]).max() <= 1e-15 + 1e-12 * loc["kappa"].max()
    assert np.abs(flat(st[c:c + 6]) - loc["epsp"]).max() <= 1e-15 + 1e-12 * np.abs(loc["epsp"]).max()


def test_fp32_refined_homogenised_stress(run128):
    for k in range(3):
        a = run128["fp32"]["stats"][k]["sigma_mean"]
        b = run128["fp64"]["stats"][k]["sigma_mean"]
        err = np.abs(a - b).max() / np.abs(b).max()
        say("increment", k, "fp32-refined vs fp64 homogenised stress", err)
        assert err <= 1e-6


# ---------------------------------------------------------------- adjoints at 128^3
# The differentiation workload's RVE (30 spheres, 128^3, lengths 6.4 / 0.128
# voxels) with the damage thresholds lowered (dC = 5e-4, dR = 0.1) so that
# damage is active within a few increments (D reaches ~0.05 at E11 = 0.004)
# while the staggered fixed point still contracts fast enough to be converged
# to 1e-9 in about ten passes.  The oracle cannot run these
# increments, so the adjoints are checked against a property that holds at any
# size: central differences of the GPU forward itself.
ADJ_TOLS = dict(cg_tol=1e-10, pcg_tol=1e-10, newton_tol=1e-9, stagger_tol=1e-9,
                max_stagger=60)
ADJ_E11 = (2e-3, 4e-3, 6e-3)


def _adj_table(ell=None):
    w = ms.workload("spheres30_128")
    table = [dict(t) for t in w["table"]]
    table[0].update(dC=5e-4, dR=0.1)
    if ell is not None:
        for t, e in zip(table, ell):
            t["ell"] = [e]
    return w, table


def _adj_path(s, ph, table, e11s, state0=None):
    """Runs the increments from state0 (virgin if None); returns the packed
    states before each increment and after the last, and <sigma_11>."""
    S = tuple(ph.shape)
    state = (torch.zeros((6 + 7 + 2,) + S, dtype=torch.float64, device="cuda")
             if state0 is None else state0.clone())
    sig = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
    states = [state.clone()]
    d = None
    for e in e11s:
        t0 = time.perf_counter()
        d = s.staggered_step(ph, table, 1, state, ms.uniaxial_mixed(3, e), sig, **ADJ_TOLS)
        say("    E11 %.3f: %d passes, %d CG, err %.1e, %.1f s" % (
            e, d["stagger_iters"], d["cg_iters"], d["err"], time.perf_counter() - t0))
        assert d["converged"], d
        states.append(state.clone())
    return states, float(d["sigma_mean"][0])


@pytest.fixture(scope="module")
def adj128():
    from paper_2103_04770_amd import Solver
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w, table = _adj_table()
    s = Solver(tuple(reversed(w["shape"])))
    ph = torch.from_numpy(w["phase"]).cuda()
    say("128^3 adjoint path", ADJ_E11)
    states, J = _adj_path(s, ph, table, ADJ_E11)
    yield dict(s=s, ph=ph, w=w, table=table, states=states, J=J)
    s.close()


def _fd(adj, q, rel, e11s, state0):
    ells = [float(t["ell"][0]) for t in adj["table"]]
    hq = rel * ells[q]
    vals = []
    for sgn in (1, -1):
        e = list(ells)
        e[q] += sgn * hq
        _, tab = _adj_table(e)
        say("  fd phase", q, "sign", sgn)
        vals.append(_adj_path(adj["s"], adj["ph"], tab, e11s, state0)[1])
    return (vals[0] - vals[1]) / (2 * hq)


def test_increment_adjoint_128_by_central_differences(adj128):
    """d<sigma_11>/d ell_q of the last increment (E11 0.004 -> 0.006, damage
    active), its starting state held fixed: fftg_staggered_adjoint against
    central differences of that GPU increment (h = 1e-3 ell_q)."""
    from oracle import adjoint  # only to sum per phase
    a = adj128
    s, ph, table, states = a["s"], a["ph"], a["table"], a["states"]
    shape = a["w"]["shape"]
    g = torch.zeros((6,) + shape, dtype=torch.float64, device="cuda")
    g[0] = 1.0 / float(np.prod(shape))
    dl = torch.empty((1,) + shape, dtype=torch.float64, device="cuda")
    d = s.fftg_staggered_adjoint(ph, table, 1, states[-2], states[-1], ms.uniaxial_mixed(3, ADJ_E11[-1]),
                                 dl, g_sig=g, cg_tol=1e-10, pcg_tol=1e-10, tol=1e-9, maxit=100)
    assert d["converged"]
    grad = adjoint.phase_length_gradient(dl[0].cpu().numpy(), a["w"]["phase"], table, 0)
    for q in range(2):
        fd = _fd(a, q, 1e-3, ADJ_E11[-1:], states[-2])
        say("  phase", q, "adjoint %.6e fd %.6e" % (grad[q], fd))
        # J converged to ~1e-9 relative: noise of the difference ~3e-7 / (2 h ell_q),
        # 1e-4 of the matrix derivative, 1e-3 of the particle one (ell 50x smaller)
        assert grad[q] == pytest.approx(fd, rel=(2e-4, 2e-3)[q])


def test_path_gradient_128_by_central_differences(adj128):
    """d<sigma_11>/d ell_matrix after three increments from the virgin state,
    through the plastic history of every increment (autograd.path_gradient),
    against central differences of the whole GPU path; it differs from the
    last increment's own derivative."""
    from oracle import adjoint
    from paper_2103_04770_amd import autograd as ag
    a = adj128
    s, ph, table, states = a["s"], a["ph"], a["table"], a["states"]
    shape = a["w"]["shape"]
    g = torch.zeros((6,) + shape, dtype=torch.float64, device="cuda")
    g[0] = 1.0 / float(np.prod(shape))
    dl, log = ag.path_gradient(s, ph, table, 1, states, [ms.uniaxial_mixed(3, e) for e in ADJ_E11],
                               g, cg_tol=1e-10, pcg_tol=1e-10, tol=1e-9, maxit=100)
    grad = adjoint.phase_length_gradient(dl[0].cpu().numpy(), a["w"]["phase"], table, 0)
    last = torch.empty((1,) + shape, dtype=torch.float64, device="cuda")
    s.fftg_staggered_adjoint(ph, table, 1, states[-2], states[-1], ms.uniaxial_mixed(3, ADJ_E11[-1]),
                             last, g_sig=g, cg_tol=1e-10, pcg_tol=1e-10, tol=1e-9, maxit=100)
    one = adjoint.phase_length_gradient(last[0].cpu().numpy(), a["w"]["phase"], table, 0)
    fd = _fd(a, 0, 1e-3, ADJ_E11, None)
    say("  path passes", [d["stagger_iters"] for d in log], "path %.6e last-only %.6e fd %.6e" % (
        grad[0], one[0], fd))
    assert grad[0] == pytest.approx(fd, rel=2e-4)
    assert abs(one[0] - fd) > 10 * abs(grad[0] - fd)
