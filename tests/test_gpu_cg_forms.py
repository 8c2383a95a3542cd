"""The forms of one Krylov iteration give the same increments to rounding.
Galerkin CG: the default (p.Ap summed in real space by the x pass, forward
outer pass fused with the residual update), the two-pass form
(FFTG_GAL_FUSE=0: forward pass and residual pass apart) and the form with
p.Ap on the half spectrum (FFTG_GAL_XDOT=0).  Helmholtz PCG: the default
(p.Lp from the inverse and x passes, forward pass fused with the residual
update) and the two-pass form (FFTG_HELM_FUSE=0).  The forms order their
sums differently, so the states agree to rounding, not bitwise.  3D (the
fixed-length and the generic outer-axis kernels) and 2D."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2103_04770_amd import microstructure as ms  # noqa: E402

TOLS = dict(cg_tol=1e-11, pcg_tol=1e-11, newton_tol=1e-10, stagger_tol=1e-9, max_stagger=60)
FORMS = [{}, {"FFTG_GAL_FUSE": "0"}, {"FFTG_GAL_XDOT": "0"}, {"FFTG_HELM_FUSE": "0"}]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(shape, env, monkeypatch):
    from paper_2103_04770_amd import FP64, Solver
    for k in ("FFTG_GAL_FUSE", "FFTG_GAL_XDOT", "FFTG_HELM_FUSE"):
        monkeypatch.delenv(k, raising=False)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    d = len(shape)
    if d == 3:
        phase, _, _ = ms.rsa_spheres(shape, 900 + sum(shape), radius_range=(1.5, 3.0),
                                     volume_fraction=0.15)
    else:
        phase = ms.disc_2d(shape, (shape[0] / 2, shape[1] / 2), 0.25 * shape[0])
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
    table[0]["dC"], table[0]["dR"] = 0.002, 0.05
    c = 6 if d == 3 else 3
    s = Solver(tuple(reversed(shape)), prec=FP64)
    state = torch.zeros((c + 7 + 2,) + shape, dtype=torch.float64, device="cuda")
    sig = torch.empty((c,) + shape, dtype=torch.float64, device="cuda")
    ph = torch.from_numpy(phase).cuda()
    out = []
    # the 2D disc softens past E11 ~ 4e-3 (its staggered map stops
    # contracting), so it takes smaller increments
    for e11 in ((3e-3, 5e-3) if d == 3 else (2e-3, 3e-3)):
        tgt = ms.uniaxial_mixed(d, e11)
        out.append(s.staggered_step(ph, table, 1, state, tgt, sig, **TOLS))
    torch.cuda.synchronize()
    s.close()
    return out, state.cpu().numpy(), sig.cpu().numpy()


@pytest.mark.parametrize("shape", [(16, 16, 16), (12, 16, 24), (32, 32)])
def test_cg_forms_agree(shape, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = []
    for env in FORMS:
        runs.append(_run(shape, env, monkeypatch))
        say("CG form", env or "default", shape, [
            (r["converged"], r["inner_converged"], r["stagger_iters"], r["cg_iters"], r["err"])
            for r in runs[-1][0]])
    ref_stats, ref_state, ref_sig = runs[0]
    for env, (stats, state, sig) in zip(FORMS[1:], runs[1:]):
        for a, b in zip(stats, ref_stats):
            assert a["converged"] and b["converged"], env
            assert abs(a["cg_iters"] - b["cg_iters"]) <= 0.02 * b["cg_iters"] + 2, env
            assert abs(a["pcg_iters"] - b["pcg_iters"]) <= 0.02 * b["pcg_iters"] + 2, env
            rel = np.abs(a["sigma_mean"] - b["sigma_mean"]).max() / np.abs(b["sigma_mean"]).max()
            assert rel <= 1e-10, (env, rel)
        scale = np.abs(ref_state).max()
        assert np.abs(state - ref_state).max() <= 1e-9 * scale, env
        assert np.abs(sig - ref_sig).max() <= 1e-9 * np.abs(ref_sig).max(), env
