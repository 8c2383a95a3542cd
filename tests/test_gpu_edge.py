"""Edge and degenerate cases through the C ABI, against the oracle or the
closed forms they reduce to."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import galerkin, helmholtz, spectral, staggered  # noqa: E402
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


def mech(s, shape, phase, table, J, D, tgt, **kw):
    c = 6 if len(shape) == 3 else 3
    eps = dev(np.zeros((c,) + shape))
    sig = torch.empty((c,) + shape, dtype=torch.float64, device="cuda")
    st1 = torch.empty((7,) + shape, dtype=torch.float64, device="cuda")
    al = torch.empty((max(J, 1),) + shape, dtype=torch.float64, device="cuda") if J else None
    d = s.fftg_solve(dev(phase, torch.uint8), table, J, dev(D) if J else None,
                     dev(np.zeros((7,) + shape)), tgt, eps, sig, st1, al, **kw)
    torch.cuda.synchronize()
    return d, eps.cpu().numpy(), sig.cpu().numpy()


def test_zero_load_gives_zero_fields():
    shape = (8, 8, 8)
    say("zero load")
    s = solver(shape)
    phase = (np.random.default_rng(0).uniform(size=shape) < 0.3).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
    d, eps, sig = mech(s, shape, phase, table, 1, np.zeros((1,) + shape),
                       ms.uniaxial_mixed(3, 0.0))
    assert d["converged"] and d["cg_iters"] == 0
    assert np.abs(eps).max() == 0 and np.abs(sig).max() == 0


def test_pure_stress_control_and_no_damage_fields():
    """mask all 1, nfields = 0: <sigma> = S exactly; matches the oracle."""
    shape = (12, 8, 16)
    say("pure stress control")
    s = solver(shape)
    phase = (np.random.default_rng(1).uniform(size=shape) < 0.3).astype(np.uint8)
    table = [ms.elastic_phase(70000.0, 0.3), ms.elastic_phase(400000.0, 0.2)]
    for t in table:
        t["ell"] = []
    S = np.array([50.0, -20.0, 10.0, 5.0, 0.0, -8.0])
    tgt = (np.ones(6, np.uint8), np.zeros(6), S)
    d, eps, sig = mech(s, shape, phase, table, 0, None, tgt, cg_tol=1e-12, newton_tol=1e-12)
    ref = galerkin.fftg_solve(phase, table, np.zeros((0,) + shape), np.zeros((6,) + shape),
                              np.zeros(shape), tgt, np.zeros((6,) + shape), cg_tol=1e-12,
                              newton_tol=1e-12, nfields=0)
    assert np.allclose(sig.reshape(6, -1).mean(1), S, rtol=0, atol=1e-9)
    assert np.abs(eps - ref["eps"]).max() <= 1e-10 * np.abs(ref["eps"]).max()


def test_helmholtz_zero_length_and_zero_source():
    shape = (16, 12, 8)
    say("helmholtz l=0, alpha=0")
    s = solver(shape)
    a = np.abs(np.random.default_rng(2).standard_normal(shape))
    ab = dev(np.zeros(shape))
    d = s.helmholtz_solve(dev(a), dev(np.zeros(shape)), ab, tol=1e-12)
    assert np.abs(ab.cpu().numpy() - a).max() <= 1e-14 * a.max()
    ab2 = dev(np.ones(shape))
    d = s.helmholtz_solve(dev(np.zeros(shape)), dev(np.full(shape, 4.0)), ab2, tol=1e-12)
    assert d["converged"] and d["pcg_iters"] == 0 and np.abs(ab2.cpu().numpy()).max() == 0


@pytest.mark.parametrize("shape", [(1, 6, 12), (4, 1, 8), (1, 1, 16), (1, 32)])
def test_thin_grids(shape):
    """Degenerate grids (an axis of length 1) against the oracle."""
    say("thin grid", shape)
    s = solver(shape)
    rng = np.random.default_rng(3)
    phase = (rng.uniform(size=shape) < 0.4).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
    c = 6 if len(shape) == 3 else 3
    tgt = ms.uniaxial_mixed(len(shape), 4e-3)
    D = np.zeros((1,) + shape)
    d, eps, sig = mech(s, shape, phase, table, 1, D, tgt, cg_tol=1e-12, newton_tol=1e-11)
    ref = galerkin.fftg_solve(phase, table, D, np.zeros((6,) + shape), np.zeros(shape), tgt,
                              np.zeros((c,) + shape), cg_tol=1e-12, newton_tol=1e-11)
    assert np.abs(eps - ref["eps"]).max() <= 1e-10 * np.abs(ref["eps"]).max()
    a = np.abs(rng.standard_normal(shape))
    ell2 = np.where(phase, 0.01, 4.0)
    ab = dev(np.zeros(shape))
    s.helmholtz_solve(dev(a), dev(ell2), ab, tol=1e-12)
    r = helmholtz.helmholtz_solve(a, ell2, tol=1e-12)
    assert np.abs(ab.cpu().numpy() - r["abar"]).max() <= 1e-10 * r["abar"].max()


@pytest.mark.parametrize("shape", [(256, 256, 256), (512, 512)])
def test_maximum_sizes_transform(shape):
    say("max size transform", shape)
    s = solver(shape)
    x = np.random.default_rng(4).standard_normal((1,) + shape)
    n1h = shape[-1] // 2 + 1
    out = torch.empty((1,) + shape[:-1] + (n1h, 2), dtype=torch.float64, device="cuda")
    s.fftg_forward(dev(x), out)
    got = out.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    ref = np.fft.rfftn(x[0])
    assert np.abs(got[0] - ref).max() <= 1e-12 * np.abs(ref).max()
    back = torch.empty((1,) + shape, dtype=torch.float64, device="cuda")
    s.fftg_inverse(out, back)
    assert np.abs(back.cpu().numpy() - x).max() <= 1e-13 * np.abs(x).max()


def test_invalid_arguments_are_rejected():
    from paper_2103_04770_amd import FFTGError
    shape = (8, 8, 8)
    s = solver(shape)
    phase = np.zeros(shape, np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0])]
    bad_mask = (np.array([2, 1, 1, 1, 1, 1], np.uint8), np.zeros(6), np.zeros(6))
    with pytest.raises(FFTGError) as e:
        mech(s, shape, phase, table, 1, np.zeros((1,) + shape), bad_mask)
    assert e.value.code == -1
    bad_table = [dict(table[0], dfield=3)]
    with pytest.raises(FFTGError) as e:
        mech(s, shape, phase, bad_table, 1, np.zeros((1,) + shape), ms.uniaxial_mixed(3, 1e-3))
    assert e.value.code == -1
    with pytest.raises(TypeError):
        s.helmholtz_solve(dev(np.zeros(shape)).float(), dev(np.zeros(shape)), dev(np.zeros(shape)))


def test_not_converged_is_a_warning_with_last_iterate():
    shape = (16, 16, 16)
    say("maxit=1")
    s = solver(shape)
    rng = np.random.default_rng(5)
    a = np.abs(rng.standard_normal(shape))
    ell2 = np.where(rng.uniform(size=shape) < 0.3, 0.01, 9.0)
    ab = dev(np.zeros(shape))
    d = s.helmholtz_solve(dev(a), dev(ell2), ab, tol=1e-12, maxit=1)
    assert not d["converged"] and d["pcg_iters"] == 1
    # one PCG step from zero: x = (r.z / p.Ap) z with z = M b
    assert np.isfinite(ab.cpu().numpy()).all() and np.abs(ab.cpu().numpy()).max() > 0


def test_non_finite_input_is_reported():
    """A NaN in the frozen damage makes the stress non-finite: FFTG_E_NONFINITE
    (forced from the host; every kernel still runs to completion)."""
    from paper_2103_04770_amd import FFTGError
    shape = (8, 8, 8)
    say("nan damage")
    s = solver(shape)
    phase = np.zeros(shape, np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0])]
    D = np.zeros((1,) + shape)
    D[0, 3, 4, 5] = np.nan
    with pytest.raises(FFTGError) as e:
        mech(s, shape, phase, table, 1, D, ms.uniaxial_mixed(3, 1e-3))
    assert e.value.code == -5


def test_zero_stiffness_is_a_breakdown():
    """Fully damaged material (frozen D = 1, zero tangent) under an imposed
    mean stress: p.Ap = 0 in the first CG step, FFTG_E_BREAKDOWN."""
    from paper_2103_04770_amd import FFTGError
    shape = (8, 8, 8)
    say("zero stiffness")
    s = solver(shape)
    phase = np.zeros(shape, np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0])]
    tgt = (np.ones(6, np.uint8), np.zeros(6), np.array([100.0, 0, 0, 0, 0, 0]))
    with pytest.raises(FFTGError) as e:
        mech(s, shape, phase, table, 1, np.ones((1,) + shape), tgt)
    assert e.value.code == -4


def test_staggered_error_met_with_a_capped_inner_solve_is_not_converged():
    """Algorithm 1 stops on ERR <= TOL, but the increment is only converged
    when the inner solves of its last pass met their own tolerances
    (Algorithm 2's ConjGrad test).  With one PCG iteration per Helmholtz solve
    the staggered error falls below a loose tolerance while every PCG is cut
    at maxit: FFTG_NOT_CONVERGED, inner_converged = 0 (forced from the host)."""
    shape = (12, 12, 12)
    say("capped inner PCG")
    s = solver(shape)
    phase = (np.random.default_rng(6).uniform(size=shape) < 0.3).astype(np.uint8)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
    state = dev(np.zeros((6 + 7 + 2,) + shape))
    sig = torch.empty((6,) + shape, dtype=torch.float64, device="cuda")
    ph = dev(phase, torch.uint8)
    d = s.staggered_step(ph, table, 1, state, ms.uniaxial_mixed(3, 6e-3), sig, pcg_maxit=1,
                         stagger_tol=5e-2, max_stagger=50)
    say("  ", {k: d[k] for k in ("stagger_iters", "err", "pcg_iters", "inner_converged")})
    assert d["err"] <= 5e-2
    assert not d["inner_converged"] and not d["converged"]
    # the same increment with uncapped solves converges
    state.zero_()
    d = s.staggered_step(ph, table, 1, state, ms.uniaxial_mixed(3, 6e-3), sig, stagger_tol=5e-2,
                         max_stagger=50)
    assert d["inner_converged"] and d["converged"]


def test_phase_ids_and_damage_cap_are_validated():
    """A phase id >= nphase anywhere in the phase array (checked on the device)
    and a damage cap dmax >= 1 are FFTG_E_INVALID."""
    from paper_2103_04770_amd import FFTGError
    shape = (8, 8, 8)
    say("phase ids, dmax")
    s = solver(shape)
    table = [ms.matrix_j2_damage(ell=[2.0]), ms.particle_elastic(ell=[1.0])]
    phase = np.zeros(shape, np.uint8)
    phase[7, 7, 7] = 2
    with pytest.raises(FFTGError) as e:
        mech(s, shape, phase, table, 1, np.zeros((1,) + shape), ms.uniaxial_mixed(3, 1e-3))
    assert e.value.code == -1
    phase[7, 7, 7] = 1
    d, _, _ = mech(s, shape, phase, table, 1, np.zeros((1,) + shape), ms.uniaxial_mixed(3, 1e-3))
    assert d["converged"]
    with pytest.raises(FFTGError) as e:
        mech(s, shape, phase, [dict(table[0], dmax=1.0), table[1]], 1, np.zeros((1,) + shape),
             ms.uniaxial_mixed(3, 1e-3))
    assert e.value.code == -1
