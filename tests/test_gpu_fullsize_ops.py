"""Element-wise parity of every single operator at the benchmark's full size:
the 128^3 RVE with 25% spheres and two non-local fields (the C3 phase array
and table), through the C ABI, against the oracle applied to the same seeded
inputs.  Bound: 1e-13 of the largest magnitude (FP64 rounding of O(log N)
transform passes), 1e-12 for quantities that go through the return map's
square roots and the tangent.

Sec. 3.2.1 (transforms and the rotated derivative symbols), Sec. 3.2.2
(Galerkin projection with mixed control, the linearised operator G*(K:p)),
Sec. 2.1.2 / 2.2 (return map, consistent tangent, local sources), Sec. 3.2.3
(the Helmholtz operator with per-voxel lengths).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import galerkin, helmholtz, material, spectral, staggered  # noqa: E402
from paper_2103_04770_amd import microstructure as ms  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def c3():
    from paper_2103_04770_amd import Solver
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = ms.workload("spheres_two_fields_128")
    s = Solver(tuple(reversed(w["shape"])))
    yield dict(w=w, s=s, ph=dev(w["phase"], torch.uint8))
    s.close()


def _state_inputs(w, seed):
    """Strain, plastic history and damage of the magnitudes met along the
    benchmark path (strains ~5e-3, plastic strains ~1e-3, damage in [0, 0.6))."""
    rng = np.random.default_rng(seed)
    S = w["shape"]
    eps = rng.standard_normal((6,) + S) * 4e-3
    eps[0] += 5e-3
    epsp = rng.standard_normal((6,) + S) * 1e-3
    epsp[:3] -= epsp[:3].mean(axis=0)
    kap = np.abs(rng.standard_normal(S)) * 5e-3
    D = rng.uniform(0.0, 0.6, size=(w["nfields"],) + S)
    return eps, epsp, kap, D


def test_forward_inverse_six_components_128(c3):
    s, w = c3["s"], c3["w"]
    S = w["shape"]
    say("128^3 forward/inverse, 6 components")
    x = np.random.default_rng(21).standard_normal((6,) + S)
    out = torch.empty((6,) + S[:-1] + (S[-1] // 2 + 1, 2), dtype=torch.float64, device="cuda")
    s.fftg_forward(dev(x), out)
    got = host(out)
    got = got[..., 0] + 1j * got[..., 1]
    ref = np.fft.rfftn(x, axes=(1, 2, 3))
    e = relerr(got, ref)
    say("  forward", e)
    assert e <= 1e-13
    del got, ref
    back = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
    s.fftg_inverse(out, back)
    e = relerr(host(back), x)
    say("  inverse", e)
    assert e <= 1e-13


def test_projection_mixed_control_128(c3):
    s, w = c3["s"], c3["w"]
    S = w["shape"]
    say("128^3 projection, uniaxial mixed-control mask")
    tau = np.random.default_rng(22).standard_normal((6,) + S)
    mask, _, _ = ms.uniaxial_mixed(3, 1e-3)
    out = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
    s.fftg_project((mask, np.zeros(6), np.zeros(6)), dev(tau), out)
    ref = galerkin.project(tau, spectral.projection_symbol(S), np.asarray(mask))
    e = relerr(host(out), ref)
    say("  projection", e)
    assert e <= 1e-13


def test_constitutive_and_tangent_every_voxel_128(c3):
    """The return map of the C3 table (J2 damage matrix, cracking particles)
    on all 2,097,152 voxels, and G*(K:p) with the tangent it stored."""
    s, w, ph = c3["s"], c3["w"], c3["ph"]
    S, J, table = w["shape"], w["nfields"], w["table"]
    say("128^3 constitutive, C3 table")
    eps, epsp, kap, D = _state_inputs(w, 23)
    ref = material.constitutive(eps, epsp, kap, D, w["phase"], table, J)
    sig = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
    st1 = torch.empty((7,) + S, dtype=torch.float64, device="cuda")
    al = torch.empty((J,) + S, dtype=torch.float64, device="cuda")
    s.fftg_constitutive(ph, table, J, dev(D), dev(np.concatenate([epsp, kap[None]])), dev(eps),
                        sig, st1, al)
    e_sig = relerr(host(sig), ref["sigma"])
    st1h = host(st1)
    e_ep, e_k = relerr(st1h[:6], ref["epsp"]), relerr(st1h[6], ref["kappa"])
    e_al = relerr(host(al), ref["alpha"])
    say("  sigma %.2e epsp %.2e kappa %.2e alpha %.2e, plastic voxels %d" % (
        e_sig, e_ep, e_k, e_al, int((ref["kappa"] > kap).sum())))
    assert e_sig <= 1e-13 and e_ep <= 1e-13 and e_k <= 1e-13
    assert e_al <= 1e-12
    assert (ref["kappa"] > kap).sum() > 10000
    assert (ref["alpha"][1] > table[1]["dC"]).sum() > 1000  # cracking sources active
    del st1h
    mask, _, _ = ms.uniaxial_mixed(3, 1e-3)
    p = np.random.default_rng(24).standard_normal((6,) + S)
    out = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
    s.fftg_apply_galerkin((mask, np.zeros(6), np.zeros(6)), dev(p), out)
    refo = galerkin.project(material.apply_tangent(ref["C"], p), spectral.projection_symbol(S),
                            np.asarray(mask))
    e = relerr(host(out), refo)
    say("  G*(K:p)", e)
    assert e <= 1e-12


@pytest.mark.parametrize("field", [0, 1])
def test_apply_helmholtz_c3_lengths_128(c3, field):
    """L u with the per-voxel lengths of field 0 (matrix 3, particles 0.06)
    and field 1 (particles 1.5, matrix 0.03)."""
    s, w = c3["s"], c3["w"]
    S = w["shape"]
    say("128^3 Helmholtz operator, field", field)
    ell2 = staggered.ell2_field(w["phase"], w["table"], field)
    u = np.random.default_rng(25 + field).standard_normal(S)
    out = torch.empty(S, dtype=torch.float64, device="cuda")
    s.fftg_apply_helmholtz(dev(ell2), dev(u), out)
    _, qt = spectral.symbols(S)
    qt = [np.broadcast_to(v, S) for v in qt]
    ref = np.real(spectral.ifftn(helmholtz.operator(spectral.fftn(u), ell2, qt)))
    e = relerr(host(out), ref)
    say("  L u", e)
    assert e <= 1e-13
