"""The allocation-free Helmholtz solve (helmholtz_solve_noalloc, for callers
that cannot allocate device memory) against the handle-based helmholtz_solve
on the same seeded inputs, through the C ABI: two calls in a row, the second
on a smaller grid (the shared scratch array keeps the first call's contents),
plus the size limit.  Both run the same PCG of Algorithm 2 with the same
kernels in the same order, so the solutions must agree to rounding."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


def _case(shape, seed):
    rng = np.random.default_rng(seed)
    phase = rng.uniform(size=shape) < 0.3
    ell2 = np.where(phase, 0.06 ** 2, 3.0 ** 2)
    alpha = np.where(phase, 0.0, np.abs(rng.standard_normal(shape)) * 1e-2)
    x0 = np.abs(rng.standard_normal(shape)) * 1e-3
    return alpha, ell2, x0


def test_noalloc_matches_handle_solve_two_calls():
    from paper_2103_04770_amd import Solver
    from paper_2103_04770_amd.binding import helmholtz_solve_noalloc
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for shape, seed in (((48, 36, 64), 1), ((12, 18, 16), 2)):
        say("noalloc vs handle", shape)
        alpha, ell2, x0 = _case(shape, seed)
        a_ref = dev(x0)
        s = Solver(tuple(reversed(shape)))
        ref = s.helmholtz_solve(dev(alpha), dev(ell2), a_ref, tol=1e-11, maxit=2000)
        torch.cuda.synchronize()
        s.close()
        a_na = dev(x0)
        got = helmholtz_solve_noalloc(dev(alpha), dev(ell2), a_na, tol=1e-11, maxit=2000)
        torch.cuda.synchronize()
        r, g = a_ref.cpu().numpy(), a_na.cpu().numpy()
        err = float(np.abs(g - r).max() / np.abs(r).max())
        say("  iters handle %d noalloc %d, max rel diff %.2e" % (ref["pcg_iters"], got["pcg_iters"],
                                                                 err))
        assert ref["converged"] and got["converged"]
        assert got["pcg_iters"] == ref["pcg_iters"]
        assert err <= 1e-13


def test_noalloc_rejects_grids_above_its_scratch_limit():
    from paper_2103_04770_amd import FFTGError
    from paper_2103_04770_amd.binding import helmholtz_solve_noalloc
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    shape = (64, 64, 72)  # 294912 voxels > 64^3
    z = torch.zeros(shape, dtype=torch.float64, device="cuda")
    with pytest.raises(FFTGError) as e:
        helmholtz_solve_noalloc(z, z.clone(), z.clone())
    assert e.value.code == -2 and "262144" in str(e.value)
