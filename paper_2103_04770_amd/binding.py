"""ctypes binding of libfftg.so (argument marshalling only).

Every entry point of include/fftg.h has a method of the same name on
`Solver`.  Device arrays are torch CUDA tensors (float64, contiguous,
component-major [comp][z][y][x]); phase images are uint8 CUDA tensors.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

# kernel classes of fftg_profile / fftg_kernel_name (FFTG_NKERNELS)
NKERNELS = 17

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB = None

FP64, FP32_REFINED = 0, 1
ROTATED, SPECTRAL = 0, 1
_MODELS = {"elastic": 0, "j2_damage": 1, "elastic_cracking": 2, "gtn": 3}
_GTN_KEYS = ("n", "q1", "q2", "q3", "fC", "fF", "fN", "eN", "sN", "fu")

STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "E_INVALID", -2: "E_UNSUPPORTED", -3: "E_HIP",
          -4: "E_BREAKDOWN", -5: "E_NONFINITE"}


class FFTGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class Grid(ct.Structure):
    _fields_ = [("ndim", ct.c_int), ("n", ct.c_int * 3), ("h", ct.c_double),
                ("scheme", ct.c_int), ("prec", ct.c_int)]


class Phase(ct.Structure):
    _fields_ = [("model", ct.c_int), ("E", ct.c_double), ("nu", ct.c_double),
                ("sy", ct.c_double), ("H", ct.c_double), ("dfield", ct.c_int),
                ("dC", ct.c_double), ("dR", ct.c_double), ("dmax", ct.c_double),
                ("ell", ct.c_double * 4),
                ("n_hard", ct.c_double), ("q1", ct.c_double), ("q2", ct.c_double),
                ("q3", ct.c_double), ("fC", ct.c_double), ("fF", ct.c_double),
                ("fN", ct.c_double), ("eN", ct.c_double), ("sN", ct.c_double),
                ("fu", ct.c_double)]


class Macro(ct.Structure):
    _fields_ = [("mask", ct.c_ubyte * 6), ("E", ct.c_double * 6), ("S", ct.c_double * 6)]


class KrylovOpts(ct.Structure):
    _fields_ = [("tol", ct.c_double), ("maxit", ct.c_int)]


class DriveOpts(ct.Structure):
    _fields_ = [("t", ct.c_double), ("t_end", ct.c_double), ("dt", ct.c_double),
                ("dt_min", ct.c_double), ("dt_max", ct.c_double), ("grow", ct.c_double),
                ("max_attempts", ct.c_int), ("newton_div", ct.c_int), ("reason", ct.c_int),
                ("attempts", ct.c_int)]


class DriveRecord(ct.Structure):
    _fields_ = [("t", ct.c_double), ("homog", ct.c_double * 12), ("err", ct.c_double),
                ("cutbacks", ct.c_int), ("stagger_iters", ct.c_int), ("newton_iters", ct.c_int),
                ("cg_iters", ct.c_int), ("pcg_iters", ct.c_int), ("ms", ct.c_double)]


class Stats(ct.Structure):
    _fields_ = [("newton_iters", ct.c_int), ("cg_iters", ct.c_int), ("pcg_iters", ct.c_int),
                ("stagger_iters", ct.c_int), ("relres", ct.c_double), ("err", ct.c_double),
                ("t_ms", ct.c_double * 4), ("inner_converged", ct.c_int)]

    def as_dict(self):
        return dict(newton_iters=self.newton_iters, cg_iters=self.cg_iters,
                    pcg_iters=self.pcg_iters, stagger_iters=self.stagger_iters,
                    relres=self.relres, err=self.err, t_ms=list(self.t_ms),
                    inner_converged=bool(self.inner_converged))


class BatchItem(ct.Structure):
    _fields_ = [("h", ct.c_void_p), ("phase", ct.c_void_p), ("tab", ct.POINTER(Phase)),
                ("nphase", ct.c_int), ("nfields", ct.c_int), ("state", ct.c_void_p),
                ("target", Macro), ("sigma_out", ct.c_void_p), ("homog_out", ct.c_double * 12),
                ("stats", Stats), ("status", ct.c_int)]


def lib_path():
    return os.path.join(_PKG, "libfftg.so")


def load_library():
    """Load libfftg.so from the package directory; raises if it is not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    p = lib_path()
    if not os.path.exists(p):
        raise ImportError("libfftg.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2103_04770_amd.build)")
    lib = ct.CDLL(p)
    P = ct.c_void_p
    I, D = ct.c_int, ct.c_double
    sig = {
        "fftg_create": [ct.POINTER(Grid), P, ct.POINTER(P)],
        "fftg_destroy": [P],
        "fftg_forward": [P, I, P, P],
        "fftg_inverse": [P, I, P, P],
        "fftg_project": [P, ct.POINTER(Macro), P, P],
        "fftg_constitutive": [P, P, ct.POINTER(Phase), I, I, P, P, P, P, P, P],
        "fftg_apply_galerkin": [P, ct.POINTER(Macro), P, P],
        "fftg_apply_helmholtz": [P, P, P, P],
        "helmholtz_solve": [P, P, P, D, P, ct.POINTER(KrylovOpts), ct.POINTER(Stats)],
        "helmholtz_solve_noalloc": [ct.POINTER(Grid), P, P, P, D, P, ct.POINTER(KrylovOpts),
                                    ct.POINTER(Stats)],
        "fftg_solve": [P, P, ct.POINTER(Phase), I, I, P, P, ct.POINTER(Macro), P, P, P, P,
                       ct.POINTER(KrylovOpts), D, I, ct.POINTER(Stats)],
        "staggered_step": [P, P, ct.POINTER(Phase), I, I, P, ct.POINTER(Macro),
                           ct.POINTER(KrylovOpts), ct.POINTER(KrylovOpts), D, I, D, I, P,
                           ct.POINTER(ct.c_double), ct.POINTER(Stats)],
        "helmholtz_adjoint": [P, P, D, P, P, P, P, ct.POINTER(KrylovOpts), ct.POINTER(Stats)],
        "fftg_solve_adjoint": [P, P, ct.POINTER(Phase), I, I, P, P, ct.POINTER(Macro), P, P, P,
                               P, P, ct.POINTER(KrylovOpts), ct.POINTER(Stats)],
        "fftg_staggered_adjoint": [P, P, ct.POINTER(Phase), I, I, P, P, ct.POINTER(Macro), P, P,
                                   P, P, P, P, ct.POINTER(KrylovOpts), ct.POINTER(KrylovOpts), D,
                                   I, ct.POINTER(Stats)],
        "fftg_increment_adjoint": [P, P, ct.POINTER(Phase), I, I, P, P, ct.POINTER(Macro), P, P,
                                   P, P, P, P, P, P, ct.POINTER(KrylovOpts),
                                   ct.POINTER(KrylovOpts), D, I, ct.POINTER(Stats)],
        "fftg_damage": [P, P, ct.POINTER(Phase), I, I, P, P, P],
        "fftg_damage_adjoint": [P, P, ct.POINTER(Phase), I, I, P, P, P, P],
        "fftg_ell2": [P, P, ct.POINTER(Phase), I, I, P],
        "fftg_phase_sums": [P, P, I, P, ct.POINTER(ct.c_double)],
        "fftg_batch_step": [ct.POINTER(BatchItem), I, I, ct.POINTER(KrylovOpts),
                            ct.POINTER(KrylovOpts), D, I, D, I],
        "fftg_drive": [P, P, ct.POINTER(Phase), I, I, P, ct.POINTER(Macro),
                       ct.POINTER(KrylovOpts), ct.POINTER(KrylovOpts), D, I, D, I,
                       ct.POINTER(DriveOpts), P, ct.POINTER(DriveRecord), I, ct.POINTER(I)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ct.c_int
    lib.fftg_last_error.argtypes = [P]
    lib.fftg_last_error.restype = ct.c_char_p
    lib.helmholtz_noalloc_last_error.argtypes = []
    lib.helmholtz_noalloc_last_error.restype = ct.c_char_p
    lib.fftg_profile.argtypes = [P, I, ct.POINTER(ct.c_double), ct.POINTER(ct.c_longlong)]
    lib.fftg_profile.restype = ct.c_int
    lib.fftg_tile_config.argtypes = [P, ct.POINTER(I), ct.POINTER(I), ct.POINTER(ct.c_double)]
    lib.fftg_tile_config.restype = ct.c_int
    lib.fftg_copy_rate.argtypes = [P, P, P, ct.c_longlong, I, ct.POINTER(ct.c_double)]
    lib.fftg_copy_rate.restype = ct.c_int
    lib.fftg_time_kernel.argtypes = [P, I, I, ct.POINTER(ct.c_double)]
    lib.fftg_time_kernel.restype = ct.c_int
    lib.fftg_kernel_name.argtypes = [I]
    lib.fftg_kernel_name.restype = ct.c_char_p
    _LIB = lib
    return lib


def phase_table(table):
    """Phase dicts (see microstructure) -> ctypes array of fftg_phase."""
    arr = (Phase * len(table))()
    for i, ph in enumerate(table):
        a = arr[i]
        a.model = _MODELS[ph["model"]]
        a.E, a.nu, a.sy, a.H = ph["E"], ph["nu"], ph["sy"], ph["H"]
        a.dfield = int(ph["dfield"])
        a.dC, a.dR, a.dmax = ph["dC"], ph["dR"], ph["dmax"]
        ell = list(ph["ell"]) + [0.0] * (4 - len(ph["ell"]))
        for j in range(4):
            a.ell[j] = float(ell[j])
        if ph["model"] == "gtn":
            for k in _GTN_KEYS:
                setattr(a, "n_hard" if k == "n" else k, float(ph[k]))
    return arr


def _macro(target):
    mask, E, S = target
    m = Macro()
    for k in range(len(mask)):
        m.mask[k] = int(mask[k])
        m.E[k] = float(E[k])
        m.S[k] = float(S[k])
    return m


def _ptr(t, dtype, numel=None, name="array"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))
    return ct.c_void_p(t.data_ptr())


def helmholtz_solve_noalloc(alpha, ell2, abar, h=1.0, scheme=ROTATED, tol=1e-8, maxit=1000,
                            ell2_ref=-1.0, stream=None):
    """Algorithm 2 through the allocation-free entry point (no handle; FP64;
    at most 64^3 voxels).  alpha, ell2, abar: contiguous float64 CUDA tensors
    of the grid's numpy shape (z, y, x) or (y, x); abar in = initial guess,
    out = solution.  Returns the stats dict with "converged"."""
    import torch
    lib = load_library()
    shape = tuple(reversed(alpha.shape))
    nd = len(shape)
    n = list(shape) + [1] * (3 - nd)
    N = int(np.prod(n))
    g = Grid(nd, (ct.c_int * 3)(*n), float(h), int(scheme), FP64)
    st = torch.cuda.current_stream() if stream is None else stream
    stats = Stats()
    f64 = torch.float64
    rc = lib.helmholtz_solve_noalloc(ct.byref(g), ct.c_void_p(st.cuda_stream),
                                     _ptr(alpha, f64, N, "alpha"), _ptr(ell2, f64, N, "ell2"),
                                     float(ell2_ref), _ptr(abar, f64, N, "abar"),
                                     ct.byref(KrylovOpts(tol, maxit)), ct.byref(stats))
    if rc < 0:
        raise FFTGError(rc, lib.helmholtz_noalloc_last_error().decode())
    d = stats.as_dict()
    d["converged"] = rc == 0
    return d


class Solver:
    """One grid, one stream.  shape is (N1, N2) in 2D or (N1, N2, N3) in 3D
    (x first, as in the C ABI); device fields use numpy axis order
    [comp][z][y][x]."""

    def __init__(self, shape, h=1.0, scheme=ROTATED, prec=FP64, stream=None):
        import torch
        self.lib = load_library()
        self.torch = torch
        self.ndim = len(shape)
        n = list(shape) + [1] * (3 - len(shape))
        g = Grid(self.ndim, (ct.c_int * 3)(*n), float(h), int(scheme), int(prec))
        self.n = n
        self.N = int(np.prod(n))
        self.c = 6 if self.ndim == 3 else 3
        self.n1h = n[0] // 2 + 1
        self.Ns = self.n1h * n[1] * n[2]
        self.prec = prec
        st = torch.cuda.current_stream() if stream is None else stream
        self.stream = st
        hnd = ct.c_void_p()
        rc = self.lib.fftg_create(ct.byref(g), ct.c_void_p(st.cuda_stream), ct.byref(hnd))
        if rc != 0:
            raise FFTGError(rc, self.lib.fftg_last_error(None).decode())
        self.h = hnd

    # numpy-order spatial shape
    @property
    def spatial(self):
        return tuple(reversed(self.n[: self.ndim]))

    def close(self):
        if getattr(self, "h", None):
            self.lib.fftg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc < 0:
            raise FFTGError(rc, self.lib.fftg_last_error(self.h).decode())
        return rc == 0

    # ---------------------------------------------------------------- ops
    def fftg_forward(self, x, out):
        ncomp = x.numel() // self.N
        self._check(self.lib.fftg_forward(self.h, ncomp, _ptr(x, self.torch.float64, ncomp * self.N, "in"),
                                          _ptr(out, self.torch.float64, 2 * ncomp * self.Ns, "out")))

    def fftg_inverse(self, x, out):
        ncomp = out.numel() // self.N
        self._check(self.lib.fftg_inverse(self.h, ncomp, _ptr(x, self.torch.float64, 2 * ncomp * self.Ns, "in"),
                                          _ptr(out, self.torch.float64, ncomp * self.N, "out")))

    def fftg_project(self, target, tau, out):
        m = _macro(target)
        f64 = self.torch.float64
        self._check(self.lib.fftg_project(self.h, ct.byref(m), _ptr(tau, f64, self.c * self.N, "tau"),
                                          _ptr(out, f64, self.c * self.N, "out")))

    def fftg_constitutive(self, phase, table, nfields, D, state_n, eps, sigma, state_np1, alpha):
        tab = phase_table(table)
        f64 = self.torch.float64
        self._check(self.lib.fftg_constitutive(
            self.h, _ptr(phase, self.torch.uint8, self.N, "phase"), tab, len(table), nfields,
            _ptr(D, f64, nfields * self.N, "D") if nfields else None,
            _ptr(state_n, f64, 7 * self.N, "state_n"), _ptr(eps, f64, self.c * self.N, "eps"),
            _ptr(sigma, f64, self.c * self.N, "sigma"), _ptr(state_np1, f64, 7 * self.N, "state_np1"),
            _ptr(alpha, f64, nfields * self.N, "alpha") if nfields else None))

    def fftg_apply_galerkin(self, target, p, out):
        m = _macro(target)
        f64 = self.torch.float64
        self._check(self.lib.fftg_apply_galerkin(self.h, ct.byref(m), _ptr(p, f64, self.c * self.N, "p"),
                                                 _ptr(out, f64, self.c * self.N, "out")))

    def fftg_apply_helmholtz(self, ell2, u, out):
        f64 = self.torch.float64
        self._check(self.lib.fftg_apply_helmholtz(self.h, _ptr(ell2, f64, self.N, "ell2"),
                                                  _ptr(u, f64, self.N, "u"), _ptr(out, f64, self.N, "out")))

    def helmholtz_solve(self, alpha, ell2, abar, tol=1e-8, maxit=1000, ell2_ref=-1.0):
        f64 = self.torch.float64
        st = Stats()
        opts = KrylovOpts(tol, maxit)
        ok = self._check(self.lib.helmholtz_solve(self.h, _ptr(alpha, f64, self.N, "alpha"),
                                                  _ptr(ell2, f64, self.N, "ell2"), float(ell2_ref),
                                                  _ptr(abar, f64, self.N, "abar"), ct.byref(opts),
                                                  ct.byref(st)))
        d = st.as_dict()
        d["converged"] = ok
        return d

    def fftg_solve(self, phase, table, nfields, D, state_n, target, eps, sigma, state_np1, alpha,
                   cg_tol=1e-8, cg_maxit=5000, newton_tol=1e-8, newton_maxit=50):
        f64 = self.torch.float64
        tab = phase_table(table)
        m = _macro(target)
        st = Stats()
        opts = KrylovOpts(cg_tol, cg_maxit)
        ok = self._check(self.lib.fftg_solve(
            self.h, _ptr(phase, self.torch.uint8, self.N, "phase"), tab, len(table), nfields,
            _ptr(D, f64, nfields * self.N, "D") if nfields else None,
            _ptr(state_n, f64, 7 * self.N, "state_n"), ct.byref(m),
            _ptr(eps, f64, self.c * self.N, "eps"), _ptr(sigma, f64, self.c * self.N, "sigma"),
            _ptr(state_np1, f64, 7 * self.N, "state_np1"),
            _ptr(alpha, f64, nfields * self.N, "alpha") if nfields else None,
            ct.byref(opts), float(newton_tol), int(newton_maxit), ct.byref(st)))
        d = st.as_dict()
        d["converged"] = ok
        return d

    def staggered_step(self, phase, table, nfields, state, target, sigma_out, cg_tol=1e-8,
                       cg_maxit=5000, pcg_tol=1e-8, pcg_maxit=2000, newton_tol=1e-8,
                       newton_maxit=50, stagger_tol=1e-6, max_stagger=20):
        f64 = self.torch.float64
        tab = phase_table(table)
        m = _macro(target)
        st = Stats()
        hom = (ct.c_double * 12)()
        ok = self._check(self.lib.staggered_step(
            self.h, _ptr(phase, self.torch.uint8, self.N, "phase"), tab, len(table), nfields,
            _ptr(state, f64, (self.c + 7 + 2 * nfields) * self.N, "state"), ct.byref(m),
            ct.byref(KrylovOpts(cg_tol, cg_maxit)), ct.byref(KrylovOpts(pcg_tol, pcg_maxit)),
            float(newton_tol), int(newton_maxit), float(stagger_tol), int(max_stagger),
            _ptr(sigma_out, f64, self.c * self.N, "sigma_out"), hom, ct.byref(st)))
        d = st.as_dict()
        d["converged"] = ok
        c = self.c
        d["sigma_mean"] = np.array(hom[:c])
        d["eps_mean"] = np.array(hom[6:6 + c])
        return d

    def helmholtz_adjoint(self, ell2, abar, gbar, dalpha, dell2, tol=1e-8, maxit=1000,
                          ell2_ref=-1.0):
        """dalpha <- dJ/dalpha = L^-1 gbar (in: initial guess), dell2 <- dJ/dell2."""
        f64 = self.torch.float64
        st = Stats()
        ok = self._check(self.lib.helmholtz_adjoint(
            self.h, _ptr(ell2, f64, self.N, "ell2"), float(ell2_ref), _ptr(abar, f64, self.N, "abar"),
            _ptr(gbar, f64, self.N, "gbar"), _ptr(dalpha, f64, self.N, "dalpha"),
            _ptr(dell2, f64, self.N, "dell2"), ct.byref(KrylovOpts(tol, maxit)), ct.byref(st)))
        d = st.as_dict()
        d["converged"] = ok
        return d

    def fftg_solve_adjoint(self, phase, table, nfields, D, state_n, target, eps, gbar, mu, dD,
                           cg_tol=1e-8, cg_maxit=5000, gsig=None):
        """mu <- (G* K)^-1 G*(gbar + K gsig) at the converged eps; dD <- dJ/dD
        (gbar = dJ/deps, gsig = dJ/dsigma or None)."""
        f64 = self.torch.float64
        tab = phase_table(table)
        m = _macro(target)
        st = Stats()
        ok = self._check(self.lib.fftg_solve_adjoint(
            self.h, _ptr(phase, self.torch.uint8, self.N, "phase"), tab, len(table), nfields,
            _ptr(D, f64, nfields * self.N, "D") if nfields else None,
            _ptr(state_n, f64, 7 * self.N, "state_n"), ct.byref(m),
            _ptr(eps, f64, self.c * self.N, "eps"), _ptr(gbar, f64, self.c * self.N, "gbar"),
            _ptr(gsig, f64, self.c * self.N, "gsig") if gsig is not None else None,
            _ptr(mu, f64, self.c * self.N, "mu"),
            _ptr(dD, f64, nfields * self.N, "dD") if nfields else None,
            ct.byref(KrylovOpts(cg_tol, cg_maxit)), ct.byref(st)))
        d = st.as_dict()
        d["converged"] = ok
        return d

    def fftg_staggered_adjoint(self, phase, table, nfields, state_n, state_np1, target, dell2,
                               lam=None, g_eps=None, g_sig=None, g_abar=None, g_D=None,
                               cg_tol=1e-10, cg_maxit=5000, pcg_tol=1e-10, pcg_maxit=5000,
                               tol=1e-10, maxit=200):
        """dell2 <- dJ/dell2_j(x) of a converged staggered increment (total
        derivative at the fixed point); lam <- the Helmholtz adjoint fields."""
        f64 = self.torch.float64
        n = nfields * self.N
        nst = (self.c + 7 + 2 * nfields) * self.N
        m = _macro(target)
        st = Stats()
        opt = lambda t, k, name: _ptr(t, f64, k, name) if t is not None else None  # noqa: E731
        ok = self._check(self.lib.fftg_staggered_adjoint(
            self.h, _ptr(phase, self.torch.uint8, self.N, "phase"), phase_table(table), len(table),
            nfields, _ptr(state_n, f64, nst, "state_n"), _ptr(state_np1, f64, nst, "state_np1"),
            ct.byref(m), opt(g_eps, self.c * self.N, "g_eps"), opt(g_sig, self.c * self.N, "g_sig"),
            opt(g_abar, n, "g_abar"), opt(g_D, n, "g_D"), _ptr(dell2, f64, n, "dell2"),
            opt(lam, n, "lam"), ct.byref(KrylovOpts(cg_tol, cg_maxit)),
            ct.byref(KrylovOpts(pcg_tol, pcg_maxit)), float(tol), int(maxit), ct.byref(st)))
        d = st.as_dict()
        d["converged"] = ok
        return d

    def fftg_increment_adjoint(self, phase, table, nfields, state_n, state_np1, target, dell2,
                               g_epsp_n, g_kappa_n, g_hist_n, g_sig=None, g_epsp=None,
                               g_kappa=None, g_hist=None, cg_tol=1e-10, cg_maxit=5000,
                               pcg_tol=1e-10, pcg_maxit=5000, tol=1e-10, maxit=200):
        """Adjoint of one converged increment: dell2 <- dJ/dell2_j(x) through
        this increment; g_epsp_n (6, *S), g_kappa_n (*S), g_hist_n (J, *S) <-
        the cotangents of the plastic state and damage history it started
        from, given g_sig (c, *S) and the cotangents g_epsp, g_kappa, g_hist of
        the history it committed."""
        f64 = self.torch.float64
        n = nfields * self.N
        nst = (self.c + 7 + 2 * nfields) * self.N
        m = _macro(target)
        st = Stats()
        opt = lambda t, k, name: _ptr(t, f64, k, name) if t is not None else None  # noqa: E731
        ok = self._check(self.lib.fftg_increment_adjoint(
            self.h, _ptr(phase, self.torch.uint8, self.N, "phase"), phase_table(table), len(table),
            nfields, _ptr(state_n, f64, nst, "state_n"), _ptr(state_np1, f64, nst, "state_np1"),
            ct.byref(m), opt(g_sig, self.c * self.N, "g_sig"), opt(g_epsp, 6 * self.N, "g_epsp"),
            opt(g_kappa, self.N, "g_kappa"), opt(g_hist, n, "g_hist"), _ptr(dell2, f64, n, "dell2"),
            _ptr(g_epsp_n, f64, 6 * self.N, "g_epsp_n"), _ptr(g_kappa_n, f64, self.N, "g_kappa_n"),
            _ptr(g_hist_n, f64, n, "g_hist_n"),
            ct.byref(KrylovOpts(cg_tol, cg_maxit)), ct.byref(KrylovOpts(pcg_tol, pcg_maxit)),
            float(tol), int(maxit), ct.byref(st)))
        d = st.as_dict()
        d["converged"] = ok
        return d

    def fftg_damage(self, phase, table, nfields, abar, hist, D):
        f64 = self.torch.float64
        n = nfields * self.N
        self._check(self.lib.fftg_damage(self.h, _ptr(phase, self.torch.uint8, self.N, "phase"),
                                         phase_table(table), len(table), nfields,
                                         _ptr(abar, f64, n, "abar"), _ptr(hist, f64, n, "hist"),
                                         _ptr(D, f64, n, "D")))

    def fftg_damage_adjoint(self, phase, table, nfields, abar, hist, gD, gabar):
        f64 = self.torch.float64
        n = nfields * self.N
        self._check(self.lib.fftg_damage_adjoint(
            self.h, _ptr(phase, self.torch.uint8, self.N, "phase"), phase_table(table), len(table),
            nfields, _ptr(abar, f64, n, "abar"), _ptr(hist, f64, n, "hist"),
            _ptr(gD, f64, n, "gD"), _ptr(gabar, f64, n, "gabar")))

    def fftg_ell2(self, phase, table, field, ell2):
        self._check(self.lib.fftg_ell2(self.h, _ptr(phase, self.torch.uint8, self.N, "phase"),
                                       phase_table(table), len(table), int(field),
                                       _ptr(ell2, self.torch.float64, self.N, "ell2")))

    def tile_config(self):
        """(yz_code, outer_code, times_ms[8]) chosen by the tile autotuner
        (codes 0..3 = 32, 16, 8, 64 KB tiles)."""
        a, b = ct.c_int(), ct.c_int()
        t = (ct.c_double * 8)()
        self._check(self.lib.fftg_tile_config(self.h, ct.byref(a), ct.byref(b), t))
        return a.value, b.value, list(t)

    def fftg_copy_rate(self, src, dst, reps=20):
        """GB/s of the library's streaming copy src -> dst (same-size tensors)."""
        nb = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() != nb or not (src.is_cuda and dst.is_cuda):
            raise ValueError("fftg_copy_rate: two CUDA tensors of the same byte size")
        out = ct.c_double()
        self._check(self.lib.fftg_copy_rate(self.h, ct.c_void_p(src.data_ptr()),
                                            ct.c_void_p(dst.data_ptr()), nb, int(reps),
                                            ct.byref(out)))
        return out.value

    def fftg_phase_sums(self, phase, nphase, f):
        out = (ct.c_double * nphase)()
        self._check(self.lib.fftg_phase_sums(self.h, _ptr(phase, self.torch.uint8, self.N, "phase"),
                                             int(nphase), _ptr(f, self.torch.float64, self.N, "f"),
                                             out))
        return np.array(out[:])

    def fftg_drive(self, phase, table, nfields, state, target_end, sigma_out, t=0.0, t_end=1.0,
                   dt=0.1, dt_min=1e-5, dt_max=1.0, grow=1.5, max_attempts=1000,
                   max_records=1000, newton_div=3, cg_tol=1e-8, cg_maxit=5000, pcg_tol=1e-8,
                   pcg_maxit=2000, newton_tol=1e-8, newton_maxit=50, stagger_tol=1e-6,
                   max_stagger=20):
        """Variable-increment loading from load factor t towards t_end (see
        fftg_drive in include/fftg.h).  Returns dict(t, dt, reason, attempts,
        converged, records) with one record dict per accepted increment."""
        f64 = self.torch.float64
        tab = phase_table(table)
        m = _macro(target_end)
        o = DriveOpts(float(t), float(t_end), float(dt), float(dt_min), float(dt_max),
                      float(grow), int(max_attempts), int(newton_div), 0, 0)
        recs = (DriveRecord * max(1, int(max_records)))()
        n = ct.c_int(0)
        ok = self._check(self.lib.fftg_drive(
            self.h, _ptr(phase, self.torch.uint8, self.N, "phase"), tab, len(table), nfields,
            _ptr(state, f64, (self.c + 7 + 2 * nfields) * self.N, "state"), ct.byref(m),
            ct.byref(KrylovOpts(cg_tol, cg_maxit)), ct.byref(KrylovOpts(pcg_tol, pcg_maxit)),
            float(newton_tol), int(newton_maxit), float(stagger_tol), int(max_stagger),
            ct.byref(o), _ptr(sigma_out, f64, self.c * self.N, "sigma_out"), recs,
            int(max_records), ct.byref(n)))
        c = self.c
        records = []
        for r in recs[: n.value]:
            records.append(dict(t=r.t, sigma=np.array(r.homog[:c]), eps=np.array(r.homog[6:6 + c]),
                                err=r.err, cutbacks=r.cutbacks, stagger_iters=r.stagger_iters,
                                newton_iters=r.newton_iters, cg_iters=r.cg_iters,
                                pcg_iters=r.pcg_iters, ms=r.ms))
        return dict(t=o.t, dt=o.dt, reason=o.reason, attempts=o.attempts, converged=ok,
                    records=records)

    def profile(self, enable):
        """Per-kernel-class GPU time (HIP events on the handle's stream).
        Returns (ms, launches) accumulated since profiling was last enabled."""
        n = NKERNELS
        ms = (ct.c_double * n)()
        cnt = (ct.c_longlong * n)()
        self._check(self.lib.fftg_profile(self.h, int(bool(enable)), ms, cnt))
        return list(ms), list(cnt)

    def time_kernel(self, name, reps=50):
        """Average milliseconds of one launch of a kernel class, back to back."""
        kid = self.kernel_names().index(name)
        ms = ct.c_double()
        self._check(self.lib.fftg_time_kernel(self.h, kid, int(reps), ct.byref(ms)))
        return ms.value

    def kernel_names(self):
        return [self.lib.fftg_kernel_name(i).decode() for i in range(NKERNELS)]

    # ---------------------------------------------------------------- helpers
    def state_layout(self, nfields):
        """Slices of the packed staggered state [c + 7 + 2J][N]."""
        c, J = self.c, nfields
        return dict(eps=slice(0, c), epsp=slice(c, c + 6), kappa=c + 6,
                    hist=slice(c + 7, c + 7 + J), abar=slice(c + 7 + J, c + 7 + 2 * J))
