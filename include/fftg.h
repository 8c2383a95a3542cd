/*
 * fftg.h -- C ABI of the MI355X (gfx950) staggered FFT solver for non-local
 * ductile damage on periodic voxel RVEs.
 *
 * Method: Magri, Lucarini, Lemoine, Adam, Segurado, "An FFT framework for
 * simulating non-local ductile failure in heterogeneous materials" (CMAME).
 *   - fftg_solve      : FFT-Galerkin mechanics with mixed macroscopic control,
 *                       Newton + conjugate gradients (Sec. 3.2.2, eq. weakeq,
 *                       eq. eqdiscrete2, eq. lin_stress).
 *   - helmholtz_solve : generalised Helmholtz equation with a per-voxel length,
 *                       preconditioned CG in Fourier space (Sec. 3.2.3,
 *                       eq. LhelmFourier, eq. preconditioner, Algorithm 2).
 *   - staggered_step  : one load increment of the iterated staggered scheme
 *                       (Sec. 3.2, Algorithm 1).
 *   - fftg_drive      : variable-increment loading with cutback (Sec. 4.2).
 *   - fftg_batch_step : staggered increments of many independent RVEs at once.
 *   - helmholtz_adjoint, fftg_solve_adjoint : gradients of the two solves by
 *                       implicit differentiation at the converged state.
 *
 * Conventions shared by every entry point
 *   Grid       N1 x N2 x N3 voxels (N3 = 1 in 2D plane strain), voxel size h.
 *              Every N_i must be of the form 2^a 3^b, at most 256 in 3D and 512
 *              in 2D, and N1 must be even.  N = N1 N2 N3.
 *   Fields     FP64, contiguous, component-major [comp][z][y][x] (x fastest).
 *   Tensors    Mandel order (11, 22, 33, sqrt2*23, sqrt2*13, sqrt2*12) in 3D,
 *              (11, 22, sqrt2*12) in 2D; c = 6 (3D) or 3 (2D) components.
 *              Macro targets (fftg_macro) and homogenised outputs use the
 *              same Mandel values.
 *   Pointers   Arguments marked "dev" are device pointers owned by the caller
 *              (the library never frees them); "host" pointers are read or
 *              written before the call returns.
 *   Streams    All work is enqueued on the stream given to fftg_create; every
 *              call returns after its host-visible outputs are valid.  One
 *              handle per stream and per host thread.
 *   Errors     No exception crosses the ABI.  FFTG_NOT_CONVERGED is a warning:
 *              outputs hold the last iterate and stats are valid.  Negative
 *              codes leave outputs unspecified; fftg_last_error() explains.
 */
#ifndef FFTG_H
#define FFTG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fftg_handle fftg_handle;

typedef enum {
  FFTG_OK = 0,
  FFTG_NOT_CONVERGED = 1,
  FFTG_E_INVALID = -1,     /* bad argument: null pointer, ndim, mask entry, phase id, ... */
  FFTG_E_UNSUPPORTED = -2, /* grid size with a prime factor other than 2 and 3, odd N1, ... */
  FFTG_E_HIP = -3,         /* a HIP runtime call failed */
  FFTG_E_BREAKDOWN = -4,   /* Krylov breakdown: p.Ap <= 0 (operator not positive) */
  FFTG_E_NONFINITE = -5    /* NaN or Inf met in a Krylov scalar */
} fftg_status;

typedef enum { FFTG_FP64 = 0, FFTG_FP32_REFINED = 1 } fftg_precision;

/* Derivative symbol (Sec. 3.2.1).  ROTATED: Willot's rotated finite-difference
 * scheme, q_j = (2/h) sin(theta_j/2) prod_{m!=j} cos(theta_m/2);
 * SPECTRAL: q_j = theta_j / h. */
typedef enum { FFTG_ROTATED = 0, FFTG_SPECTRAL = 1 } fftg_scheme;

/* Phase models.
 * ELASTIC          isotropic elasticity, never damages.
 * J2_DAMAGE        Lemaitre-type: J2 plasticity with linear hardening
 *                  sy + H eps_p on the effective stress, sigma = (1-D) sigma_eff,
 *                  D = clip((abar - dC)/(dR - dC), 0, dmax) from non-local field
 *                  `dfield`; local source eps_p (Sec. 2.1.2, Sec. 2.2.3).
 * ELASTIC_CRACKING isotropic elasticity with sigma = (1-D) C:eps,
 *                  D = clip((max(hist, abar) - dC)/(dR - dC), 0, dmax); local
 *                  source = Mazars equivalent strain sqrt(sum <e_i>_+^2).  Not in
 *                  the paper: a second damage mechanism with its own field.
 * GTN              non-local Gurson-Tvergaard-Needleman matrix (Sec. 2.1.1 and
 *                  the non-local Gurson extension; appendix A.1): yield
 *                  (q/s0)^2 + 2 q1 f* cosh(3 q2 sm/(2 s0)) - 1 - q3 f*^2 <= 0
 *                  (sm = tr(sigma)/3), normality, matrix plastic strain e0 from
 *                  the plastic work sigma:d eps_p = (1 - f) s0 de0, Aravas
 *                  hardening s0/sy = (s0/sy + 3 mu e0/sy)^n_hard, effective
 *                  porosity f*(f) capped at fu.  It drives TWO non-local fields:
 *                  dfield (source e0) and dfield + 1 (source tr eps_p).  Its
 *                  "damage" is the porosity f, fixed within a mechanics solve by
 *                  the non-local fields (backward Euler of the porosity rate,
 *                  f_{n+1} = (f_n + A_N(ebar) d ebar + d trbar)/(1 + d trbar),
 *                  clamped at 0); f enters the yield function, the stress is not
 *                  scaled.  In the packed state its kappa slot holds e0 and
 *                  hist[dfield] the committed porosity f_n (initial porosity). */
typedef enum {
  FFTG_ELASTIC = 0,
  FFTG_J2_DAMAGE = 1,
  FFTG_ELASTIC_CRACKING = 2,
  FFTG_GTN = 3
} fftg_model;

#define FFTG_MAX_FIELDS 4
#define FFTG_MAX_PHASES 16

typedef struct {
  int ndim;         /* 2 (plane strain) or 3 */
  int n[3];         /* N1 (x), N2 (y), N3 (z); n[2] = 1 when ndim = 2 */
  double h;         /* voxel size (lengths ell are in the same unit) */
  int scheme;       /* fftg_scheme */
  int prec;         /* fftg_precision */
} fftg_grid;

typedef struct {
  int model;                    /* fftg_model */
  double E, nu;                 /* Young's modulus, Poisson ratio */
  double sy, H;                 /* yield stress and linear plastic hardening modulus */
  int dfield;                   /* non-local field driving this phase's damage, -1 none */
  double dC, dR, dmax;          /* damage law thresholds and cap */
  double ell[FFTG_MAX_FIELDS];  /* characteristic length of field j inside this phase */
  /* FFTG_GTN only (ignored otherwise): Aravas hardening exponent n_hard in
   * (0, 1); yield-surface coefficients q1, q2, q3 > 0; coalescence fC < fF;
   * nucleation fN >= 0, mean strain eN, spread sN > 0 (Chu-Needleman); cap
   * fu of f*, with the elastic domain non-empty at f* = fu
   * (1 + q3 fu^2 - 2 q1 fu > 0, fu < q1/q3).  sy is the initial yield stress
   * (> 0); H is not used. */
  double n_hard, q1, q2, q3, fC, fF, fN, eN, sN, fu;
} fftg_phase;

/* Mixed macroscopic control (Sec. 3.1): mask[k] = 1 -> component k is
 * stress-controlled with <sigma>_k = S[k]; mask[k] = 0 -> strain-controlled
 * with <eps>_k = E[k].  Only the first c entries are read. */
typedef struct {
  unsigned char mask[6];
  double E[6];
  double S[6];
} fftg_macro;

/* ConjGrad(A, M, b, TOL) of Algorithm 2: stop when ||r|| <= tol ||b||. */
typedef struct {
  double tol;
  int maxit;
} fftg_krylov_opts;

typedef struct {
  int newton_iters;   /* Newton corrections (CG solves) */
  int cg_iters;       /* Galerkin CG iterations, summed */
  int pcg_iters;      /* Helmholtz PCG iterations, summed over fields */
  int stagger_iters;  /* staggered passes */
  double relres;      /* last Newton residual ratio (fftg_solve) or PCG ratio */
  double err;         /* last staggered error ERR (Algorithm 1 (iii)) */
  double t_ms[4];     /* wall time: constitutive, Galerkin CG, Helmholtz PCG, other */
  int inner_converged; /* staggered_step, fftg_drive: 1 when every inner solve of the
                        * last staggered pass met its stop test (the Newton iteration
                        * of step (i) and each Helmholtz PCG of step (ii)), else 0 */
} fftg_stats;

/* Create a solver for one grid.  `hip_stream` is a hipStream_t (NULL = the
 * default stream).  The handle owns its workspace (spectra, Krylov vectors,
 * tangent, FFT tables, reduction scratch), sized from the grid, until
 * fftg_destroy.  Errors: INVALID (null, ndim), UNSUPPORTED (sizes), HIP.
 * Read from the environment at creation (all default to the form measured
 * fastest; the others give the same iterates, with sums in another order):
 *   FFTG_GAL_XDOT=0   Galerkin CG p.Ap on the half spectrum by the forward
 *                     outer pass instead of in real space by the x pass
 *   FFTG_GAL_FUSE=0   Galerkin forward outer pass and residual update as two
 *                     passes instead of one
 *   FFTG_GAL_FOLD=1   Galerkin scalar steps folded into the passes (with the
 *                     two-pass form)
 *   FFTG_HELM_FUSE=0  Helmholtz p.Lp on the half spectrum and the forward
 *                     pass and residual update as two passes */
fftg_status fftg_create(const fftg_grid* grid, void* hip_stream, fftg_handle** out);
fftg_status fftg_destroy(fftg_handle* h);
/* Text of the last error on this handle (or of the last failed create when h
 * is NULL).  Valid until the next call on the handle. */
const char* fftg_last_error(const fftg_handle* h);

/* Mechanics at frozen damage (Algorithm 1 step (i); Sec. 3.2.2).
 *   phase     dev u8 [N], phase id of every voxel (< nphase)
 *   tab       host [nphase] phase table
 *   D         dev [nfields][N] frozen damage per field (a voxel takes the field
 *             its phase names; for a GTN phase, D[dfield] is the frozen
 *             porosity f); may be NULL when nfields = 0
 *   state_n   dev [7][N]: eps_p (6 Mandel comps) and kappa = eq. plastic strain
 *             at t_n
 *   target    host macro targets at t_{n+1}
 *   eps       dev [c][N]: in = initial guess (its strain-controlled means are
 *             moved to E), out = converged strain
 *   sigma     dev [c][N] out
 *   state_np1 dev [7][N] out: eps_p, kappa at the solution (may alias nothing
 *             else)
 *   alpha     dev [nfields][N] out: local sources (may be NULL if nfields = 0)
 * Newton stops when ||G*(sigma - S)||_2 <= newton_tol max(||sigma||_2,
 * s_ref sqrt(N)) after at least one correction (s_ref = largest yield stress
 * in the table, 1 if none), or after newton_maxit corrections. */
fftg_status fftg_solve(fftg_handle* h, const unsigned char* phase, const fftg_phase* tab,
                       int nphase, int nfields, const double* D, const double* state_n,
                       const fftg_macro* target, double* eps, double* sigma, double* state_np1,
                       double* alpha, const fftg_krylov_opts* cg, double newton_tol,
                       int newton_maxit, fftg_stats* stats);

/* Algorithm 2: solve abar - div(ell2 grad abar) = alpha for one field.
 *   alpha     dev [N] source
 *   ell2      dev [N] squared length per voxel
 *   ell2_ref  preconditioner length^2; <= 0 -> volume mean of ell2
 *   abar      dev [N] in = initial guess, out = solution */
fftg_status helmholtz_solve(fftg_handle* h, const double* alpha, const double* ell2,
                            double ell2_ref, double* abar, const fftg_krylov_opts* opts,
                            fftg_stats* stats);

/* Algorithm 1, one load increment n -> n+1.
 *   state  dev packed [c + 6 + 1 + 2*nfields][N]:
 *          eps (c), eps_p (6), kappa (1), hist (nfields), abar (nfields);
 *          in = state at t_n, out = state at t_{n+1} (written on every return
 *          code >= 0; with FFTG_NOT_CONVERGED it holds the last iterate)
 *   sigma_out  dev [c][N] stress at t_{n+1}
 *   homog_out  host [12]: <sigma> (first c of 6 slots), <eps> (slots 6..6+c)
 * max_stagger_iters = 1 is the "simple staggered" single pass.  The loop
 * stops when ERR <= stagger_tol.  FFTG_OK needs both ERR <= stagger_tol and
 * every inner solve of the last pass at its own tolerance (Algorithm 1 (i),
 * (ii); Algorithm 2's ConjGrad test): a Newton iteration cut at newton_maxit
 * or a Helmholtz PCG cut at its maxit (or stalled at its rounding floor)
 * gives FFTG_NOT_CONVERGED with stats->inner_converged = 0, even when the
 * staggered error passed.
 * Every entry point that takes `phase` checks on the device that each id is
 * below nphase (FFTG_E_INVALID otherwise); a phase with a damage law needs
 * 0 <= dmax < 1. */
fftg_status staggered_step(fftg_handle* h, const unsigned char* phase, const fftg_phase* tab,
                           int nphase, int nfields, double* state, const fftg_macro* target,
                           const fftg_krylov_opts* cg, const fftg_krylov_opts* pcg,
                           double newton_tol, int newton_maxit, double stagger_tol,
                           int max_stagger_iters, double* sigma_out, double* homog_out,
                           fftg_stats* stats);

/* Allocation-free Algorithm 2, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same PCG as helmholtz_solve on an FP64 grid, with
 * no handle: the transform tables, spectra, Krylov vectors, reduction partials
 * and control block live in one static device array of 36 MiB that the
 * library holds on each GPU it runs on until the process ends; the call makes
 * no hipMalloc, hipFree or other device-memory allocation.  Its iterations are launched
 * directly (no HIP graph is instantiated); the call returns after its outputs
 * are valid.
 *   grid      host: as for fftg_create; prec must be FFTG_FP64; at most
 *             262144 voxels (64^3), else FFTG_E_UNSUPPORTED
 *   hip_stream  the hipStream_t to enqueue on (NULL = the default stream)
 *   alpha, ell2, ell2_ref, abar, opts, stats  as helmholtz_solve
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (each call writes all it reads): calls that overlap on one GPU, from
 * several host threads or streams, race and must be serialised by the caller.
 * Tile budgets are the fixed default (no autotuning).  Error text:
 * helmholtz_noalloc_last_error() (per host thread). */
fftg_status helmholtz_solve_noalloc(const fftg_grid* grid, void* hip_stream, const double* alpha,
                                    const double* ell2, double ell2_ref, double* abar,
                                    const fftg_krylov_opts* opts, fftg_stats* stats);
const char* helmholtz_noalloc_last_error(void);

/* ---- adjoints (implicit differentiation at the converged state) ---- */

/* Adjoint of Algorithm 2.  In real space the operator is
 * L u = u + sum_j G_j^T (ell2 G_j u), G_j = F^-1 diag(i q~_j) F, symmetric
 * positive definite.  For abar = L^-1 alpha and a scalar J with
 * gbar = dJ/dabar:
 *   dalpha = dJ/dalpha = L^-1 gbar   (the same PCG as helmholtz_solve)
 *   dell2  = dJ/dell2(x) = -sum_j (G_j dalpha)(x) (G_j abar)(x)
 *   ell2, abar, gbar  dev [N] (abar: the converged solution)
 *   dalpha            dev [N] in = initial guess, out = dJ/dalpha
 *   dell2             dev [N] out
 * FFTG_NOT_CONVERGED: the adjoint PCG stopped at opts->maxit. */
fftg_status helmholtz_adjoint(fftg_handle* h, const double* ell2, double ell2_ref,
                              const double* abar, const double* gbar, double* dalpha,
                              double* dell2, const fftg_krylov_opts* opts, fftg_stats* stats);

/* Adjoint of the mechanics solve at frozen damage (Sec. 3.2.2).  At the
 * converged strain eps of fftg_solve (same phase, tab, D, state_n, target),
 * for a scalar J(eps, sigma) with partial derivatives gbar = dJ/deps and
 * gsig = dJ/dsigma:
 *   mu = (G* K)^-1 G*(gbar + K gsig) on the admissible space (compatible
 *        fluctuations and the means of the stress-controlled components), K
 *        the consistent tangent recomputed at eps, solved by the same CG;
 *   dD_j(x) = dJ/dD_j(x) = (mu(x) - gsig(x)) : sigma(x) / (1 - D_j(x)) on
 *        voxels whose phase has a damage law driven by field j (d sigma / dD
 *        is minus the effective stress), 0 elsewhere.
 *   eps, gbar  dev [c][N];  gsig dev [c][N] or NULL (= 0);  mu dev [c][N]
 *   out;  dD dev [nfields][N] out (may be NULL when nfields = 0).
 * For J = <sigma_11>, gsig = e_11 / N and gbar = 0.
 * Tables with a GTN phase: FFTG_E_UNSUPPORTED (its stress does not depend on
 * the frozen field through a stiffness factor). */
fftg_status fftg_solve_adjoint(fftg_handle* h, const unsigned char* phase, const fftg_phase* tab,
                               int nphase, int nfields, const double* D, const double* state_n,
                               const fftg_macro* target, const double* eps, const double* gbar,
                               const double* gsig, double* mu, double* dD,
                               const fftg_krylov_opts* cg, fftg_stats* stats);

/* Adjoint of a converged staggered increment (Algorithm 1 at its fixed
 * point: mechanics at D(abar), Helmholtz with the sources alpha(eps)).  For a
 * scalar J(eps, sigma, abar, D) with partial derivatives g_eps, g_sig (dev
 * [c][N]), g_abar, g_D (dev [nfields][N]; each may be NULL = 0), returns
 *   dell2  dev [nfields][N]: dJ/dell2_j(x), with the damage feeding back into
 *          the local sources through the mechanics (total derivative at the
 *          fixed point); dJ/d ell_q = 2 ell_q sum over phase q (fftg_phase_sums)
 *   lam    dev [nfields][N] or NULL: the Helmholtz adjoint fields L^-1 z.
 * Linearising both equations, a change of ell2 moves abar by
 * -(I - T)^-1 L^-1 dL abar with the staggered map T = L^-1 alpha' A^-1 G*
 * sigma_eff D' (A = G* K); so dell2_j = -sum_i (G_i lam_j)(G_i abar_j),
 * lam = L^-1 z, where z solves the transposed staggered fixed point
 *   z = h + D' (sigma_eff : A^-1 G*(alpha'^T L^-1 z)),
 *   h = D' ((mu0 - g_sig) : sigma_eff + g_D) + g_abar,  mu0 = A^-1 G*(g_eps + K g_sig),
 * iterated (one Helmholtz PCG per field and one Galerkin CG per pass) until
 * ||z_new - z|| <= tol ||z_new|| or maxit passes (then FFTG_NOT_CONVERGED, as
 * when an inner Krylov solve stops at its own maxit).
 *   state_n    dev packed state at t_n (staggered_step's input)
 *   state_np1  dev packed state at t_{n+1} (its output): eps and abar are read
 * stats: cg_iters, pcg_iters, stagger_iters = passes, err = last change.
 * Sources covered: the J2 damage matrix (d alpha/d eps of its return) and the
 * cracking phase (Mazars equivalent strain, gradient <eps>_+ / alpha).  Tables
 * with a Gurson phase: FFTG_E_UNSUPPORTED. */
fftg_status fftg_staggered_adjoint(fftg_handle* h, const unsigned char* phase,
                                   const fftg_phase* tab, int nphase, int nfields,
                                   const double* state_n, const double* state_np1,
                                   const fftg_macro* target, const double* g_eps,
                                   const double* g_sig, const double* g_abar, const double* g_D,
                                   double* dell2, double* lam, const fftg_krylov_opts* cg,
                                   const fftg_krylov_opts* pcg, double tol, int maxit,
                                   fftg_stats* stats);

/* Adjoint of one converged staggered increment with respect to the squared
 * lengths AND to the history it started from, so that increments can be
 * chained backwards along a load path (Sec. 2.1: the J2 return and its
 * history eps_p, kappa; Sec. 2.2: the particle cracking law and its damage
 * history; Sec. 2.3 and Algorithm 1: the increment).  A functional J depends
 * on this increment through the stress (g_sig), through the committed plastic
 * state eps_p,{n+1}, kappa_{n+1} (g_epsp, g_kappa) and through the committed
 * damage history hist_{n+1} = max(hist_n, abar) (g_hist): the history
 * cotangents a later increment returned.  The call
 *   1. turns g_epsp, g_kappa into a strain cotangent through the derivatives
 *      of the return map at the converged strain, and g_hist into an abar
 *      cotangent where abar is the max (abar >= hist_n),
 *   2. runs fftg_staggered_adjoint's coupled adjoint (dell2, lam) and the
 *      total mechanics adjoint mu = A^-1 G*(g_eps + K g_sig + alpha'^T lam),
 *   3. writes the cotangents of the history the increment started from: on a
 *      J2 damage voxel
 *        g_epsp_n  = (1 - D) C_eff (mu - g_sig) - lam dkappa/deps
 *                    + (I - deps_p/deps)^T g_epsp - dkappa/deps g_kappa
 *        g_kappa_n = (1 - D) dsigma_eff/dkappa_n . (g_sig - mu)
 *                    + lam dkappa/dkappa_n + deps_p/dkappa_n . g_epsp
 *                    + dkappa/dkappa_n g_kappa
 *      (C_eff the consistent tangent of the return, lam of the phase's field);
 *      an elastic or cracking voxel passes g_epsp, g_kappa through unchanged;
 *      and, per field, g_hist_n = g_hist where hist_n > abar, plus
 *      zeta / (dR - dC) on a cracking voxel whose history drives its damage
 *      inside the slope band (zeta = dJ/dD, the total damage cotangent).
 * Summing dell2 over the increments of a path, last to first, feeding each
 * call the g_epsp_n, g_kappa_n of the one after it (g_sig only on the last),
 * gives dJ/dell2 of the whole path.
 *   state_n, state_np1 dev packed states before / after the increment
 *   g_sig      dev [c][N] or NULL;  g_epsp dev [6][N] or NULL (Mandel);
 *   g_kappa    dev [N] or NULL;  g_hist dev [nfields][N] or NULL
 *   dell2      dev [nfields][N] out;  g_epsp_n dev [6][N] out;  g_kappa_n dev [N] out;
 *   g_hist_n   dev [nfields][N] out
 *   cg, pcg, tol, maxit, stats as fftg_staggered_adjoint
 * Tables with a Gurson phase return FFTG_E_UNSUPPORTED (J2 damage with linear
 * hardening, elastic and cracking phases are covered); an inner solve at its
 * cap or the fixed point at maxit gives FFTG_NOT_CONVERGED with the outputs
 * written. */
fftg_status fftg_increment_adjoint(fftg_handle* h, const unsigned char* phase,
                                   const fftg_phase* tab, int nphase, int nfields,
                                   const double* state_n, const double* state_np1,
                                   const fftg_macro* target, const double* g_sig,
                                   const double* g_epsp, const double* g_kappa,
                                   const double* g_hist, double* dell2, double* g_epsp_n,
                                   double* g_kappa_n, double* g_hist_n,
                                   const fftg_krylov_opts* cg, const fftg_krylov_opts* pcg,
                                   double tol, int maxit, fftg_stats* stats);

/* Pieces of the differentiable one-pass chain alpha -> abar -> D -> (eps,
 * sigma) (see paper_2103_04770_amd/autograd.py), all on the handle's grid.
 *   fftg_damage        D dev [nfields][N] from abar, hist dev [nfields][N]
 *                      (eq. non-local_damage_lemaitre; cracking phases take
 *                      max(hist, abar)), the same law staggered_step applies
 *   fftg_damage_adjoint gabar = gD dD/dabar: slope 1/(dR - dC) strictly inside
 *                      (dC, dR) below the cap, where abar drives D; 0 elsewhere
 *   fftg_ell2          ell2 dev [N] = ell_q^2 of `field` on phase q
 *   fftg_phase_sums    out host [nphase] = sum of f dev [N] over each phase
 *                      (dJ/d ell_q = 2 ell_q sum_q dJ/dell2)
 * fftg_damage and fftg_damage_adjoint return FFTG_E_UNSUPPORTED for tables
 * with a GTN phase (its porosity update needs the committed fields too). */
fftg_status fftg_damage(fftg_handle* h, const unsigned char* phase, const fftg_phase* tab,
                        int nphase, int nfields, const double* abar, const double* hist,
                        double* D);
fftg_status fftg_damage_adjoint(fftg_handle* h, const unsigned char* phase, const fftg_phase* tab,
                                int nphase, int nfields, const double* abar, const double* hist,
                                const double* gD, double* gabar);
fftg_status fftg_ell2(fftg_handle* h, const unsigned char* phase, const fftg_phase* tab,
                      int nphase, int field, double* ell2);
fftg_status fftg_phase_sums(fftg_handle* h, const unsigned char* phase, int nphase,
                            const double* f, double* out);

/* ---- adaptive load driver ---- */

/* Variable-increment loading (Sec. 4.2: the strain increment is reduced where
 * the response softens, down to a smallest admissible increment).  The macro
 * target is proportional to a load factor t: E(t) = t E_end on the
 * strain-controlled components, S(t) = t S_end on the stress-controlled ones
 * (mask of target_end).  An attempt t -> t' = min(t + dt, t_end) runs one
 * staggered increment (as staggered_step) that stops early when a mechanics
 * solve fails or Newton's residual grows newton_div times in a row; it is
 * accepted when ERR <= stagger_tol and every inner solve of its last pass
 * converged (the Newton iteration and each Helmholtz PCG; then
 * dt <- min(grow dt, dt_max)).  A rejected attempt restores the state
 * and the stress and halves dt; the run stops once dt < dt_min. */
typedef struct {
  double t;         /* in: load factor of `state`; out: load factor reached */
  double t_end;     /* load factor to reach (t = 1 is target_end itself) */
  double dt;        /* in: first increment to try; out: the next one to try */
  double dt_min;    /* smallest admissible increment (> 0) */
  double dt_max;    /* largest increment (> 0) */
  double grow;      /* growth factor after an accepted increment (>= 1) */
  int max_attempts; /* attempts allowed in this call */
  int newton_div;   /* Newton divergence guard: consecutive residual increases (0 = off) */
  int reason;       /* out: 0 t_end reached, 1 dt < dt_min, 2 attempts used up, 3 records full */
  int attempts;     /* out: attempts made in this call */
} fftg_drive_opts;

typedef struct {
  double t;          /* load factor of the accepted increment */
  double homog[12];  /* <sigma>, <eps> as staggered_step's homog_out */
  double err;        /* staggered error of its last pass */
  int cutbacks;      /* rejected attempts just before it */
  int stagger_iters, newton_iters, cg_iters, pcg_iters;
  double ms;         /* wall time of the accepted attempt */
} fftg_drive_record;

/*   state       dev packed state as in staggered_step; in at opts->t, out at
 *               the last accepted increment
 *   sigma_out   dev [c][N] stress of the last accepted increment (left as
 *               passed in when none was accepted)
 *   records     host [max_records], one per accepted increment; *n_records
 *               of them are written
 * (state, opts->t, opts->dt) is the driver's whole position: a later call
 * with them continues the same run (checkpoint / resume).  Returns FFTG_OK
 * when t_end was reached, FFTG_NOT_CONVERGED when it stopped for another
 * reason (opts->reason); invalid options give FFTG_E_INVALID. */
fftg_status fftg_drive(fftg_handle* h, const unsigned char* phase, const fftg_phase* tab,
                       int nphase, int nfields, double* state, const fftg_macro* target_end,
                       const fftg_krylov_opts* cg, const fftg_krylov_opts* pcg,
                       double newton_tol, int newton_maxit, double stagger_tol,
                       int max_stagger_iters, fftg_drive_opts* opts, double* sigma_out,
                       fftg_drive_record* records, int max_records, int* n_records);

/* ---- batches of independent RVEs ---- */

typedef struct {
  fftg_handle* h;              /* this RVE's handle: own grid, own stream */
  const unsigned char* phase;  /* dev [N] */
  const fftg_phase* tab;       /* host phase table */
  int nphase, nfields;
  double* state;               /* dev packed state (staggered_step layout), in/out */
  fftg_macro target;           /* macro target of this increment */
  double* sigma_out;           /* dev [c][N] out */
  double homog_out[12];        /* out, as staggered_step */
  fftg_stats stats;            /* out */
  int status;                  /* out: this item's staggered_step return code */
} fftg_batch_item;

/* One staggered increment (Algorithm 1) of each of n independent RVEs.
 * Items of one grid, voxel size, derivative scheme, precision, field count
 * and macro mask form a class that advances in lockstep on the handle of its
 * first item (on that handle's stream): every Galerkin CG and Helmholtz PCG
 * iteration is one set of launches over all RVEs of the class, each RVE with
 * its own scalars, stop test and targets, and an RVE that has met its test
 * skipped by every launch.  The class grows that handle's workspace to hold
 * all its RVEs (kept until the handle is destroyed).  nworkers host threads
 * take the classes (and lone items), largest first, so that different
 * classes overlap on the GPU.  FFTG_BATCH_LOCKSTEP=0 in the environment runs
 * every item alone on its own handle and stream instead.  Either way each
 * item gets exactly (bitwise) the result of staggered_step on its own.
 * Every item must have a distinct handle (FFTG_E_INVALID otherwise).
 * Returns FFTG_OK when every item converged, FFTG_NOT_CONVERGED when one did
 * not, else the most negative item code; the per-item codes and error texts
 * (fftg_last_error(item.h)) remain valid.  The handles must not be used by
 * other threads during the call. */
fftg_status fftg_batch_step(fftg_batch_item* items, int n, int nworkers,
                            const fftg_krylov_opts* cg, const fftg_krylov_opts* pcg,
                            double newton_tol, int newton_maxit, double stagger_tol,
                            int max_stagger_iters);

/* ---- single-operator entry points (same kernels as the solvers) ---- */

/* Forward real-to-half-spectrum transform of `ncomp` fields (Sec. 3.2.1):
 * in dev [ncomp][N] real, out dev [ncomp][N3][N2][N1/2+1] complex
 * (interleaved re, im).  Unnormalised: X[k] = sum_x u[x] exp(-i theta.x). */
fftg_status fftg_forward(fftg_handle* h, int ncomp, const double* in, double* out);
/* Inverse of fftg_forward, normalised by 1/N (Hermitian input assumed; the
 * imaginary parts of self-conjugate coefficients are ignored). */
fftg_status fftg_inverse(fftg_handle* h, int ncomp, const double* in, double* out);
/* out = G*(tau) for a real Mandel field (dev [c][N] both), with the mixed
 * control mask of `target` at the zero frequency (Sec. 3.2.2). */
fftg_status fftg_project(fftg_handle* h, const fftg_macro* target, const double* tau,
                         double* out);
/* Constitutive update on the grid (the per-voxel step of fftg_solve):
 * sigma dev [c][N], state_np1 dev [7][N], alpha dev [nfields][N] out; also
 * keeps the consistent tangent inside the handle for fftg_apply_tangent_op. */
fftg_status fftg_constitutive(fftg_handle* h, const unsigned char* phase, const fftg_phase* tab,
                              int nphase, int nfields, const double* D, const double* state_n,
                              const double* eps, double* sigma, double* state_np1,
                              double* alpha);
/* out = G*(K : p) with the tangent of the last fftg_constitutive call;
 * p, out dev [c][N] real; `target` supplies the zero-frequency mask. */
fftg_status fftg_apply_galerkin(fftg_handle* h, const fftg_macro* target, const double* p,
                                double* out);
/* out = L(u) = u - div(ell2 grad u) for real u, out, ell2 dev [N] (the
 * operator of Algorithm 2 taken back to real space). */
fftg_status fftg_apply_helmholtz(fftg_handle* h, const double* ell2, const double* u,
                                 double* out);

/* ---- kernel timing ---- */

#define FFTG_NKERNELS 17
/* Per-kernel-class GPU time, measured with HIP events recorded on the
 * handle's stream around every launch while profiling is on.  Returns (when
 * non-NULL) the milliseconds and launch counts accumulated since profiling was
 * last enabled, then: enable = 1 clears the counters and (re)starts, enable =
 * 0 stops.  Class names: fftg_kernel_name(id), 0 <= id < FFTG_NKERNELS.
 * While profiling, Krylov loops run without HIP graphs, and launches of
 * iterations past convergence (which return at once) are not counted. */
fftg_status fftg_profile(fftg_handle* h, int enable, double* ms, long long* launches);
const char* fftg_kernel_name(int id);
/* Average GPU time of one launch of kernel class `kid`, launched `reps` times
 * back to back on the handle's stream between one pair of HIP events, on the
 * handle's own workspace, zeroed first (the passes do the same work whatever
 * the values).  The workspace contents, the stored tangent included, are lost:
 * fftg_apply_galerkin needs a new fftg_constitutive afterwards. */
fftg_status fftg_time_kernel(fftg_handle* h, int kid, int reps, double* avg_ms);

/* Tile autotuner result of this handle.  At creation the library times the
 * inner y pass and the outer inverse Galerkin pass back to back with tile
 * budgets of 32, 16, 8 and 64 KB (codes 0, 1, 2, 3) and keeps the fastest
 * (another than 32 KB only when >= 3% faster; results are bitwise identical
 * for every choice).  times_ms (may be NULL) receives 8 averages: y pass codes
 * 0..3, then outer pass codes 0..3 (0 where not timed).  The environment
 * variable FFTG_TILE_SHIFT=0|1|2|3 fixes both codes instead of timing. */
fftg_status fftg_tile_config(const fftg_handle* h, int* yz_shift, int* outer_shift,
                             double* times_ms);

/* HBM reference rate: a streaming copy of nbytes (a multiple of 16, both
 * pointers 16-byte aligned, dev) from src to dst with one 16-byte load and
 * store per lane, `reps` back-to-back copies between one event pair on the
 * handle's stream, for a few grid sizes; *gbps = 2 nbytes reps / best time.
 * Use buffers well above the 256 MB last-level cache. */
fftg_status fftg_copy_rate(fftg_handle* h, const void* src, void* dst, long long nbytes, int reps,
                           double* gbps);

#ifdef __cplusplus
}
#endif
#endif /* FFTG_H */
