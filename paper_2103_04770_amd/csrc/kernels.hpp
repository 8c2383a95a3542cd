// Shared declarations between the kernels and the host solver.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "fft_device.hpp"

namespace fftg {

// Grid geometry.  Real fields: [comp][n3][n2][n1]; half spectra:
// [comp][n3][n2][n1h], n1h = n1/2 + 1.
struct Geo {
  int ndim, n1, n2, n3, n1h;
  long long N;   // n1 n2 n3
  long long Ns;  // n1h n2 n3
};

// Per-axis derivative tables (Sec. 3.2.1), packed in one device array:
//   pq[a][k] : projection numerator   ROTATED (2/h) sin(theta/2); SPECTRAL theta/h
//              (zero on the Nyquist frequency for SPECTRAL)
//   gq[a][k] : gradient numerator, as pq but zero on the Nyquist frequency
//   cs[a][k] : ROTATED cos(theta/2) (exactly zero on Nyquist); SPECTRAL 1
// theta = 2 pi k'/n with k' the signed frequency (x axis: 0..n1/2).
template <typename T>
struct Sym {
  const T* base;
  int pq[3], gq[3], cs[3];  // offsets into base
};

// Krylov control block kept in device memory.  The finalize kernels update
// it; every iteration kernel reads it and returns at once when done != 0, so
// that the host can launch iterations in chunks and read it back rarely.
struct KrylovCtl {
  double rz;      // r.z (PCG) or r.r (CG) of the current residual
  double rr;      // r.r of the current residual (stopping test)
  double pAp;
  double alpha;   // step of the current iteration (applied to x lazily)
  double beta;
  double bb;      // ||b||^2
  double tol2;    // tol^2 ||b||^2
  double ell2ref; // preconditioner length^2 (Helmholtz)
  double rrmin;   // smallest r.r seen so far, and the iteration it was seen at
  int itmin;
  int iters, maxit;
  int window;     // stagnation window (0: none)
  int done;       // 0 running, 1 converged, 2 max iterations, 3 breakdown,
                  // 4 non-finite, 5 stagnated (no new smallest residual for
                  // `window` iterations: the rounding floor of FP32 vectors)
  // Galerkin CG with the scalar steps folded into the passes: the state of
  // iteration k lives in slot k & 1 (the pass that writes slot k & 1 reads
  // slot (k & 1) ^ 1 in every workgroup, so no workgroup sees a half-updated
  // value); first = 1 until the first residual pass has run.
  double rzs[2], rrmins[2];
  int its[2], itmins[2];
  int first;
};

struct Mat {
  int model;  // 0 elastic, 1 J2 damage, 2 elastic cracking, 3 Gurson (GTN)
  int dfield;
  double K, mu, sy, H, dC, dR, dmax;
  double ell2[4];
  // Gurson only: hardening exponent, yield-surface coefficients, coalescence,
  // nucleation, cap of f* and the porosity fV at which the surface vanishes
  double n, q1, q2, q3, fC, fF, fN, eN, sN, fu, fV;
};
constexpr int kMaxPhases = 16;  // phases of a material table
struct MatTable {
  int nphase;
  int gtn;  // 1 when some phase is a Gurson matrix
  Mat m[kMaxPhases];
};

constexpr int RED_BLOCKS = 2048;  // largest grid of the pointwise kernels
// Every reduction launcher returns its block count; the finalisers take it.

// ---------------------------------------------------------------- launchers
template <typename T>
void launch_x_r2c(const Plan& p, const cpx<T>* tw, const T* in, cpx<T>* out, long long S,
                  int n1, int n1h, hipStream_t st);
template <typename T, typename TO>
void launch_x_c2r(const Plan& p, const cpx<T>* tw, const cpx<T>* in, TO* out, long long S,
                  int n1, int n1h, T scale, bool acc, hipStream_t st);
template <typename T>
void launch_strided(const Plan& p, const cpx<T>* tw, cpx<T>* data, long long nlines,
                    long long inner, long long ostride, long long es, bool fwd,
                    const KrylovCtl* ctl, hipStream_t st, int sh = 0, long long lps = 0);

// Galerkin CG passes.  Several systems of one grid (RVEs solved in lockstep)
// are stacked: spectra [sys][comp][Ns], tangents [sys][N][8], control blocks
// ctl[sys], partial sums [sys][...] (the int returned is the count per
// system).
template <typename T>
int launch_gal_dir_inv(const Plan& p, const cpx<T>* tw, const Geo& g, int c, bool zouter,
                       cpx<T>* r, cpx<T>* pp, cpx<T>* x, cpx<T>* w, KrylovCtl* ctl,
                       hipStream_t st, int sh = 0, int nsys = 1, int parity = 0,
                       const double* rpart = nullptr, int nbr = 0);
template <typename T>
int launch_gal_dot_fwd(const Plan& p, const cpx<T>* tw, const Geo& g, int c, bool zouter,
                       const cpx<T>* pp, cpx<T>* w, double* partials, const KrylovCtl* ctl,
                       hipStream_t st, int nsys = 1);
// partials (optional): the CG's p . A p summed in real space, [sys][count]
// with count = gal_xdot_count (returned); the forward pass then takes pp =
// nullptr and writes no partials.
template <typename T, typename TT>
int launch_x_fused_gal(const Plan& p, const cpx<T>* tw, const Geo& g, int c, cpx<T>* w,
                       const TT* tan, T scale, const KrylovCtl* ctl, hipStream_t st,
                       int nsys = 1, double* partials = nullptr);
template <typename T>
int gal_xdot_count(const Geo& g, int c);
// Forward outer pass fused with the residual update r <- r - alpha G*(Z(w))
// (alpha in the control blocks), partial sums of weighted |r|^2 [sys][count]
// with count = gal_fwd_resid_count (returned).
template <typename T>
int launch_gal_fwd_resid(const Plan& p, const cpx<T>* tw, const Geo& g, int c, bool zouter,
                         const Sym<T>& sym, const unsigned char* mask6, const cpx<T>* w,
                         cpx<T>* r, double* partials, const KrylovCtl* ctl, hipStream_t st,
                         int nsys = 1);
template <typename T>
int gal_fwd_resid_count(const Plan& p, const Geo& g, int c, bool zouter);
template <typename T>
int launch_gal_resid(const Geo& g, int c, const Sym<T>& sym, const unsigned char* mask6,
                      cpx<T>* r, const cpx<T>* w, double* partials, KrylovCtl* ctl,
                      hipStream_t st, int nsys = 1, int parity = 0,
                      const double* dpart = nullptr, int nbd = 0);
// Folded scalar steps (rpart / dpart given): the inverse pass reads the r.r
// partial sums of the previous residual pass ([sys][gal_resid_count]), the
// residual pass the p.Ap partial sums of the forward pass
// ([sys][gal_dot_count]); the two sets must live in different buffers.
template <typename T>
int gal_dot_count(const Plan& p, const Geo& g, int c, bool zouter);
int gal_resid_count(const Geo& g);
// S_sys (optional): per-system mean stress targets [sys][6] in place of Sbar6;
// partials [sys][2][count].
template <typename T>
int launch_gal_rhs(const Geo& g, int c, const Sym<double>& sym, const unsigned char* mask6,
                    const double* Sbar6, const cpx<double>* sig_hat, cpx<T>* r,
                    double* partials, hipStream_t st, int nsys = 1,
                    const double* S_sys = nullptr);
template <typename T>
void launch_project(const Geo& g, int c, const Sym<T>& sym, const unsigned char* mask6,
                    cpx<T>* data, hipStream_t st);

// Helmholtz PCG passes.  On 3D grids with n2 > 1 (helm_split) the outer
// passes transform two fields instead of three and launch_h_y_split, in
// place of the plain y passes, forms and folds the gradient components.
inline bool helm_split(const Geo& g) { return g.ndim == 3 && g.n2 > 1; }
//
// Several Helmholtz systems of one grid (one per non-local field, solved in
// lockstep) are stacked: scalar spectra [sys][Ns], the gradient buffer
// [comp][sys][Ns], ell2 [sys][N], one control block per system ctl[sys],
// and the reductions return per-system partial counts (partials of system s
// at s * count * nred).  nsys = 1 is the single-system case.
template <typename T>
void launch_h_y_split(const Plan& p, const cpx<T>* tw, const Geo& g, const Sym<T>& sym,
                      cpx<T>* w, bool fwd, const KrylovCtl* ctl, hipStream_t st, int nsys = 1);
// ppart (optional, with update): weighted |p|^2 of the new p, [sys][count]
// with count the returned tiles per system.
template <typename T>
int launch_h_dir_inv(const Plan& p, const cpx<T>* tw, const Geo& g, bool zouter,
                     const Sym<T>& sym, bool update, const cpx<T>* r, cpx<T>* pp, cpx<T>* x,
                     cpx<T>* w, const KrylovCtl* ctl, hipStream_t st, int nsys = 1,
                     double* ppart = nullptr);
// The forward pass fused with the residual update r <- r - alpha L p (alpha
// in the control blocks), partials [sys][2][count] (weighted r.Mr, |r|^2),
// count returned.
template <typename T>
int launch_h_fwd_resid(const Plan& p, const cpx<T>* tw, const Geo& g, bool zouter,
                       const Sym<T>& sym, const cpx<T>* pp, cpx<T>* w, cpx<T>* r,
                       double* partials, const KrylovCtl* ctl, hipStream_t st, int nsys = 1);
template <typename T>
int launch_h_div_fwd(const Plan& p, const cpx<T>* tw, const Geo& g, bool zouter,
                     const Sym<T>& sym, const cpx<T>* pp, cpx<T>* w, cpx<T>* Ap,
                     double* partials, const KrylovCtl* ctl, hipStream_t st, int nsys = 1);
// phase / ptab (optional): ell^2 from a per-phase table ptab [sys][kMaxPhases]
// indexed by the phase array shared by the systems, instead of ell2.
// partials (optional): sum of ell^2 |grad p|^2 per workgroup, [sys][count]
// with count returned.
template <typename T, typename TL>
int launch_x_fused_helm(const Plan& p, const cpx<T>* tw, const Geo& g, cpx<T>* w,
                        const TL* ell2, T scale, const KrylovCtl* ctl, hipStream_t st,
                        int nsys = 1, const unsigned char* phase = nullptr,
                        const TL* ptab = nullptr, double* partials = nullptr);
template <typename T>
int launch_h_resid(const Geo& g, const Sym<T>& sym, bool init, cpx<T>* r, const cpx<T>* b,
                   const cpx<T>* Ap, double* partials, const KrylovCtl* ctl, hipStream_t st,
                   int nsys = 1);

// Krylov scalars: one workgroup per system (partials of system s at s * nb,
// or s * nred * nb)
void launch_fin_alpha(double* partials, int nb, KrylovCtl* ctl, hipStream_t st, int nsys = 1);
void launch_fin_alpha2(const double* pa, int na, const double* pb, int nb, KrylovCtl* ctl,
                       hipStream_t st, int nsys = 1);
void launch_fin_beta(double* partials, int nb, int nred, KrylovCtl* ctl, hipStream_t st,
                     int nsys = 1);
void launch_fin_sums(const double* partials, int nb, int nred, double* out, hipStream_t st);

// adjoint helpers (FP64)
template <typename T>
void launch_grad_comp(const Geo& g, const Sym<T>& sym, int j, const cpx<T>* in, cpx<T>* out,
                      hipStream_t st);
void launch_sub_prod(long long n, const double* a, const double* b, double* out, bool acc,
                     hipStream_t st);
void launch_scale(long long n, double s, const double* x, double* y, hipStream_t st);
void launch_adj_damage(const MatTable& tab, long long N, int c, int J,
                       const unsigned char* phase, const double* D, const double* sigma,
                       const double* mu, const double* gsig, double* dD, hipStream_t st);
void launch_damage_adj(const MatTable& tab, long long N, int J, const unsigned char* phase,
                       const double* abar, const double* hist, const double* gD, double* gabar,
                       hipStream_t st);
int launch_phase_sums(long long N, int nphase, const unsigned char* phase, const double* f,
                      double* partials, hipStream_t st);
int launch_count_bad_phase(long long N, int nphase, const unsigned char* phase,
                           double* partials, hipStream_t st);
template <typename TT>
void launch_tangent_apply(long long N, int c, const TT* tan, const double* gsig,
                          const double* gin, double* gout, hipStream_t st);
// x += alpha p per system: n elements each, nsys systems back to back
template <typename T>
void launch_xfinal(cpx<T>* x, const cpx<T>* p, long long n, const KrylovCtl* ctl,
                   hipStream_t st, int nsys = 1);
template <typename T>
void launch_hermitize(const Geo& g, int ncomp, cpx<T>* d, hipStream_t st);
template <typename T>
int launch_wnorm2(const Geo& g, int ncomp, const cpx<T>* a, double* partials, hipStream_t st,
                  int nsys = 1);

// grid-space kernels (FP64)
template <typename TT>
void launch_constitutive(const MatTable& tab, const Geo& g, int c, int J,
                         const unsigned char* phase, const double* eps, const double* state_n,
                         const double* D, double* sigma, double* state_np1, double* alpha,
                         TT* tan, hipStream_t st);
void launch_damage(const MatTable& tab, long long N, int J, const unsigned char* phase,
                   const double* abar, const double* hist, const double* abar_n, double* D,
                   hipStream_t st);
void launch_source_adj(const MatTable& tab, long long N, int c, int J, const unsigned char* phase,
                       const double* eps, const double* state_n, const double* lam, double* out,
                       hipStream_t st);
void launch_stream_copy(const void* src, void* dst, long long n16, int blocks, hipStream_t st);
void launch_hist_out_cot(const MatTable& tab, long long N, int c, const unsigned char* phase,
                         const double* eps, const double* state_n, const double* g_epsp,
                         const double* g_kappa, double* g_eps, hipStream_t st);
void launch_hist_in_cot(const MatTable& tab, long long N, int c, int J, const unsigned char* phase,
                        const double* eps, const double* state_n, const double* D,
                        const double* mu, const double* g_sig, const double* lam,
                        const double* g_epsp, const double* g_kappa, double* g_epsp_n,
                        double* g_kappa_n, hipStream_t st);
void launch_hist_split(long long n, const double* abar, const double* hist_n,
                       const double* g_hist, double* g_abar, hipStream_t st);
void launch_hist_damage_cot(const MatTable& tab, long long N, int J, const unsigned char* phase,
                            const double* abar, const double* hist_n, const double* zeta,
                            const double* g_hist, double* g_hist_n, hipStream_t st);
int launch_diff2(long long n, const double* a, const double* b, double* partials, hipStream_t st);
void launch_axpby(long long n, double a, const double* x, double b, const double* y, double* out,
                  hipStream_t st);
void launch_commit_hist(const MatTable& tab, long long N, int J, const unsigned char* phase,
                        const double* abar, const double* abar_n, double* hist, hipStream_t st);
template <typename TL>
void launch_ell2(const MatTable& tab, long long N, int j, const unsigned char* phase, TL* ell2,
                 hipStream_t st);
int launch_comp_sums(long long N, int ncomp, const double* f, double* partials,
                      hipStream_t st);
void launch_add_const(long long N, int ncomp, double* f, const double* delta6,
                      hipStream_t st);
int launch_stagger_err(long long N, int c, int J, const double* eps_new, const double* eps_old,
                        const double* ab_new, const double* ab_old, double* partials,
                        hipStream_t st);
void launch_vmax(long long n, double* a, const double* b, hipStream_t st);
template <typename TA, typename TB>
void launch_convert(long long n, const TA* a, TB* b, hipStream_t st);
template <typename T>
int launch_sum_ell2(long long N, const T* ell2, double* partials, hipStream_t st, int nsys = 1);
template <typename TA>
void launch_acc_wide(long long n, const TA* a, double* b, hipStream_t st);
int launch_h_refine_resid(const Geo& g, const cpx<double>* b, const cpx<double>* Ap,
                          cpx<float>* r32, double* partials, hipStream_t st, int nsys = 1);

}  // namespace fftg
