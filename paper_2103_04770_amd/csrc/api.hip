// Host side of the solver: handle, transform plans and tables, the Krylov,
// Newton and staggered drivers, and the C ABI declared in include/fftg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "fftg.h"
#include "host_logic.hpp"
#include "kernels.hpp"

using fftg::cpx;
using fftg::Geo;
using fftg::KrylovCtl;
using fftg::MatTable;
using fftg::Plan;
using fftg::Sym;

namespace {

thread_local std::string g_create_error;

// Smallest relative residual asked of a Krylov solve with FP32 vectors.
constexpr double kFp32KrylovFloor = 1e-5;
// A Krylov loop with FP32 vectors stops as stagnated when its residual has
// not reached a new minimum for this many iterations (its rounding floor).
// FP64 loops have no such test: like the paper's ConjGrad they run to the
// tolerance or to maxit (the residual of CG on an ill-conditioned operator
// can rise for hundreds of iterations while the error still falls).
constexpr int kFp32StagnationWindow = 400;

// FFTG_VERBOSE=1 prints one line per Newton correction and per Krylov solve.
bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("FFTG_VERBOSE");
    return e && e[0] == '1';
  }();
  return v;
}

struct HipError {
  std::string msg;
};

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw HipError{std::string(#expr) + ": " + hipGetErrorString(e_)};               \
  } while (0)

using fftg_host::Fail;

// Workspace of a lockstep batch class (several RVEs of one grid solved as
// stacked systems): FP64 fields [sys][comp][N], ell2 [sys][J][N].
struct BatchWS {
  int cap_sys = 0, cap_J = 0;
  double *eps_k = nullptr, *eps_prev = nullptr, *sig_k = nullptr, *st1 = nullptr,
         *Dj = nullptr, *alph = nullptr, *ab_k = nullptr, *ab_prev = nullptr,
         *ell2j64 = nullptr;
  void* ell2j = nullptr;  // work precision
};

}  // namespace

struct fftg_handle {
  Geo g{};
  int c = 0;
  double h = 1.0;
  int scheme = 0, prec = 0;
  hipStream_t st = nullptr;
  Plan plan[3]{};
  cpx<double>* tw64[3]{};
  cpx<float>* tw32[3]{};
  double* sym64 = nullptr;
  float* sym32 = nullptr;
  Sym<double> S64{};
  Sym<float> S32{};
  // Galerkin workspace (work precision), c-component half spectra
  void *kx = nullptr, *kr = nullptr, *kp = nullptr, *kw = nullptr;
  cpx<double>* spec64 = nullptr;  // FP64 c-component spectrum (stress, residual)
  void* tan = nullptr;            // compact tangent [N][8] (a, b, m0..m5), work precision
  bool tan_valid = false;
  unsigned char mask_last[6] = {0, 1, 1, 1, 1, 1};
  double* partials = nullptr;
  size_t npartials = 0;
  long long psys = 0;  // partial sums one system of a lockstep solve may need
  double* dsums = nullptr;
  KrylovCtl* ctl = nullptr;
  KrylovCtl* hctl = nullptr;  // pinned
  double* hsums = nullptr;    // pinned
  // control blocks held (and 16 sys_cap + 64 sums); systems the Galerkin
  // workspace holds (stacked [sys][c][Ns], tangent [sys][N][8])
  int sys_cap = FFTG_MAX_FIELDS, gal_cap = 1;
  BatchWS* bws = nullptr;  // lockstep batch class workspace (lead handle of a class)
  // Helmholtz workspace (work precision), scalar half spectra + ndim gradient comps
  void *hx = nullptr, *hr = nullptr, *hp = nullptr, *hAp = nullptr, *hb = nullptr,
       *hw = nullptr;
  int helm_cap = 0;       // systems the Helmholtz workspace holds (one per field)
  // ell^2 of the Helmholtz x pass from a per-phase table (staggered step of
  // one RVE: hphase is its phase array while the solve runs, else null):
  // ptab [field][kMaxPhases] in work precision, ptab64 in FP64, hptab pinned
  const unsigned char* hphase = nullptr;
  void* ptab = nullptr;
  double* ptab64 = nullptr;
  double* hptab = nullptr;
  void* rtmp = nullptr;   // real scratch [max(c, 2)][N] in work precision
  void* ell2w = nullptr;  // work-precision ell2 [N]
  cpx<double>* ref64 = nullptr;  // FP64 refinement workspace, 6 spectra per system
  int ref64_cap = 0;
  // staggered workspace (FP64)
  int stJ = -1;
  double *eps_k = nullptr, *eps_prev = nullptr, *ab_k = nullptr, *ab_prev = nullptr,
         *Dj = nullptr, *alph = nullptr, *st1 = nullptr, *sig_k = nullptr;
  void* ell2j = nullptr;  // [J][N] work precision
  double* ell2j64 = nullptr;  // [J][N] FP64 copy (FP32-refined handles: refinement residuals)
  // adaptive driver: copy of the packed state and the stress before an attempt
  double* drive_bak = nullptr;
  double* adj_r = nullptr;  // adjoint: two FP64 real scratch fields
  double* sadj = nullptr;   // staggered adjoint: (2c + 5J) FP64 real fields
  double* hadj = nullptr;   // increment adjoint: history cotangents (c + J fields)
  int hadjJ = 0;
  // tile-budget shifts of the fixed-length strided passes (inner y passes,
  // outer-axis passes), chosen at creation by timing; times of each choice
  int tsh_y = 0, tsh_o = 0;
  double tune_ms[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  int sadjJ = 0;
  size_t drive_bak_n = 0;
  hipEvent_t ev[8]{};
  // per-kernel-class timing (fftg_profile): event pairs resolved at sync points
  bool prof = false;
  double kt_ms[FFTG_NKERNELS]{};
  long long kt_n[FFTG_NKERNELS]{};
  std::vector<hipEvent_t> evpool;
  struct Pend {
    hipEvent_t a, b;
    int kid;
    int iter;  // iteration index inside a profiled Krylov chunk, -1 outside
  };
  int kt_iter = -1;
  std::vector<Pend> pend;
  // captured Krylov iteration chunks: kGraphIters iterations per launch, or
  // kTailIters near the stop test
  hipStream_t cap = nullptr;
  struct GraphSlot {
    hipGraphExec_t exec[2] = {nullptr, nullptr};  // kGraphIters, kTailIters iterations
    unsigned long long key = 0;
    const void* kell = nullptr;    // Helmholtz graphs: the ell2 field they read
    const void* kphase = nullptr;  // Helmholtz graphs: the phase array they read
    int knsys = 0;
    void drop() {
      for (auto& e : exec) {
        if (e) (void)hipGraphExecDestroy(e);
        e = nullptr;
      }
      key = 0;
    }
  };
  GraphSlot ggal;
  GraphSlot ghelm[4];
  int ghelm_next = 0;
  std::string err;

  // Krylov loops launch their iterations directly instead of through HIP
  // graphs (the allocation-free entry point: instantiating a graph allocates)
  bool nograph = false;
  // Galerkin CG scalar steps folded into the passes instead of two scalar
  // kernels per iteration (FFTG_GAL_FOLD=1 at creation).  Off by default: the
  // redundant per-workgroup reductions cost about what the two launches do.
  bool fold = false;
  // Galerkin CG p.Ap summed in real space by the fused x pass (so that the
  // forward outer pass does not read p) instead of on the half spectrum by
  // the forward outer pass (FFTG_GAL_XDOT=0 at creation)
  bool xdot = true;
  // with xdot (and without fold): the forward outer pass and the residual
  // update as one pass that does not store the transform (FFTG_GAL_FUSE=0 at
  // creation: two passes)
  bool fuse_res = true;
  // Helmholtz PCG: p.Lp summed by the inverse pass (|p|^2) and the x pass
  // (ell^2 |grad p|^2), and the forward pass fused with the residual update
  // (FFTG_HELM_FUSE=0 at creation: forward pass, scalar kernel and residual
  // pass apart)
  bool hfuse = true;
  bool fp32() const { return prec == FFTG_FP32_REFINED; }
  size_t wsz() const { return fp32() ? sizeof(float) : sizeof(double); }
};

namespace {

// ------------------------------------------------------------ tables
bool smooth23(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

Plan make_plan(int n) {
  Plan p{};
  p.n = n;
  int a = 0, b = 0, m = n;
  while (m % 2 == 0) m /= 2, ++a;
  while (m % 3 == 0) m /= 3, ++b;
  int n8 = a / 3, rem = a % 3, n4 = 0, n2 = 0;
  if (rem == 1 && n8 >= 1) {
    --n8;
    n4 = 2;
  } else if (rem == 2) {
    n4 = 1;
  } else if (rem == 1) {
    n2 = 1;
  }
  int s = 0;
  for (int i = 0; i < n8; ++i) p.radix[s++] = 8;
  for (int i = 0; i < n4; ++i) p.radix[s++] = 4;
  for (int i = 0; i < n2; ++i) p.radix[s++] = 2;
  for (int i = 0; i < b; ++i) p.radix[s++] = 3;
  p.nst = s;
  return p;
}

// exp(-2 pi i k / n), evaluated in extended precision and rounded.
std::vector<double> twiddles(int n) {
  std::vector<double> t(2 * (size_t)n);
  const long double tp = 6.283185307179586476925286766559005768L;
  for (int k = 0; k < n; ++k) {
    long double a = tp * (long double)k / (long double)n;
    t[2 * k] = (double)cosl(a);
    t[2 * k + 1] = (double)(-sinl(a));
  }
  return t;
}

// Per-axis derivative tables: signed frequency k' (x axis: 0..n/2), theta = 2 pi k'/n.
void axis_tables(int n, bool xaxis, double h, int scheme, std::vector<double>& pq,
                 std::vector<double>& gq, std::vector<double>& cs) {
  const int len = xaxis ? n / 2 + 1 : n;
  pq.assign(len, 0.0);
  gq.assign(len, 0.0);
  cs.assign(len, 1.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < len; ++k) {
    const int ks = xaxis ? k : (k <= (n - 1) / 2 ? k : k - n);
    const bool nyq = (n % 2 == 0) && (2 * (ks < 0 ? -ks : ks) == n);
    const long double th = 2.0L * pi * (long double)ks / (long double)n;
    if (scheme == FFTG_ROTATED) {
      pq[k] = (double)(2.0L / (long double)h * sinl(th / 2.0L));
      gq[k] = nyq ? 0.0 : pq[k];
      cs[k] = nyq ? 0.0 : (double)cosl(th / 2.0L);
    } else {
      pq[k] = nyq ? 0.0 : (double)(th / (long double)h);
      gq[k] = pq[k];
      cs[k] = 1.0;
    }
  }
}

template <typename T>
const cpx<T>* TW(fftg_handle* H, int a);
template <>
const cpx<double>* TW<double>(fftg_handle* H, int a) { return H->tw64[a]; }
template <>
const cpx<float>* TW<float>(fftg_handle* H, int a) { return H->tw32[a]; }
template <typename T>
const Sym<T>& SY(fftg_handle* H);
template <>
const Sym<double>& SY<double>(fftg_handle* H) { return H->S64; }
template <>
const Sym<float>& SY<float>(fftg_handle* H) { return H->S32; }
template <typename T>
cpx<T>* C(void* p) { return reinterpret_cast<cpx<T>*>(p); }

void* dalloc(size_t bytes) {
  void* p = nullptr;
  HIPCHK(hipMalloc(&p, bytes < 256 ? 256 : bytes));
  return p;
}
void dfree(void*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

enum Kid {
  K_GAL_X = 0, K_GAL_YI, K_GAL_YF, K_GAL_OI, K_GAL_OF, K_GAL_RES,
  K_HLM_X, K_HLM_YI, K_HLM_YF, K_HLM_OI, K_HLM_OF, K_HLM_RES,
  K_CONST, K_TR_X, K_TR_YZ, K_SMALL, K_GAL_OFR
};
const char* const kKernelNames[FFTG_NKERNELS] = {
    "galerkin_x_fused",       "galerkin_y_inv",       "galerkin_y_fwd",
    "galerkin_outer_dir_inv", "galerkin_outer_dot_fwd", "galerkin_resid",
    "helmholtz_x_fused",      "helmholtz_y_inv",      "helmholtz_y_fwd",
    "helmholtz_outer_dir_inv", "helmholtz_outer_div_fwd", "helmholtz_resid",
    "constitutive",           "transform_x",          "transform_yz",
    "small",                  "galerkin_outer_fwd_resid"};

// Waits for the stream, then books the timed launches; launches of Krylov
// chunk iterations at index >= keep (run past convergence, so they returned
// at once) are not booked.
void sync(fftg_handle* H, int keep = INT_MAX) {
  HIPCHK(hipStreamSynchronize(H->st));
  for (auto& p : H->pend) {
    if (p.iter < keep) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
      H->kt_ms[p.kid] += ms;
      H->kt_n[p.kid] += 1;
    }
    H->evpool.push_back(p.a);
    H->evpool.push_back(p.b);
  }
  H->pend.clear();
}

// Scope timer around one kernel launch (active only while profiling).
struct KT {
  fftg_handle* H;
  int kid;
  hipEvent_t a = nullptr, b = nullptr;
  hipEvent_t take() {
    if (H->evpool.empty()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      return e;
    }
    hipEvent_t e = H->evpool.back();
    H->evpool.pop_back();
    return e;
  }
  KT(fftg_handle* h, int k) : H(h), kid(k) {
    if (H->prof) {
      a = take();
      b = take();
      HIPCHK(hipEventRecord(a, H->st));
    }
  }
  ~KT() {
    if (a) {
      (void)hipEventRecord(b, H->st);
      H->pend.push_back({a, b, kid, H->kt_iter});
    }
  }
};
void check_launch() { HIPCHK(hipGetLastError()); }

// read back the control block
// read back the control block; `before` = the iteration count when the
// profiled chunk just waited for started (-1: not a profiled chunk)
KrylovCtl read_ctl(fftg_handle* H, int before = -1) {
  HIPCHK(hipMemcpyAsync(H->hctl, H->ctl, sizeof(KrylovCtl), hipMemcpyDeviceToHost, H->st));
  HIPCHK(hipStreamSynchronize(H->st));
  sync(H, before >= 0 ? H->hctl->iters - before : INT_MAX);
  return *H->hctl;
}
void write_ctl(fftg_handle* H, const KrylovCtl& k) {
  *H->hctl = k;
  HIPCHK(hipMemcpyAsync(H->ctl, H->hctl, sizeof(KrylovCtl), hipMemcpyHostToDevice, H->st));
}
// the control blocks of n systems solved in lockstep; a profiled chunk books
// the launches of the iterations the most advanced system ran
void read_ctls(fftg_handle* H, int n, KrylovCtl* out, int before = -1) {
  HIPCHK(hipMemcpyAsync(H->hctl, H->ctl, sizeof(KrylovCtl) * n, hipMemcpyDeviceToHost, H->st));
  HIPCHK(hipStreamSynchronize(H->st));
  int most = 0;
  for (int s = 0; s < n; ++s) most = std::max(most, H->hctl[s].iters);
  sync(H, before >= 0 ? most - before : INT_MAX);
  for (int s = 0; s < n; ++s) out[s] = H->hctl[s];
}
void write_ctls(fftg_handle* H, int n, const KrylovCtl* k) {
  for (int s = 0; s < n; ++s) H->hctl[s] = k[s];
  HIPCHK(hipMemcpyAsync(H->ctl, H->hctl, sizeof(KrylovCtl) * n, hipMemcpyHostToDevice, H->st));
}
// finalise nred sums of partials [nred][nb] and read them back
void read_sums(fftg_handle* H, int nb, int nred, double* out) {
  fftg::launch_fin_sums(H->partials, nb, nred, H->dsums, H->st);
  HIPCHK(hipMemcpyAsync(H->hsums, H->dsums, sizeof(double) * nred, hipMemcpyDeviceToHost, H->st));
  sync(H);
  for (int i = 0; i < nred; ++i) out[i] = H->hsums[i];
}
// finalise nred sums of partials into the device sums from slot `at`, to be
// read later together with others (read_dsums)
void stage_sums(fftg_handle* H, int nb, int nred, int at) {
  fftg::launch_fin_sums(H->partials, nb, nred, H->dsums + at, H->st);
}
void read_dsums(fftg_handle* H, int n, double* out) {
  HIPCHK(hipMemcpyAsync(H->hsums, H->dsums, sizeof(double) * n, hipMemcpyDeviceToHost, H->st));
  sync(H);
  for (int i = 0; i < n; ++i) out[i] = H->hsums[i];
}

// The captured Krylov graphs hold the workspace pointers: drop them before a
// buffer they use is reallocated.
void drop_graphs(fftg_handle* H) {
  HIPCHK(hipStreamSynchronize(H->st));
  H->ggal.drop();
  for (auto& sl : H->ghelm) sl.drop();
}

// Control blocks, sums and partials for a lockstep solve of n systems.
void ensure_sys(fftg_handle* H, int n) {
  const bool ctl_ok = n <= H->sys_cap;
  const bool part_ok = (size_t)n * (size_t)H->psys <= H->npartials;
  if (ctl_ok && part_ok) return;
  if (H->nograph) throw Fail{FFTG_E_UNSUPPORTED, "lockstep solve too large for this workspace"};
  drop_graphs(H);
  if (!ctl_ok) {
    dfree((void*&)H->ctl);
    dfree((void*&)H->dsums);
    if (H->hctl) (void)hipHostFree(H->hctl);
    if (H->hsums) (void)hipHostFree(H->hsums);
    H->hctl = nullptr;
    H->hsums = nullptr;
    H->ctl = (KrylovCtl*)dalloc(sizeof(KrylovCtl) * (size_t)n);
    H->dsums = (double*)dalloc(sizeof(double) * (16 * (size_t)n + 64));
    HIPCHK(hipHostMalloc((void**)&H->hctl, sizeof(KrylovCtl) * (size_t)n, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&H->hsums, sizeof(double) * (16 * (size_t)n + 64),
                         hipHostMallocDefault));
    H->sys_cap = n;
  }
  if (!part_ok) {
    dfree((void*&)H->partials);
    H->npartials = (size_t)n * (size_t)H->psys;
    H->partials = (double*)dalloc(sizeof(double) * H->npartials);
  }
}

void free_bws(fftg_handle* H) {
  BatchWS* B = H->bws;
  if (!B) return;
  for (double** p : {&B->eps_k, &B->eps_prev, &B->sig_k, &B->st1, &B->Dj, &B->alph, &B->ab_k,
                     &B->ab_prev, &B->ell2j64})
    dfree((void*&)*p);
  dfree(B->ell2j);
  delete B;
  H->bws = nullptr;
}

// Galerkin workspace for nsys stacked systems.
void alloc_gal(fftg_handle* H, int nsys) {
  if (nsys <= H->gal_cap) return;
  drop_graphs(H);
  const Geo& g = H->g;
  for (void** p : {&H->kx, &H->kr, &H->kp, &H->kw, &H->tan}) dfree(*p);
  dfree((void*&)H->spec64);
  const size_t cs_bytes = 2 * H->wsz() * (size_t)H->c * g.Ns * (size_t)nsys;
  H->kx = dalloc(cs_bytes);
  H->kr = dalloc(cs_bytes);
  H->kp = dalloc(cs_bytes);
  H->kw = dalloc(cs_bytes);
  H->spec64 = (cpx<double>*)dalloc(sizeof(cpx<double>) * 6 * g.Ns * (size_t)nsys);
  H->tan = dalloc(H->wsz() * 8 * (size_t)g.N * (size_t)nsys);
  H->tan_valid = false;
  H->gal_cap = nsys;
}

// tile shift of a strided pass along plan axis a (1 = y, 2 = z): the outer
// axis (z in 3D, y in 2D) takes the outer-pass choice, y in 3D the inner one
int tsh(const fftg_handle* H, int a) { return a == (H->g.ndim == 3 ? 2 : 1) ? H->tsh_o : H->tsh_y; }

// ------------------------------------------------------------ 3D transforms
template <typename T>
void fwd3(fftg_handle* H, int ncomp, const T* in, cpx<T>* out, const KrylovCtl* ctl = nullptr) {
  const Geo& g = H->g;
  {
    KT t(H, K_TR_X);
    fftg::launch_x_r2c<T>(H->plan[0], TW<T>(H, 0), in, out, (long long)ncomp * g.n2 * g.n3, g.n1,
                          g.n1h, H->st);
  }
  if (g.n2 > 1) {
    KT t(H, K_TR_YZ);
    fftg::launch_strided<T>(H->plan[1], TW<T>(H, 1), out, (long long)ncomp * g.n3 * g.n1h, g.n1h,
                            (long long)g.n2 * g.n1h, g.n1h, true, ctl, H->st, tsh(H, 1));
  }
  if (g.n3 > 1) {
    KT t(H, K_TR_YZ);
    fftg::launch_strided<T>(H->plan[2], TW<T>(H, 2), out, (long long)ncomp * g.n2 * g.n1h,
                            (long long)g.n2 * g.n1h, g.Ns, (long long)g.n2 * g.n1h, true, ctl,
                            H->st, tsh(H, 2));
  }
}

// in is destroyed; out (=|+=) scale * inverse
template <typename T, typename TO>
void inv3(fftg_handle* H, int ncomp, cpx<T>* in, TO* out, T scale, bool acc) {
  const Geo& g = H->g;
  if (g.n3 > 1) {
    KT t(H, K_TR_YZ);
    fftg::launch_strided<T>(H->plan[2], TW<T>(H, 2), in, (long long)ncomp * g.n2 * g.n1h,
                            (long long)g.n2 * g.n1h, g.Ns, (long long)g.n2 * g.n1h, false,
                            nullptr, H->st, tsh(H, 2));
  }
  if (g.n2 > 1) {
    KT t(H, K_TR_YZ);
    fftg::launch_strided<T>(H->plan[1], TW<T>(H, 1), in, (long long)ncomp * g.n3 * g.n1h, g.n1h,
                            (long long)g.n2 * g.n1h, g.n1h, false, nullptr, H->st, tsh(H, 1));
  }
  KT t(H, K_TR_X);
  fftg::launch_x_c2r<T, TO>(H->plan[0], TW<T>(H, 0), in, out, (long long)ncomp * g.n2 * g.n3,
                            g.n1, g.n1h, scale, acc, H->st);
}

// inner (non-outer) passes of an operator application on an ncomp spectrum;
// ctl: the control blocks of the stacked systems, lps lines each (0: one
// system)
template <typename T>
void inner_inv(fftg_handle* H, int ncomp, cpx<T>* w, const KrylovCtl* ctl, int kid,
               long long lps = 0) {
  const Geo& g = H->g;
  KT t(H, kid);
  if (g.ndim == 3 && g.n2 > 1)
    fftg::launch_strided<T>(H->plan[1], TW<T>(H, 1), w, (long long)ncomp * g.n3 * g.n1h, g.n1h,
                            (long long)g.n2 * g.n1h, g.n1h, false, ctl, H->st, H->tsh_y, lps);
}
template <typename T>
void inner_fwd(fftg_handle* H, int ncomp, cpx<T>* w, const KrylovCtl* ctl, int kid,
               long long lps = 0) {
  const Geo& g = H->g;
  KT t(H, kid);
  if (g.ndim == 3 && g.n2 > 1)
    fftg::launch_strided<T>(H->plan[1], TW<T>(H, 1), w, (long long)ncomp * g.n3 * g.n1h, g.n1h,
                            (long long)g.n2 * g.n1h, g.n1h, true, ctl, H->st, H->tsh_y, lps);
}
int outer_axis(fftg_handle* H) { return H->g.ndim == 3 ? 2 : 1; }

// y passes of the Helmholtz operator on its gradient buffer: the split form
// (two fields to three and back, launch_h_y_split) where the outer passes
// use it, the plain per-component passes otherwise.
// nsys stacked systems: the gradient buffer is [comp][sys][Ns], so the plain
// y passes transform ndim * nsys spectra.
template <typename T>
void helm_inner(fftg_handle* H, bool fwd, cpx<T>* w, const KrylovCtl* ctl, int kid,
                int nsys = 1) {
  const Geo& g = H->g;
  if (fftg::helm_split(g)) {
    KT t(H, kid);
    fftg::launch_h_y_split<T>(H->plan[1], TW<T>(H, 1), g, SY<T>(H), w, fwd, ctl, H->st, nsys);
  } else if (fwd) {
    inner_fwd<T>(H, g.ndim * nsys, w, nsys == 1 ? ctl : nullptr, kid);
  } else {
    inner_inv<T>(H, g.ndim * nsys, w, nsys == 1 ? ctl : nullptr, kid);
  }
}

MatTable make_table(const fftg_phase* tab, int nphase, int J) {
  MatTable t{};
  t.nphase = nphase;
  for (int p = 0; p < nphase; ++p) {
    const fftg_phase& q = tab[p];
    fftg::Mat& m = t.m[p];
    m.model = q.model;
    m.dfield = q.dfield;
    m.mu = q.E / (2.0 * (1.0 + q.nu));
    m.K = q.E / (3.0 * (1.0 - 2.0 * q.nu));
    m.sy = q.sy;
    m.H = q.H;
    m.dC = q.dC;
    m.dR = q.dR;
    m.dmax = q.dmax;
    for (int j = 0; j < FFTG_MAX_FIELDS; ++j) m.ell2[j] = q.ell[j] * q.ell[j];
    if (q.model == FFTG_GTN) {
      t.gtn = 1;
      m.n = q.n_hard;
      m.q1 = q.q1;
      m.q2 = q.q2;
      m.q3 = q.q3;
      m.fC = q.fC;
      m.fF = q.fF;
      m.fN = q.fN;
      m.eN = q.eN;
      m.sN = q.sN;
      m.fu = q.fu;
      // porosity at which the yield surface shrinks to the origin
      m.fV = (q.q1 + std::sqrt(std::max(q.q1 * q.q1 - q.q3, 0.0))) / q.q3;
    }
  }
  (void)J;
  return t;
}

bool has_gtn(const fftg_phase* tab, int nphase) {
  for (int p = 0; p < nphase; ++p)
    if (tab[p].model == FFTG_GTN) return true;
  return false;
}

void validate_table(const fftg_phase* tab, int nphase, int nfields) {
  fftg_host::check_table(tab, nphase, nfields);
}

// Every phase id must index the table: counted on the device, one read-back.
void validate_phase(fftg_handle* H, const unsigned char* phase, int nphase) {
  if (!phase) throw Fail{FFTG_E_INVALID, "null phase array"};
  double bad = 0.0;
  read_sums(H, fftg::launch_count_bad_phase(H->g.N, nphase, phase, H->partials, H->st), 1, &bad);
  if (bad != 0.0) throw Fail{FFTG_E_INVALID, "phase id >= nphase in the phase array"};
}

void validate_macro(const fftg_macro* t, int c) {
  if (!t) throw Fail{FFTG_E_INVALID, "null macro target"};
  for (int k = 0; k < c; ++k)
    if (t->mask[k] > 1) throw Fail{FFTG_E_INVALID, "macro mask entries must be 0 or 1"};
}

// One Galerkin CG iteration of nsys stacked systems (RVEs of one grid, each
// with its own scalars; spectra [sys][c][Ns], tangent [sys][N][8]): 6 passes
// and 2 scalar kernels on H->st.  With H->fold the scalar steps are folded
// into the passes instead: the inverse outer pass finishes the previous
// iteration (r.r, stop test, beta) from the residual pass's partial sums, the
// residual pass forms alpha from the forward pass's; parity = the
// iteration's index & 1 (the slot of the control block it writes).
template <typename T>
void gal_iteration(fftg_handle* H, const unsigned char* mask, int nsys = 1, int parity = 0) {
  const Geo& g = H->g;
  const int c = H->c;
  const bool zo = g.ndim == 3;
  const int oa = outer_axis(H);
  const T scl = T(1.0 / (double)g.N);
  const long long lps = (long long)c * g.n3 * g.n1h;  // y lines per system
  const bool xdot = H->xdot;
  const bool fold = H->fold;
  const bool fused = xdot && !fold && H->fuse_res;
  const int nbd = xdot ? fftg::gal_xdot_count<T>(g, c) : fftg::gal_dot_count<T>(H->plan[oa], g, c, zo);
  const int nbr = fused ? fftg::gal_fwd_resid_count<T>(H->plan[oa], g, c, zo)
                        : fftg::gal_resid_count(g);
  double* dpart = H->partials;                             // p.Ap, [sys][nbd]
  double* rpart = H->partials + (long long)nsys * nbd;     // r.r, [sys][nbr]
  {
    KT t(H, K_GAL_OI);
    fftg::launch_gal_dir_inv<T>(H->plan[oa], TW<T>(H, oa), g, c, zo, C<T>(H->kr), C<T>(H->kp),
                                C<T>(H->kx), C<T>(H->kw), H->ctl, H->st, H->tsh_o, nsys, parity,
                                fold ? rpart : nullptr, nbr);
  }
  inner_inv<T>(H, c * nsys, C<T>(H->kw), H->ctl, K_GAL_YI, lps);
  {
    KT t(H, K_GAL_X);
    const int nb = fftg::launch_x_fused_gal<T, T>(
        H->plan[0], TW<T>(H, 0), g, c, C<T>(H->kw), reinterpret_cast<const T*>(H->tan), scl,
        H->ctl, H->st, nsys, xdot ? dpart : nullptr);
    if (xdot && nb != nbd) throw Fail{FFTG_E_HIP, "Galerkin x pass: partial count mismatch"};
  }
  if (fused) {
    // alpha from the x pass's p.Ap, then one forward pass that updates r
    {
      KT t(H, K_SMALL);
      fftg::launch_fin_alpha(dpart, nbd, H->ctl, H->st, nsys);
    }
    inner_fwd<T>(H, c * nsys, C<T>(H->kw), H->ctl, K_GAL_YF, lps);
    {
      KT t(H, K_GAL_OFR);
      const int nb = fftg::launch_gal_fwd_resid<T>(H->plan[oa], TW<T>(H, oa), g, c, zo, SY<T>(H),
                                                   mask, C<T>(H->kw), C<T>(H->kr), rpart, H->ctl,
                                                   H->st, nsys);
      if (nb != nbr) throw Fail{FFTG_E_HIP, "Galerkin forward pass: partial count mismatch"};
    }
    {
      KT t(H, K_SMALL);
      fftg::launch_fin_beta(rpart, nbr, 1, H->ctl, H->st, nsys);
    }
    return;
  }
  inner_fwd<T>(H, c * nsys, C<T>(H->kw), H->ctl, K_GAL_YF, lps);
  {
    KT t(H, K_GAL_OF);
    const int nb = fftg::launch_gal_dot_fwd<T>(H->plan[oa], TW<T>(H, oa), g, c, zo,
                                               xdot ? nullptr : C<T>(H->kp), C<T>(H->kw),
                                               xdot ? nullptr : dpart, H->ctl, H->st, nsys);
    if (!xdot && nb != nbd) throw Fail{FFTG_E_HIP, "Galerkin forward pass: partial count mismatch"};
  }
  if (!fold) {
    KT t(H, K_SMALL);
    fftg::launch_fin_alpha(dpart, nbd, H->ctl, H->st, nsys);
  }
  {
    KT t(H, K_GAL_RES);
    fftg::launch_gal_resid<T>(g, c, SY<T>(H), mask, C<T>(H->kr), C<T>(H->kw), rpart, H->ctl,
                              H->st, nsys, parity, fold ? dpart : nullptr, nbd);
  }
  if (!fold) {
    KT t(H, K_SMALL);
    fftg::launch_fin_beta(rpart, nbr, 1, H->ctl, H->st, nsys);
  }
}

// Capture `body` `iters` times on the private capture stream into an
// executable graph.  Every launch inside reads the device control block, so
// iterations past convergence return at once.  Krylov loops launch graphs of
// kGraphIters iterations, and graphs of kTailIters (even, so that the
// parity of an iteration is its index & 1 in either) near the stop test.
constexpr int kGraphIters = 8;
constexpr int kTailIters = 2;

template <typename F>
hipGraphExec_t capture(fftg_handle* H, F body, int iters = kGraphIters) {
  hipStream_t saved = H->st;
  H->st = H->cap;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(H->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    try {
      for (int i = 0; i < iters; ++i) body(i);
    } catch (...) {
      (void)hipStreamEndCapture(H->cap, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      H->st = saved;
      throw;
    }
    e = hipStreamEndCapture(H->cap, &graph);
  }
  H->st = saved;
  if (e != hipSuccess) throw HipError{std::string("graph capture: ") + hipGetErrorString(e)};
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) throw HipError{std::string("graph instantiate: ") + hipGetErrorString(e)};
  return ex;
}

// Graph launches of a lockstep Krylov solve until every system is done, in
// rounds planned by fftg_host::plan_round from the predicted iterations
// left (fftg_host::predict_left); the control blocks are read after each
// round.  Several full graphs queued in one round keep the GPU from waiting
// on the host's read between them.
void run_krylov_graphs(fftg_handle* H, int nsys, KrylovCtl* k, hipGraphExec_t full,
                       hipGraphExec_t tail) {
  std::vector<KrylovCtl> prev(k, k + nsys);
  for (;;) {
    bool all = true;
    for (int q = 0; q < nsys; ++q) all = all && k[q].done;
    if (all) return;
    const auto round = fftg_host::plan_round(fftg_host::predict_left(nsys, k, prev.data()),
                                             kGraphIters, kTailIters);
    prev.assign(k, k + nsys);
    for (int i = 0; i < round.full; ++i) HIPCHK(hipGraphLaunch(full, H->st));
    for (int i = 0; i < round.tail; ++i) HIPCHK(hipGraphLaunch(tail, H->st));
    read_ctls(H, nsys, k);
  }
}

// The Galerkin CG graphs (kGraphIters and kTailIters iterations) of a mask,
// system count, precision and scalar-step form.
template <typename T>
fftg_handle::GraphSlot& gal_graphs(fftg_handle* H, const unsigned char* mask, int nsys) {
  unsigned long long key = 1ull + (H->fp32() ? 2ull : 0ull);
  for (int i = 0; i < 6; ++i) key |= (unsigned long long)(mask[i] & 1) << (8 + i);
  key |= (unsigned long long)nsys << 16;
  key |= H->fold ? 4ull : 0ull;
  key |= H->xdot ? 8ull : 0ull;
  key |= H->fuse_res ? 16ull : 0ull;
  auto& sl = H->ggal;
  if (sl.exec[0] && sl.key == key) return sl;
  sl.drop();
  unsigned char m[6];
  std::memcpy(m, mask, 6);
  sl.exec[0] = capture(H, [&](int i) { gal_iteration<T>(H, m, nsys, i & 1); }, kGraphIters);
  sl.exec[1] = capture(H, [&](int i) { gal_iteration<T>(H, m, nsys, i & 1); }, kTailIters);
  sl.key = key;
  return sl;
}

// ------------------------------------------------------------ Galerkin CG
// Solves G*(K_s : dx_s) = b_s in the half spectrum for nsys stacked systems
// in lockstep (b in H->kr, dx -> H->kx, [sys][c][Ns]), each with its own
// scalars and stop test; systems with need[s] = 0 or bb[s] = 0 start as done
// (dx_s = 0).  k[s]: the final control block of system s.
template <typename T>
void galerkin_cg_n(fftg_handle* H, const unsigned char* mask, int nsys, const double* bb,
                   const unsigned char* need, double tol, int maxit, KrylovCtl* k) {
  const Geo& g = H->g;
  const int c = H->c;
  bool all = true;
  for (int q = 0; q < nsys; ++q) {
    k[q] = KrylovCtl{};
    k[q].rz = bb[q];
    k[q].rr = bb[q];
    k[q].bb = bb[q];
    k[q].tol2 = tol * tol * bb[q];
    k[q].rrmin = bb[q];
    k[q].maxit = maxit;
    k[q].window = std::is_same<T, float>::value ? kFp32StagnationWindow : 0;
    k[q].done = (!need[q] || bb[q] == 0.0) ? 1 : (maxit <= 0 ? 2 : 0);
    // slot 0: the state before the first iteration
    k[q].rzs[0] = bb[q];
    k[q].rrmins[0] = bb[q];
    k[q].its[0] = 0;
    k[q].itmins[0] = 0;
    k[q].first = 1;
    all = all && k[q].done;
  }
  write_ctls(H, nsys, k);
  HIPCHK(hipMemsetAsync(H->kx, 0, sizeof(cpx<T>) * c * g.Ns * nsys, H->st));
  HIPCHK(hipMemsetAsync(H->kp, 0, sizeof(cpx<T>) * c * g.Ns * nsys, H->st));
  if (!H->prof) {
    if (!all) {
      auto& sl = gal_graphs<T>(H, mask, nsys);
      run_krylov_graphs(H, nsys, k, sl.exec[0], sl.exec[1]);
    }
  } else {
    int chunk = 2;
    while (!all) {
      int before = 0;
      for (int q = 0; q < nsys; ++q) before = std::max(before, k[q].iters);
      // chunks of even length: the iteration's parity is it & 1
      for (int it = 0; it < chunk; ++it) {
        H->kt_iter = it;
        gal_iteration<T>(H, mask, nsys, it & 1);
      }
      H->kt_iter = -1;
      check_launch();
      read_ctls(H, nsys, k, before);
      all = true;
      for (int q = 0; q < nsys; ++q) all = all && k[q].done;
      if (chunk < 16) chunk *= 2;
    }
  }
  fftg::launch_xfinal<T>(C<T>(H->kx), C<T>(H->kp), (long long)c * g.Ns, H->ctl, H->st, nsys);
  check_launch();
}

// One system: b in H->kr, dx -> H->kx.
template <typename T>
void galerkin_cg(fftg_handle* H, const unsigned char* mask, double bb, double tol, int maxit,
                 int& iters, int& status) {
  const unsigned char need = 1;
  KrylovCtl k{};
  galerkin_cg_n<T>(H, mask, 1, &bb, &need, tol, maxit, &k);
  iters = k.iters;
  status = k.done;
}

// the per-phase ell^2 table of the work precision, while a phase array is set
template <typename T>
const T* phase_tab(fftg_handle* H) {
  return H->hphase ? static_cast<const T*>(H->ptab) : nullptr;
}

// One Helmholtz PCG iteration of nsys stacked systems (one per non-local
// field, each with its own scalars): 5 passes + 2 scalar kernels, all on H->st.
template <typename T>
void helm_iteration(fftg_handle* H, const T* ell2, int nsys) {
  const Geo& g = H->g;
  const bool zo = g.ndim == 3;
  const int oa = outer_axis(H);
  const T scl = T(1.0 / (double)g.N);
  if (H->hfuse) {
    // p.Lp = weighted |p|^2 (inverse pass, [sys][nbp]) + the sum of
    // ell^2 |grad p|^2 over the voxels (x pass, [sys][nbx], after them); alpha
    // from both, then the forward pass updates r ([sys][2][nbr], from the
    // start again).  The counts stay below the workspace's partials: nbp is
    // at most the lines of one slab, nbx the x lines, nbr the slab's lines.
    double* ppart = H->partials;
    int nbp, nbx;
    {
      KT t(H, K_HLM_OI);
      nbp = fftg::launch_h_dir_inv<T>(H->plan[oa], TW<T>(H, oa), g, zo, SY<T>(H), true,
                                      C<T>(H->hr), C<T>(H->hp), C<T>(H->hx), C<T>(H->hw), H->ctl,
                                      H->st, nsys, ppart);
    }
    double* xpart = H->partials + (long long)nsys * nbp;
    helm_inner<T>(H, false, C<T>(H->hw), H->ctl, K_HLM_YI, nsys);
    {
      KT t(H, K_HLM_X);
      nbx = fftg::launch_x_fused_helm<T, T>(H->plan[0], TW<T>(H, 0), g, C<T>(H->hw), ell2, scl,
                                            H->ctl, H->st, nsys, H->hphase, phase_tab<T>(H),
                                            xpart);
    }
    {
      KT t(H, K_SMALL);
      fftg::launch_fin_alpha2(ppart, nbp, xpart, nbx, H->ctl, H->st, nsys);
    }
    helm_inner<T>(H, true, C<T>(H->hw), H->ctl, K_HLM_YF, nsys);
    int nr;
    {
      KT t(H, K_HLM_OF);
      nr = fftg::launch_h_fwd_resid<T>(H->plan[oa], TW<T>(H, oa), g, zo, SY<T>(H), C<T>(H->hp),
                                       C<T>(H->hw), C<T>(H->hr), H->partials, H->ctl, H->st,
                                       nsys);
    }
    {
      KT t(H, K_SMALL);
      fftg::launch_fin_beta(H->partials, nr, 2, H->ctl, H->st, nsys);
    }
    return;
  }
  {
    KT t(H, K_HLM_OI);
    fftg::launch_h_dir_inv<T>(H->plan[oa], TW<T>(H, oa), g, zo, SY<T>(H), true, C<T>(H->hr),
                              C<T>(H->hp), C<T>(H->hx), C<T>(H->hw), H->ctl, H->st, nsys);
  }
  helm_inner<T>(H, false, C<T>(H->hw), H->ctl, K_HLM_YI, nsys);
  {
    KT t(H, K_HLM_X);
    fftg::launch_x_fused_helm<T, T>(H->plan[0], TW<T>(H, 0), g, C<T>(H->hw), ell2, scl,
                                    H->ctl, H->st, nsys, H->hphase, phase_tab<T>(H));
  }
  helm_inner<T>(H, true, C<T>(H->hw), H->ctl, K_HLM_YF, nsys);
  int nb;
  {
    KT t(H, K_HLM_OF);
    nb = fftg::launch_h_div_fwd<T>(H->plan[oa], TW<T>(H, oa), g, zo, SY<T>(H), C<T>(H->hp),
                                   C<T>(H->hw), C<T>(H->hAp), H->partials, H->ctl, H->st, nsys);
  }
  {
    KT t(H, K_SMALL);
    fftg::launch_fin_alpha(H->partials, nb, H->ctl, H->st, nsys);
  }
  int nr;
  {
    KT t(H, K_HLM_RES);
    nr = fftg::launch_h_resid<T>(g, SY<T>(H), false, C<T>(H->hr), C<T>(H->hb), C<T>(H->hAp),
                                 H->partials, H->ctl, H->st, nsys);
  }
  {
    KT t(H, K_SMALL);
    fftg::launch_fin_beta(H->partials, nr, 2, H->ctl, H->st, nsys);
  }
}

// The Helmholtz PCG graphs (kGraphIters and kTailIters iterations) of an
// ell2 field, system count, precision and phase array (the four most recent).
template <typename T>
fftg_handle::GraphSlot& helm_graphs(fftg_handle* H, const T* ell2, int nsys) {
  const unsigned long long key = (H->fp32() ? 1ull : 2ull) | (H->hfuse ? 4ull : 0ull);
  for (auto& sl : H->ghelm)
    if (sl.exec[0] && sl.key == key && sl.kell == ell2 && sl.knsys == nsys &&
        sl.kphase == H->hphase)
      return sl;
  auto& sl = H->ghelm[H->ghelm_next];
  H->ghelm_next = (H->ghelm_next + 1) % 4;
  sl.drop();
  sl.exec[0] = capture(H, [&](int) { helm_iteration<T>(H, ell2, nsys); }, kGraphIters);
  sl.exec[1] = capture(H, [&](int) { helm_iteration<T>(H, ell2, nsys); }, kTailIters);
  sl.key = key;
  sl.kell = ell2;
  sl.knsys = nsys;
  sl.kphase = H->hphase;
  return sl;
}

// ------------------------------------------------------------ Helmholtz PCG
// Workspace for nsys stacked Helmholtz systems (scalar spectra [sys][Ns],
// gradient buffer [comp][sys][Ns]).  Growing it drops the captured graphs,
// which hold the old buffers.
void alloc_helm(fftg_handle* H, int nsys = 1) {
  if (H->hx && H->helm_cap >= nsys) return;
  const Geo& g = H->g;
  if (H->hx) {
    HIPCHK(hipStreamSynchronize(H->st));
    for (auto& sl : H->ghelm) sl.drop();
    for (void** p : {&H->hx, &H->hr, &H->hp, &H->hAp, &H->hb, &H->hw}) dfree(*p);
  }
  const size_t cs = 2 * H->wsz() * (size_t)g.Ns * (size_t)nsys;
  H->hx = dalloc(cs);
  H->hr = dalloc(cs);
  H->hp = dalloc(cs);
  H->hAp = dalloc(cs);
  H->hb = dalloc(cs);
  H->hw = dalloc(cs * g.ndim);
  if (!H->ell2w) H->ell2w = dalloc(H->wsz() * (size_t)g.N);
  H->helm_cap = nsys;
}

// PCG of Algorithm 2 on the half spectrum in work precision T for nsys
// stacked systems in lockstep, each with its own scalars and stop test:
// b in H->hb (weighted |b_s|^2 = bb[s]), x0 in H->hx (x0_zero: x0 = 0, H->hx
// is cleared); systems with bb[s] = 0 or tol[s] < 0 start as done.  On
// return H->hx holds x and k[s] the final control block of system s.
// bb_staged: the |b_s|^2 are still on the device (device sums 0 .. nsys-1)
// and are read into bb together with the initial residual; a system with
// bb[s] = 0 then gets x = 0 (the solution for a zero source).
template <typename T>
void helm_krylov(fftg_handle* H, const T* ell2, int nsys, const double* ell2_ref, double* bb,
                 const double* tol, const int* maxit, bool x0_zero, KrylovCtl* k,
                 bool bb_staged = false) {
  const Geo& g = H->g;
  const bool zo = g.ndim == 3;
  const int oa = outer_axis(H);
  const T scl = T(1.0 / (double)g.N);
  for (int q = 0; q < nsys; ++q) {
    k[q] = KrylovCtl{};
    k[q].bb = bb_staged ? 0.0 : bb[q];
    k[q].tol2 = tol[q] * tol[q] * k[q].bb;
    k[q].maxit = maxit[q];
    k[q].window = std::is_same<T, float>::value ? kFp32StagnationWindow : 0;
    k[q].ell2ref = ell2_ref[q];
  }
  write_ctls(H, nsys, k);
  if (x0_zero) {
    // r = b - 0 (H->hx doubles as the zero operator output)
    HIPCHK(hipMemsetAsync(H->hx, 0, sizeof(cpx<T>) * g.Ns * nsys, H->st));
  } else {
    // r = b - L x0
    fftg::launch_h_dir_inv<T>(H->plan[oa], TW<T>(H, oa), g, zo, SY<T>(H), false, C<T>(H->hr),
                              C<T>(H->hx), C<T>(H->hx), C<T>(H->hw), H->ctl, H->st, nsys);
    helm_inner<T>(H, false, C<T>(H->hw), nullptr, K_HLM_YI, nsys);
    fftg::launch_x_fused_helm<T, T>(H->plan[0], TW<T>(H, 0), g, C<T>(H->hw), ell2, scl, nullptr,
                                    H->st, nsys, H->hphase, phase_tab<T>(H));
    helm_inner<T>(H, true, C<T>(H->hw), nullptr, K_HLM_YF, nsys);
    fftg::launch_h_div_fwd<T>(H->plan[oa], TW<T>(H, oa), g, zo, SY<T>(H), C<T>(H->hx),
                              C<T>(H->hw), C<T>(H->hAp), nullptr, H->ctl, H->st, nsys);
  }
  const int nr0 = fftg::launch_h_resid<T>(g, SY<T>(H), true, C<T>(H->hr), C<T>(H->hb),
                                          x0_zero ? C<T>(H->hx) : C<T>(H->hAp), H->partials,
                                          H->ctl, H->st, nsys);
  std::vector<double> s2(2 * (size_t)nsys);
  if (bb_staged) {
    std::vector<double> all3(3 * (size_t)nsys);
    stage_sums(H, nr0, 2 * nsys, nsys);
    read_dsums(H, 3 * nsys, all3.data());
    for (int q = 0; q < nsys; ++q) {
      bb[q] = all3[q];
      s2[2 * q] = all3[nsys + 2 * q];
      s2[2 * q + 1] = all3[nsys + 2 * q + 1];
      k[q].bb = bb[q];
      k[q].tol2 = tol[q] * tol[q] * bb[q];
      if (bb[q] == 0.0)
        HIPCHK(hipMemsetAsync(C<T>(H->hx) + q * g.Ns, 0, sizeof(cpx<T>) * g.Ns, H->st));
    }
  } else {
    read_sums(H, nr0, 2 * nsys, s2.data());
  }
  bool all = true;
  for (int q = 0; q < nsys; ++q) {
    k[q].rz = s2[2 * q];
    k[q].rr = s2[2 * q + 1];
    k[q].rrmin = s2[2 * q + 1];
    if (bb[q] == 0.0 || tol[q] < 0.0 || s2[2 * q + 1] <= k[q].tol2)
      k[q].done = 1;
    else if (maxit[q] <= 0)
      k[q].done = 2;
    all = all && k[q].done;
  }
  write_ctls(H, nsys, k);
  HIPCHK(hipMemsetAsync(H->hp, 0, sizeof(cpx<T>) * g.Ns * nsys, H->st));
  if (!H->prof && !H->nograph) {
    if (!all) {
      auto& sl = helm_graphs<T>(H, ell2, nsys);
      run_krylov_graphs(H, nsys, k, sl.exec[0], sl.exec[1]);
    }
  } else {
    int chunk = 2;
    while (!all) {
      int before = 0;
      for (int q = 0; q < nsys; ++q) before = std::max(before, k[q].iters);
      for (int it = 0; it < chunk; ++it) {
        H->kt_iter = it;
        helm_iteration<T>(H, ell2, nsys);
      }
      H->kt_iter = -1;
      check_launch();
      read_ctls(H, nsys, k, H->prof ? before : -1);
      all = true;
      for (int q = 0; q < nsys; ++q) all = all && k[q].done;
      if (chunk < 16) chunk *= 2;
    }
  }
  fftg::launch_xfinal<T>(C<T>(H->hx), C<T>(H->hp), g.Ns, H->ctl, H->st, nsys);
  check_launch();
  if (verbose())
    for (int q = 0; q < nsys; ++q)
      std::fprintf(stderr, "[fftg]   %s pcg system %d/%d: bb %.3e tol %.1e iters %d done %d "
                   "rr/bb %.3e pAp %.3e\n", std::is_same<T, float>::value ? "fp32" : "fp64", q,
                   nsys, bb[q], tol[q], k[q].iters, k[q].done, bb[q] > 0 ? k[q].rr / bb[q] : 0.0,
                   k[q].pAp);
}

// preconditioner length^2 of each system: the given one, else the volume
// mean of its ell2 [sys][N].  cache (optional): the means of an earlier call
// on the same ell2 fields when it holds nsys of them, else filled here (the
// staggered loops solve with unchanged lengths pass after pass).
template <typename T>
void ell2_reference(fftg_handle* H, const T* ell2, double ell2_ref, int nsys, double* out,
                    std::vector<double>* cache = nullptr) {
  if (ell2_ref > 0.0) {
    for (int q = 0; q < nsys; ++q) out[q] = ell2_ref;
    return;
  }
  if (cache && (int)cache->size() == nsys) {
    std::copy(cache->begin(), cache->end(), out);
    return;
  }
  read_sums(H, fftg::launch_sum_ell2<T>(H->g.N, ell2, H->partials, H->st, nsys), nsys, out);
  for (int q = 0; q < nsys; ++q) out[q] /= (double)H->g.N;
  if (cache) cache->assign(out, out + nsys);
}

// Transforms of nsys stacked scalar fields, one field at a time: the x pass
// transforms two real lines as one complex line, which would leave rounding
// of one field's magnitude in the other.  Fields with skip[q] set are left
// alone.
void fwd_fields(fftg_handle* H, int nsys, const double* in, cpx<double>* out,
                const unsigned char* skip = nullptr) {
  for (int q = 0; q < nsys; ++q)
    if (!skip || !skip[q]) fwd3<double>(H, 1, in + q * H->g.N, out + q * H->g.Ns);
}
void inv_fields(fftg_handle* H, int nsys, cpx<double>* in, double* out,
                const unsigned char* skip = nullptr) {
  for (int q = 0; q < nsys; ++q)
    if (!skip || !skip[q])
      inv3<double, double>(H, 1, in + q * H->g.Ns, out + q * H->g.N, 1.0 / (double)H->g.N,
                           false);
}

// Outcome of one Helmholtz system: PCG iterations, final relative residual,
// status (KrylovCtl::done codes).
struct HelmOut {
  int iters = 0;
  double relres = 0.0;
  int status = 0;
};

// FP64 handles: solves L abar_s = alpha_s for nsys stacked fields (alpha,
// ell2, abar [sys][N] FP64; abar in = x0), the whole PCG in FP64.  Fields
// with skip[q] set are not solved and their abar is left alone.
void helmholtz_pcg64(fftg_handle* H, const double* alpha, const double* ell2, double ell2_ref,
                     double* abar, double tol, int maxit, int nsys, HelmOut* out,
                     const unsigned char* skip = nullptr, std::vector<double>* refc = nullptr) {
  const Geo& g = H->g;
  fwd_fields(H, nsys, alpha, C<double>(H->hb), skip);
  std::vector<double> bb(nsys), ref(nsys), tols(nsys);
  std::vector<int> mits(nsys);
  for (int q = 0; q < nsys; ++q)
    if (skip && skip[q])
      HIPCHK(hipMemsetAsync(C<double>(H->hb) + q * g.Ns, 0, sizeof(cpx<double>) * g.Ns, H->st));
  fftg::launch_hermitize<double>(g, nsys, C<double>(H->hb), H->st);
  ell2_reference<double>(H, ell2, ell2_ref, nsys, ref.data(), refc);
  // |b|^2 stays on the device until the initial residual is read with it
  stage_sums(H, fftg::launch_wnorm2<double>(g, 1, C<double>(H->hb), H->partials, H->st, nsys),
             nsys, 0);
  fwd_fields(H, nsys, abar, C<double>(H->hx), skip);
  for (int q = 0; q < nsys; ++q) {
    tols[q] = skip && skip[q] ? -1.0 : tol;
    mits[q] = maxit;
  }
  std::vector<KrylovCtl> k(nsys);
  helm_krylov<double>(H, ell2, nsys, ref.data(), bb.data(), tols.data(), mits.data(), false,
                      k.data(), true);
  inv_fields(H, nsys, C<double>(H->hx), abar, skip);
  check_launch();
  for (int q = 0; q < nsys; ++q) {
    if (verbose())
      std::fprintf(stderr, "[fftg] pcg field %d iters %d status %d rr/bb %.3e ell2ref %.4g\n", q,
                   k[q].iters, k[q].done, bb[q] > 0 ? k[q].rr / bb[q] : 0.0, ref[q]);
    out[q].iters = k[q].iters;
    out[q].relres = bb[q] > 0 ? std::sqrt(k[q].rr / bb[q]) : 0.0;
    out[q].status = k[q].done;
  }
}

// FP64 application of the Helmholtz operator on nsys stacked half spectra,
// Ap = L x, through the same fused passes as the PCG (w: the gradient buffer,
// [comp][sys][Ns]; ell2 [sys][N]).
void helm_apply64(fftg_handle* H, const cpx<double>* x, cpx<double>* w, cpx<double>* Ap,
                  const double* ell2, int nsys) {
  const Geo& g = H->g;
  const bool zo = g.ndim == 3;
  const int oa = outer_axis(H);
  cpx<double>* xm = const_cast<cpx<double>*>(x);  // read only (update = false)
  fftg::launch_h_dir_inv<double>(H->plan[oa], TW<double>(H, oa), g, zo, H->S64, false, nullptr,
                                 xm, xm, w, nullptr, H->st, nsys);
  helm_inner<double>(H, false, w, nullptr, K_HLM_YI, nsys);
  fftg::launch_x_fused_helm<double, double>(H->plan[0], TW<double>(H, 0), g, w, ell2,
                                            1.0 / (double)g.N, nullptr, H->st, nsys, H->hphase,
                                            H->hphase ? H->ptab64 : nullptr);
  helm_inner<double>(H, true, w, nullptr, K_HLM_YF, nsys);
  fftg::launch_h_div_fwd<double>(H->plan[oa], TW<double>(H, oa), g, zo, H->S64, x, w, Ap,
                                 nullptr, nullptr, H->st, nsys);
}

// Largest number of FP64 refinement sweeps of one FP32-refined Helmholtz solve.
constexpr int kHelmSweeps = 30;

// FP32-refined handles: iterative refinement of Algorithm 2 (Sec. 3.2.3) for
// nsys stacked fields in lockstep.  x and b live in FP64 on the half
// spectrum; each sweep forms the FP64 residual r = b - L x with the FP64
// operator (FP64 ell2), solves L d = r with the FP32 PCG (b rounded to FP32,
// d0 = 0), and adds d to x in FP64.  A field stops when its FP64 residual
// meets ||r|| <= tol ||b|| (status 1), when its FP32 iterations reach maxit
// (2), on a breakdown (3, 4), or when a sweep no longer halves its FP64
// residual (5: the attainable accuracy is reached); the others go on.
void helmholtz_refined(fftg_handle* H, const double* alpha, const float* ell2_32,
                       const double* ell2_64, double ell2_ref, double* abar, double tol,
                       int maxit, int nsys, HelmOut* out, const unsigned char* skip = nullptr,
                       std::vector<double>* refc = nullptr) {
  const Geo& g = H->g;
  const long long Ns = g.Ns;
  cpx<double>* S = H->spec64;
  if (nsys > 1) {
    if (H->ref64_cap < nsys) {
      dfree((void*&)H->ref64);
      H->ref64 = (cpx<double>*)dalloc(sizeof(cpx<double>) * 6 * (size_t)nsys * Ns);
      H->ref64_cap = nsys;
    }
    S = H->ref64;
  }
  // b [sys], x [sys], gradient fields [3][sys], L x [sys]
  cpx<double>* b = S;
  cpx<double>* x = S + nsys * Ns;
  cpx<double>* w = S + 2 * nsys * Ns;
  cpx<double>* Ax = S + 5 * nsys * Ns;
  fwd_fields(H, nsys, alpha, b, skip);
  for (int q = 0; q < nsys; ++q)
    if (skip && skip[q]) {
      HIPCHK(hipMemsetAsync(b + q * Ns, 0, sizeof(cpx<double>) * Ns, H->st));
      HIPCHK(hipMemsetAsync(x + q * Ns, 0, sizeof(cpx<double>) * Ns, H->st));
    }
  fftg::launch_hermitize<double>(g, nsys, b, H->st);
  std::vector<double> bb(nsys), ref(nsys), rr(nsys), rr_prev(nsys), tin(nsys);
  std::vector<int> mits(nsys);
  read_sums(H, fftg::launch_wnorm2<double>(g, 1, b, H->partials, H->st, nsys), nsys, bb.data());
  ell2_reference<float>(H, ell2_32, ell2_ref, nsys, ref.data(), refc);
  fwd_fields(H, nsys, abar, x, skip);
  fftg::launch_hermitize<double>(g, nsys, x, H->st);
  int active = 0;
  for (int q = 0; q < nsys; ++q) {
    out[q] = HelmOut{};
    rr[q] = 0.0;
    rr_prev[q] = HUGE_VAL;
    if (skip && skip[q]) {
      out[q].status = 1;  // not solved here
    } else if (bb[q] == 0.0) {
      // a zero source has the zero solution
      HIPCHK(hipMemsetAsync(x + q * Ns, 0, sizeof(cpx<double>) * Ns, H->st));
      out[q].status = 1;
    } else {
      ++active;
    }
  }
  for (int sweep = 0; active > 0; ++sweep) {
    helm_apply64(H, x, w, Ax, ell2_64, nsys);
    read_sums(H, fftg::launch_h_refine_resid(g, b, Ax, C<float>(H->hb), H->partials, H->st, nsys),
              nsys, rr.data());
    for (int q = 0; q < nsys; ++q) {
      tin[q] = -1.0;  // no correction for this field
      mits[q] = 0;
      if (out[q].status != 0) continue;
      if (!std::isfinite(rr[q])) throw Fail{FFTG_E_NONFINITE, "non-finite Helmholtz residual"};
      if (rr[q] <= tol * tol * bb[q])
        out[q].status = 1;
      else if (sweep > 0 && !(rr[q] < 0.25 * rr_prev[q]))
        out[q].status = 5;
      else if (out[q].iters >= maxit || sweep >= kHelmSweeps)
        out[q].status = 2;
      if (out[q].status != 0) {
        --active;
        continue;
      }
      rr_prev[q] = rr[q];
      // the correction only has to bring ||r|| below tol ||b|| (with a
      // margin); FP32 vectors do not resolve more than ~1e-5 of their
      // right-hand side
      tin[q] = std::min(0.5, std::max(kFp32KrylovFloor, 0.5 * tol * std::sqrt(bb[q] / rr[q])));
      mits[q] = maxit - out[q].iters;
    }
    if (active == 0) break;
    std::vector<KrylovCtl> k(nsys);
    helm_krylov<float>(H, ell2_32, nsys, ref.data(), rr.data(), tin.data(), mits.data(), true,
                       k.data());
    for (int q = 0; q < nsys; ++q) {
      if (tin[q] < 0.0) continue;
      out[q].iters += k[q].iters;
      if (k[q].done == 3 || k[q].done == 4) {
        out[q].status = k[q].done;
        --active;
      }
    }
    fftg::launch_acc_wide<float>(2 * Ns * nsys, reinterpret_cast<const float*>(H->hx),
                                 reinterpret_cast<double*>(x), H->st);
  }
  inv_fields(H, nsys, x, abar, skip);
  check_launch();
  for (int q = 0; q < nsys; ++q) {
    if (skip && skip[q]) continue;
    if (verbose())
      std::fprintf(stderr, "[fftg] refined pcg field %d iters %d status %d rr/bb %.3e ell2ref %.4g\n",
                   q, out[q].iters, out[q].status, bb[q] > 0 ? rr[q] / bb[q] : 0.0, ref[q]);
    out[q].relres = bb[q] > 0 ? std::sqrt(rr[q] / bb[q]) : 0.0;
  }
}

// Algorithm 2 for nsys stacked fields on the handle's precision: ell2w is
// the work-precision ell2 [sys][N] (FP32 on FP32-refined handles), ell2_64
// the FP64 one (read by the FP64 residuals of the refinement; equal to ell2w
// on FP64 handles).  skip (optional): fields not to solve (abar untouched).
// refc (optional): reference lengths of earlier solves on the same fields
// (ell2_reference).
void helm_solve(fftg_handle* H, const double* alpha, const void* ell2w, const double* ell2_64,
                double ell2_ref, double* abar, double tol, int maxit, int nsys, HelmOut* out,
                const unsigned char* skip = nullptr, std::vector<double>* refc = nullptr) {
  if (nsys < 1) throw Fail{FFTG_E_INVALID, "no Helmholtz field"};
  ensure_sys(H, nsys);
  alloc_helm(H, nsys);
  if (H->fp32())
    helmholtz_refined(H, alpha, reinterpret_cast<const float*>(ell2w), ell2_64, ell2_ref, abar,
                      tol, maxit, nsys, out, skip, refc);
  else
    helmholtz_pcg64(H, alpha, ell2_64, ell2_ref, abar, tol, maxit, nsys, out, skip, refc);
}

// ------------------------------------------------------------ mechanics
// out (=|+=) F^-1(x) for the Galerkin CG solution x in H->kx.  With FP32
// Krylov vectors the solution is widened to FP64, projected again with the
// FP64 G* (its zero frequency: the mask) and transformed back in FP64: the
// FP32 iteration and an FP32 inverse leave rounding outside the compatible
// space range(G*) (~1e-7 of the correction), which the FP64 Newton residual
// G*(sigma - Sbar) cannot see and so would never remove from the strain.
// kx: the solution spectrum (work precision), spec: an FP64 c-component
// spectrum of scratch.
template <typename T>
void galerkin_solution_at(fftg_handle* H, const unsigned char* mask, void* kx,
                          cpx<double>* spec, double* out, bool acc) {
  const Geo& g = H->g;
  const int c = H->c;
  if (std::is_same<T, float>::value) {
    fftg::launch_convert<float, double>(2LL * c * g.Ns, reinterpret_cast<const float*>(kx),
                                        reinterpret_cast<double*>(spec), H->st);
    fftg::launch_project<double>(g, c, H->S64, mask, spec, H->st);
    inv3<double, double>(H, c, spec, out, 1.0 / (double)g.N, acc);
  } else {
    inv3<T, double>(H, c, C<T>(kx), out, T(1.0 / (double)g.N), acc);
  }
}
template <typename T>
void galerkin_solution(fftg_handle* H, const unsigned char* mask, double* out, bool acc) {
  galerkin_solution_at<T>(H, mask, H->kx, H->spec64, out, acc);
}

struct MechOut {
  int newton = 0, cg = 0;
  double relres = 0.0;
  bool converged = false;
  double t_const = 0.0, t_cg = 0.0;
};

void comp_means(fftg_handle* H, int ncomp, const double* f, double* out) {
  read_sums(H, fftg::launch_comp_sums(H->g.N, ncomp, f, H->partials, H->st), ncomp, out);
  for (int k = 0; k < ncomp; ++k) out[k] /= (double)H->g.N;
}

// Means of ncomp fields of several RVEs with one read-back: f[k] (device,
// [ncomp][N]) -> out[6 k + i].  Each is summed as comp_means sums it.  Needs
// ensure_sys(n) for n >= f.size() / 2.
void batch_means(fftg_handle* H, int ncomp, const std::vector<const double*>& f,
                 std::vector<double>& out) {
  const int n = (int)f.size();
  out.assign(6 * (size_t)n, 0.0);
  if (n == 0) return;
  const long long stride = 6LL * fftg::RED_BLOCKS;  // comp_sums partials of one field set
  for (int k = 0; k < n; ++k) {
    double* part = H->partials + k * stride;
    const int nb = fftg::launch_comp_sums(H->g.N, ncomp, f[k], part, H->st);
    fftg::launch_fin_sums(part, nb, ncomp, H->dsums + 6 * k, H->st);
  }
  HIPCHK(hipMemcpyAsync(H->hsums, H->dsums, sizeof(double) * 6 * n, hipMemcpyDeviceToHost,
                        H->st));
  sync(H);
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < ncomp; ++i) out[6 * k + i] = H->hsums[6 * k + i] / (double)H->g.N;
}

double wall_ms(std::chrono::steady_clock::time_point a) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
}

template <typename T>
MechOut mechanics(fftg_handle* H, const unsigned char* phase, const MatTable& tab, int J,
                  const double* D, const double* state_n, const fftg_macro* tgt, double* eps,
                  double* sigma, double* st_np1, double* alpha, const fftg_krylov_opts* cg,
                  double ntol, int nmaxit, int newton_div = 0) {
  const Geo& g = H->g;
  const int c = H->c;
  MechOut o;
  o.relres = HUGE_VAL;
  int grown = 0;  // consecutive corrections after which the residual grew
  // move the strain-controlled means to their targets
  double mean[6], delta[6] = {0, 0, 0, 0, 0, 0};
  comp_means(H, c, eps, mean);
  bool any = false;
  for (int k = 0; k < c; ++k)
    if (!tgt->mask[k]) {
      delta[k] = tgt->E[k] - mean[k];
      any = any || delta[k] != 0.0;
    }
  if (any) fftg::launch_add_const(g.N, c, eps, delta, H->st);
  double sref = 0.0;
  for (int p = 0; p < tab.nphase; ++p) sref = std::max(sref, tab.m[p].sy);
  if (!(sref > 0.0)) sref = 1.0;
  double Sbar[6] = {0, 0, 0, 0, 0, 0};
  for (int k = 0; k < c; ++k) Sbar[k] = tgt->mask[k] ? tgt->S[k] : 0.0;
  const double sqN = std::sqrt((double)g.N);
  int r = 0;
  while (true) {
    auto t0 = std::chrono::steady_clock::now();
    {
      KT t(H, K_CONST);
      fftg::launch_constitutive<T>(tab, g, c, J, phase, eps, state_n, D, sigma, st_np1, alpha,
                                   reinterpret_cast<T*>(H->tan), H->st);
    }
    H->tan_valid = true;
    check_launch();
    sync(H);
    o.t_const += wall_ms(t0);
    t0 = std::chrono::steady_clock::now();
    fwd3<double>(H, c, sigma, H->spec64);
    fftg::launch_hermitize<double>(g, c, H->spec64, H->st);
    const int nr = fftg::launch_gal_rhs<T>(g, c, H->S64, tgt->mask, Sbar, H->spec64, C<T>(H->kr),
                                           H->partials, H->st);
    double s2[2];
    read_sums(H, nr, 2, s2);
    const double nb = std::sqrt(s2[0] / (double)g.N), ns = std::sqrt(s2[1] / (double)g.N);
    const double prev = o.relres;
    o.relres = nb / std::max(ns, sref * sqN);
    if (!std::isfinite(o.relres)) throw Fail{FFTG_E_NONFINITE, "non-finite Newton residual"};
    grown = (r >= 1 && o.relres > prev) ? grown + 1 : 0;
    if (r >= 1 && o.relres <= ntol) {
      o.converged = true;
      o.t_cg += wall_ms(t0);
      break;
    }
    if (newton_div > 0 && grown >= newton_div) {
      o.t_cg += wall_ms(t0);
      break;
    }
    if (r >= nmaxit) {
      o.t_cg += wall_ms(t0);
      break;
    }
    int it = 0, status = 0;
    // FP32 Krylov vectors cannot push the residual much below 1e-6 of |b|
    // (rounding of b itself); the FP64 Newton residual refines the rest.
    const double cgtol = H->fp32() ? std::max(cg->tol, kFp32KrylovFloor) : cg->tol;
    std::memcpy(H->mask_last, tgt->mask, 6);
    galerkin_cg<T>(H, tgt->mask, s2[0], cgtol, cg->maxit, it, status);
    if (verbose()) {
      const KrylovCtl kk = *H->hctl;
      std::fprintf(stderr, "[fftg] newton %d relres %.3e |b| %.3e cg %d status %d rr/bb %.3e\n", r,
                   o.relres, nb, it, status, kk.rr / kk.bb);
    }
    if (status == 3) throw Fail{FFTG_E_BREAKDOWN, "Galerkin CG breakdown (p.Ap <= 0)"};
    if (status == 4) throw Fail{FFTG_E_NONFINITE, "non-finite value in Galerkin CG"};
    o.cg += it;
    galerkin_solution<T>(H, tgt->mask, eps, true);
    check_launch();
    sync(H);
    o.t_cg += wall_ms(t0);
    ++r;
  }
  o.newton = r;
  return o;
}

// ------------------------------------------------------------ workspace
// squared lengths of every field on the grid: work precision in H->ell2j, and
// FP64 in H->ell2j64 on FP32-refined handles
void fill_ell2(fftg_handle* H, const MatTable& t, int J, const unsigned char* phase) {
  const long long N = H->g.N;
  for (int j = 0; j < J; ++j) {
    if (H->fp32()) {
      fftg::launch_ell2<float>(t, N, j, phase, reinterpret_cast<float*>(H->ell2j) + j * N, H->st);
      fftg::launch_ell2<double>(t, N, j, phase, H->ell2j64 + j * N, H->st);
    } else {
      fftg::launch_ell2<double>(t, N, j, phase, reinterpret_cast<double*>(H->ell2j) + j * N,
                                H->st);
    }
  }
}
// field j's squared lengths: work precision, FP64
const void* ell2w_of(fftg_handle* H, int j) {
  return static_cast<const char*>(H->ell2j) + H->wsz() * (size_t)j * (size_t)H->g.N;
}
const double* ell2d_of(fftg_handle* H, int j) {
  return (H->fp32() ? H->ell2j64 : reinterpret_cast<const double*>(H->ell2j)) + (long long)j * H->g.N;
}

void alloc_stagger(fftg_handle* H, int J) {
  if (H->stJ >= J) return;
  dfree((void*&)H->eps_k);
  dfree((void*&)H->eps_prev);
  dfree((void*&)H->ab_k);
  dfree((void*&)H->ab_prev);
  dfree((void*&)H->Dj);
  dfree((void*&)H->alph);
  dfree((void*&)H->st1);
  dfree((void*&)H->sig_k);
  dfree(H->ell2j);
  dfree((void*&)H->ell2j64);
  const size_t N = H->g.N;
  const size_t Jm = J > 0 ? J : 1;
  H->eps_k = (double*)dalloc(sizeof(double) * H->c * N);
  H->eps_prev = (double*)dalloc(sizeof(double) * H->c * N);
  H->sig_k = (double*)dalloc(sizeof(double) * H->c * N);
  H->ab_k = (double*)dalloc(sizeof(double) * Jm * N);
  H->ab_prev = (double*)dalloc(sizeof(double) * Jm * N);
  H->Dj = (double*)dalloc(sizeof(double) * Jm * N);
  H->alph = (double*)dalloc(sizeof(double) * Jm * N);
  H->st1 = (double*)dalloc(sizeof(double) * 7 * N);
  H->ell2j = dalloc(H->wsz() * Jm * N);
  if (H->fp32()) H->ell2j64 = (double*)dalloc(sizeof(double) * Jm * N);
  H->stJ = J;
}

void destroy(fftg_handle* H) {
  for (int a = 0; a < 3; ++a) {
    dfree((void*&)H->tw64[a]);
    dfree((void*&)H->tw32[a]);
  }
  dfree((void*&)H->sym64);
  dfree((void*&)H->sym32);
  dfree(H->kx);
  dfree(H->kr);
  dfree(H->kp);
  dfree(H->kw);
  dfree((void*&)H->spec64);
  dfree(H->tan);
  dfree((void*&)H->partials);
  dfree((void*&)H->dsums);
  dfree((void*&)H->ctl);
  if (H->hctl) (void)hipHostFree(H->hctl);
  if (H->hsums) (void)hipHostFree(H->hsums);
  dfree(H->ptab);
  dfree((void*&)H->ptab64);
  if (H->hptab) (void)hipHostFree(H->hptab);
  dfree(H->hx);
  dfree(H->hr);
  dfree(H->hp);
  dfree(H->hAp);
  dfree(H->hb);
  dfree(H->hw);
  dfree(H->rtmp);
  dfree(H->ell2w);
  dfree((void*&)H->ref64);
  dfree((void*&)H->eps_k);
  dfree((void*&)H->eps_prev);
  dfree((void*&)H->ab_k);
  dfree((void*&)H->ab_prev);
  dfree((void*&)H->Dj);
  dfree((void*&)H->alph);
  dfree((void*&)H->st1);
  dfree((void*&)H->sig_k);
  dfree(H->ell2j);
  dfree((void*&)H->ell2j64);
  dfree((void*&)H->drive_bak);
  free_bws(H);
  dfree((void*&)H->adj_r);
  dfree((void*&)H->sadj);
  dfree((void*&)H->hadj);
  for (auto& e : H->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& p : H->pend) {
    H->evpool.push_back(p.a);
    H->evpool.push_back(p.b);
  }
  for (auto e : H->evpool) (void)hipEventDestroy(e);
  H->evpool.clear();
  H->ggal.drop();
  for (auto& sl : H->ghelm) sl.drop();
  if (H->cap) (void)hipStreamDestroy(H->cap);
}

fftg_status run_guarded(fftg_handle* H, const std::function<fftg_status()>& f) {
  try {
    return f();
  } catch (const Fail& e) {
    if (H) H->err = e.msg;
    return e.code;
  } catch (const HipError& e) {
    if (H) H->err = e.msg;
    return FFTG_E_HIP;
  } catch (const std::exception& e) {
    if (H) H->err = e.what();
    return FFTG_E_HIP;
  }
}
}  // namespace

// ============================================================ C ABI
// ------------------------------------------------------------ adjoints
// dell2(x) = -sum_j (G_j a)(x) (G_j b)(x), G_j = F^-1 diag(i q~_j) F, all in
// FP64 (spec64 components 0..3 and two real scratch fields as workspace).
void grad_dot(fftg_handle* H, const double* a, const double* b, double* out) {
  const Geo& g = H->g;
  const long long Ns = g.Ns;
  if (!H->adj_r) H->adj_r = (double*)dalloc(sizeof(double) * 2 * (size_t)g.N);
  cpx<double>* S = H->spec64;
  fwd3<double>(H, 1, a, S);
  fwd3<double>(H, 1, b, S + Ns);
  for (int j = 0; j < g.ndim; ++j) {
    fftg::launch_grad_comp<double>(g, H->S64, j, S, S + 2 * Ns, H->st);
    inv3<double, double>(H, 1, S + 2 * Ns, H->adj_r, 1.0 / (double)g.N, false);
    fftg::launch_grad_comp<double>(g, H->S64, j, S + Ns, S + 3 * Ns, H->st);
    inv3<double, double>(H, 1, S + 3 * Ns, H->adj_r + g.N, 1.0 / (double)g.N, false);
    fftg::launch_sub_prod(g.N, H->adj_r, H->adj_r + g.N, out, j > 0, H->st);
  }
  check_launch();
}

// Adjoint of the mechanics solve at frozen damage: mu = (G* K)^-1 G*(gbar)
// with the tangent at eps, then dD.
template <typename T>
int mech_adjoint(fftg_handle* H, const unsigned char* phase, const MatTable& tab, int J,
                 const double* D, const double* state_n, const fftg_macro* tgt,
                 const double* eps, const double* gbar, const double* gsig, double* mu,
                 double* dD, const fftg_krylov_opts* cg, int& status) {
  const Geo& g = H->g;
  const int c = H->c;
  alloc_stagger(H, J);
  fftg::launch_constitutive<T>(tab, g, c, J, phase, eps, state_n, D, H->sig_k, H->st1, H->alph,
                               reinterpret_cast<T*>(H->tan), H->st);
  H->tan_valid = true;
  // strain cotangent g = gbar + K gsig; b = -G*(F(-g) - 0) = G* F(g)
  const double* gtot = gbar;
  if (gsig) {
    fftg::launch_tangent_apply<T>(g.N, c, reinterpret_cast<const T*>(H->tan), gsig, gbar,
                                  H->eps_k, H->st);
    gtot = H->eps_k;
  }
  fftg::launch_scale((long long)c * g.N, -1.0, gtot, H->eps_prev, H->st);
  fwd3<double>(H, c, H->eps_prev, H->spec64);
  fftg::launch_hermitize<double>(g, c, H->spec64, H->st);
  const double zero6[6] = {0, 0, 0, 0, 0, 0};
  const int nr = fftg::launch_gal_rhs<T>(g, c, H->S64, tgt->mask, zero6, H->spec64, C<T>(H->kr),
                                         H->partials, H->st);
  double s2[2];
  read_sums(H, nr, 2, s2);
  const double cgtol = H->fp32() ? std::max(cg->tol, kFp32KrylovFloor) : cg->tol;
  std::memcpy(H->mask_last, tgt->mask, 6);
  int it = 0;
  galerkin_cg<T>(H, tgt->mask, s2[0], cgtol, cg->maxit, it, status);
  if (status == 3) throw Fail{FFTG_E_BREAKDOWN, "Galerkin CG breakdown (p.Ap <= 0)"};
  if (status == 4) throw Fail{FFTG_E_NONFINITE, "non-finite value in Galerkin CG"};
  galerkin_solution<T>(H, tgt->mask, mu, false);
  if (J > 0) fftg::launch_adj_damage(tab, g.N, c, J, phase, D, H->sig_k, mu, gsig, dD, H->st);
  check_launch();
  sync(H);
  return it;
}

// ell^2 of the fields of one RVE as per-phase tables for the Helmholtz x
// pass (the values k_ell2 writes into the ell^2 fields), and its phase array;
// the guard clears the phase array again when the staggered step ends.
void set_helm_phase(fftg_handle* H, const unsigned char* phase, const MatTable& t, int J) {
  const int nt = FFTG_MAX_FIELDS * fftg::kMaxPhases;
  double* h64 = H->hptab;
  float* h32 = reinterpret_cast<float*>(H->hptab + nt);
  for (int j = 0; j < J; ++j)
    for (int p = 0; p < fftg::kMaxPhases; ++p) {
      const double v = t.m[p < t.nphase ? p : 0].ell2[j];
      h64[j * fftg::kMaxPhases + p] = v;
      h32[j * fftg::kMaxPhases + p] = (float)v;
    }
  const size_t n = (size_t)J * fftg::kMaxPhases;
  HIPCHK(hipMemcpyAsync(H->ptab64, h64, sizeof(double) * n, hipMemcpyHostToDevice, H->st));
  if (H->fp32())
    HIPCHK(hipMemcpyAsync(H->ptab, h32, sizeof(float) * n, hipMemcpyHostToDevice, H->st));
  else
    HIPCHK(hipMemcpyAsync(H->ptab, h64, sizeof(double) * n, hipMemcpyHostToDevice, H->st));
  H->hphase = phase;
}
struct PhaseGuard {
  fftg_handle* H;
  ~PhaseGuard() { H->hphase = nullptr; }
};

// One increment of Algorithm 1 on a validated call.  abort_on_mech: leave
// the staggered loop as soon as a mechanics solve fails (adaptive driver);
// newton_div: Newton divergence guard (0 = off).
struct StaggerOut {
  fftg_stats stats{};
  bool converged = false;  // ERR <= stagger_tol
  bool mech_ok = false;    // the last mechanics solve converged
  bool inner_ok = false;   // every inner solve of the last pass met its stop test
};

StaggerOut stagger_core(fftg_handle* H, const unsigned char* phase, const MatTable& t, int J,
                        double* state, const fftg_macro* target, const fftg_krylov_opts* cg,
                        const fftg_krylov_opts* pcg, double newton_tol, int newton_maxit,
                        double stagger_tol, int max_stagger_iters, double* sigma_out,
                        double* homog_out, bool abort_on_mech, int newton_div) {
  StaggerOut out;
  auto t_all = std::chrono::steady_clock::now();
  const Geo& g = H->g;
  const int c = H->c;
  const long long N = g.N;
  alloc_stagger(H, J);
  alloc_helm(H);
  double* s_eps = state;
  double* s_epsp = state + (long long)c * N;  // eps_p (6) followed by kappa (1)
  double* s_hist = state + (long long)(c + 7) * N;
  double* s_abar = state + (long long)(c + 7 + J) * N;
  HIPCHK(hipMemcpyAsync(H->eps_k, s_eps, sizeof(double) * c * N, hipMemcpyDeviceToDevice, H->st));
  if (J > 0)
    HIPCHK(hipMemcpyAsync(H->ab_k, s_abar, sizeof(double) * J * N, hipMemcpyDeviceToDevice,
                          H->st));
  fill_ell2(H, t, J, phase);
  PhaseGuard pg{H};
  if (J > 0) set_helm_phase(H, phase, t, J);
  fftg_stats acc{};
  bool converged = false;
  int k = 0;
  double err = 0.0;
  std::vector<double> ell2_means;  // preconditioner lengths, fixed within the step
  for (k = 0; k < max_stagger_iters; ++k) {
    if (J > 0) fftg::launch_damage(t, N, J, phase, H->ab_k, s_hist, s_abar, H->Dj, H->st);
    HIPCHK(hipMemcpyAsync(H->eps_prev, H->eps_k, sizeof(double) * c * N,
                          hipMemcpyDeviceToDevice, H->st));
    MechOut o = H->fp32()
                    ? mechanics<float>(H, phase, t, J, H->Dj, s_epsp, target, H->eps_k,
                                       H->sig_k, H->st1, H->alph, cg, newton_tol, newton_maxit, newton_div)
                    : mechanics<double>(H, phase, t, J, H->Dj, s_epsp, target, H->eps_k,
                                        H->sig_k, H->st1, H->alph, cg, newton_tol,
                                        newton_maxit, newton_div);
    acc.newton_iters += o.newton;
    out.mech_ok = o.converged;
    out.inner_ok = o.converged;
    acc.cg_iters += o.cg;
    acc.relres = o.relres;
    acc.t_ms[0] += o.t_const;
    acc.t_ms[1] += o.t_cg;
    if (abort_on_mech && !o.converged) {
      acc.stagger_iters = k + 1;
      break;
    }
    auto th = std::chrono::steady_clock::now();
    if (J > 0)
      HIPCHK(hipMemcpyAsync(H->ab_prev, H->ab_k, sizeof(double) * J * N,
                            hipMemcpyDeviceToDevice, H->st));
    if (J > 0) {
      // every field's Helmholtz solve (Algorithm 1 (ii)) at once, in lockstep
      HelmOut ho[FFTG_MAX_FIELDS];
      helm_solve(H, H->alph, ell2w_of(H, 0), ell2d_of(H, 0), -1.0, H->ab_k, pcg->tol,
                 pcg->maxit, J, ho, nullptr, &ell2_means);
      for (int j = 0; j < J; ++j) {
        if (ho[j].status == 3) throw Fail{FFTG_E_BREAKDOWN, "Helmholtz PCG breakdown"};
        if (ho[j].status == 4) throw Fail{FFTG_E_NONFINITE, "non-finite value in Helmholtz PCG"};
        // maxit (2) or a stall at the rounding floor (5): not at tolerance
        out.inner_ok = out.inner_ok && ho[j].status == 1;
        acc.pcg_iters += ho[j].iters;
      }
    }
    sync(H);
    acc.t_ms[2] += wall_ms(th);
    // staggered error (Algorithm 1 (iii))
    const int nbe = fftg::launch_stagger_err(N, c, J, H->eps_k, H->eps_prev, H->ab_k,
                                             H->ab_prev, H->partials, H->st);
    // block partials: [0] max of |d eps|^2, then per field sum d^2, sum abar^2
    std::vector<double> part((size_t)nbe * (1 + 2 * J));
    HIPCHK(hipMemcpyAsync(part.data(), H->partials, sizeof(double) * part.size(),
                          hipMemcpyDeviceToHost, H->st));
    sync(H);
    double mx = 0.0;
    for (int b = 0; b < nbe; ++b) mx = std::max(mx, part[b]);
    double mean[6];
    comp_means(H, c, H->eps_k, mean);
    double mn = 0.0;
    for (int i = 0; i < c; ++i) mn += mean[i] * mean[i];
    mn = std::sqrt(mn);
    err = std::sqrt(mx) / (mn > 0.0 ? mn : 1.0);
    for (int j = 0; j < J; ++j) {
      double d2 = 0.0, a2 = 0.0;
      for (int b = 0; b < nbe; ++b) {
        d2 += part[(size_t)(1 + 2 * j) * nbe + b];
        a2 += part[(size_t)(2 + 2 * j) * nbe + b];
      }
      if (d2 > 0.0) err = std::max(err, std::sqrt(d2) / std::max(std::sqrt(a2), 1e-12 * std::sqrt((double)N)));
    }
    acc.stagger_iters = k + 1;
    acc.err = err;
    if (err <= stagger_tol) {
      converged = true;
      break;
    }
  }
  // commit the increment
  HIPCHK(hipMemcpyAsync(s_eps, H->eps_k, sizeof(double) * c * N, hipMemcpyDeviceToDevice, H->st));
  HIPCHK(hipMemcpyAsync(s_epsp, H->st1, sizeof(double) * 7 * N, hipMemcpyDeviceToDevice, H->st));
  if (J > 0) {
    fftg::launch_commit_hist(t, N, J, phase, H->ab_k, s_abar, s_hist, H->st);
    HIPCHK(hipMemcpyAsync(s_abar, H->ab_k, sizeof(double) * J * N, hipMemcpyDeviceToDevice,
                          H->st));
  }
  HIPCHK(hipMemcpyAsync(sigma_out, H->sig_k, sizeof(double) * c * N, hipMemcpyDeviceToDevice,
                        H->st));
  double ms[6], me[6];
  comp_means(H, c, H->sig_k, ms);
  comp_means(H, c, H->eps_k, me);
  for (int i = 0; i < 12; ++i) homog_out[i] = 0.0;
  for (int i = 0; i < c; ++i) {
    homog_out[i] = ms[i];
    homog_out[6 + i] = me[i];
  }
  check_launch();
  sync(H);
  const double tot = wall_ms(t_all);
  acc.t_ms[3] = std::max(0.0, tot - acc.t_ms[0] - acc.t_ms[1] - acc.t_ms[2]);
  acc.inner_converged = out.inner_ok ? 1 : 0;
  out.stats = acc;
  out.converged = converged;
  return out;
}

// ------------------------------------------------------------ lockstep batch
// Several RVEs of one grid, precision, field count and macro mask (a class)
// advance through one increment of Algorithm 1 together, stacked on the lead
// handle's workspace: each Galerkin CG iteration and each Helmholtz PCG
// iteration is one set of launches over all of them (per-RVE scalars, stop
// tests and control blocks; an RVE that has met its test returns at once
// from every launch), while the per-voxel and once-per-Newton-step work runs
// RVE by RVE.  Every RVE takes exactly the arithmetic of its own
// staggered_step: no tile, line pair or reduction spans two RVEs.

// One RVE of a class: its item, table and packed state, its slot views of
// the class workspace, and its progress through the increment.
struct BSys {
  fftg_batch_item* it = nullptr;
  MatTable tab{};
  int q = 0;  // slot
  double *s_eps = nullptr, *s_epsp = nullptr, *s_hist = nullptr, *s_abar = nullptr;
  double *eps = nullptr, *eps_prev = nullptr, *sig = nullptr, *st1 = nullptr, *D = nullptr,
         *alph = nullptr, *ab = nullptr, *ab_prev = nullptr;
  void *tan = nullptr, *kx = nullptr, *kr = nullptr;
  cpx<double>* spec = nullptr;
  double Sbar[6] = {0, 0, 0, 0, 0, 0};
  double sref = 1.0;
  bool live = true;  // still in the staggered loop
  bool converged = false, inner_ok = false, committed = false;
  fftg_status fail = FFTG_OK;
  std::string msg;
  fftg_stats acc{};
  // Newton loop of the current pass
  MechOut o;
  int r = 0;
  bool nl = false;
};

void bsys_fail(BSys& s, fftg_status code, const char* msg) {
  s.fail = code;
  s.msg = msg;
  s.live = false;
  s.nl = false;
}

void alloc_bws(fftg_handle* H, int nsys, int J) {
  const int Jm = std::max(J, 1);
  if (H->bws && H->bws->cap_sys >= nsys && H->bws->cap_J >= Jm) return;
  drop_graphs(H);  // the Helmholtz graphs may hold the old ell2
  free_bws(H);
  BatchWS* B = new BatchWS();
  H->bws = B;
  const size_t N = H->g.N, n = nsys, c = H->c;
  B->eps_k = (double*)dalloc(sizeof(double) * c * N * n);
  B->eps_prev = (double*)dalloc(sizeof(double) * c * N * n);
  B->sig_k = (double*)dalloc(sizeof(double) * c * N * n);
  B->st1 = (double*)dalloc(sizeof(double) * 7 * N * n);
  B->Dj = (double*)dalloc(sizeof(double) * Jm * N * n);
  B->alph = (double*)dalloc(sizeof(double) * Jm * N * n);
  B->ab_k = (double*)dalloc(sizeof(double) * Jm * N * n);
  B->ab_prev = (double*)dalloc(sizeof(double) * Jm * N * n);
  B->ell2j = dalloc(H->wsz() * Jm * N * n);
  if (H->fp32()) B->ell2j64 = (double*)dalloc(sizeof(double) * Jm * N * n);
  B->cap_sys = nsys;
  B->cap_J = Jm;
}

// The Newton loop of Algorithm 1 (i) for every live RVE of a class (the
// steps of mechanics(), RVE by RVE, with one lockstep Galerkin CG per Newton
// step over the RVEs that need a correction).
template <typename T>
void mechanics_batch(fftg_handle* H, std::vector<BSys>& S, const unsigned char* mask,
                     const fftg_krylov_opts* cg, double ntol, int nmaxit) {
  const Geo& g = H->g;
  const int c = H->c;
  const int n = (int)S.size();
  const double sqN = std::sqrt((double)g.N);
  std::vector<const double*> fl;
  for (auto& s : S) {
    s.nl = s.live;
    s.o = MechOut{};
    s.o.relres = HUGE_VAL;
    s.r = 0;
    if (s.nl) fl.push_back(s.eps);
  }
  std::vector<double> mv;
  batch_means(H, c, fl, mv);
  int km = 0;
  for (auto& s : S) {
    if (!s.nl) continue;
    // move the strain-controlled means to their targets
    const double* mean = &mv[6 * km++];
    double delta[6] = {0, 0, 0, 0, 0, 0};
    bool any = false;
    for (int k = 0; k < c; ++k)
      if (!mask[k]) {
        delta[k] = s.it->target.E[k] - mean[k];
        any = any || delta[k] != 0.0;
      }
    if (any) fftg::launch_add_const(g.N, c, s.eps, delta, H->st);
  }
  std::vector<double> bb(n, 0.0);
  std::vector<unsigned char> need(n, 0);
  std::vector<KrylovCtl> k(n);
  while (true) {
    auto t0 = std::chrono::steady_clock::now();
    bool any = false;
    for (auto& s : S) {
      if (!s.nl) continue;
      any = true;
      KT t(H, K_CONST);
      fftg::launch_constitutive<T>(s.tab, g, c, s.it->nfields, s.it->phase, s.eps, s.s_epsp,
                                   s.D, s.sig, s.st1, s.alph, reinterpret_cast<T*>(s.tan),
                                   H->st);
    }
    if (!any) break;
    check_launch();  // no wait: the residual read-back below waits for the stream
    const double tc = wall_ms(t0);
    t0 = std::chrono::steady_clock::now();
    for (auto& s : S) {
      if (!s.nl) continue;
      s.o.t_const += tc;
      fwd3<double>(H, c, s.sig, s.spec);
      fftg::launch_hermitize<double>(g, c, s.spec, H->st);
      double* part = H->partials + (long long)s.q * H->psys;
      const int nr = fftg::launch_gal_rhs<T>(g, c, H->S64, mask, s.Sbar, s.spec, C<T>(s.kr),
                                             part, H->st);
      fftg::launch_fin_sums(part, nr, 2, H->dsums + 2 * s.q, H->st);
    }
    HIPCHK(hipMemcpyAsync(H->hsums, H->dsums, sizeof(double) * 2 * n, hipMemcpyDeviceToHost,
                          H->st));
    sync(H);
    bool anycg = false;
    for (auto& s : S) {
      need[s.q] = 0;
      if (!s.nl) continue;
      const double* s2 = H->hsums + 2 * s.q;
      const double nb = std::sqrt(s2[0] / (double)g.N), ns = std::sqrt(s2[1] / (double)g.N);
      s.o.relres = nb / std::max(ns, s.sref * sqN);
      if (!std::isfinite(s.o.relres)) {
        bsys_fail(s, FFTG_E_NONFINITE, "non-finite Newton residual");
        continue;
      }
      if ((s.r >= 1 && s.o.relres <= ntol) || s.r >= nmaxit) {
        s.o.converged = s.r >= 1 && s.o.relres <= ntol;
        s.nl = false;
        s.o.t_cg += wall_ms(t0);
        continue;
      }
      need[s.q] = 1;
      bb[s.q] = s2[0];
      anycg = true;
    }
    if (!anycg) break;
    // FP32 Krylov vectors cannot push the residual much below 1e-6 of |b|;
    // the FP64 Newton residual refines the rest
    const double cgtol = H->fp32() ? std::max(cg->tol, kFp32KrylovFloor) : cg->tol;
    std::memcpy(H->mask_last, mask, 6);
    galerkin_cg_n<T>(H, mask, n, bb.data(), need.data(), cgtol, cg->maxit, k.data());
    for (auto& s : S) {
      if (!need[s.q]) continue;
      if (k[s.q].done == 3) {
        bsys_fail(s, FFTG_E_BREAKDOWN, "Galerkin CG breakdown (p.Ap <= 0)");
        continue;
      }
      if (k[s.q].done == 4) {
        bsys_fail(s, FFTG_E_NONFINITE, "non-finite value in Galerkin CG");
        continue;
      }
      s.o.cg += k[s.q].iters;
      galerkin_solution_at<T>(H, mask, s.kx, s.spec, s.eps, true);
    }
    check_launch();  // the next Newton step's read-back waits for these
    const double tcg = wall_ms(t0);
    for (auto& s : S)
      if (need[s.q] && s.nl) {
        s.o.t_cg += tcg;
        ++s.r;
      }
  }
  for (auto& s : S) s.o.newton = s.r;
}

// Commit the increments of RVEs to their items (the end of stagger_core),
// their means read back together.
void commit_many(fftg_handle* H, const std::vector<BSys*>& L, int J,
                 std::chrono::steady_clock::time_point t_all) {
  if (L.empty()) return;
  const int c = H->c;
  const long long N = H->g.N;
  std::vector<const double*> f;
  for (BSys* s : L) {
    fftg_batch_item& it = *s->it;
    HIPCHK(hipMemcpyAsync(s->s_eps, s->eps, sizeof(double) * c * N, hipMemcpyDeviceToDevice,
                          H->st));
    HIPCHK(hipMemcpyAsync(s->s_epsp, s->st1, sizeof(double) * 7 * N, hipMemcpyDeviceToDevice,
                          H->st));
    if (J > 0) {
      fftg::launch_commit_hist(s->tab, N, J, it.phase, s->ab, s->s_abar, s->s_hist, H->st);
      HIPCHK(hipMemcpyAsync(s->s_abar, s->ab, sizeof(double) * J * N, hipMemcpyDeviceToDevice,
                            H->st));
    }
    HIPCHK(hipMemcpyAsync(it.sigma_out, s->sig, sizeof(double) * c * N,
                          hipMemcpyDeviceToDevice, H->st));
    f.push_back(s->sig);
  }
  for (BSys* s : L) f.push_back(s->eps);
  std::vector<double> mv;
  batch_means(H, c, f, mv);  // synchronises: the copies above are done
  check_launch();
  const int n = (int)L.size();
  const double tot = wall_ms(t_all);
  for (int k = 0; k < n; ++k) {
    BSys& s = *L[k];
    fftg_batch_item& it = *s.it;
    for (int i = 0; i < 12; ++i) it.homog_out[i] = 0.0;
    for (int i = 0; i < c; ++i) {
      it.homog_out[i] = mv[6 * k + i];
      it.homog_out[6 + i] = mv[6 * (n + k) + i];
    }
    s.acc.t_ms[3] = std::max(0.0, tot - s.acc.t_ms[0] - s.acc.t_ms[1] - s.acc.t_ms[2]);
    s.acc.inner_converged = s.inner_ok ? 1 : 0;
    it.stats = s.acc;
    it.status = s.converged && s.inner_ok ? FFTG_OK : FFTG_NOT_CONVERGED;
    s.committed = true;
    s.live = false;
  }
}

// One increment of Algorithm 1 for every RVE of a class (stagger_core's
// steps, RVE by RVE where they are per voxel, in lockstep for the Krylov
// solves).  An RVE leaves the loop when its staggered error meets the
// tolerance (committed at once) or on a failure (not committed).
template <typename T>
void stagger_batch(fftg_handle* H, std::vector<BSys>& S, const unsigned char* mask, int J,
                   const fftg_krylov_opts* cg, const fftg_krylov_opts* pcg, double ntol,
                   int nmaxit, double stol, int maxk) {
  const auto t_all = std::chrono::steady_clock::now();
  const Geo& g = H->g;
  const int c = H->c;
  const long long N = g.N, Ns = g.Ns;
  const int n = (int)S.size();
  const int Jm = std::max(J, 1);
  ensure_sys(H, std::max(n, n * J));
  alloc_gal(H, n);
  alloc_bws(H, n, J);
  if (J > 0) alloc_helm(H, n * J);
  BatchWS* B = H->bws;
  const size_t w = H->wsz();
  for (auto& s : S) {
    const long long q = s.q;
    s.eps = B->eps_k + q * c * N;
    s.eps_prev = B->eps_prev + q * c * N;
    s.sig = B->sig_k + q * c * N;
    s.st1 = B->st1 + q * 7 * N;
    s.D = B->Dj + q * Jm * N;
    s.alph = B->alph + q * Jm * N;
    s.ab = B->ab_k + q * Jm * N;
    s.ab_prev = B->ab_prev + q * Jm * N;
    s.tan = static_cast<char*>(H->tan) + w * 8 * N * q;
    s.kx = static_cast<char*>(H->kx) + 2 * w * c * Ns * q;
    s.kr = static_cast<char*>(H->kr) + 2 * w * c * Ns * q;
    s.spec = H->spec64 + 6 * Ns * q;
    double* st = s.it->state;
    s.s_eps = st;
    s.s_epsp = st + (long long)c * N;
    s.s_hist = st + (long long)(c + 7) * N;
    s.s_abar = st + (long long)(c + 7 + J) * N;
    HIPCHK(hipMemcpyAsync(s.eps, s.s_eps, sizeof(double) * c * N, hipMemcpyDeviceToDevice,
                          H->st));
    if (J > 0)
      HIPCHK(hipMemcpyAsync(s.ab, s.s_abar, sizeof(double) * J * N, hipMemcpyDeviceToDevice,
                            H->st));
    for (int j = 0; j < J; ++j) {
      const long long o = (q * J + j) * N;
      if (H->fp32()) {
        fftg::launch_ell2<float>(s.tab, N, j, s.it->phase, static_cast<float*>(B->ell2j) + o,
                                 H->st);
        fftg::launch_ell2<double>(s.tab, N, j, s.it->phase, B->ell2j64 + o, H->st);
      } else {
        fftg::launch_ell2<double>(s.tab, N, j, s.it->phase, static_cast<double*>(B->ell2j) + o,
                                  H->st);
      }
    }
    s.sref = 0.0;
    for (int p = 0; p < s.tab.nphase; ++p) s.sref = std::max(s.sref, s.tab.m[p].sy);
    if (!(s.sref > 0.0)) s.sref = 1.0;
    for (int k = 0; k < 6; ++k) s.Sbar[k] = (k < c && mask[k]) ? s.it->target.S[k] : 0.0;
  }
  const double* ell2_64 = H->fp32() ? B->ell2j64 : static_cast<const double*>(B->ell2j);
  std::vector<unsigned char> skip((size_t)n * Jm, 0);
  std::vector<HelmOut> ho((size_t)n * Jm);
  std::vector<double> ell2_means;  // preconditioner lengths, fixed within the step
  std::vector<std::vector<double>> part(n);
  std::vector<int> nbe(n, 0);
  for (int k = 0; k < maxk; ++k) {
    bool any = false;
    for (auto& s : S) any = any || s.live;
    if (!any) break;
    for (auto& s : S) {
      if (!s.live) continue;
      if (J > 0)
        fftg::launch_damage(s.tab, N, J, s.it->phase, s.ab, s.s_hist, s.s_abar, s.D, H->st);
      HIPCHK(hipMemcpyAsync(s.eps_prev, s.eps, sizeof(double) * c * N, hipMemcpyDeviceToDevice,
                            H->st));
    }
    mechanics_batch<T>(H, S, mask, cg, ntol, nmaxit);
    for (auto& s : S) {
      if (!s.live) continue;
      s.acc.newton_iters += s.o.newton;
      s.inner_ok = s.o.converged;
      s.acc.cg_iters += s.o.cg;
      s.acc.relres = s.o.relres;
      s.acc.t_ms[0] += s.o.t_const;
      s.acc.t_ms[1] += s.o.t_cg;
    }
    auto th = std::chrono::steady_clock::now();
    if (J > 0) {
      for (auto& s : S) {
        for (int j = 0; j < J; ++j) skip[(size_t)s.q * J + j] = s.live ? 0 : 1;
        if (s.live)
          HIPCHK(hipMemcpyAsync(s.ab_prev, s.ab, sizeof(double) * J * N,
                                hipMemcpyDeviceToDevice, H->st));
      }
      // every field of every live RVE (Algorithm 1 (ii)) in one lockstep solve
      helm_solve(H, B->alph, B->ell2j, ell2_64, -1.0, B->ab_k, pcg->tol, pcg->maxit, n * J,
                 ho.data(), skip.data(), &ell2_means);
      for (auto& s : S) {
        if (!s.live) continue;
        for (int j = 0; j < J && s.live; ++j) {
          const HelmOut& h = ho[(size_t)s.q * J + j];
          if (h.status == 3) {
            bsys_fail(s, FFTG_E_BREAKDOWN, "Helmholtz PCG breakdown");
          } else if (h.status == 4) {
            bsys_fail(s, FFTG_E_NONFINITE, "non-finite value in Helmholtz PCG");
          } else {
            s.inner_ok = s.inner_ok && h.status == 1;
            s.acc.pcg_iters += h.iters;
          }
        }
      }
    }
    const double thm = wall_ms(th);
    // staggered error (Algorithm 1 (iii)), per RVE
    for (auto& s : S) {
      if (!s.live) continue;
      s.acc.t_ms[2] += thm;
      nbe[s.q] = fftg::launch_stagger_err(N, c, J, s.eps, s.eps_prev, s.ab, s.ab_prev,
                                          H->partials + (long long)s.q * H->psys, H->st);
      part[s.q].resize((size_t)nbe[s.q] * (1 + 2 * J));
      HIPCHK(hipMemcpyAsync(part[s.q].data(), H->partials + (long long)s.q * H->psys,
                            sizeof(double) * part[s.q].size(), hipMemcpyDeviceToHost, H->st));
    }
    sync(H);
    std::vector<const double*> fl;
    for (auto& s : S)
      if (s.live) fl.push_back(s.eps);
    std::vector<double> mv;
    batch_means(H, c, fl, mv);
    std::vector<BSys*> done;
    int km = 0;
    for (auto& s : S) {
      if (!s.live) continue;
      const int nb = nbe[s.q];
      const std::vector<double>& pt = part[s.q];
      double mx = 0.0;
      for (int b = 0; b < nb; ++b) mx = std::max(mx, pt[b]);
      const double* mean = &mv[6 * km++];
      double mn = 0.0;
      for (int i = 0; i < c; ++i) mn += mean[i] * mean[i];
      mn = std::sqrt(mn);
      double err = std::sqrt(mx) / (mn > 0.0 ? mn : 1.0);
      for (int j = 0; j < J; ++j) {
        double d2 = 0.0, a2 = 0.0;
        for (int b = 0; b < nb; ++b) {
          d2 += pt[(size_t)(1 + 2 * j) * nb + b];
          a2 += pt[(size_t)(2 + 2 * j) * nb + b];
        }
        if (d2 > 0.0)
          err = std::max(err, std::sqrt(d2) / std::max(std::sqrt(a2), 1e-12 * std::sqrt((double)N)));
      }
      s.acc.stagger_iters = k + 1;
      s.acc.err = err;
      if (err <= stol) {
        s.converged = true;
        done.push_back(&s);
      }
    }
    commit_many(H, done, J, t_all);
  }
  std::vector<BSys*> rest;
  for (auto& s : S)
    if (s.live) rest.push_back(&s);
  commit_many(H, rest, J, t_all);
  H->tan_valid = false;  // the tangent buffer holds the class's tangents
}

// One increment of every item of a class on the first item's handle; the
// items' codes, stats and results are those of staggered_step on each alone.
void run_class(fftg_batch_item* items, const std::vector<int>& idx, const fftg_krylov_opts* cg,
               const fftg_krylov_opts* pcg, double newton_tol, int newton_maxit,
               double stagger_tol, int max_stagger_iters) {
  fftg_handle* H = items[idx[0]].h;
  std::vector<BSys> S;
  for (int i : idx) {
    fftg_batch_item& it = items[i];
    BSys b;
    const fftg_status rc = run_guarded(it.h, [&]() -> fftg_status {
      validate_table(it.tab, it.nphase, it.nfields);
      validate_macro(&it.target, H->c);
      if (!it.phase || !it.state || !cg || !pcg || !it.sigma_out)
        throw Fail{FFTG_E_INVALID, "staggered_step: null pointer"};
      if (max_stagger_iters < 1) throw Fail{FFTG_E_INVALID, "max_stagger_iters must be >= 1"};
      validate_phase(H, it.phase, it.nphase);
      b.tab = make_table(it.tab, it.nphase, it.nfields);
      return FFTG_OK;
    });
    if (rc != FFTG_OK) {
      it.status = rc;
      continue;
    }
    b.it = &it;
    b.q = (int)S.size();
    S.push_back(b);
  }
  if (S.empty()) return;
  if (S.size() == 1) {
    fftg_batch_item& it = *S[0].it;
    it.status = staggered_step(it.h, it.phase, it.tab, it.nphase, it.nfields, it.state,
                               &it.target, cg, pcg, newton_tol, newton_maxit, stagger_tol,
                               max_stagger_iters, it.sigma_out, it.homog_out, &it.stats);
    return;
  }
  const unsigned char* mask = S[0].it->target.mask;
  const int J = S[0].it->nfields;
  const fftg_status rc = run_guarded(H, [&]() -> fftg_status {
    if (H->fp32())
      stagger_batch<float>(H, S, mask, J, cg, pcg, newton_tol, newton_maxit, stagger_tol,
                           max_stagger_iters);
    else
      stagger_batch<double>(H, S, mask, J, cg, pcg, newton_tol, newton_maxit, stagger_tol,
                            max_stagger_iters);
    return FFTG_OK;
  });
  const std::string herr = H->err;
  for (auto& s : S) {
    if (s.committed) continue;
    if (s.fail != FFTG_OK) {
      s.it->status = s.fail;
      s.it->h->err = s.msg;
    } else {
      s.it->status = rc != FFTG_OK ? rc : FFTG_E_HIP;
      s.it->h->err = herr;
    }
  }
}

// Tile autotuner: time the inner y pass and the outer inverse Galerkin pass
// back to back with each tile budget (code 0..3 = 32, 16, 8, 64 KB for the
// fixed-length kernels) and keep the fastest; another budget than 32 KB is
// taken only when it is at least 3% faster.  The per-line arithmetic does not
// depend on the tile, so results are bitwise the same for every choice.
// FFTG_TILE_SHIFT=0|1|2|3 fixes the choice instead.
void tune_tiles(fftg_handle* H) {
  const char* e = std::getenv("FFTG_TILE_SHIFT");
  if (e && e[0] >= '0' && e[0] <= '3' && e[1] == '\0') {
    H->tsh_y = H->tsh_o = e[0] - '0';
    return;
  }
  const int kids[2] = {K_GAL_YI, K_GAL_OI};
  for (int k = 0; k < 2; ++k) {
    int& sh = k == 0 ? H->tsh_y : H->tsh_o;
    if (k == 0 && !(H->g.ndim == 3 && H->g.n2 > 1)) continue;  // no inner pass
    int best = 0;
    for (int v = 0; v < 4; ++v) {
      sh = v;
      double ms = 0.0;
      if (fftg_time_kernel(H, kids[k], 10, &ms) != FFTG_OK || !(ms > 0.0)) ms = HUGE_VAL;
      H->tune_ms[k][v] = ms;
      if (ms < 0.97 * H->tune_ms[k][best]) best = v;
    }
    sh = best;
  }
  H->err.clear();
}

namespace {

// Coupled adjoint of a converged staggered increment on a validated call
// (J2 damage, cracking and elastic phases).  Leaves lam (J x N) and, with
// total_mu, the total mechanics adjoint mu = A^-1 G*(g_eps + K g_sig +
// alpha'^T lam) (c x N) and the total damage cotangent zeta = dJ/dD (J x N)
// in the handle's adjoint buffers; dell2 receives
// -sum_i G_i lam_j G_i abar_j.
struct AdjOut {
  fftg_stats stats{};
  bool converged = false;
  bool inner_capped = false;
  const double* lam = nullptr;
  const double* mu = nullptr;
  const double* zeta = nullptr;  // with total_mu: the total damage cotangent dJ/dD [J][N]
};

AdjOut stag_adjoint_core(fftg_handle* H, const unsigned char* phase, const MatTable& t, int J,
                         const double* state_n, const double* state_np1,
                         const fftg_macro* target, const double* g_eps, const double* g_sig,
                         const double* g_abar, const double* g_D, double* dell2,
                         const fftg_krylov_opts* cg, const fftg_krylov_opts* pcg, double tol,
                         int maxit, bool total_mu) {
  AdjOut out;
  const Geo& g = H->g;
  const int c = H->c;
  const long long N = g.N;
  alloc_stagger(H, J);
  alloc_helm(H);
  if (H->sadjJ < J) {
    dfree((void*&)H->sadj);
    H->sadj = (double*)dalloc(sizeof(double) * (size_t)(2 * c + 5 * J) * N);
    H->sadjJ = J;
  }
  double* mu = H->sadj;
  double* rhs = mu + (long long)c * N;
  double* dD = rhs + (long long)c * N;
  double* hv = dD + (long long)J * N;
  double* z = hv + (long long)J * N;
  double* zn = z + (long long)J * N;
  double* lam = zn + (long long)J * N;
  const double* epsp_n = state_n + (long long)c * N;  // eps_p (6), kappa
  const double* hist_n = state_n + (long long)(c + 7) * N;
  const double* abar_n = state_n + (long long)(c + 7 + J) * N;
  const double* eps = state_np1;
  const double* abar = state_np1 + (long long)(c + 7 + J) * N;
  // frozen damage of the converged state, squared lengths per field
  fftg::launch_damage(t, N, J, phase, abar, hist_n, abar_n, H->Dj, H->st);
  fill_ell2(H, t, J, phase);
  fftg_stats& acc = out.stats;
  int status = 0;
  auto mech = [&](const double* gb, const double* gs) {
    const int it = H->fp32() ? mech_adjoint<float>(H, phase, t, J, H->Dj, epsp_n, target, eps, gb,
                                                   gs, mu, dD, cg, status)
                             : mech_adjoint<double>(H, phase, t, J, H->Dj, epsp_n, target, eps,
                                                    gb, gs, mu, dD, cg, status);
    out.inner_capped = out.inner_capped || status == 2;
    acc.cg_iters += it;
    acc.newton_iters += 1;
  };
  auto helm = [&](const double* src, double* x) {
    // every field at once, in lockstep
    HelmOut ho[FFTG_MAX_FIELDS];
    helm_solve(H, src, ell2w_of(H, 0), ell2d_of(H, 0), -1.0, x, pcg->tol, pcg->maxit, J, ho);
    for (int j = 0; j < J; ++j) {
      if (ho[j].status == 3) throw Fail{FFTG_E_BREAKDOWN, "Helmholtz PCG breakdown"};
      if (ho[j].status == 4) throw Fail{FFTG_E_NONFINITE, "non-finite value in Helmholtz PCG"};
      out.inner_capped = out.inner_capped || ho[j].status == 2 || ho[j].status == 5;
      acc.pcg_iters += ho[j].iters;
    }
  };

  // hv = D' ((mu0 - g_sig) : sigma_eff + g_D) + g_abar, mu0 = A^-1 G*(g_eps + K g_sig)
  if (g_eps)
    HIPCHK(hipMemcpyAsync(rhs, g_eps, sizeof(double) * c * N, hipMemcpyDeviceToDevice, H->st));
  else
    fftg::launch_scale((long long)c * N, 0.0, eps, rhs, H->st);
  mech(rhs, g_sig);
  if (g_D) fftg::launch_axpby((long long)J * N, 1.0, dD, 1.0, g_D, dD, H->st);
  fftg::launch_damage_adj(t, N, J, phase, abar, hist_n, dD, hv, H->st);
  if (g_abar) fftg::launch_axpby((long long)J * N, 1.0, hv, 1.0, g_abar, hv, H->st);
  HIPCHK(hipMemcpyAsync(z, hv, sizeof(double) * J * N, hipMemcpyDeviceToDevice, H->st));
  fftg::launch_scale((long long)J * N, 0.0, hv, lam, H->st);
  // transposed staggered fixed point z <- hv + D' (sigma_eff : A^-1 G*(alpha'^T L^-1 z))
  int k = 0;
  double err = 0.0;
  for (k = 1; k <= maxit; ++k) {
    helm(z, lam);
    fftg::launch_source_adj(t, N, c, J, phase, eps, epsp_n, lam, rhs, H->st);
    mech(rhs, nullptr);
    fftg::launch_damage_adj(t, N, J, phase, abar, hist_n, dD, zn, H->st);
    fftg::launch_axpby((long long)J * N, 1.0, hv, 1.0, zn, zn, H->st);
    double s2[2];
    read_sums(H, fftg::launch_diff2((long long)J * N, zn, z, H->partials, H->st), 2, s2);
    std::swap(z, zn);
    err = std::sqrt(s2[0]) / std::max(std::sqrt(s2[1]), 1e-300);
    if (!std::isfinite(err)) throw Fail{FFTG_E_NONFINITE, "non-finite adjoint iterate"};
    if (err <= tol) {
      out.converged = true;
      break;
    }
  }
  helm(z, lam);
  for (int j = 0; j < J; ++j) grad_dot(H, lam + j * N, abar + j * N, dell2 + j * N);
  if (total_mu) {
    // mu = A^-1 G*(g_eps + K g_sig + alpha'^T lam)
    fftg::launch_source_adj(t, N, c, J, phase, eps, epsp_n, lam, rhs, H->st);
    if (g_eps) fftg::launch_axpby((long long)c * N, 1.0, rhs, 1.0, g_eps, rhs, H->st);
    mech(rhs, g_sig);
    if (g_D) fftg::launch_axpby((long long)J * N, 1.0, dD, 1.0, g_D, dD, H->st);
    out.mu = mu;
    out.zeta = dD;
  }
  acc.stagger_iters = out.converged ? k : maxit;
  acc.err = err;
  out.lam = lam;
  return out;
}

}  // namespace

extern "C" {

fftg_status fftg_tile_config(const fftg_handle* H, int* yz_shift, int* outer_shift,
                             double* times_ms) {
  if (!H || !yz_shift || !outer_shift) return FFTG_E_INVALID;
  *yz_shift = H->tsh_y;
  *outer_shift = H->tsh_o;
  if (times_ms)
    for (int k = 0; k < 2; ++k)
      for (int v = 0; v < 4; ++v) times_ms[4 * k + v] = H->tune_ms[k][v];
  return FFTG_OK;
}

fftg_status fftg_create(const fftg_grid* grid, void* hip_stream, fftg_handle** out) {
  g_create_error.clear();
  if (!grid || !out) {
    g_create_error = "fftg_create: null argument";
    return FFTG_E_INVALID;
  }
  *out = nullptr;
  if (grid->ndim != 2 && grid->ndim != 3) {
    g_create_error = "fftg_create: ndim must be 2 or 3";
    return FFTG_E_INVALID;
  }
  const int n1 = grid->n[0], n2 = grid->n[1], n3 = grid->ndim == 3 ? grid->n[2] : 1;
  if (grid->ndim == 2 && grid->n[2] != 1 && grid->n[2] != 0) {
    g_create_error = "fftg_create: n[2] must be 1 in 2D";
    return FFTG_E_INVALID;
  }
  if (n1 < 2 || n2 < 1 || n3 < 1 || !(grid->h > 0.0)) {
    g_create_error = "fftg_create: bad grid size or voxel size";
    return FFTG_E_INVALID;
  }
  if (grid->scheme != FFTG_ROTATED && grid->scheme != FFTG_SPECTRAL) {
    g_create_error = "fftg_create: unknown derivative scheme";
    return FFTG_E_INVALID;
  }
  if (grid->prec != FFTG_FP64 && grid->prec != FFTG_FP32_REFINED) {
    g_create_error = "fftg_create: unknown precision";
    return FFTG_E_INVALID;
  }
  const int nmax = grid->ndim == 3 ? 256 : 512;
  if (!smooth23(n1) || !smooth23(n2) || !smooth23(n3) || n1 % 2 != 0 || n1 > nmax || n2 > nmax ||
      n3 > nmax) {
    g_create_error =
        "fftg_create: unsupported size (need N = 2^a 3^b, N1 even, N <= 256 in 3D, 512 in 2D)";
    return FFTG_E_UNSUPPORTED;
  }
  fftg_handle* H = new fftg_handle();
  fftg_status rc = run_guarded(H, [&]() -> fftg_status {
    H->g.ndim = grid->ndim;
    H->g.n1 = n1;
    H->g.n2 = n2;
    H->g.n3 = n3;
    H->g.n1h = n1 / 2 + 1;
    H->g.N = (long long)n1 * n2 * n3;
    H->g.Ns = (long long)H->g.n1h * n2 * n3;
    H->c = grid->ndim == 3 ? 6 : 3;
    H->h = grid->h;
    H->scheme = grid->scheme;
    H->prec = grid->prec;
    H->st = reinterpret_cast<hipStream_t>(hip_stream);
    const int ns[3] = {n1, n2, n3};
    std::vector<double> pq[3], gq[3], cs[3];
    for (int a = 0; a < 3; ++a) {
      H->plan[a] = make_plan(ns[a]);
      std::vector<double> t = twiddles(ns[a]);
      H->tw64[a] = (cpx<double>*)dalloc(sizeof(double) * t.size());
      HIPCHK(hipMemcpy(H->tw64[a], t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice));
      std::vector<float> tf(t.begin(), t.end());
      H->tw32[a] = (cpx<float>*)dalloc(sizeof(float) * tf.size());
      HIPCHK(hipMemcpy(H->tw32[a], tf.data(), sizeof(float) * tf.size(), hipMemcpyHostToDevice));
      axis_tables(ns[a], a == 0, grid->h, grid->scheme, pq[a], gq[a], cs[a]);
    }
    std::vector<double> all;
    int off = 0;
    for (int a = 0; a < 3; ++a) {
      H->S64.pq[a] = off;
      all.insert(all.end(), pq[a].begin(), pq[a].end());
      off += (int)pq[a].size();
    }
    for (int a = 0; a < 3; ++a) {
      H->S64.gq[a] = off;
      all.insert(all.end(), gq[a].begin(), gq[a].end());
      off += (int)gq[a].size();
    }
    for (int a = 0; a < 3; ++a) {
      H->S64.cs[a] = off;
      all.insert(all.end(), cs[a].begin(), cs[a].end());
      off += (int)cs[a].size();
    }
    H->sym64 = (double*)dalloc(sizeof(double) * all.size());
    HIPCHK(hipMemcpy(H->sym64, all.data(), sizeof(double) * all.size(), hipMemcpyHostToDevice));
    std::vector<float> allf(all.begin(), all.end());
    H->sym32 = (float*)dalloc(sizeof(float) * allf.size());
    HIPCHK(hipMemcpy(H->sym32, allf.data(), sizeof(float) * allf.size(), hipMemcpyHostToDevice));
    H->S64.base = H->sym64;
    H->S32.base = H->sym32;
    for (int a = 0; a < 3; ++a) {
      H->S32.pq[a] = H->S64.pq[a];
      H->S32.gq[a] = H->S64.gq[a];
      H->S32.cs[a] = H->S64.cs[a];
    }
    const Geo& g = H->g;
    const size_t cs_bytes = 2 * H->wsz() * (size_t)H->c * g.Ns;
    H->kx = dalloc(cs_bytes);
    H->kr = dalloc(cs_bytes);
    H->kp = dalloc(cs_bytes);
    H->kw = dalloc(cs_bytes);
    H->spec64 = (cpx<double>*)dalloc(sizeof(cpx<double>) * 6 * g.Ns);
    H->tan = dalloc(H->wsz() * 8 * (size_t)g.N);
    H->rtmp = dalloc(H->wsz() * (size_t)std::max(H->c, 2) * g.N);
    // partials: largest block count of any reduction of one system (a
    // lockstep solve of n systems needs n times as many)
    long long maxb = fftg::RED_BLOCKS * 16;
    for (int a = 1; a < 3; ++a) {
      const long long nl = (long long)H->c * g.Ns / std::max(1, ns[a]);
      maxb = std::max(maxb, 2 * (nl + 1));
      maxb = std::max(maxb, g.Ns / std::max(1, ns[a]) + 1);
    }
    // the Galerkin x pass's p.Ap partials and the residual pass's r.r
    maxb = std::max(maxb, (long long)fftg::gal_xdot_count<double>(g, H->c) +
                              fftg::gal_resid_count(g));
    maxb = std::max(maxb, (long long)fftg::gal_xdot_count<float>(g, H->c) +
                              fftg::gal_resid_count(g));
    for (int a = 1; a < 3; ++a) {
      if (a >= g.ndim) break;
      maxb = std::max(maxb, (long long)fftg::gal_xdot_count<double>(g, H->c) +
                                fftg::gal_fwd_resid_count<double>(H->plan[a], g, H->c, g.ndim == 3));
      maxb = std::max(maxb, (long long)fftg::gal_xdot_count<float>(g, H->c) +
                                fftg::gal_fwd_resid_count<float>(H->plan[a], g, H->c, g.ndim == 3));
    }
    H->psys = maxb;
    // up to FFTG_MAX_FIELDS lockstep systems (the Helmholtz solves of the
    // non-local fields) without growing
    H->npartials = (size_t)maxb * FFTG_MAX_FIELDS;
    H->partials = (double*)dalloc(sizeof(double) * H->npartials);
    H->dsums = (double*)dalloc(sizeof(double) * (16 * FFTG_MAX_FIELDS + 64));
    // one Krylov control block per system of a lockstep solve
    H->ctl = (KrylovCtl*)dalloc(sizeof(KrylovCtl) * FFTG_MAX_FIELDS);
    HIPCHK(hipHostMalloc((void**)&H->hctl, sizeof(KrylovCtl) * FFTG_MAX_FIELDS,
                         hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&H->hsums, sizeof(double) * (16 * FFTG_MAX_FIELDS + 64),
                         hipHostMallocDefault));
    // per-phase ell^2 tables of the Helmholtz x pass (FP64 and work precision)
    const size_t nt = (size_t)FFTG_MAX_FIELDS * fftg::kMaxPhases;
    H->ptab = dalloc(H->wsz() * nt);
    H->ptab64 = (double*)dalloc(sizeof(double) * nt);
    HIPCHK(hipHostMalloc((void**)&H->hptab, sizeof(double) * 2 * nt, hipHostMallocDefault));
    for (auto& e : H->ev) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipStreamCreateWithFlags(&H->cap, hipStreamNonBlocking));
    return FFTG_OK;
  });
  if (const char* f = std::getenv("FFTG_GAL_FOLD")) H->fold = f[0] == '1' && f[1] == '\0';
  if (const char* f = std::getenv("FFTG_GAL_XDOT")) H->xdot = !(f[0] == '0' && f[1] == '\0');
  if (const char* f = std::getenv("FFTG_GAL_FUSE")) H->fuse_res = !(f[0] == '0' && f[1] == '\0');
  if (const char* f = std::getenv("FFTG_HELM_FUSE")) H->hfuse = !(f[0] == '0' && f[1] == '\0');
  if (rc == FFTG_OK) tune_tiles(H);
  if (rc != FFTG_OK) {
    g_create_error = H->err;
    destroy(H);
    delete H;
    return rc;
  }
  *out = H;
  return FFTG_OK;
}

fftg_status fftg_destroy(fftg_handle* H) {
  if (!H) return FFTG_E_INVALID;
  (void)hipStreamSynchronize(H->st);
  destroy(H);
  delete H;
  return FFTG_OK;
}

const char* fftg_last_error(const fftg_handle* H) {
  return H ? H->err.c_str() : g_create_error.c_str();
}

fftg_status fftg_profile(fftg_handle* H, int enable, double* ms, long long* launches) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    sync(H);
    if (ms)
      for (int i = 0; i < FFTG_NKERNELS; ++i) ms[i] = H->kt_ms[i];
    if (launches)
      for (int i = 0; i < FFTG_NKERNELS; ++i) launches[i] = H->kt_n[i];
    if (enable) {
      for (int i = 0; i < FFTG_NKERNELS; ++i) {
        H->kt_ms[i] = 0.0;
        H->kt_n[i] = 0;
      }
    }
    H->prof = enable != 0;
    return FFTG_OK;
  });
}

fftg_status fftg_copy_rate(fftg_handle* H, const void* src, void* dst, long long nbytes,
                           int reps, double* gbps) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    if (!src || !dst || !gbps || reps < 1 || nbytes < 16 || nbytes % 16 != 0 ||
        (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
      throw Fail{FFTG_E_INVALID, "fftg_copy_rate: bad arguments"};
    const long long n16 = nbytes / 16;
    int best_blocks = 0;
    float best = 0.0f;
    // a few grid sizes (multiples of the compute-unit count); keep the fastest
    for (int blocks : {1024, 2048, 4096, 8192}) {
      fftg::launch_stream_copy(src, dst, n16, blocks, H->st);  // warm-up
      HIPCHK(hipEventRecord(H->ev[0], H->st));
      for (int r = 0; r < reps; ++r) fftg::launch_stream_copy(src, dst, n16, blocks, H->st);
      HIPCHK(hipEventRecord(H->ev[1], H->st));
      HIPCHK(hipEventSynchronize(H->ev[1]));
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, H->ev[0], H->ev[1]));
      if (best_blocks == 0 || ms < best) {
        best = ms;
        best_blocks = blocks;
      }
    }
    check_launch();
    *gbps = 2.0 * (double)nbytes * reps / (best * 1e-3) / 1e9;
    return FFTG_OK;
  });
}

fftg_status fftg_time_kernel(fftg_handle* H, int kid, int reps, double* avg_ms) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    if (!avg_ms || reps < 1) throw Fail{FFTG_E_INVALID, "fftg_time_kernel: bad arguments"};
    const Geo& g = H->g;
    const int c = H->c;
    const bool zo = g.ndim == 3;
    const int oa = outer_axis(H);
    alloc_helm(H);
    const size_t cs = 2 * H->wsz() * (size_t)c * g.Ns;
    for (void* p : {H->kx, H->kr, H->kp, H->kw}) HIPCHK(hipMemsetAsync(p, 0, cs, H->st));
    const size_t ss = 2 * H->wsz() * (size_t)g.Ns;
    for (void* p : {H->hx, H->hr, H->hp, H->hAp, H->hb}) HIPCHK(hipMemsetAsync(p, 0, ss, H->st));
    HIPCHK(hipMemsetAsync(H->hw, 0, ss * g.ndim, H->st));
    HIPCHK(hipMemsetAsync(H->ell2w, 0, H->wsz() * (size_t)g.N, H->st));
    HIPCHK(hipMemsetAsync(H->tan, 0, H->wsz() * 8 * (size_t)g.N, H->st));
    KrylovCtl k{};
    k.maxit = 1 << 30;
    write_ctl(H, k);
    auto launch = [&](auto tag) {
      using T = decltype(tag);
      const T scl = T(1.0 / (double)g.N);
      switch (kid) {
        case K_GAL_X:
          fftg::launch_x_fused_gal<T, T>(H->plan[0], TW<T>(H, 0), g, c, C<T>(H->kw),
                                         reinterpret_cast<const T*>(H->tan), scl, H->ctl, H->st,
                                         1, H->xdot ? H->partials : nullptr);
          break;
        case K_GAL_YI:
          inner_inv<T>(H, c, C<T>(H->kw), H->ctl, K_GAL_YI);
          break;
        case K_GAL_YF:
          inner_fwd<T>(H, c, C<T>(H->kw), H->ctl, K_GAL_YF);
          break;
        case K_GAL_OI:
          fftg::launch_gal_dir_inv<T>(H->plan[oa], TW<T>(H, oa), g, c, zo, C<T>(H->kr),
                                      C<T>(H->kp), C<T>(H->kx), C<T>(H->kw), H->ctl, H->st, H->tsh_o);
          break;
        case K_GAL_OF:
          fftg::launch_gal_dot_fwd<T>(H->plan[oa], TW<T>(H, oa), g, c, zo,
                                      H->xdot ? nullptr : C<T>(H->kp), C<T>(H->kw),
                                      H->xdot ? nullptr : H->partials, H->ctl, H->st);
          break;
        case K_GAL_RES:
          fftg::launch_gal_resid<T>(g, c, SY<T>(H), H->mask_last, C<T>(H->kr), C<T>(H->kw),
                                    H->partials, H->ctl, H->st);
          break;
        case K_GAL_OFR:
          fftg::launch_gal_fwd_resid<T>(H->plan[oa], TW<T>(H, oa), g, c, zo, SY<T>(H),
                                        H->mask_last, C<T>(H->kw), C<T>(H->kr), H->partials,
                                        H->ctl, H->st);
          break;
        case K_HLM_X:
          fftg::launch_x_fused_helm<T, T>(H->plan[0], TW<T>(H, 0), g, C<T>(H->hw),
                                          reinterpret_cast<const T*>(H->ell2w), scl, H->ctl,
                                          H->st);
          break;
        case K_HLM_OI:
          fftg::launch_h_dir_inv<T>(H->plan[oa], TW<T>(H, oa), g, zo, SY<T>(H), true,
                                    C<T>(H->hr), C<T>(H->hp), C<T>(H->hx), C<T>(H->hw), H->ctl,
                                    H->st);
          break;
        case K_HLM_OF:
          if (H->hfuse)
            fftg::launch_h_fwd_resid<T>(H->plan[oa], TW<T>(H, oa), g, zo, SY<T>(H),
                                        C<T>(H->hp), C<T>(H->hw), C<T>(H->hr), H->partials,
                                        H->ctl, H->st);
          else
            fftg::launch_h_div_fwd<T>(H->plan[oa], TW<T>(H, oa), g, zo, SY<T>(H), C<T>(H->hp),
                                      C<T>(H->hw), C<T>(H->hAp), H->partials, H->ctl, H->st);
          break;
        case K_HLM_RES:
          fftg::launch_h_resid<T>(g, SY<T>(H), false, C<T>(H->hr), C<T>(H->hb), C<T>(H->hAp),
                                  H->partials, H->ctl, H->st);
          break;
        default:
          throw Fail{FFTG_E_UNSUPPORTED, "fftg_time_kernel: kernel class not timeable"};
      }
    };
    const bool was = H->prof;
    H->prof = false;
    auto one = [&]() {
      if (H->fp32())
        launch(float{});
      else
        launch(double{});
    };
    one();  // warm
    check_launch();
    HIPCHK(hipEventRecord(H->ev[0], H->st));
    for (int i = 0; i < reps; ++i) one();
    HIPCHK(hipEventRecord(H->ev[1], H->st));
    check_launch();
    sync(H);
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, H->ev[0], H->ev[1]));
    *avg_ms = ms / reps;
    H->prof = was;
    H->tan_valid = false;  // the workspace was overwritten
    return FFTG_OK;
  });
}

const char* fftg_kernel_name(int id) {
  return (id >= 0 && id < FFTG_NKERNELS) ? kKernelNames[id] : "";
}

fftg_status fftg_forward(fftg_handle* H, int ncomp, const double* in, double* out) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    if (!in || !out || ncomp < 1 || ncomp > 8) throw Fail{FFTG_E_INVALID, "fftg_forward: bad args"};
    // transform through the work buffer so `in` is not modified
    fwd3<double>(H, ncomp, in, reinterpret_cast<cpx<double>*>(out));
    check_launch();
    sync(H);
    return FFTG_OK;
  });
}

fftg_status fftg_inverse(fftg_handle* H, int ncomp, const double* in, double* out) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    if (!in || !out || ncomp < 1 || ncomp > 6) throw Fail{FFTG_E_INVALID, "fftg_inverse: bad args"};
    const Geo& g = H->g;
    HIPCHK(hipMemcpyAsync(H->spec64, in, sizeof(cpx<double>) * ncomp * g.Ns,
                          hipMemcpyDeviceToDevice, H->st));
    inv3<double, double>(H, ncomp, H->spec64, out, 1.0 / (double)g.N, false);
    check_launch();
    sync(H);
    return FFTG_OK;
  });
}

fftg_status fftg_project(fftg_handle* H, const fftg_macro* tgt, const double* tau, double* out) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    if (!tau || !out) throw Fail{FFTG_E_INVALID, "fftg_project: null pointer"};
    validate_macro(tgt, H->c);
    const Geo& g = H->g;
    fwd3<double>(H, H->c, tau, H->spec64);
    fftg::launch_project<double>(g, H->c, H->S64, tgt->mask, H->spec64, H->st);
    inv3<double, double>(H, H->c, H->spec64, out, 1.0 / (double)g.N, false);
    check_launch();
    sync(H);
    return FFTG_OK;
  });
}

fftg_status fftg_constitutive(fftg_handle* H, const unsigned char* phase, const fftg_phase* tab,
                              int nphase, int nfields, const double* D, const double* state_n,
                              const double* eps, double* sigma, double* state_np1,
                              double* alpha) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    validate_table(tab, nphase, nfields);
    if (!phase || !state_n || !eps || !sigma || !state_np1 || (nfields > 0 && (!D || !alpha)))
      throw Fail{FFTG_E_INVALID, "fftg_constitutive: null pointer"};
    validate_phase(H, phase, nphase);
    MatTable t = make_table(tab, nphase, nfields);
    if (H->fp32())
      fftg::launch_constitutive<float>(t, H->g, H->c, nfields, phase, eps, state_n, D, sigma,
                                       state_np1, alpha, reinterpret_cast<float*>(H->tan), H->st);
    else
      fftg::launch_constitutive<double>(t, H->g, H->c, nfields, phase, eps, state_n, D, sigma,
                                        state_np1, alpha, reinterpret_cast<double*>(H->tan), H->st);
    H->tan_valid = true;
    check_launch();
    sync(H);
    return FFTG_OK;
  });
}

fftg_status fftg_apply_galerkin(fftg_handle* H, const fftg_macro* tgt, const double* p,
                                double* out) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    if (!p || !out) throw Fail{FFTG_E_INVALID, "fftg_apply_galerkin: null pointer"};
    validate_macro(tgt, H->c);
    if (!H->tan_valid) throw Fail{FFTG_E_INVALID, "fftg_apply_galerkin: no tangent yet"};
    if (H->fp32()) throw Fail{FFTG_E_UNSUPPORTED, "fftg_apply_galerkin: FP64 handles only"};
    const Geo& g = H->g;
    const int c = H->c;
    // out = G*(K : p) through the same passes as the CG operator
    fwd3<double>(H, c, p, C<double>(H->kw));
    const int oa = outer_axis(H);
    if (g.ndim == 3)
      fftg::launch_strided<double>(H->plan[oa], TW<double>(H, oa), C<double>(H->kw),
                                   (long long)c * g.n2 * g.n1h, (long long)g.n2 * g.n1h, g.Ns,
                                   (long long)g.n2 * g.n1h, false, nullptr, H->st, H->tsh_o);
    else
      fftg::launch_strided<double>(H->plan[oa], TW<double>(H, oa), C<double>(H->kw),
                                   (long long)c * g.n1h, g.n1h, g.Ns, g.n1h, false, nullptr,
                                   H->st, H->tsh_o);
    inner_inv<double>(H, c, C<double>(H->kw), nullptr, K_GAL_YI);
    fftg::launch_x_fused_gal<double, double>(H->plan[0], TW<double>(H, 0), g, c, C<double>(H->kw),
                                             reinterpret_cast<const double*>(H->tan),
                                             1.0 / (double)g.N, nullptr, H->st);
    inner_fwd<double>(H, c, C<double>(H->kw), nullptr, K_GAL_YF);
    if (g.ndim == 3)
      fftg::launch_strided<double>(H->plan[oa], TW<double>(H, oa), C<double>(H->kw),
                                   (long long)c * g.n2 * g.n1h, (long long)g.n2 * g.n1h, g.Ns,
                                   (long long)g.n2 * g.n1h, true, nullptr, H->st, H->tsh_o);
    else
      fftg::launch_strided<double>(H->plan[oa], TW<double>(H, oa), C<double>(H->kw),
                                   (long long)c * g.n1h, g.n1h, g.Ns, g.n1h, true, nullptr,
                                   H->st, H->tsh_o);
    fftg::launch_project<double>(g, c, H->S64, tgt->mask, C<double>(H->kw), H->st);
    inv3<double, double>(H, c, C<double>(H->kw), out, 1.0 / (double)g.N, false);
    check_launch();
    sync(H);
    return FFTG_OK;
  });
}

fftg_status fftg_apply_helmholtz(fftg_handle* H, const double* ell2, const double* u,
                                 double* out) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    if (!ell2 || !u || !out) throw Fail{FFTG_E_INVALID, "fftg_apply_helmholtz: null pointer"};
    if (H->fp32()) throw Fail{FFTG_E_UNSUPPORTED, "fftg_apply_helmholtz: FP64 handles only"};
    alloc_helm(H);
    const Geo& g = H->g;
    const bool zo = g.ndim == 3;
    const int oa = outer_axis(H);
    KrylovCtl k{};
    write_ctl(H, k);
    fwd3<double>(H, 1, u, C<double>(H->hx));
    fftg::launch_h_dir_inv<double>(H->plan[oa], TW<double>(H, oa), g, zo, H->S64, false,
                                   C<double>(H->hr), C<double>(H->hx), C<double>(H->hx),
                                   C<double>(H->hw), H->ctl, H->st);
    helm_inner<double>(H, false, C<double>(H->hw), nullptr, K_HLM_YI);
    fftg::launch_x_fused_helm<double, double>(H->plan[0], TW<double>(H, 0), g, C<double>(H->hw),
                                              ell2, 1.0 / (double)g.N, nullptr, H->st);
    helm_inner<double>(H, true, C<double>(H->hw), nullptr, K_HLM_YF);
    fftg::launch_h_div_fwd<double>(H->plan[oa], TW<double>(H, oa), g, zo, H->S64,
                                   C<double>(H->hx), C<double>(H->hw), C<double>(H->hAp), nullptr,
                                   H->ctl, H->st);
    inv3<double, double>(H, 1, C<double>(H->hAp), out, 1.0 / (double)g.N, false);
    check_launch();
    sync(H);
    return FFTG_OK;
  });
}

fftg_status helmholtz_solve(fftg_handle* H, const double* alpha, const double* ell2,
                            double ell2_ref, double* abar, const fftg_krylov_opts* opts,
                            fftg_stats* stats) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    if (!alpha || !ell2 || !abar || !opts)
      throw Fail{FFTG_E_INVALID, "helmholtz_solve: null pointer"};
    alloc_helm(H);
    auto t0 = std::chrono::steady_clock::now();
    int it = 0, status = 0;
    double rel = 0.0;
    if (H->fp32())
      fftg::launch_convert<double, float>(H->g.N, ell2, reinterpret_cast<float*>(H->ell2w), H->st);
    HelmOut ho;
    helm_solve(H, alpha, H->fp32() ? H->ell2w : ell2, ell2, ell2_ref, abar, opts->tol,
               opts->maxit, 1, &ho);
    it = ho.iters;
    rel = ho.relres;
    status = ho.status;
    sync(H);
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->pcg_iters = it;
      stats->relres = rel;
      stats->t_ms[2] = wall_ms(t0);
    }
    if (status == 3) throw Fail{FFTG_E_BREAKDOWN, "Helmholtz PCG breakdown"};
    if (status == 4) throw Fail{FFTG_E_NONFINITE, "non-finite value in Helmholtz PCG"};
    return status == 1 ? FFTG_OK : FFTG_NOT_CONVERGED;
  });
}

fftg_status helmholtz_adjoint(fftg_handle* H, const double* ell2, double ell2_ref,
                              const double* abar, const double* gbar, double* dalpha,
                              double* dell2, const fftg_krylov_opts* opts, fftg_stats* stats) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    if (!ell2 || !abar || !gbar || !dalpha || !dell2 || !opts)
      throw Fail{FFTG_E_INVALID, "helmholtz_adjoint: null pointer"};
    alloc_helm(H);
    auto t0 = std::chrono::steady_clock::now();
    int it = 0, status = 0;
    double rel = 0.0;
    if (H->fp32())
      fftg::launch_convert<double, float>(H->g.N, ell2, reinterpret_cast<float*>(H->ell2w), H->st);
    HelmOut ho;
    helm_solve(H, gbar, H->fp32() ? H->ell2w : ell2, ell2, ell2_ref, dalpha, opts->tol,
               opts->maxit, 1, &ho);
    it = ho.iters;
    rel = ho.relres;
    status = ho.status;
    if (status == 3) throw Fail{FFTG_E_BREAKDOWN, "Helmholtz PCG breakdown"};
    if (status == 4) throw Fail{FFTG_E_NONFINITE, "non-finite value in Helmholtz PCG"};
    grad_dot(H, dalpha, abar, dell2);
    sync(H);
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->pcg_iters = it;
      stats->relres = rel;
      stats->t_ms[2] = wall_ms(t0);
    }
    return status == 1 ? FFTG_OK : FFTG_NOT_CONVERGED;
  });
}

fftg_status fftg_solve_adjoint(fftg_handle* H, const unsigned char* phase, const fftg_phase* tab,
                               int nphase, int nfields, const double* D, const double* state_n,
                               const fftg_macro* target, const double* eps, const double* gbar,
                               const double* gsig, double* mu, double* dD,
                               const fftg_krylov_opts* cg, fftg_stats* stats) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    validate_table(tab, nphase, nfields);
    validate_macro(target, H->c);
    if (!phase || !state_n || !eps || !gbar || !mu || !cg || (nfields > 0 && (!D || !dD)))
      throw Fail{FFTG_E_INVALID, "fftg_solve_adjoint: null pointer"};
    validate_phase(H, phase, nphase);
    if (has_gtn(tab, nphase))
      throw Fail{FFTG_E_UNSUPPORTED, "fftg_solve_adjoint: no adjoint of the Gurson return"};
    const MatTable t = make_table(tab, nphase, nfields);
    auto t0 = std::chrono::steady_clock::now();
    int status = 0;
    const int it = H->fp32() ? mech_adjoint<float>(H, phase, t, nfields, D, state_n, target, eps,
                                                   gbar, gsig, mu, dD, cg, status)
                             : mech_adjoint<double>(H, phase, t, nfields, D, state_n, target,
                                                    eps, gbar, gsig, mu, dD, cg, status);
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->cg_iters = it;
      stats->t_ms[1] = wall_ms(t0);
    }
    return status == 1 ? FFTG_OK : FFTG_NOT_CONVERGED;
  });
}

fftg_status fftg_staggered_adjoint(fftg_handle* H, const unsigned char* phase,
                                   const fftg_phase* tab, int nphase, int nfields,
                                   const double* state_n, const double* state_np1,
                                   const fftg_macro* target, const double* g_eps,
                                   const double* g_sig, const double* g_abar, const double* g_D,
                                   double* dell2, double* lam_out, const fftg_krylov_opts* cg,
                                   const fftg_krylov_opts* pcg, double tol, int maxit,
                                   fftg_stats* stats) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    validate_table(tab, nphase, nfields);
    validate_macro(target, H->c);
    if (!phase || !state_n || !state_np1 || !dell2 || !cg || !pcg || nfields < 1 || maxit < 1)
      throw Fail{FFTG_E_INVALID, "fftg_staggered_adjoint: null pointer, no field or maxit < 1"};
    validate_phase(H, phase, nphase);
    if (has_gtn(tab, nphase))
      throw Fail{FFTG_E_UNSUPPORTED, "fftg_staggered_adjoint: Gurson sources are not covered"};
    auto t0 = std::chrono::steady_clock::now();
    const MatTable t = make_table(tab, nphase, nfields);
    const AdjOut r = stag_adjoint_core(H, phase, t, nfields, state_n, state_np1, target, g_eps,
                                       g_sig, g_abar, g_D, dell2, cg, pcg, tol, maxit, false);
    if (lam_out)
      HIPCHK(hipMemcpyAsync(lam_out, r.lam, sizeof(double) * nfields * H->g.N,
                            hipMemcpyDeviceToDevice, H->st));
    check_launch();
    sync(H);
    if (stats) {
      *stats = r.stats;
      stats->t_ms[3] = wall_ms(t0);
    }
    return r.converged && !r.inner_capped ? FFTG_OK : FFTG_NOT_CONVERGED;
  });
}

fftg_status fftg_increment_adjoint(fftg_handle* H, const unsigned char* phase,
                                   const fftg_phase* tab, int nphase, int nfields,
                                   const double* state_n, const double* state_np1,
                                   const fftg_macro* target, const double* g_sig,
                                   const double* g_epsp, const double* g_kappa,
                                   const double* g_hist, double* dell2, double* g_epsp_n,
                                   double* g_kappa_n, double* g_hist_n,
                                   const fftg_krylov_opts* cg, const fftg_krylov_opts* pcg,
                                   double tol, int maxit, fftg_stats* stats) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    validate_table(tab, nphase, nfields);
    validate_macro(target, H->c);
    if (!phase || !state_n || !state_np1 || !dell2 || !g_epsp_n || !g_kappa_n || !g_hist_n ||
        !cg || !pcg || nfields < 1 || maxit < 1)
      throw Fail{FFTG_E_INVALID, "fftg_increment_adjoint: null pointer, no field or maxit < 1"};
    validate_phase(H, phase, nphase);
    for (int p = 0; p < nphase; ++p)
      if (tab[p].model == FFTG_GTN)
        throw Fail{FFTG_E_UNSUPPORTED,
                   "fftg_increment_adjoint: no adjoint of the Gurson return and porosity"};
    auto t0 = std::chrono::steady_clock::now();
    const int c = H->c, J = nfields;
    const long long N = H->g.N;
    const MatTable t = make_table(tab, nphase, J);
    const double* epsp_n = state_n + (long long)c * N;
    const double* hist_n = state_n + (long long)(c + 7) * N;
    const double* eps = state_np1;
    const double* abar = state_np1 + (long long)(c + 7 + J) * N;
    if (H->hadjJ < J) {
      dfree((void*&)H->hadj);
      H->hadj = (double*)dalloc(sizeof(double) * (size_t)(c + J) * N);
      H->hadjJ = J;
    }
    // strain cotangent of the committed plastic state; abar cotangent of the
    // committed damage history where abar is its max
    const double* g_eps = nullptr;
    if (g_epsp || g_kappa) {
      fftg::launch_hist_out_cot(t, N, c, phase, eps, epsp_n, g_epsp, g_kappa, H->hadj, H->st);
      g_eps = H->hadj;
    }
    const double* g_abar = nullptr;
    if (g_hist) {
      double* ga = H->hadj + (long long)c * N;
      fftg::launch_hist_split((long long)J * N, abar, hist_n, g_hist, ga, H->st);
      g_abar = ga;
    }
    const AdjOut r = stag_adjoint_core(H, phase, t, J, state_n, state_np1, target, g_eps, g_sig,
                                       g_abar, nullptr, dell2, cg, pcg, tol, maxit, true);
    fftg::launch_hist_in_cot(t, N, c, J, phase, eps, epsp_n, H->Dj, r.mu, g_sig, r.lam, g_epsp,
                             g_kappa, g_epsp_n, g_kappa_n, H->st);
    fftg::launch_hist_damage_cot(t, N, J, phase, abar, hist_n, r.zeta, g_hist, g_hist_n, H->st);
    check_launch();
    sync(H);
    if (stats) {
      *stats = r.stats;
      stats->t_ms[3] = wall_ms(t0);
    }
    return r.converged && !r.inner_capped ? FFTG_OK : FFTG_NOT_CONVERGED;
  });
}

fftg_status fftg_damage(fftg_handle* H, const unsigned char* phase, const fftg_phase* tab,
                        int nphase, int nfields, const double* abar, const double* hist,
                        double* D) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    validate_table(tab, nphase, nfields);
    if (nfields < 1 || !phase || !abar || !hist || !D)
      throw Fail{FFTG_E_INVALID, "fftg_damage: null pointer or no field"};
    validate_phase(H, phase, nphase);
    if (has_gtn(tab, nphase))
      throw Fail{FFTG_E_UNSUPPORTED, "fftg_damage: Gurson phases need the committed fields"};
    const MatTable t = make_table(tab, nphase, nfields);
    fftg::launch_damage(t, H->g.N, nfields, phase, abar, hist, nullptr, D, H->st);
    check_launch();
    sync(H);
    return FFTG_OK;
  });
}

fftg_status fftg_damage_adjoint(fftg_handle* H, const unsigned char* phase, const fftg_phase* tab,
                                int nphase, int nfields, const double* abar, const double* hist,
                                const double* gD, double* gabar) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    validate_table(tab, nphase, nfields);
    if (nfields < 1 || !phase || !abar || !hist || !gD || !gabar)
      throw Fail{FFTG_E_INVALID, "fftg_damage_adjoint: null pointer or no field"};
    validate_phase(H, phase, nphase);
    if (has_gtn(tab, nphase))
      throw Fail{FFTG_E_UNSUPPORTED, "fftg_damage_adjoint: no adjoint of the Gurson porosity"};
    const MatTable t = make_table(tab, nphase, nfields);
    fftg::launch_damage_adj(t, H->g.N, nfields, phase, abar, hist, gD, gabar, H->st);
    check_launch();
    sync(H);
    return FFTG_OK;
  });
}

fftg_status fftg_ell2(fftg_handle* H, const unsigned char* phase, const fftg_phase* tab,
                      int nphase, int field, double* ell2) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    validate_table(tab, nphase, FFTG_MAX_FIELDS);
    if (!phase || !ell2 || field < 0 || field >= FFTG_MAX_FIELDS)
      throw Fail{FFTG_E_INVALID, "fftg_ell2: null pointer or bad field"};
    validate_phase(H, phase, nphase);
    const MatTable t = make_table(tab, nphase, FFTG_MAX_FIELDS);
    fftg::launch_ell2<double>(t, H->g.N, field, phase, ell2, H->st);
    check_launch();
    sync(H);
    return FFTG_OK;
  });
}

fftg_status fftg_phase_sums(fftg_handle* H, const unsigned char* phase, int nphase,
                            const double* f, double* out) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    if (!phase || !f || !out || nphase < 1 || nphase > FFTG_MAX_PHASES)
      throw Fail{FFTG_E_INVALID, "fftg_phase_sums: bad arguments"};
    validate_phase(H, phase, nphase);
    read_sums(H, fftg::launch_phase_sums(H->g.N, nphase, phase, f, H->partials, H->st), nphase,
              out);
    return FFTG_OK;
  });
}

fftg_status fftg_solve(fftg_handle* H, const unsigned char* phase, const fftg_phase* tab,
                       int nphase, int nfields, const double* D, const double* state_n,
                       const fftg_macro* target, double* eps, double* sigma, double* state_np1,
                       double* alpha, const fftg_krylov_opts* cg, double newton_tol,
                       int newton_maxit, fftg_stats* stats) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    validate_table(tab, nphase, nfields);
    validate_macro(target, H->c);
    if (!phase || !state_n || !eps || !sigma || !state_np1 || !cg ||
        (nfields > 0 && (!D || !alpha)))
      throw Fail{FFTG_E_INVALID, "fftg_solve: null pointer"};
    validate_phase(H, phase, nphase);
    MatTable t = make_table(tab, nphase, nfields);
    MechOut o = H->fp32() ? mechanics<float>(H, phase, t, nfields, D, state_n, target, eps, sigma,
                                             state_np1, alpha, cg, newton_tol, newton_maxit)
                          : mechanics<double>(H, phase, t, nfields, D, state_n, target, eps,
                                              sigma, state_np1, alpha, cg, newton_tol,
                                              newton_maxit);
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->newton_iters = o.newton;
      stats->cg_iters = o.cg;
      stats->relres = o.relres;
      stats->t_ms[0] = o.t_const;
      stats->t_ms[1] = o.t_cg;
    }
    return o.converged ? FFTG_OK : FFTG_NOT_CONVERGED;
  });
}

fftg_status staggered_step(fftg_handle* H, const unsigned char* phase, const fftg_phase* tab,
                           int nphase, int nfields, double* state, const fftg_macro* target,
                           const fftg_krylov_opts* cg, const fftg_krylov_opts* pcg,
                           double newton_tol, int newton_maxit, double stagger_tol,
                           int max_stagger_iters, double* sigma_out, double* homog_out,
                           fftg_stats* stats) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    validate_table(tab, nphase, nfields);
    validate_macro(target, H->c);
    if (!phase || !state || !cg || !pcg || !sigma_out || !homog_out)
      throw Fail{FFTG_E_INVALID, "staggered_step: null pointer"};
    validate_phase(H, phase, nphase);
    if (max_stagger_iters < 1) throw Fail{FFTG_E_INVALID, "max_stagger_iters must be >= 1"};
    const MatTable t = make_table(tab, nphase, nfields);
    const StaggerOut o = stagger_core(H, phase, t, nfields, state, target, cg, pcg, newton_tol,
                                      newton_maxit, stagger_tol, max_stagger_iters, sigma_out,
                                      homog_out, false, 0);
    if (stats) *stats = o.stats;
    return o.converged && o.inner_ok ? FFTG_OK : FFTG_NOT_CONVERGED;
  });
}


fftg_status fftg_drive(fftg_handle* H, const unsigned char* phase, const fftg_phase* tab,
                       int nphase, int nfields, double* state, const fftg_macro* target_end,
                       const fftg_krylov_opts* cg, const fftg_krylov_opts* pcg,
                       double newton_tol, int newton_maxit, double stagger_tol,
                       int max_stagger_iters, fftg_drive_opts* opts, double* sigma_out,
                       fftg_drive_record* records, int max_records, int* n_records) {
  if (!H) return FFTG_E_INVALID;
  return run_guarded(H, [&]() -> fftg_status {
    validate_table(tab, nphase, nfields);
    validate_macro(target_end, H->c);
    if (!phase || !state || !cg || !pcg || !opts || !sigma_out || !n_records ||
        (max_records > 0 && !records))
      throw Fail{FFTG_E_INVALID, "fftg_drive: null pointer"};
    validate_phase(H, phase, nphase);
    if (max_stagger_iters < 1) throw Fail{FFTG_E_INVALID, "max_stagger_iters must be >= 1"};
    if (!(opts->dt > 0.0) || !(opts->dt_min > 0.0) || !(opts->dt_max > 0.0) ||
        !(opts->grow >= 1.0) || max_records < 0 || opts->max_attempts < 0 ||
        opts->newton_div < 0 || !std::isfinite(opts->t) || !std::isfinite(opts->t_end))
      throw Fail{FFTG_E_INVALID, "fftg_drive: bad options"};
    const Geo& g = H->g;
    const int c = H->c, J = nfields;
    const size_t nstate = (size_t)(c + 7 + 2 * J) * (size_t)g.N;
    const size_t nsig = (size_t)c * (size_t)g.N;
    if (H->drive_bak_n < nstate + nsig) {
      dfree((void*&)H->drive_bak);
      H->drive_bak = (double*)dalloc(sizeof(double) * (nstate + nsig));
      H->drive_bak_n = nstate + nsig;
    }
    const MatTable t = make_table(tab, nphase, J);
    fftg_host::DriveCtl dc{opts->t,      opts->dt,    opts->t_end,       opts->dt_min,
                           opts->dt_max, opts->grow,  max_records,       opts->max_attempts};
    double tn = 0.0;
    while (dc.next(tn)) {
      fftg_macro tgt = *target_end;
      for (int k = 0; k < 6; ++k) {
        tgt.E[k] = tn * target_end->E[k];
        tgt.S[k] = tn * target_end->S[k];
      }
      HIPCHK(hipMemcpyAsync(H->drive_bak, state, sizeof(double) * nstate,
                            hipMemcpyDeviceToDevice, H->st));
      HIPCHK(hipMemcpyAsync(H->drive_bak + nstate, sigma_out, sizeof(double) * nsig,
                            hipMemcpyDeviceToDevice, H->st));
      auto t0 = std::chrono::steady_clock::now();
      double homog[12];
      const StaggerOut o =
          stagger_core(H, phase, t, J, state, &tgt, cg, pcg, newton_tol, newton_maxit,
                       stagger_tol, max_stagger_iters, sigma_out, homog, true, opts->newton_div);
      if (o.converged && o.inner_ok) {
        const int cuts = dc.cut;
        fftg_drive_record& r = records[dc.accepted(tn)];
        r.t = tn;
        for (int i = 0; i < 12; ++i) r.homog[i] = homog[i];
        r.err = o.stats.err;
        r.cutbacks = cuts;
        r.stagger_iters = o.stats.stagger_iters;
        r.newton_iters = o.stats.newton_iters;
        r.cg_iters = o.stats.cg_iters;
        r.pcg_iters = o.stats.pcg_iters;
        r.ms = wall_ms(t0);
      } else {
        HIPCHK(hipMemcpyAsync(state, H->drive_bak, sizeof(double) * nstate,
                              hipMemcpyDeviceToDevice, H->st));
        HIPCHK(hipMemcpyAsync(sigma_out, H->drive_bak + nstate, sizeof(double) * nsig,
                              hipMemcpyDeviceToDevice, H->st));
        if (!dc.rejected()) break;
      }
    }
    const double tl = dc.t, dt = dc.dt;
    const int reason = dc.reason, attempts = dc.attempts, recs = dc.recs;
    sync(H);
    opts->t = tl;
    opts->dt = dt;
    opts->reason = reason;
    opts->attempts = attempts;
    *n_records = recs;
    return reason == 0 ? FFTG_OK : FFTG_NOT_CONVERGED;
  });
}


}  // extern "C"

// ------------------------------------------------------------ allocation-free Helmholtz solve
// Device memory of helmholtz_solve_noalloc: one static array per GPU, held
// until the process ends.  Host code must never pass `scratch` itself to a
// kernel or a copy (on the host it is only a stand-in for the symbol): it uses
// the device address hipGetSymbolAddress returns for the current device.
constexpr long long kNoallocMaxVoxels = 64LL * 64 * 64;
constexpr size_t kNoallocBytes = (size_t)36 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
thread_local std::string g_noalloc_error;

// device address of `scratch` on the current device, looked up once per device
void* scratch_address() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Fail{FFTG_E_UNSUPPORTED, "device index above 63"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw HipError{std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// bump allocator over the scratch array (256-byte aligned slices)
struct Carve {
  char* base;
  size_t off = 0, cap;
  void* take(size_t bytes) {
    const size_t b = (bytes + 255) & ~(size_t)255;
    if (off + b > cap) throw Fail{FFTG_E_UNSUPPORTED, "helmholtz_solve_noalloc: scratch too small"};
    void* p = base + off;
    off += b;
    return p;
  }
};

}  // namespace

extern "C" {

fftg_status helmholtz_solve_noalloc(const fftg_grid* grid, void* hip_stream, const double* alpha,
                                    const double* ell2, double ell2_ref, double* abar,
                                    const fftg_krylov_opts* opts, fftg_stats* stats) {
  g_noalloc_error.clear();
  auto fail = [](fftg_status c, const std::string& m) {
    g_noalloc_error = m;
    return c;
  };
  if (!grid || !alpha || !ell2 || !abar || !opts)
    return fail(FFTG_E_INVALID, "helmholtz_solve_noalloc: null pointer");
  if (grid->ndim != 2 && grid->ndim != 3)
    return fail(FFTG_E_INVALID, "helmholtz_solve_noalloc: ndim must be 2 or 3");
  if (grid->prec != FFTG_FP64)
    return fail(FFTG_E_UNSUPPORTED, "helmholtz_solve_noalloc: FP64 grids only");
  if (grid->scheme != FFTG_ROTATED && grid->scheme != FFTG_SPECTRAL)
    return fail(FFTG_E_INVALID, "helmholtz_solve_noalloc: unknown derivative scheme");
  const int n1 = grid->n[0], n2 = grid->n[1], n3 = grid->ndim == 3 ? grid->n[2] : 1;
  if (n1 < 2 || n2 < 1 || n3 < 1 || !(grid->h > 0.0) ||
      (grid->ndim == 2 && grid->n[2] != 1 && grid->n[2] != 0))
    return fail(FFTG_E_INVALID, "helmholtz_solve_noalloc: bad grid size or voxel size");
  const int nmax = grid->ndim == 3 ? 256 : 512;
  if (!smooth23(n1) || !smooth23(n2) || !smooth23(n3) || n1 % 2 != 0 || n1 > nmax ||
      n2 > nmax || n3 > nmax)
    return fail(FFTG_E_UNSUPPORTED, "helmholtz_solve_noalloc: unsupported size (need N = "
                                     "2^a 3^b, N1 even, N <= 256 in 3D, 512 in 2D)");
  if ((long long)n1 * n2 * n3 > kNoallocMaxVoxels)
    return fail(FFTG_E_UNSUPPORTED,
                "helmholtz_solve_noalloc: more than 262144 voxels (64^3), the scratch limit");
  // a handle on the stack whose workspace is carved from the scratch array;
  // nothing it points to is freed (destroy() is never called on it)
  fftg_handle hd;
  fftg_handle* H = &hd;
  KrylovCtl hctl_host{};
  double hsums_host[64];
  fftg_status rc = run_guarded(H, [&]() -> fftg_status {
    Carve cv{static_cast<char*>(scratch_address()), 0, kNoallocBytes};
    Geo& g = H->g;
    g.ndim = grid->ndim;
    g.n1 = n1;
    g.n2 = n2;
    g.n3 = n3;
    g.n1h = n1 / 2 + 1;
    g.N = (long long)n1 * n2 * n3;
    g.Ns = (long long)g.n1h * n2 * n3;
    H->c = grid->ndim == 3 ? 6 : 3;
    H->h = grid->h;
    H->scheme = grid->scheme;
    H->prec = FFTG_FP64;
    H->st = reinterpret_cast<hipStream_t>(hip_stream);
    H->nograph = true;
    H->hctl = &hctl_host;
    H->hsums = hsums_host;
    const int ns[3] = {n1, n2, n3};
    std::vector<double> tw[3], pq[3], gq[3], cs[3];
    for (int a = 0; a < 3; ++a) {
      H->plan[a] = make_plan(ns[a]);
      tw[a] = twiddles(ns[a]);
      H->tw64[a] = static_cast<cpx<double>*>(cv.take(sizeof(double) * tw[a].size()));
      HIPCHK(hipMemcpyAsync(H->tw64[a], tw[a].data(), sizeof(double) * tw[a].size(),
                            hipMemcpyHostToDevice, H->st));
      axis_tables(ns[a], a == 0, grid->h, grid->scheme, pq[a], gq[a], cs[a]);
    }
    std::vector<double> all;
    int off = 0;
    for (auto* tab : {pq, gq, cs}) {
      int* dst = tab == pq ? H->S64.pq : tab == gq ? H->S64.gq : H->S64.cs;
      for (int a = 0; a < 3; ++a) {
        dst[a] = off;
        all.insert(all.end(), tab[a].begin(), tab[a].end());
        off += (int)tab[a].size();
      }
    }
    H->sym64 = static_cast<double*>(cv.take(sizeof(double) * all.size()));
    HIPCHK(hipMemcpyAsync(H->sym64, all.data(), sizeof(double) * all.size(),
                          hipMemcpyHostToDevice, H->st));
    H->S64.base = H->sym64;
    const size_t ss = sizeof(cpx<double>) * (size_t)g.Ns;
    H->hx = cv.take(ss);
    H->hr = cv.take(ss);
    H->hp = cv.take(ss);
    H->hAp = cv.take(ss);
    H->hb = cv.take(ss);
    H->hw = cv.take(ss * g.ndim);
    // reductions: at most one partial per outer-axis tile of the divergence
    // pass (<= Ns), two sets of at most RED_BLOCKS for the pointwise kernels
    H->npartials = (size_t)std::max<long long>(g.Ns, 2LL * fftg::RED_BLOCKS) + 64;
    H->partials = static_cast<double*>(cv.take(sizeof(double) * H->npartials));
    H->dsums = static_cast<double*>(cv.take(sizeof(double) * 64));
    H->ctl = static_cast<KrylovCtl*>(cv.take(sizeof(KrylovCtl)));
    int it = 0, status = 0;
    double rel = 0.0;
    auto t0 = std::chrono::steady_clock::now();
    HelmOut ho;
    helmholtz_pcg64(H, alpha, ell2, ell2_ref, abar, opts->tol, opts->maxit, 1, &ho);
    it = ho.iters;
    rel = ho.relres;
    status = ho.status;
    sync(H);
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->pcg_iters = it;
      stats->relres = rel;
      stats->t_ms[2] = wall_ms(t0);
    }
    if (status == 3) throw Fail{FFTG_E_BREAKDOWN, "Helmholtz PCG breakdown"};
    if (status == 4) throw Fail{FFTG_E_NONFINITE, "non-finite value in Helmholtz PCG"};
    return status == 1 ? FFTG_OK : FFTG_NOT_CONVERGED;
  });
  if (rc < 0) g_noalloc_error = H->err;
  return rc;
}

const char* helmholtz_noalloc_last_error(void) { return g_noalloc_error.c_str(); }

// voxels a lockstep sub-class of large grids aims at
constexpr long long kClassVoxels = 4LL << 20;

fftg_status fftg_batch_step(fftg_batch_item* items, int n, int nworkers,
                            const fftg_krylov_opts* cg, const fftg_krylov_opts* pcg,
                            double newton_tol, int newton_maxit, double stagger_tol,
                            int max_stagger_iters) {
  if (n < 0 || (n > 0 && !items) || nworkers < 1 || !cg || !pcg) return FFTG_E_INVALID;
  // every item needs its own handle: a handle is driven by one thread at a time
  std::vector<fftg_handle*> hs;
  for (int i = 0; i < n; ++i) {
    if (!items[i].h) return FFTG_E_INVALID;
    hs.push_back(items[i].h);
  }
  std::sort(hs.begin(), hs.end());
  if (std::adjacent_find(hs.begin(), hs.end()) != hs.end()) return FFTG_E_INVALID;
  // classes of items that run in lockstep (FFTG_BATCH_LOCKSTEP=0: every item
  // alone on its own handle and stream); a class of large grids is split into
  // sub-classes of about kClassVoxels voxels (FFTG_BATCH_CLASS_VOXELS
  // overrides), run by different workers: a sub-class already fills the GPU,
  // and several of them in flight keep it busy while one waits on its host
  // decisions or on its slowest RVE.
  const char* ls = std::getenv("FFTG_BATCH_LOCKSTEP");
  const bool lockstep = !(ls && ls[0] == '0' && ls[1] == '\0');
  long long cap = kClassVoxels;
  if (const char* cv = std::getenv("FFTG_BATCH_CLASS_VOXELS")) {
    const long long v = std::atoll(cv);
    if (v > 0) cap = v;
  }
  std::vector<fftg_host::ItemKey> keys(n);
  for (int i = 0; i < n; ++i) {
    const fftg_handle* x = items[i].h;
    fftg_host::ItemKey& k = keys[i];
    k.ndim = x->g.ndim;
    k.n1 = x->g.n1;
    k.n2 = x->g.n2;
    k.n3 = x->g.n3;
    k.c = x->c;
    k.scheme = x->scheme;
    k.prec = x->prec;
    k.nfields = items[i].nfields;
    k.h = x->h;
    std::memcpy(k.mask, items[i].target.mask, 6);
    k.voxels = x->g.N;
  }
  const std::vector<std::vector<int>> units = fftg_host::batch_units(keys, lockstep, cap);
  const int nu = (int)units.size();
  std::atomic<int> next{0};
  auto work = [&]() {
    for (int k = next.fetch_add(1); k < nu; k = next.fetch_add(1)) {
      const std::vector<int>& u = units[k];
      if (u.size() > 1) {
        run_class(items, u, cg, pcg, newton_tol, newton_maxit, stagger_tol, max_stagger_iters);
        continue;
      }
      fftg_batch_item& it = items[u[0]];
      it.status = staggered_step(it.h, it.phase, it.tab, it.nphase, it.nfields, it.state,
                                 &it.target, cg, pcg, newton_tol, newton_maxit, stagger_tol,
                                 max_stagger_iters, it.sigma_out, it.homog_out, &it.stats);
    }
  };
  const int nw = std::min(nworkers, std::max(nu, 1));
  std::vector<std::thread> pool;
  for (int w = 1; w < nw; ++w) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  fftg_status rc = FFTG_OK;
  for (int i = 0; i < n; ++i) {
    const int st = items[i].status;
    if (st < 0 && (rc >= 0 || st < rc)) rc = (fftg_status)st;
    if (st == FFTG_NOT_CONVERGED && rc == FFTG_OK) rc = FFTG_NOT_CONVERGED;
  }
  return rc;
}
}  // extern "C"
