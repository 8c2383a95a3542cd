// Device building blocks for the LDS-staged mixed-radix (2, 3, 4, 8) Stockham
// FFT used by every transform pass.  One workgroup of FFT_THREADS threads
// transforms a batch of lines that sits in LDS; each stage reads its inputs
// into registers, synchronises, and writes the autosorted outputs back, so a
// single LDS buffer suffices.
//
// Stockham autosort (decimation in time), natural order in and out: for a
// stage of radix R after stages whose radices multiply to Ns, butterfly j of
// a line reads elements j + r n/R, multiplies element r by W_n^(k r n/(Ns R))
// with k = j mod Ns, applies the length-R DFT and writes output r to
// (j div Ns) Ns R + k + r Ns.
#pragma once
#include <hip/hip_runtime.h>

namespace fftg {

constexpr int FFT_THREADS = 256;
constexpr int LDS_ELEMS = 2048;  // complex elements of one batch held in LDS
constexpr int MAX_STAGES = 12;

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

// The complex arithmetic fixes its own roundings: products are never fused
// into a following sum by the compiler (fp contract off), and the complex
// product uses one explicit fma per component.  So a transform rounds the
// same way in every instantiation (tile size, lines per thread), and results
// do not depend on the tile the autotuner picks.
template <typename T>
__device__ __forceinline__ cpx<T> mk(T a, T b) { return cpx<T>{a, b}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) {
#pragma clang fp contract(off)
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) {
#pragma clang fp contract(off)
  return {a.x - b.x, a.y - b.y};
}
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename T>
__device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
#pragma clang fp contract(off)
  const T ry = a.y * b.y, iy = a.y * b.x;
  return {fma_t(a.x, b.x, -ry), fma_t(a.x, b.y, iy)};
}
template <typename T>
__device__ __forceinline__ cpx<T> scale(cpx<T> a, T s) {
#pragma clang fp contract(off)
  return {a.x * s, a.y * s};
}
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.x, -a.y}; }
// a * i
template <typename T>
__device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return {-a.y, a.x}; }
// a * (-i)
template <typename T>
__device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) { return {a.y, -a.x}; }

// a * W4, W4 = exp(-i pi/2) = -i (forward) or +i (inverse)
template <bool FWD, typename T>
__device__ __forceinline__ cpx<T> rot4(cpx<T> a) { return FWD ? mul_mi(a) : mul_i(a); }

template <bool FWD, typename T>
__device__ __forceinline__ void dft2(cpx<T>* v) {
  cpx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <bool FWD, typename T>
__device__ __forceinline__ void dft3(cpx<T>* v) {
#pragma clang fp contract(off)
  const T s3 = T(0.86602540378443864676372317075294);  // sqrt(3)/2
  cpx<T> t = v[1] + v[2];
  cpx<T> m = v[0] - scale(t, T(0.5));
  cpx<T> d = scale(v[1] - v[2], s3);
  cpx<T> s = FWD ? mul_mi(d) : mul_i(d);
  v[0] = v[0] + t;
  v[1] = m + s;
  v[2] = m - s;
}

template <bool FWD, typename T>
__device__ __forceinline__ void dft4(cpx<T>& v0, cpx<T>& v1, cpx<T>& v2, cpx<T>& v3) {
  cpx<T> t0 = v0 + v2, t1 = v0 - v2, t2 = v1 + v3, t3 = rot4<FWD>(v1 - v3);
  v0 = t0 + t2;
  v1 = t1 + t3;
  v2 = t0 - t2;
  v3 = t1 - t3;
}

template <bool FWD, typename T>
__device__ __forceinline__ void dft4(cpx<T>* v) { dft4<FWD>(v[0], v[1], v[2], v[3]); }

template <bool FWD, typename T>
__device__ __forceinline__ void dft8(cpx<T>* v) {
#pragma clang fp contract(off)
  const T c = T(0.70710678118654752440084436210485);  // sqrt(1/2)
  cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<FWD>(e0, e1, e2, e3);
  dft4<FWD>(o0, o1, o2, o3);
  // o_k *= W8^k
  cpx<T> w1, w3;
  if (FWD) {
    w1 = mk(c * (o1.x + o1.y), c * (o1.y - o1.x));
    w3 = mk(c * (o3.y - o3.x), -c * (o3.x + o3.y));
  } else {
    w1 = mk(c * (o1.x - o1.y), c * (o1.x + o1.y));
    w3 = mk(-c * (o3.x + o3.y), c * (o3.x - o3.y));
  }
  cpx<T> w2 = rot4<FWD>(o2);
  v[0] = e0 + o0;
  v[4] = e0 - o0;
  v[1] = e1 + w1;
  v[5] = e1 - w1;
  v[2] = e2 + w2;
  v[6] = e2 - w2;
  v[3] = e3 + w3;
  v[7] = e3 - w3;
}

// One 1D transform plan: length and radix sequence.
struct Plan {
  int n;
  int nst;
  int radix[MAX_STAGES];
};

// LDS addressing: LINEFAST -> element t of line l at t*ld + l (lines adjacent);
// otherwise at l*ld + t (each line contiguous).
template <bool LINEFAST>
__device__ __forceinline__ int laddr(int line, int t, int ld) {
  return LINEFAST ? t * ld + line : line * ld + t;
}

// Line-contiguous layout with one pad slot after every 8 elements: the
// radix-R Stockham writes (stride R elements across threads) and the
// contiguous reads then fall into distinct LDS banks.  Line pitch >=
// n + n / 8.
__device__ __forceinline__ int paddr(int line, int t, int ld) { return line * ld + t + (t >> 3); }
constexpr int padded_pitch(int n) { return n + n / 8 + 1; }

template <typename T, int R, bool FWD, bool LINEFAST>
__device__ __forceinline__ void stage(cpx<T>* buf, int n, int nlines, int ld, int Ns,
                                      const cpx<T>* __restrict__ tw) {
  constexpr int MAXB = (LDS_ELEMS / R + FFT_THREADS - 1) / FFT_THREADS;
  const int m = n / R;
  const int total = nlines * m;
  const int tid = threadIdx.x;
  cpx<T> v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = tid + q * FFT_THREADS;
    if (b < total) {
      const int line = LINEFAST ? b % nlines : b / m;
      const int j = LINEFAST ? b / nlines : b % m;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[laddr<LINEFAST>(line, j + r * m, ld)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = tid + q * FFT_THREADS;
    if (b < total) {
      const int line = LINEFAST ? b % nlines : b / m;
      const int j = LINEFAST ? b / nlines : b % m;
      const int k = j % Ns;
      if (Ns > 1) {
        const int step = n / (Ns * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = tw[k * r * step];
          if (!FWD) w.y = -w.y;
          v[q][r] = v[q][r] * w;
        }
      }
      if (R == 2) dft2<FWD>(v[q]);
      if (R == 3) dft3<FWD>(v[q]);
      if (R == 4) dft4<FWD>(v[q]);
      if (R == 8) dft8<FWD>(v[q]);
      const int o = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[laddr<LINEFAST>(line, o + r * Ns, ld)] = v[q][r];
    }
  }
  __syncthreads();
}

// Transform `nlines` lines of length plan.n held in LDS (nlines * n must not
// exceed LDS_ELEMS).  FWD: exp(-i ...), unnormalised; otherwise exp(+i ...).
// The caller synchronises before the call; the call ends synchronised.
template <typename T, bool FWD, bool LINEFAST>
__device__ void lds_fft(cpx<T>* buf, const Plan& plan, int nlines, int ld,
                        const cpx<T>* __restrict__ tw) {
  int Ns = 1;
  for (int s = 0; s < plan.nst; ++s) {
    const int R = plan.radix[s];
    if (R == 8)
      stage<T, 8, FWD, LINEFAST>(buf, plan.n, nlines, ld, Ns, tw);
    else if (R == 4)
      stage<T, 4, FWD, LINEFAST>(buf, plan.n, nlines, ld, Ns, tw);
    else if (R == 3)
      stage<T, 3, FWD, LINEFAST>(buf, plan.n, nlines, ld, Ns, tw);
    else
      stage<T, 2, FWD, LINEFAST>(buf, plan.n, nlines, ld, Ns, tw);
    Ns *= R;
  }
}

// ---------------------------------------------------------------------------
// Compile-time variant for fixed lengths: the radix sequence, the number of
// lines and the LDS pitch are constants, so every index division becomes a
// shift or a multiply and the butterfly loops unroll.  The radix rule is the
// host's: as many 8s as possible (two 4s instead of 8 x 2), then 4 or 2, then 3s.
constexpr int c_pow(int n, int p) {
  int c = 0;
  while (n % p == 0) {
    n /= p;
    ++c;
  }
  return c;
}
constexpr int c_n8(int n) {
  const int a = c_pow(n, 2);
  return (a % 3 == 1 && a / 3 >= 1) ? a / 3 - 1 : a / 3;
}
constexpr int c_n4(int n) {
  const int a = c_pow(n, 2);
  return (a % 3 == 1 && a / 3 >= 1) ? 2 : (a % 3 == 2 ? 1 : 0);
}
constexpr int c_n2(int n) {
  const int a = c_pow(n, 2);
  return (a % 3 == 1 && a / 3 == 0) ? 1 : 0;
}
constexpr int c_nst(int n) { return c_n8(n) + c_n4(n) + c_n2(n) + c_pow(n, 3); }
constexpr int c_radix(int n, int s) {
  return s < c_n8(n)                         ? 8
         : s < c_n8(n) + c_n4(n)             ? 4
         : s < c_n8(n) + c_n4(n) + c_n2(n)   ? 2
                                             : 3;
}

template <typename T, int R, bool FWD, bool LINEFAST, int N, int NL, int LD, int NS, int NT,
          bool PAD = false>
__device__ __forceinline__ void stage_c(cpx<T>* buf, const cpx<T>* __restrict__ tw) {
  constexpr int M = N / R;
  constexpr int TOTAL = NL * M;
  constexpr int MAXB = (TOTAL + NT - 1) / NT;
  const int tid = threadIdx.x;
  cpx<T> v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = tid + q * NT;
    if (TOTAL % NT == 0 || b < TOTAL) {
      const int line = LINEFAST ? b % NL : b / M;
      const int j = LINEFAST ? b / NL : b % M;
#pragma unroll
      for (int r = 0; r < R; ++r)
        v[q][r] = buf[PAD ? paddr(line, j + r * M, LD) : laddr<LINEFAST>(line, j + r * M, LD)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = tid + q * NT;
    if (TOTAL % NT == 0 || b < TOTAL) {
      const int line = LINEFAST ? b % NL : b / M;
      const int j = LINEFAST ? b / NL : b % M;
      const int k = j % NS;
      if (NS > 1) {
        constexpr int STEP = N / (NS * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = tw[k * r * STEP];
          if (!FWD) w.y = -w.y;
          v[q][r] = v[q][r] * w;
        }
      }
      if (R == 2) dft2<FWD>(v[q]);
      if (R == 3) dft3<FWD>(v[q]);
      if (R == 4) dft4<FWD>(v[q]);
      if (R == 8) dft8<FWD>(v[q]);
      const int o = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r)
        buf[PAD ? paddr(line, o + r * NS, LD) : laddr<LINEFAST>(line, o + r * NS, LD)] = v[q][r];
    }
  }
  __syncthreads();
}

template <typename T, bool FWD, bool LINEFAST, int N, int NL, int LD, int NT, bool PAD, int S,
          int NS>
__device__ __forceinline__ void lds_fft_stages(cpx<T>* buf, const cpx<T>* __restrict__ tw) {
  if constexpr (S < c_nst(N)) {
    constexpr int R = c_radix(N, S);
    stage_c<T, R, FWD, LINEFAST, N, NL, LD, NS, NT, PAD>(buf, tw);
    lds_fft_stages<T, FWD, LINEFAST, N, NL, LD, NT, PAD, S + 1, NS * R>(buf, tw);
  }
}

// Fixed-length transform of NL lines of length N in LDS by a workgroup of NT
// threads (same contract as lds_fft).
template <typename T, bool FWD, bool LINEFAST, int N, int NL, int LD, int NT = FFT_THREADS,
          bool PAD = false>
__device__ __forceinline__ void lds_fft_c(cpx<T>* buf, const cpx<T>* __restrict__ tw) {
  static_assert(!PAD || (!LINEFAST && LD >= N + N / 8), "padded layout: line pitch");
  lds_fft_stages<T, FWD, LINEFAST, N, NL, LD, NT, PAD, 0, 1>(buf, tw);
}

// Direct-stage form of lds_fft_c for line-fast tiles: the first stage takes
// its inputs from ld(t) (element t of the thread's line, tid % NL) straight
// into registers, the last stage hands its outputs to st(t, v), and only the
// stages in between go through LDS (element t of line l at t * NL + l).  The
// butterflies, twiddles and their order are those of lds_fft_c, so the
// results are the same bit for bit; a 3-stage transform makes 2 LDS round
// trips and 3 barriers instead of 4 and 7.
// FIRST / LAST: this stage reads from ld / writes to st (else from / to LDS).
template <typename T, int R, bool FWD, int N, int NL, int NS, int NT, bool FIRST, bool LAST,
          typename LDF, typename STF>
__device__ __forceinline__ void stage_d(cpx<T>* buf, const cpx<T>* __restrict__ tw, LDF& ld,
                                        STF& st) {
  static_assert(NT % NL == 0, "each thread keeps one line");
  constexpr int M = N / R;
  constexpr int TOTAL = NL * M;
  constexpr int MAXB = (TOTAL + NT - 1) / NT;
  const int tid = threadIdx.x;
  const int line = tid % NL;
  cpx<T> v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = tid + q * NT;
    if (TOTAL % NT == 0 || b < TOTAL) {
      const int j = b / NL;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = FIRST ? ld(j + r * M) : buf[(j + r * M) * NL + line];
    }
  }
  if (!FIRST && !LAST) __syncthreads();  // every read of the stage before its writes
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = tid + q * NT;
    if (TOTAL % NT == 0 || b < TOTAL) {
      const int j = b / NL;
      const int k = j % NS;
      if (NS > 1) {
        constexpr int STEP = N / (NS * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = tw[k * r * STEP];
          if (!FWD) w.y = -w.y;
          v[q][r] = v[q][r] * w;
        }
      }
      if (R == 2) dft2<FWD>(v[q]);
      if (R == 3) dft3<FWD>(v[q]);
      if (R == 4) dft4<FWD>(v[q]);
      if (R == 8) dft8<FWD>(v[q]);
      const int o = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (LAST)
          st(o + r * NS, v[q][r]);
        else
          buf[(o + r * NS) * NL + line] = v[q][r];
      }
    }
  }
  if (!LAST) __syncthreads();  // the stage's writes before the next stage reads
}

template <typename T, bool FWD, int N, int NL, int NT, bool GIN, bool GOUT, int S, int NS,
          typename LDF, typename STF>
__device__ __forceinline__ void direct_stages(cpx<T>* buf, const cpx<T>* __restrict__ tw, LDF& ld,
                                              STF& st) {
  if constexpr (S < c_nst(N)) {
    constexpr int R = c_radix(N, S);
    stage_d<T, R, FWD, N, NL, NS, NT, GIN && S == 0, GOUT && S + 1 == c_nst(N)>(buf, tw, ld, st);
    direct_stages<T, FWD, N, NL, NT, GIN, GOUT, S + 1, NS * R>(buf, tw, ld, st);
  }
}

// GIN = false: the input is already in LDS (line-fast, pitch NL, after a
// barrier); GOUT = false: the output stays in LDS (a barrier follows).
template <typename T, bool FWD, int N, int NL, int NT, typename LDF, typename STF,
          bool GIN = true, bool GOUT = true>
__device__ __forceinline__ void lds_fft_direct(cpx<T>* buf, const cpx<T>* __restrict__ tw, LDF ld,
                                               STF st) {
  direct_stages<T, FWD, N, NL, NT, GIN, GOUT, 0, 1>(buf, tw, ld, st);
}

// LDS budgets of the fixed-length kernels (bytes).  A smaller tile leaves
// room for more workgroups per CU, i.e. more loads in flight.
#ifndef FFTG_TILE_BYTES
#define FFTG_TILE_BYTES 32768   // y / z passes, one component per line
#endif
#ifndef FFTG_FUSED_BYTES
#define FFTG_FUSED_BYTES 16384  // x passes fused with the pointwise operator
#endif
#ifndef FFTG_WIDE_BYTES
#define FFTG_WIDE_BYTES 49152   // outer Helmholtz passes, all gradient components
#endif
static_assert((FFTG_TILE_BYTES & (FFTG_TILE_BYTES - 1)) == 0 && FFTG_TILE_BYTES >= 4096,
              "y/z tile budget must be a power of two (tile lines must divide the workgroup)");
static_assert(FFTG_FUSED_BYTES >= 4096 && FFTG_WIDE_BYTES >= 4096, "LDS budgets too small");
template <typename T>
constexpr int kElems = 32768 / (int)sizeof(cpx<T>);   // plain x R2C / C2R
template <typename T>
constexpr int kElemsFused = FFTG_FUSED_BYTES / (int)sizeof(cpx<T>);
template <typename T>
constexpr int kElemsWide = FFTG_WIDE_BYTES / (int)sizeof(cpx<T>);

// Tile shapes shared by kernels and launchers (fixed-length path).
template <typename T>
constexpr int fx_pairs(int n) { return kElems<T> / n; }                 // x R2C / C2R
// Fused x passes: half the LDS budget for lines of up to 64 points, where
// small grids need more workgroups in flight (measured: 25-30% faster at
// 32^3-64^3, slower at 96^3 and 128^3).
template <typename T>
constexpr int fused_elems(int n) { return (n <= 64 ? kElemsFused<T> / 2 : kElemsFused<T>); }
template <typename T>
constexpr int lines_in(int elems, int n, int c) {
  return (2 * elems / (c * n)) - (2 * elems / (c * n)) % 2 < 2
             ? 2
             : (2 * elems / (c * n)) - (2 * elems / (c * n)) % 2;
}
template <typename T>
constexpr int fx_fused_lines(int n, int c) { return lines_in<T>(fused_elems<T>(n), n, c); }
// Helmholtz fused x pass: the half budget also at 96 and 128 points in FP32
// (measured 14.2 -> 11.3 us at 96^3, 19.5 -> 18.8 us at 128^3; FP64 keeps
// 16 KB there)
template <typename T>
constexpr int fx_helm_lines(int n, int nd) {
  return lines_in<T>(sizeof(T) == 4 ? kElemsFused<T> / 2 : fused_elems<T>(n), n, nd);
}
// Workgroup size of the fixed-length y / z passes: more threads over the same
// tile keep more loads in flight without shrinking the tile rows.
#ifndef FFTG_STRIDED_THREADS
#define FFTG_STRIDED_THREADS 512
#endif
#ifndef FFTG_WIDE_THREADS
#define FFTG_WIDE_THREADS 512
#endif
#ifndef FFTG_FUSED_THREADS
#define FFTG_FUSED_THREADS 256
#endif
constexpr int kFusedThreads = FFTG_FUSED_THREADS;  // fused x passes
static_assert(kFusedThreads == 128 || kFusedThreads == 256, "x-pass workgroup size");
constexpr int kStridedThreads = FFTG_STRIDED_THREADS;
constexpr int kWideThreads = FFTG_WIDE_THREADS;
static_assert((kStridedThreads == 256 || kStridedThreads == 512) &&
                  (kWideThreads == 256 || kWideThreads == 512),
              "outer-pass workgroup sizes");
// Outer Galerkin forward pass with the p.Ap partial sums (measured best:
// FP64 a 32 KB tile over 512 threads, FP32 a 16 KB tile over 256 threads).
template <typename T>
constexpr int kDotBytes = sizeof(T) == 8 ? 32768 : 16384;
template <typename T>
constexpr int kDotThreads = sizeof(T) == 8 ? 512 : 256;
constexpr int pow2_floor(int v) {
  int p = 1;
  while (2 * p <= v) p *= 2;
  return p;
}
// lines per y / z tile: a power of two (it must divide the workgroup)
template <typename T, int BYTES = FFTG_TILE_BYTES>
constexpr int fs_tile(int n) {                                          // y / z passes
  return pow2_floor(BYTES / (int)sizeof(cpx<T>) / n) < FFT_THREADS
             ? pow2_floor(BYTES / (int)sizeof(cpx<T>) / n)
             : FFT_THREADS;
}
template <typename T>
constexpr int fs_tile_wide(int n, int nc) { return pow2_floor(kElemsWide<T> / (n * nc)); }
// Galerkin forward pass fused with the residual update: every component of
// a tile's lines in LDS at once
#ifndef FFTG_FWDRES_BYTES
#define FFTG_FWDRES_BYTES 49152
#endif
#ifndef FFTG_FWDRES_THREADS
#define FFTG_FWDRES_THREADS 512
#endif
constexpr int kFwdResThreads = FFTG_FWDRES_THREADS;
template <typename T>
constexpr int fr_tile(int n, int nc) {
  return pow2_floor(FFTG_FWDRES_BYTES / (int)sizeof(cpx<T>) / (n * nc)) < 1
             ? 1
             : pow2_floor(FFTG_FWDRES_BYTES / (int)sizeof(cpx<T>) / (n * nc));
}

// Deterministic workgroup sum (fixed tree over NT lanes); the result is valid
// in thread 0.  `red` must hold NT doubles of LDS.
template <int NT = FFT_THREADS>
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  __syncthreads();
  red[tid] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  return red[0];
}

// Sum of nb partial sums in a fixed order: lane l adds p[l], p[l + NT], ...,
// then the fixed tree.  Every lane gets the result; `red` (NT doubles of LDS)
// may be reused only after a barrier.
template <int NT = FFT_THREADS>
__device__ __forceinline__ double ordered_sum_t(const double* __restrict__ p, int nb,
                                                double* red) {
  double acc = 0.0;
  // unrolled so that several loads are in flight; the additions keep their order
#pragma unroll 8
  for (int i = threadIdx.x; i < nb; i += NT) acc += p[i];
  return block_sum<NT>(acc, red);
}

}  // namespace fftg
