// HIP kernels for gfx950: transform passes, fused Galerkin / Helmholtz
// operator passes with their Krylov prologues and epilogues, pointwise
// projection and residual kernels, deterministic reductions, and the
// per-voxel constitutive update.
#include "kernels.hpp"

#include <cmath>
#include <stdexcept>

namespace fftg {

#define FFTG_KERNEL __global__ __launch_bounds__(FFT_THREADS)
#define FFTG_KERNEL_WIDE __global__ __launch_bounds__(512)

// Hermitian weight of a half-spectrum coefficient: its mirror image is not
// stored except on the planes kx = 0 and kx = n1/2.
__device__ __forceinline__ double hweight(int kx, int n1h) {
  return (kx == 0 || kx == n1h - 1) ? 1.0 : 2.0;
}

// Frequency indices of half-spectrum coefficient gi (gi < 2^31: grids are at
// most 256^3, so 32-bit division is exact and far cheaper than 64-bit).
__device__ __forceinline__ void decode(const Geo& g, long long gi, int& kx, int& ky, int& kz) {
  const unsigned u = (unsigned)gi, n1h = (unsigned)g.n1h, n2 = (unsigned)g.n2;
  const unsigned r = u / n1h;
  kx = (int)(u - r * n1h);
  const unsigned s = r / n2;
  ky = (int)(r - s * n2);
  kz = (int)(s % (unsigned)g.n3);
}

template <typename T>
__device__ __forceinline__ void qvec(const Sym<T>& s, bool grad, int kx, int ky, int kz, T q[3]) {
  const T* b = s.base;
  const T cx = b[s.cs[0] + kx], cy = b[s.cs[1] + ky], cz = b[s.cs[2] + kz];
  const int* o = grad ? s.gq : s.pq;
  q[0] = b[o[0] + kx] * cy * cz;
  q[1] = cx * b[o[1] + ky] * cz;
  q[2] = cx * cy * b[o[2] + kz];
}

// Orthogonal projection of a symmetric Mandel tensor onto {sym(u (x) q)}
// (Sec. 3.2.2): t = tau q, P tau = (t(x)q + q(x)t)/|q|^2 - (q(x)q)(q.t)/|q|^4;
// zero where |q| = 0.
template <typename T, int C>
__device__ __forceinline__ void project_point(const T q[3], cpx<T>* v) {
  const T q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
  if (!(q2 > T(0))) {
#pragma unroll
    for (int i = 0; i < C; ++i) v[i] = mk(T(0), T(0));
    return;
  }
  const T ir2 = T(0.70710678118654752440084436210485);
  const T inv = T(1) / q2;
  if (C == 6) {
    // full tensor from Mandel
    cpx<T> t11 = v[0], t22 = v[1], t33 = v[2];
    cpx<T> t23 = scale(v[3], ir2), t13 = scale(v[4], ir2), t12 = scale(v[5], ir2);
    cpx<T> a0 = scale(t11, q[0]) + scale(t12, q[1]) + scale(t13, q[2]);
    cpx<T> a1 = scale(t12, q[0]) + scale(t22, q[1]) + scale(t23, q[2]);
    cpx<T> a2 = scale(t13, q[0]) + scale(t23, q[1]) + scale(t33, q[2]);
    cpx<T> s = scale(a0, q[0]) + scale(a1, q[1]) + scale(a2, q[2]);
    cpx<T> si = scale(s, inv * inv);
    cpx<T> p11 = scale(scale(a0, q[0]), T(2) * inv) - scale(si, q[0] * q[0]);
    cpx<T> p22 = scale(scale(a1, q[1]), T(2) * inv) - scale(si, q[1] * q[1]);
    cpx<T> p33 = scale(scale(a2, q[2]), T(2) * inv) - scale(si, q[2] * q[2]);
    cpx<T> p23 = scale(scale(a1, q[2]) + scale(a2, q[1]), inv) - scale(si, q[1] * q[2]);
    cpx<T> p13 = scale(scale(a0, q[2]) + scale(a2, q[0]), inv) - scale(si, q[0] * q[2]);
    cpx<T> p12 = scale(scale(a0, q[1]) + scale(a1, q[0]), inv) - scale(si, q[0] * q[1]);
    const T r2 = T(1.4142135623730950488016887242097);
    v[0] = p11;
    v[1] = p22;
    v[2] = p33;
    v[3] = scale(p23, r2);
    v[4] = scale(p13, r2);
    v[5] = scale(p12, r2);
  } else {
    cpx<T> t11 = v[0], t22 = v[1], t12 = scale(v[2], ir2);
    cpx<T> a0 = scale(t11, q[0]) + scale(t12, q[1]);
    cpx<T> a1 = scale(t12, q[0]) + scale(t22, q[1]);
    cpx<T> s = scale(a0, q[0]) + scale(a1, q[1]);
    cpx<T> si = scale(s, inv * inv);
    cpx<T> p11 = scale(scale(a0, q[0]), T(2) * inv) - scale(si, q[0] * q[0]);
    cpx<T> p22 = scale(scale(a1, q[1]), T(2) * inv) - scale(si, q[1] * q[1]);
    cpx<T> p12 = scale(scale(a0, q[1]) + scale(a1, q[0]), inv) - scale(si, q[0] * q[1]);
    const T r2 = T(1.4142135623730950488016887242097);
    v[0] = p11;
    v[1] = p22;
    v[2] = scale(p12, r2);
  }
}

// ============================================================ x passes
// Two real lines a, b are transformed together as z = a + i b.  After the
// forward transform A[k] = (Z[k] + conj Z[n-k])/2, B[k] = -i (Z[k] - conj Z[n-k])/2;
// the inverse rebuilds Z[k] = A[k] + i B[k] and Z[n-k] = conj A[k] + i conj B[k].

// element j of complex line p in LDS: contiguous lines of pitch ld, padded
// (one slot after every 8 elements) when PAD
template <bool PAD>
__device__ __forceinline__ int xaddr(int p, int j, int ld) {
  return PAD ? paddr(p, j, ld) : p * ld + j;
}

template <bool PAD, typename T>
__device__ __forceinline__ void pack_inverse(cpx<T>* buf, int p, int k, int n1, int ld,
                                             cpx<T> A, cpx<T> B) {
  if (k == 0 || 2 * k == n1) {
    A.y = T(0);
    B.y = T(0);
  }
  buf[xaddr<PAD>(p, k, ld)] = mk(A.x - B.y, A.y + B.x);
  if (k > 0 && 2 * k < n1) buf[xaddr<PAD>(p, n1 - k, ld)] = mk(A.x + B.y, B.x - A.y);
}

template <bool PAD, typename T>
__device__ __forceinline__ void unpack_forward(const cpx<T>* buf, int p, int k, int n1, int ld,
                                               cpx<T>& A, cpx<T>& B) {
  const cpx<T> Z = buf[xaddr<PAD>(p, k, ld)];
  const cpx<T> Zm = buf[xaddr<PAD>(p, (n1 - k) % n1, ld)];
  A = mk(T(0.5) * (Z.x + Zm.x), T(0.5) * (Z.y - Zm.y));
  B = mk(T(0.5) * (Z.y + Zm.y), T(0.5) * (Zm.x - Z.x));
}

// Every transform kernel takes a compile-time length NF: NF > 0 selects the
// fixed-length path (constant tile shapes, lds_fft_c), NF = 0 the run-time
// path (tile shapes passed in, lds_fft).

template <typename T, int NF>
FFTG_KERNEL void k_x_r2c(Plan plan, const cpx<T>* __restrict__ tw, const T* __restrict__ in,
                         cpx<T>* __restrict__ out, long long S, int n1_rt, int n1h_rt, int P_rt) {
  constexpr bool FIX = NF > 0;
  __shared__ cpx<T> buf[FIX ? kElems<T> : LDS_ELEMS];
  const int n1 = FIX ? NF : n1_rt;
  const int n1h = FIX ? NF / 2 + 1 : n1h_rt;
  const int P = FIX ? fx_pairs<T>(NF) : P_rt;
  const long long s0 = (long long)blockIdx.x * (2 * P);
  for (int e = threadIdx.x; e < P * n1; e += FFT_THREADS) {
    const int p = e / n1, x = e % n1;
    const long long sa = s0 + p, sb = s0 + p + P;
    const T a = sa < S ? in[sa * n1 + x] : T(0);
    const T b = sb < S ? in[sb * n1 + x] : T(0);
    buf[p * n1 + x] = mk(a, b);
  }
  __syncthreads();
  if constexpr (FIX)
    lds_fft_c<T, true, false, NF, fx_pairs<T>(NF), NF>(buf, tw);
  else
    lds_fft<T, true, false>(buf, plan, P, n1, tw);
  for (int e = threadIdx.x; e < P * n1h; e += FFT_THREADS) {
    const int p = e / n1h, k = e % n1h;
    const long long sa = s0 + p, sb = s0 + p + P;
    cpx<T> A, B;
    unpack_forward<false>(buf, p, k, n1, n1, A, B);
    if (sa < S) out[sa * n1h + k] = A;
    if (sb < S) out[sb * n1h + k] = B;
  }
}

template <typename T, typename TO, int NF>
FFTG_KERNEL void k_x_c2r(Plan plan, const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ in,
                         TO* __restrict__ out, long long S, int n1_rt, int n1h_rt, int P_rt, T scl,
                         int acc) {
  constexpr bool FIX = NF > 0;
  __shared__ cpx<T> buf[FIX ? kElems<T> : LDS_ELEMS];
  const int n1 = FIX ? NF : n1_rt;
  const int n1h = FIX ? NF / 2 + 1 : n1h_rt;
  const int P = FIX ? fx_pairs<T>(NF) : P_rt;
  const long long s0 = (long long)blockIdx.x * (2 * P);
  for (int e = threadIdx.x; e < P * n1h; e += FFT_THREADS) {
    const int p = e / n1h, k = e % n1h;
    const long long sa = s0 + p, sb = s0 + p + P;
    const cpx<T> A = sa < S ? in[sa * n1h + k] : mk(T(0), T(0));
    const cpx<T> B = sb < S ? in[sb * n1h + k] : mk(T(0), T(0));
    pack_inverse<false>(buf, p, k, n1, n1, A, B);
  }
  __syncthreads();
  if constexpr (FIX)
    lds_fft_c<T, false, false, NF, fx_pairs<T>(NF), NF>(buf, tw);
  else
    lds_fft<T, false, false>(buf, plan, P, n1, tw);
  for (int e = threadIdx.x; e < P * n1; e += FFT_THREADS) {
    const int p = e / n1, x = e % n1;
    const long long sa = s0 + p, sb = s0 + p + P;
    const cpx<T> z = buf[p * n1 + x];
    if (sa < S) {
      TO v = (TO)(z.x * scl);
      out[sa * n1 + x] = acc ? (TO)(out[sa * n1 + x] + v) : v;
    }
    if (sb < S) {
      TO v = (TO)(z.y * scl);
      out[sb * n1 + x] = acc ? (TO)(out[sb * n1 + x] + v) : v;
    }
  }
}

// Fused x pass of the Galerkin operator: half spectrum -> real (C2R), then
// sigma = scale * K : eps per voxel with the compact tangent
// K:e = a tr(e) I + b dev(e) - (m.e) m, then real -> half spectrum (R2C).
// A workgroup owns NL whole x-lines with all C components; sequence
// s = comp * NL + line, and sequences s and s + P share one complex line.
//
// Stacked systems: spectra [sys][comp][Ns], tangent [sys][N][8]; a workgroup
// holds lines of one system only (system blockIdx.x / bps).
//
// partials (optional): the CG's p . A p, summed in real space.  The forward
// pass of the CG takes p in the range of the projection G* (an orthogonal
// projection, frequency by frequency), so p . G*(F(K:eps_p)) = p . F(K:eps_p),
// and by Parseval's identity that is the sum over voxels of eps_p : K : eps_p
// (the inverse transform here carries no 1/N, `scl` does): each workgroup
// writes the sum over its voxels to partials[blockIdx.x], [sys][bps].  The
// forward pass then need not read p.
template <typename T, typename TT, int NF, int C>
FFTG_KERNEL void k_x_fused_gal(Plan plan, const cpx<T>* __restrict__ tw, Geo g, int NL_rt,
                               cpx<T>* __restrict__ w_all, const TT* __restrict__ tan_all, T scl,
                               const KrylovCtl* __restrict__ ctl,
                               double* __restrict__ partials) {
  constexpr bool FIX = NF > 0;
  constexpr int NT = FIX ? kFusedThreads : FFT_THREADS;
  // fixed-length path: padded line pitch (conflict-free Stockham stages)
  constexpr int LDX = FIX ? padded_pitch(NF) : 1;
  __shared__ cpx<T> buf[FIX ? C * fx_fused_lines<T>(NF, C) / 2 * LDX : LDS_ELEMS];
  const long long nlines = (long long)g.n2 * g.n3;
  const int NL = FIX ? fx_fused_lines<T>(NF, C) : NL_rt;
  const long long bps = (nlines + NL - 1) / NL;
  const long long sys = blockIdx.x / bps;
  if (ctl && ctl[sys].done) return;
  cpx<T>* __restrict__ w = w_all + sys * C * g.Ns;
  const TT* __restrict__ tan = tan_all + sys * 8 * g.N;
  const long long line0 = (blockIdx.x % bps) * NL;
  const int n1 = FIX ? NF : g.n1, n1h = FIX ? NF / 2 + 1 : g.n1h;
  const int ld = FIX ? LDX : n1;
  const int P = C * NL / 2;
  for (int e = threadIdx.x; e < P * n1h; e += NT) {
    const int p = e / n1h, k = e % n1h;
    const int sa = p, sb = p + P;
    const long long la = line0 + sa % NL, lb = line0 + sb % NL;
    const cpx<T> A = la < nlines ? w[(sa / NL) * g.Ns + la * n1h + k] : mk(T(0), T(0));
    const cpx<T> B = lb < nlines ? w[(sb / NL) * g.Ns + lb * n1h + k] : mk(T(0), T(0));
    pack_inverse<FIX>(buf, p, k, n1, ld, A, B);
  }
  __syncthreads();
  if constexpr (FIX)
    lds_fft_c<T, false, false, NF, C * fx_fused_lines<T>(NF, C) / 2, LDX, NT, true>(buf,
                                                                                             tw);
  else
    lds_fft<T, false, false>(buf, plan, P, n1, tw);
  T* fb = reinterpret_cast<T*>(buf);
  double dot = 0.0;
  for (int e = threadIdx.x; e < NL * n1; e += NT) {
    const int l = e / n1, x = e % n1;
    const long long line = line0 + l;
    if (line >= nlines) continue;
    const long long v = line * n1 + x;
    int slot[C];
    T ev[C];
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int s = q * NL + l;
      slot[q] = s < P ? 2 * xaddr<FIX>(s, x, ld) : 2 * xaddr<FIX>(s - P, x, ld) + 1;
      ev[q] = fb[slot[q]];
    }
    const TT* tv = tan + 8 * v;  // [a, b, m0..m5] of the voxel, contiguous
    const T a = (T)tv[0], b = (T)tv[1];
    T m[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) m[i] = (T)tv[2 + i];
    T out[C];
    if constexpr (C == 6) {
      const T tr = ev[0] + ev[1] + ev[2];
      const T md = m[0] * ev[0] + m[1] * ev[1] + m[2] * ev[2] + m[3] * ev[3] + m[4] * ev[4] +
                   m[5] * ev[5];
      const T dv = tr / T(3);
#pragma unroll
      for (int i = 0; i < 3; ++i) out[i] = a * tr + b * (ev[i] - dv) - md * m[i];
#pragma unroll
      for (int i = 3; i < 6; ++i) out[i] = b * ev[i] - md * m[i];
    } else {
      const T tr = ev[0] + ev[1];
      const T md = m[0] * ev[0] + m[1] * ev[1] + m[5] * ev[2];
      const T dv = tr / T(3);
      out[0] = a * tr + b * (ev[0] - dv) - md * m[0];
      out[1] = a * tr + b * (ev[1] - dv) - md * m[1];
      out[2] = b * ev[2] - md * m[5];
    }
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const T o = out[q] * scl;
      fb[slot[q]] = o;
      dot += (double)ev[q] * (double)o;
    }
  }
  __syncthreads();
  if constexpr (FIX)
    lds_fft_c<T, true, false, NF, C * fx_fused_lines<T>(NF, C) / 2, LDX, NT, true>(buf,
                                                                                            tw);
  else
    lds_fft<T, true, false>(buf, plan, P, n1, tw);
  for (int e = threadIdx.x; e < P * n1h; e += NT) {
    const int p = e / n1h, k = e % n1h;
    const int sa = p, sb = p + P;
    const long long la = line0 + sa % NL, lb = line0 + sb % NL;
    cpx<T> A, B;
    unpack_forward<FIX>(buf, p, k, n1, ld, A, B);
    if (la < nlines) w[(sa / NL) * g.Ns + la * n1h + k] = A;
    if (lb < nlines) w[(sb / NL) * g.Ns + lb * n1h + k] = B;
  }
  if (partials) {
    // the tile is free once every wave is past the loop above (block_sum
    // starts with a barrier)
    static_assert(sizeof(buf) >= NT * sizeof(double), "reduction scratch aliases the tile");
    const double s = block_sum<NT>(dot, reinterpret_cast<double*>(buf));
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// Fused x pass of the Helmholtz operator: C2R of the ND gradient
// components, multiply by scale * ell^2(x), R2C.
// partials (optional): the PCG's sum over voxels of ell^2 |grad p|^2 (the
// gradient part of p . L p by Parseval's identity; the inverse transform
// carries no 1/N, `scale` does), one per workgroup, [sys][bps].
// Stacked systems: nsys x n2 x n3 lines per gradient component (component
// stride wstride), ell2 [sys][N].  With a phase array (shared by the
// systems: the fields of one RVE), ell^2 comes from the per-phase table
// ptab [sys][kMaxPhases] instead: 1 byte per voxel read instead of a
// real, and the same values as the field it would replace.
template <typename T, typename TL, int NF, int ND>
FFTG_KERNEL void k_x_fused_helm(Plan plan, const cpx<T>* __restrict__ tw, Geo g, int NL_rt,
                                cpx<T>* __restrict__ w, const TL* __restrict__ ell2, T scl,
                                int nsys, long long wstride, const KrylovCtl* __restrict__ ctl,
                                const unsigned char* __restrict__ phase,
                                const TL* __restrict__ ptab, double* __restrict__ partials) {
  constexpr bool FIX = NF > 0;
  constexpr int NT = FIX ? kFusedThreads : FFT_THREADS;
  constexpr int LDX = FIX ? padded_pitch(NF) : 1;
  __shared__ cpx<T> buf[FIX ? ND * fx_helm_lines<T>(NF, ND) / 2 * LDX : LDS_ELEMS];
  // A workgroup holds lines of one system only: two real lines share one
  // complex transform, which leaves rounding of the larger line's magnitude
  // in the smaller one, so lines of fields of very different size must never
  // be paired.
  const long long lpsys = (long long)g.n2 * g.n3;
  const int NL = FIX ? fx_helm_lines<T>(NF, ND) : NL_rt;
  const long long bps = (lpsys + NL - 1) / NL;  // workgroups per system
  const long long sys = blockIdx.x / bps;
  const long long line0 = sys * lpsys + (blockIdx.x % bps) * NL;
  const long long nlines = (sys + 1) * lpsys;   // end of this system's lines
  if (ctl && ctl[sys].done) return;
  const int n1 = FIX ? NF : g.n1, n1h = FIX ? NF / 2 + 1 : g.n1h;
  const int ld = FIX ? LDX : n1;
  const int P = ND * NL / 2;
  for (int e = threadIdx.x; e < P * n1h; e += NT) {
    const int p = e / n1h, k = e % n1h;
    const int sa = p, sb = p + P;
    const long long la = line0 + sa % NL, lb = line0 + sb % NL;
    const cpx<T> A = la < nlines ? w[(sa / NL) * wstride + la * n1h + k] : mk(T(0), T(0));
    const cpx<T> B = lb < nlines ? w[(sb / NL) * wstride + lb * n1h + k] : mk(T(0), T(0));
    pack_inverse<FIX>(buf, p, k, n1, ld, A, B);
  }
  __syncthreads();
  if constexpr (FIX)
    lds_fft_c<T, false, false, NF, ND * fx_helm_lines<T>(NF, ND) / 2, LDX, NT, true>(
        buf, tw);
  else
    lds_fft<T, false, false>(buf, plan, P, n1, tw);
  T* fb = reinterpret_cast<T*>(buf);
  double dot = 0.0;
  for (int e = threadIdx.x; e < NL * n1; e += NT) {
    const int l = e / n1, x = e % n1;
    const long long line = line0 + l;
    if (line >= nlines) continue;
    const TL e2 = phase ? ptab[sys * kMaxPhases + phase[(line - sys * lpsys) * n1 + x]]
                        : ell2[line * n1 + x];
    const T f = (T)e2 * scl;
#pragma unroll
    for (int q = 0; q < ND; ++q) {
      const int s = q * NL + l;
      const int slot = s < P ? 2 * xaddr<FIX>(s, x, ld) : 2 * xaddr<FIX>(s - P, x, ld) + 1;
      const T gq = fb[slot];
      const T o = gq * f;
      fb[slot] = o;
      dot += (double)gq * (double)o;
    }
  }
  __syncthreads();
  if constexpr (FIX)
    lds_fft_c<T, true, false, NF, ND * fx_helm_lines<T>(NF, ND) / 2, LDX, NT, true>(
        buf, tw);
  else
    lds_fft<T, true, false>(buf, plan, P, n1, tw);
  for (int e = threadIdx.x; e < P * n1h; e += NT) {
    const int p = e / n1h, k = e % n1h;
    const int sa = p, sb = p + P;
    const long long la = line0 + sa % NL, lb = line0 + sb % NL;
    cpx<T> A, B;
    unpack_forward<FIX>(buf, p, k, n1, ld, A, B);
    if (la < nlines) w[(sa / NL) * wstride + la * n1h + k] = A;
    if (lb < nlines) w[(sb / NL) * wstride + lb * n1h + k] = B;
  }
  if (partials) {
    // the tile is free once every wave is past the loop above (block_sum
    // starts with a barrier)
    static_assert(sizeof(buf) >= NT * sizeof(double), "reduction scratch aliases the tile");
    const double s = block_sum<NT>(dot, reinterpret_cast<double*>(buf));
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// ============================================================ strided passes
// Lines are numbered L = o * inner + i; line L starts at o * ostride + i and
// its elements are es apart.  A workgroup takes TL consecutive lines, so the
// loads of one row of the tile are contiguous within a slab.
__device__ __forceinline__ long long line_base(long long L, long long inner, long long ostride) {
  return (L / inner) * ostride + (L % inner);
}

// Workgroups go to the eight XCDs round-robin in launch order.  xcd_tile()
// renumbers them so that each XCD takes one contiguous run of tiles: the
// rows of the half spectrum (n1/2 + 1 points) are not cache-line aligned, so
// neighbouring tiles of a strided pass share lines at their edges, which are
// then fetched once into that XCD's L2 rather than once per XCD.  A bijection
// of [0, nb) for any nb.
__device__ __forceinline__ long long xcd_tile(long long b, long long nb) {
  const long long q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// Stacked systems that converge at different times: with one contiguous run
// per XCD, the tiles of a converged system would leave the XCDs that hold
// them idle while the others still work.  With chunk > 0 the XCDs take runs
// of `chunk` tiles in turn (XCD x the runs x, x + 8, x + 16, ...), so the
// tiles of every system spread over all eight XCDs, and neighbouring tiles
// still share an XCD within a run.  A bijection of [0, nb): the tail past
// the last whole round of 8 runs keeps its own order.
__device__ __forceinline__ long long xcd_tile(long long b, long long nb, int chunk) {
  if (chunk <= 0) return xcd_tile(b, nb);
  const long long span = 8LL * chunk, whole = nb / span * span;
  if (b >= whole) return b;
  const long long x = b & 7, i = b >> 3;
  return ((i / chunk) * 8 + x) * chunk + i % chunk;
}

// SH: tile budget code (chosen per handle by timing): FFTG_TILE_BYTES >> SH
// for SH = 0, 1, 2, twice FFTG_TILE_BYTES for SH = 3 (gfx950 workgroups may
// hold up to 160 KB of LDS).
template <int SH>
constexpr int tile_budget() { return SH == 3 ? 2 * FFTG_TILE_BYTES : FFTG_TILE_BYTES >> SH; }

// ctl (optional): the control blocks of the systems the lines belong to,
// lps lines each; a tile whose systems have all converged returns at once.
// chunk: the XCD run length of xcd_tile (0: one contiguous run per XCD).
template <typename T, bool FWD, int NF, int SH>
FFTG_KERNEL_WIDE void k_strided(Plan plan, const cpx<T>* __restrict__ tw, cpx<T>* __restrict__ data,
                           long long nlines, long long inner, long long ostride, long long es,
                           int TL_rt, const KrylovCtl* __restrict__ ctl, long long lps,
                           int chunk) {
  constexpr bool FIX = NF > 0;
  constexpr int TB = tile_budget<SH>();
  __shared__ cpx<T> buf[FIX ? fs_tile<T, TB>(NF) * NF : LDS_ELEMS];
  constexpr int NT = FIX ? kStridedThreads : FFT_THREADS;
  const int n = FIX ? NF : plan.n;
  const int TL = FIX ? fs_tile<T, TB>(NF) : TL_rt;
  const long long tile = xcd_tile(blockIdx.x, gridDim.x, chunk);
  if (ctl) {
    const long long last = (tile + 1) * TL - 1 < nlines ? (tile + 1) * TL - 1 : nlines - 1;
    bool live = false;
    for (long long sy = tile * TL / lps; sy <= last / lps; ++sy) live = live || !ctl[sy].done;
    if (!live) return;
  }
  // TL divides NT: each thread stays on line l of the tile
  const int l = threadIdx.x % TL, t0 = threadIdx.x / TL, dt = NT / TL;
  const long long L = tile * TL + l;
  const long long lb = L < nlines ? line_base(L, inner, ostride) : -1;
  if constexpr (FIX) {
    // first stage straight from global memory, last stage straight to it
    auto ld = [&](int t) { return lb >= 0 ? data[lb + t * es] : mk(T(0), T(0)); };
    auto st = [&](int t, cpx<T> v) {
      if (lb >= 0) data[lb + t * es] = v;
    };
    lds_fft_direct<T, FWD, NF, fs_tile<T, TB>(NF), NT>(buf, tw, ld, st);
  } else {
    for (int t = t0; t < n; t += dt)
      buf[t * TL + l] = lb >= 0 ? data[lb + t * es] : mk(T(0), T(0));
    __syncthreads();
    lds_fft<T, FWD, true>(buf, plan, TL, TL, tw);
    if (lb >= 0)
      for (int t = t0; t < n; t += dt) data[lb + t * es] = buf[t * TL + l];
  }
}

// Outer-axis inverse pass of the Galerkin CG (per component):
//   p <- r + beta p ; x <- x + alpha p_old ; w <- inverse transform of p.
//
// Stacked systems (several RVEs of one grid solved in lockstep): spectra
// [sys][comp][Ns]; the tiles of a (system, component) slab never reach into
// the next one (tpo tiles per slab), and system sys uses ctl[sys].
//
// rpart (folded scalars): the r.r partial sums of the previous iteration's
// residual pass, [sys][nbr].  Every workgroup sums them in the same fixed
// order and takes the same decisions (stop test, beta = r.r / r.r_old); the
// first workgroup of each system records them in slot `parity` of its
// control block.  Without rpart, alpha and beta come from the control block
// (the scalar kernels ran in between).
template <typename T, int NF, int SH>
FFTG_KERNEL_WIDE void k_gal_dir_inv(Plan plan, const cpx<T>* __restrict__ tw,
                               const cpx<T>* __restrict__ r, cpx<T>* __restrict__ pp,
                               cpx<T>* __restrict__ x, cpx<T>* __restrict__ w, long long inner,
                               long long ostride, long long es, int TL_rt, int tpo, int ncomp,
                               KrylovCtl* __restrict__ ctl_all, int parity,
                               const double* __restrict__ rpart, int nbr) {
  const long long o = blockIdx.x / tpo;  // (system, component) slab
  const int sys = (int)(o / ncomp);
  KrylovCtl* ctl = ctl_all + sys;
  // The first workgroup of the system may set done while this pass runs:
  // the whole workgroup acts on one reading of it, so that no wave leaves
  // while the others sum or update.
  __shared__ int s_done;
  if (threadIdx.x == 0) s_done = ctl->done;
  __syncthreads();
  if (s_done) return;
  constexpr bool FIX = NF > 0;
  constexpr int TB = tile_budget<SH>();
  __shared__ cpx<T> buf[FIX ? fs_tile<T, TB>(NF) * NF : LDS_ELEMS];
  constexpr int NT = FIX ? kStridedThreads : FFT_THREADS;
  static_assert(sizeof(buf) >= NT * sizeof(double), "reduction scratch aliases the tile");
  T alpha, beta;
  if (!rpart) {
    alpha = (T)ctl->alpha;
    beta = (T)ctl->beta;
  } else if (ctl->first) {
    alpha = T(0);
    beta = T(0);
  } else {
    const int q = parity ^ 1;  // slot of the previous iteration
    const double rz = ordered_sum_t<NT>(rpart + (long long)sys * nbr, nbr,
                                        reinterpret_cast<double*>(buf));
    __syncthreads();  // the tile below reuses the reduction scratch
    const int it = ctl->its[q] + 1;
    double rrmin = ctl->rrmins[q];
    int itmin = ctl->itmins[q];
    if (rz < rrmin) {
      rrmin = rz;
      itmin = it;
    }
    int done = 0;
    if (!isfinite(rz))
      done = 4;
    else if (rz <= ctl->tol2)
      done = 1;
    else if (it >= ctl->maxit)
      done = 2;
    else if (ctl->window > 0 && it - itmin >= ctl->window)
      done = 5;
    const double b = rz / ctl->rzs[q];
    if (blockIdx.x % (tpo * ncomp) == 0 && threadIdx.x == 0) {
      ctl->rzs[parity] = rz;
      ctl->its[parity] = it;
      ctl->rrmins[parity] = rrmin;
      ctl->itmins[parity] = itmin;
      ctl->iters = it;
      ctl->rz = rz;
      ctl->rr = rz;
      ctl->rrmin = rrmin;
      ctl->itmin = itmin;
      ctl->beta = b;
      if (done) ctl->done = done;
    }
    if (done) return;
    alpha = (T)ctl->alpha;  // step of the previous iteration (its residual pass)
    beta = (T)b;
  }
  const int n = FIX ? NF : plan.n;
  const int TL = FIX ? fs_tile<T, TB>(NF) : TL_rt;
  const int l = threadIdx.x % TL, t0 = threadIdx.x / TL, dt = NT / TL;
  const long long Lloc = (long long)(blockIdx.x % tpo) * TL + l;
  const long long lb = Lloc < inner ? line_base(o * inner + Lloc, inner, ostride) : -1;
  // the update of element t of the thread's line (each element once)
  auto upd = [&](int t) {
    cpx<T> pn = mk(T(0), T(0));
    if (lb >= 0) {
      const long long gi = lb + t * es;
      const cpx<T> po = pp[gi];
      x[gi] = x[gi] + scale(po, alpha);
      pn = r[gi] + scale(po, beta);
      pp[gi] = pn;
    }
    return pn;
  };
  if constexpr (FIX) {
    // last stage straight to w; FP32: first stage straight from the update
    // (FP64 keeps the update in its own sweep through LDS, which measures
    // faster at 96^3 and 128^3: all threads load, not only those of the
    // first stage's butterflies)
    auto st = [&](int t, cpx<T> v) {
      if (lb >= 0) w[lb + t * es] = v;
    };
    if constexpr (sizeof(T) == 4) {
      lds_fft_direct<T, false, NF, fs_tile<T, TB>(NF), NT>(buf, tw, upd, st);
    } else {
      for (int t = t0; t < n; t += dt) buf[t * TL + l] = upd(t);
      __syncthreads();
      lds_fft_direct<T, false, NF, fs_tile<T, TB>(NF), NT, decltype(upd), decltype(st), false,
                     true>(buf, tw, upd, st);
    }
  } else {
    for (int t = t0; t < n; t += dt) buf[t * TL + l] = upd(t);
    __syncthreads();
    lds_fft<T, false, true>(buf, plan, TL, TL, tw);
    if (lb >= 0)
      for (int t = t0; t < n; t += dt) w[lb + t * es] = buf[t * TL + l];
  }
}

// Outer-axis forward pass of the Galerkin CG: w <- forward transform of w,
// and the partial sums of the Hermitian-weighted p.w (= p.Ap, since p lies in
// the range of the orthogonal projector).
// Stacked systems as in k_gal_dir_inv; the partials of system sys are the
// ncomp * tpo entries from sys * ncomp * tpo.
template <typename T, int NF>
FFTG_KERNEL_WIDE void k_gal_dot_fwd(Plan plan, const cpx<T>* __restrict__ tw,
                               const cpx<T>* __restrict__ pp, cpx<T>* __restrict__ w,
                               long long inner, long long ostride, long long es, int TL_rt,
                               int tpo, int ncomp, int n1h, double* __restrict__ partials,
                               const KrylovCtl* __restrict__ ctl_all) {
  const long long o = blockIdx.x / tpo;
  const KrylovCtl* ctl = ctl_all + o / ncomp;
  if (ctl->done) return;
  constexpr bool FIX = NF > 0;
  __shared__ cpx<T> buf[FIX ? fs_tile<T, kDotBytes<T>>(NF) * NF : LDS_ELEMS];
  constexpr int NT = FIX ? kDotThreads<T> : FFT_THREADS;
  static_assert(sizeof(buf) >= NT * sizeof(double), "reduction scratch aliases the tile");
  double* red = reinterpret_cast<double*>(buf);  // reused after the transform (block_sum syncs)
  const int n = FIX ? NF : plan.n;
  const int TL = FIX ? fs_tile<T, kDotBytes<T>>(NF) : TL_rt;
  const int l = threadIdx.x % TL, t0 = threadIdx.x / TL, dt = NT / TL;
  const long long Lloc = (long long)(blockIdx.x % tpo) * TL + l;
  const long long lb = Lloc < inner ? line_base(o * inner + Lloc, inner, ostride) : -1;
  // every element of a line has the same kx (es is a multiple of n1h)
  const double wt = lb >= 0 ? hweight((int)(lb % n1h), n1h) : 0.0;
  double acc = 0.0;
  auto st = [&](int t, cpx<T> v) {
    if (lb >= 0) {
      const long long gi = lb + t * es;
      w[gi] = v;
      if (pp) {
        const cpx<T> pv = pp[gi];
        acc += wt * ((double)pv.x * (double)v.x + (double)pv.y * (double)v.y);
      }
    }
  };
  if constexpr (FIX) {
    // first stage straight from w, last stage straight back with the dot
    auto ld = [&](int t) { return lb >= 0 ? w[lb + t * es] : mk(T(0), T(0)); };
    lds_fft_direct<T, true, NF, fs_tile<T, kDotBytes<T>>(NF), NT>(buf, tw, ld, st);
  } else {
    for (int t = t0; t < n; t += dt) buf[t * TL + l] = lb >= 0 ? w[lb + t * es] : mk(T(0), T(0));
    __syncthreads();
    lds_fft<T, true, true>(buf, plan, TL, TL, tw);
    for (int t = t0; t < n; t += dt) st(t, buf[t * TL + l]);
  }
  if (pp) {
    const double s = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// Outer-axis inverse pass of the Helmholtz PCG (single scalar spectrum):
//   update: p <- M r + beta p ; x <- x + alpha p_old
//   w_j <- inverse transform of (i q~_j p), j < ND.
// ppart (optional, with update): weighted |p|^2 of the new p, one partial
// sum per workgroup [sys][tpo] (the identity part of p . L p).
// The fixed-length path uses a 48 KB tile so that tile rows stay >= 128 B.
//
// SPLIT (3D): the modified frequencies factor per axis, q_x = f_x c_y c_z,
// q_y = c_x f_y c_z, q_z = c_x c_y f_z, and on a z line only the z factors
// vary.  So the pass transforms two fields instead of three,
//   w_0 = Z^-1(i c_z p),  w_1 = Z^-1(i c_x c_y f_z p),
// and the y pass (k_h_y_split) forms the three gradient components from them.
//
// Several systems (one per non-local field, solved in lockstep) are stacked
// spectra [sys][Ns] with gradient fields [comp][sys][Ns] (component stride
// wstride); the tiles of a system never reach into the next one (tpo tiles per
// system), and each system has its own control block ctl[sys].
template <typename T, int NF, int ND, bool SPLIT>
FFTG_KERNEL_WIDE void k_h_dir_inv(Plan plan, const cpx<T>* __restrict__ tw, Geo g, Sym<T> sym,
                             int update, const cpx<T>* __restrict__ r, cpx<T>* __restrict__ pp,
                             cpx<T>* __restrict__ x, cpx<T>* __restrict__ w, long long inner,
                             long long ostride, long long es, int TL_rt, int tpo,
                             long long wstride, const KrylovCtl* __restrict__ ctl_all,
                             double* __restrict__ ppart) {
  const int sys = (int)(blockIdx.x / tpo);
  const KrylovCtl* ctl = ctl_all ? ctl_all + sys : nullptr;
  if (ctl && ctl->done) return;
  constexpr bool FIX = NF > 0;
  constexpr int NC = SPLIT ? 2 : ND;  // fields transformed
  __shared__ cpx<T> buf[FIX ? NC * fs_tile_wide<T>(NF, NC) * NF : LDS_ELEMS];
  double pp2 = 0.0;  // weighted |p|^2 of the new p (ppart)
  const int n = FIX ? NF : plan.n;
  constexpr int NT = FIX ? kWideThreads : FFT_THREADS;
  const int TL = FIX ? fs_tile_wide<T>(NF, NC) : TL_rt;
  const int ld = NC * TL;
  const int l = threadIdx.x % TL, t0 = threadIdx.x / TL, dt = NT / TL;
  const long long Lloc = (long long)(blockIdx.x % tpo) * TL + l;
  const long long L = (long long)sys * inner + Lloc;
  const long long lb = Lloc < inner ? line_base(L, inner, ostride) : -1;
  // lines are (ky, kx) in 3D (z outer) and kx in 2D (y outer)
  const bool zouter = g.ndim == 3;
  const int lkx = (int)(Lloc % g.n1h), lky = (int)(Lloc / g.n1h);
  const T alpha = ctl ? (T)ctl->alpha : T(0), beta = ctl ? (T)ctl->beta : T(0);
  const T l2 = ctl ? (T)ctl->ell2ref : T(0);
  for (int t = t0; t < n; t += dt) {
    cpx<T> pn = mk(T(0), T(0));
    T q[3] = {T(0), T(0), T(0)};
    if (lb >= 0) {
      const long long gi = lb + t * es;
      const int kx = lkx, ky = zouter ? lky : t, kz = zouter ? t : 0;
      qvec(sym, true, kx, ky, kz, q);
      if (update) {
        const T minv = T(1) / (T(1) + l2 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]));
        const cpx<T> po = pp[gi];
        x[gi] = x[gi] + scale(po, alpha);
        pn = scale(r[gi], minv) + scale(po, beta);
        pp[gi] = pn;
        pp2 += (double)pn.x * (double)pn.x + (double)pn.y * (double)pn.y;
      } else {
        pn = pp[gi];
      }
    }
    const cpx<T> ip = mul_i(pn);
    if constexpr (SPLIT) {
      T f0 = T(0), f1 = T(0);
      if (lb >= 0) {
        const T* b = sym.base;
        f0 = b[sym.cs[2] + t];
        f1 = b[sym.cs[0] + lkx] * b[sym.cs[1] + lky] * b[sym.gq[2] + t];
      }
      buf[t * ld + l] = scale(ip, f0);
      buf[t * ld + TL + l] = scale(ip, f1);
    } else {
#pragma unroll
      for (int j = 0; j < ND; ++j) buf[t * ld + j * TL + l] = scale(ip, q[j]);
    }
  }
  __syncthreads();
  constexpr int TLC = FIX ? fs_tile_wide<T>(NF, NC) : 1;
  if constexpr (FIX && NT % (NC * TLC) == 0) {
    // last stage straight to the NC fields (pseudo-line pl = field pl / TL,
    // line pl % TL of the tile)
    const int pl = threadIdx.x % (NC * TLC), jf = pl / TLC;
    const long long Lf = (long long)(blockIdx.x % tpo) * TLC + pl % TLC;
    const long long lbf = Lf < inner ? line_base((long long)sys * inner + Lf, inner, ostride) : -1;
    auto nold = [](int) { return mk(T(0), T(0)); };
    auto stf = [&](int t, cpx<T> v) {
      if (lbf >= 0) w[jf * wstride + lbf + t * es] = v;
    };
    lds_fft_direct<T, false, NF, NC * TLC, NT, decltype(nold), decltype(stf), false, true>(
        buf, tw, nold, stf);
  } else {
    if constexpr (FIX)
      lds_fft_c<T, false, true, NF, NC * fs_tile_wide<T>(NF, NC), NC * fs_tile_wide<T>(NF, NC),
                NT>(buf, tw);
    else
      lds_fft<T, false, true>(buf, plan, ld, ld, tw);
    if (lb >= 0)
      for (int t = t0; t < n; t += dt) {
        const long long gi = lb + t * es;
#pragma unroll
        for (int j = 0; j < NC; ++j) w[j * wstride + gi] = buf[t * ld + j * TL + l];
      }
  }
  if (ppart) {
    // every element of the thread's line has the same kx; the tile is free
    // once every wave is past the transform (block_sum starts with a barrier)
    static_assert(sizeof(buf) >= NT * sizeof(double), "reduction scratch aliases the tile");
    const double wt = lb >= 0 ? hweight(lkx, g.n1h) : 0.0;
    const double s = block_sum<NT>(wt * pp2, reinterpret_cast<double*>(buf));
    if (threadIdx.x == 0) ppart[blockIdx.x] = s;
  }
}

// y pass of the split Helmholtz operator (3D), lines (z, kx) of the
// half spectrum.  Inverse: from w_0, w_1 of k_h_dir_inv<SPLIT> forms and
// transforms the three gradient components
//   Y^-1(f_x c_y w_0), Y^-1(c_x f_y w_0), Y^-1(w_1)  -> w_0, w_1, w_2.
// Forward: transforms w_0, w_1, w_2 and folds the x and y components,
//   u = f_x c_y Y(w_0) + c_x f_y Y(w_1),  v = c_x c_y Y(w_2)  -> w_0, w_1,
// which the outer forward pass (k_h_div_fwd<SPLIT>) finishes with c_z, f_z.
// Stacked systems: lines (sys, z, kx) in order, gradient fields wstride apart;
// chunk as in k_strided.
template <typename T, bool FWD, int NF>
FFTG_KERNEL_WIDE void k_h_y_split(Plan plan, const cpx<T>* __restrict__ tw, Geo g, Sym<T> sym,
                                  cpx<T>* __restrict__ w, long long nlines, int TL_rt,
                                  long long wstride, const KrylovCtl* __restrict__ ctl,
                                  int chunk) {
  constexpr bool FIX = NF > 0;
  __shared__ cpx<T> buf[FIX ? 3 * fs_tile_wide<T>(NF, 3) * NF : LDS_ELEMS];
  const int n = FIX ? NF : plan.n;
  constexpr int NT = FIX ? kWideThreads : FFT_THREADS;
  const int TL = FIX ? fs_tile_wide<T>(NF, 3) : TL_rt;
  const int ld = 3 * TL;
  const int l = threadIdx.x % TL, t0 = threadIdx.x / TL, dt = NT / TL;
  const long long tile = xcd_tile(blockIdx.x, gridDim.x, chunk);
  if (ctl) {
    // skip a tile whose systems have all converged
    const long long lpsys = (long long)g.n3 * g.n1h;
    const long long last = (tile + 1) * TL - 1 < nlines ? (tile + 1) * TL - 1 : nlines - 1;
    bool live = false;
    for (long long sy = tile * TL / lpsys; sy <= last / lpsys; ++sy) live = live || !ctl[sy].done;
    if (!live) return;
  }
  const long long L = tile * TL + l;
  const long long inner = g.n1h, es = g.n1h;
  const long long lb = L < nlines ? line_base(L, inner, (long long)g.n2 * g.n1h) : -1;
  const int kx = (int)(L % inner);
  const T* b = sym.base;
  const T fx = lb >= 0 ? b[sym.gq[0] + kx] : T(0), cx = lb >= 0 ? b[sym.cs[0] + kx] : T(0);
  for (int t = t0; t < n; t += dt) {
    if (lb < 0) {
#pragma unroll
      for (int j = 0; j < 3; ++j) buf[t * ld + j * TL + l] = mk(T(0), T(0));
      continue;
    }
    const long long gi = lb + t * es;
    if constexpr (FWD) {
#pragma unroll
      for (int j = 0; j < 3; ++j) buf[t * ld + j * TL + l] = w[j * wstride + gi];
    } else {
      const cpx<T> a = w[gi], bb = w[wstride + gi];
      const T fy = b[sym.gq[1] + t], cy = b[sym.cs[1] + t];
      buf[t * ld + l] = scale(a, fx * cy);
      buf[t * ld + TL + l] = scale(a, cx * fy);
      buf[t * ld + 2 * TL + l] = bb;
    }
  }
  __syncthreads();
  if constexpr (FIX)
    lds_fft_c<T, FWD, true, NF, 3 * fs_tile_wide<T>(NF, 3), 3 * fs_tile_wide<T>(NF, 3), NT>(buf,
                                                                                            tw);
  else
    lds_fft<T, FWD, true>(buf, plan, ld, ld, tw);
  if (lb < 0) return;
  for (int t = t0; t < n; t += dt) {
    const long long gi = lb + t * es;
    if constexpr (FWD) {
      const T fy = b[sym.gq[1] + t], cy = b[sym.cs[1] + t];
      w[gi] = scale(buf[t * ld + l], fx * cy) + scale(buf[t * ld + TL + l], cx * fy);
      w[wstride + gi] = scale(buf[t * ld + 2 * TL + l], cx * cy);
    } else {
#pragma unroll
      for (int j = 0; j < 3; ++j) w[j * wstride + gi] = buf[t * ld + j * TL + l];
    }
  }
}

// Outer-axis forward pass of the Helmholtz operator:
//   Ap = p - i sum_j q~_j FFT(w_j) ; partial sums of weighted p.Ap.
// SPLIT (3D): w_0, w_1 are the u, v of k_h_y_split, and
// sum_j q_j FFT(w_j) = c_z Z(u) + f_z Z(v).
// Stacked systems as in k_h_dir_inv; partials of system sys are the tpo
// entries from sys * tpo.
template <typename T, int NF, int ND, bool SPLIT>
FFTG_KERNEL_WIDE void k_h_div_fwd(Plan plan, const cpx<T>* __restrict__ tw, Geo g, Sym<T> sym,
                             const cpx<T>* __restrict__ pp, cpx<T>* __restrict__ w,
                             cpx<T>* __restrict__ Ap, long long inner, long long ostride,
                             long long es, int TL_rt, int tpo, long long wstride,
                             double* __restrict__ partials, const KrylovCtl* __restrict__ ctl_all) {
  const int sys = (int)(blockIdx.x / tpo);
  const KrylovCtl* ctl = ctl_all ? ctl_all + sys : nullptr;
  if (ctl && ctl->done) return;
  constexpr bool FIX = NF > 0;
  constexpr int NC = SPLIT ? 2 : ND;  // fields transformed
  __shared__ cpx<T> buf[FIX ? NC * fs_tile_wide<T>(NF, NC) * NF : LDS_ELEMS];
  double* red = reinterpret_cast<double*>(buf);  // reused after the transform (block_sum syncs)
  const int n = FIX ? NF : plan.n;
  constexpr int NT = FIX ? kWideThreads : FFT_THREADS;
  static_assert(sizeof(buf) >= NT * sizeof(double), "reduction scratch aliases the tile");
  const int TL = FIX ? fs_tile_wide<T>(NF, NC) : TL_rt;
  const int ld = NC * TL;
  const int l = threadIdx.x % TL, t0 = threadIdx.x / TL, dt = NT / TL;
  const long long Lloc = (long long)(blockIdx.x % tpo) * TL + l;
  const long long L = (long long)sys * inner + Lloc;
  const long long lb = Lloc < inner ? line_base(L, inner, ostride) : -1;
  const bool zouter = g.ndim == 3;
  const int lkx = (int)(Lloc % g.n1h), lky = (int)(Lloc / g.n1h);
  constexpr int TLC = FIX ? fs_tile_wide<T>(NF, NC) : 1;
  if constexpr (FIX && NT % (NC * TLC) == 0) {
    // first stage straight from the NC fields: the thread's pseudo-line of
    // the tile is field pl / TL, line pl % TL
    const int pl = threadIdx.x % (NC * TLC), jf = pl / TLC;
    const long long Lf = (long long)(blockIdx.x % tpo) * TLC + pl % TLC;
    const long long lbf = Lf < inner ? line_base((long long)sys * inner + Lf, inner, ostride) : -1;
    auto ldf = [&](int t) { return lbf >= 0 ? w[jf * wstride + lbf + t * es] : mk(T(0), T(0)); };
    auto nost = [](int, cpx<T>) {};
    lds_fft_direct<T, true, NF, NC * TLC, NT, decltype(ldf), decltype(nost), true, false>(
        buf, tw, ldf, nost);
  } else {
    for (int t = t0; t < n; t += dt) {
      if (lb >= 0) {
        const long long gi = lb + t * es;
#pragma unroll
        for (int j = 0; j < NC; ++j) buf[t * ld + j * TL + l] = w[j * wstride + gi];
      } else {
#pragma unroll
        for (int j = 0; j < NC; ++j) buf[t * ld + j * TL + l] = mk(T(0), T(0));
      }
    }
    __syncthreads();
    if constexpr (FIX)
      lds_fft_c<T, true, true, NF, NC * fs_tile_wide<T>(NF, NC), NC * fs_tile_wide<T>(NF, NC),
                NT>(buf, tw);
    else
      lds_fft<T, true, true>(buf, plan, ld, ld, tw);
  }
  double acc = 0.0;
  for (int t = t0; t < n; t += dt) {
    if (lb >= 0) {
      const long long gi = lb + t * es;
      const int kx = lkx, ky = zouter ? lky : t, kz = zouter ? t : 0;
      const cpx<T> pv = pp[gi];
      cpx<T> div = mk(T(0), T(0));
      if constexpr (SPLIT) {
        const T* b = sym.base;
        div = scale(buf[t * ld + l], b[sym.cs[2] + kz]) +
              scale(buf[t * ld + TL + l], b[sym.gq[2] + kz]);
      } else {
        T q[3];
        qvec(sym, true, kx, ky, kz, q);
#pragma unroll
        for (int j = 0; j < ND; ++j) div = div + scale(buf[t * ld + j * TL + l], q[j]);
      }
      const cpx<T> a = pv + mul_mi(div);
      Ap[gi] = a;
      acc += hweight(kx, g.n1h) * ((double)pv.x * (double)a.x + (double)pv.y * (double)a.y);
    }
  }
  const double s = block_sum<NT>(acc, red);
  if (partials && threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Outer-axis forward pass of the Helmholtz PCG fused with the residual
// update, for the iteration whose p . L p the inverse pass (|p|^2) and the x
// pass (ell^2 |grad p|^2) summed (alpha is in the control block): the
// transform of k_h_div_fwd, then per coefficient
//   r <- r - alpha (p - i sum_j q~_j w_j),  partial sums of weighted r . M r
// and |r|^2 ([sys][2][tpo]), without storing L p.
template <typename T, int NF, int ND, bool SPLIT>
FFTG_KERNEL_WIDE void k_h_fwd_resid(Plan plan, const cpx<T>* __restrict__ tw, Geo g, Sym<T> sym,
                                    const cpx<T>* __restrict__ pp, cpx<T>* __restrict__ w,
                                    cpx<T>* __restrict__ r, long long inner, long long ostride,
                                    long long es, int TL_rt, int tpo, long long wstride,
                                    double* __restrict__ partials,
                                    const KrylovCtl* __restrict__ ctl_all) {
  const int sys = (int)(blockIdx.x / tpo);
  const KrylovCtl* ctl = ctl_all + sys;
  if (ctl->done) return;
  constexpr bool FIX = NF > 0;
  constexpr int NC = SPLIT ? 2 : ND;  // fields transformed
  __shared__ cpx<T> buf[FIX ? NC * fs_tile_wide<T>(NF, NC) * NF : LDS_ELEMS];
  double* red = reinterpret_cast<double*>(buf);  // reused after the transform (block_sum syncs)
  const int n = FIX ? NF : plan.n;
  constexpr int NT = FIX ? kWideThreads : FFT_THREADS;
  static_assert(sizeof(buf) >= NT * sizeof(double), "reduction scratch aliases the tile");
  const int TL = FIX ? fs_tile_wide<T>(NF, NC) : TL_rt;
  const int ld = NC * TL;
  const int l = threadIdx.x % TL, t0 = threadIdx.x / TL, dt = NT / TL;
  const long long Lloc = (long long)(blockIdx.x % tpo) * TL + l;
  const long long L = (long long)sys * inner + Lloc;
  const long long lb = Lloc < inner ? line_base(L, inner, ostride) : -1;
  const bool zouter = g.ndim == 3;
  const int lkx = (int)(Lloc % g.n1h), lky = (int)(Lloc / g.n1h);
  constexpr int TLC = FIX ? fs_tile_wide<T>(NF, NC) : 1;
  if constexpr (FIX && NT % (NC * TLC) == 0) {
    // first stage straight from the NC fields: the thread's pseudo-line of
    // the tile is field pl / TL, line pl % TL
    const int pl = threadIdx.x % (NC * TLC), jf = pl / TLC;
    const long long Lf = (long long)(blockIdx.x % tpo) * TLC + pl % TLC;
    const long long lbf = Lf < inner ? line_base((long long)sys * inner + Lf, inner, ostride) : -1;
    auto ldf = [&](int t) { return lbf >= 0 ? w[jf * wstride + lbf + t * es] : mk(T(0), T(0)); };
    auto nost = [](int, cpx<T>) {};
    lds_fft_direct<T, true, NF, NC * TLC, NT, decltype(ldf), decltype(nost), true, false>(
        buf, tw, ldf, nost);
  } else {
    for (int t = t0; t < n; t += dt) {
      if (lb >= 0) {
        const long long gi = lb + t * es;
#pragma unroll
        for (int j = 0; j < NC; ++j) buf[t * ld + j * TL + l] = w[j * wstride + gi];
      } else {
#pragma unroll
        for (int j = 0; j < NC; ++j) buf[t * ld + j * TL + l] = mk(T(0), T(0));
      }
    }
    __syncthreads();
    if constexpr (FIX)
      lds_fft_c<T, true, true, NF, NC * fs_tile_wide<T>(NF, NC), NC * fs_tile_wide<T>(NF, NC),
                NT>(buf, tw);
    else
      lds_fft<T, true, true>(buf, plan, ld, ld, tw);
  }
  const T alpha = (T)ctl->alpha;
  const T l2 = (T)ctl->ell2ref;
  double arz = 0.0, arr = 0.0;
  for (int t = t0; t < n; t += dt) {
    if (lb >= 0) {
      const long long gi = lb + t * es;
      const int kx = lkx, ky = zouter ? lky : t, kz = zouter ? t : 0;
      const cpx<T> pv = pp[gi];
      T q[3];
      qvec(sym, true, kx, ky, kz, q);
      cpx<T> div = mk(T(0), T(0));
      if constexpr (SPLIT) {
        const T* b = sym.base;
        div = scale(buf[t * ld + l], b[sym.cs[2] + kz]) +
              scale(buf[t * ld + TL + l], b[sym.gq[2] + kz]);
      } else {
#pragma unroll
        for (int j = 0; j < ND; ++j) div = div + scale(buf[t * ld + j * TL + l], q[j]);
      }
      const cpx<T> a = pv + mul_mi(div);
      const T minv = T(1) / (T(1) + l2 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]));
      const cpx<T> rn = r[gi] - scale(a, alpha);
      r[gi] = rn;
      const double wt = hweight(kx, g.n1h);
      const double rr = (double)rn.x * (double)rn.x + (double)rn.y * (double)rn.y;
      arr += wt * rr;
      arz += wt * rr * (double)minv;
    }
  }
  double* pt = partials + (long long)sys * 2 * tpo;
  const int loc = (int)(blockIdx.x % tpo);
  double sm = block_sum<NT>(arz, red);
  if (threadIdx.x == 0) pt[loc] = sm;
  sm = block_sum<NT>(arr, red);
  if (threadIdx.x == 0) pt[tpo + loc] = sm;
}

// ============================================================ pointwise
// r <- r - alpha G*(w) ; partial sums of weighted |r|^2
// Stacked systems: blockIdx.y is the system (spectra [sys][comp][Ns]), its
// partials at blockIdx.y * gridDim.x.
//
// dpart (folded scalars): the p.Ap partial sums of this iteration's forward
// pass, [sys][nbd]; every workgroup sums them in the same fixed order and
// forms alpha = r.r / p.Ap (r.r from slot `parity`), the first workgroup of
// each system records alpha (the step the next inverse pass, or the final
// update, applies to x).  Without dpart, alpha comes from the control block.
template <typename T, int C>
FFTG_KERNEL void k_gal_resid(Geo g, Sym<T> sym, unsigned char mk0, unsigned char mk1,
                             unsigned char mk2, unsigned char mk3, unsigned char mk4,
                             unsigned char mk5, cpx<T>* __restrict__ r_all,
                             const cpx<T>* __restrict__ w_all, double* __restrict__ partials,
                             KrylovCtl* __restrict__ ctl_all, int parity,
                             const double* __restrict__ dpart, int nbd) {
  KrylovCtl* ctl = ctl_all + blockIdx.y;
  // one reading of done per workgroup (the first workgroup may set it while
  // this pass runs)
  __shared__ int s_done;
  if (threadIdx.x == 0) s_done = ctl->done;
  __syncthreads();
  if (s_done) return;
  cpx<T>* __restrict__ r = r_all + (long long)blockIdx.y * C * g.Ns;
  const cpx<T>* __restrict__ w = w_all + (long long)blockIdx.y * C * g.Ns;
  __shared__ double red[FFT_THREADS];
  T alpha;
  if (dpart) {
    const double pAp = ordered_sum_t<FFT_THREADS>(dpart + (long long)blockIdx.y * nbd, nbd, red);
    const double rz = ctl->rzs[parity];
    int bad = 0;
    double a = 0.0;
    if (!isfinite(pAp) || !isfinite(rz))
      bad = 4;
    else if (!(pAp > 0.0))
      bad = 3;
    else
      a = rz / pAp;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctl->pAp = pAp;
      ctl->alpha = a;
      ctl->first = 0;
      if (bad) ctl->done = bad;
    }
    if (bad) return;
    alpha = (T)a;
  } else {
    alpha = (T)ctl->alpha;
  }
  const unsigned char mask[6] = {mk0, mk1, mk2, mk3, mk4, mk5};
  double acc = 0.0;
  for (long long gi = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; gi < g.Ns;
       gi += (long long)gridDim.x * FFT_THREADS) {
    int kx, ky, kz;
    decode(g, gi, kx, ky, kz);
    cpx<T> v[C];
    for (int i = 0; i < C; ++i) v[i] = w[i * g.Ns + gi];
    if (gi == 0) {
      for (int i = 0; i < C; ++i)
        if (!mask[i]) v[i] = mk(T(0), T(0));
    } else {
      T q[3];
      qvec(sym, false, kx, ky, kz, q);
      project_point<T, C>(q, v);
    }
    const double wt = hweight(kx, g.n1h);
    for (int i = 0; i < C; ++i) {
      const cpx<T> rn = r[i * g.Ns + gi] - scale(v[i], alpha);
      r[i * g.Ns + gi] = rn;
      acc += wt * ((double)rn.x * (double)rn.x + (double)rn.y * (double)rn.y);
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[(long long)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// Outer-axis forward pass of the Galerkin CG fused with the residual update,
// for the iteration whose p.Ap the x pass summed (alpha is in the control
// block): the C components of TL lines are transformed together in LDS, so
// that every frequency has all of them for the projection G* (its zero
// frequency: the mixed-control mask), and
//   r <- r - alpha G*(Z(w)),  partial sums of weighted |r|^2,
// without storing the transform.  Lines are (ky, kx) in 3D (z outer) and kx
// in 2D (y outer), inner per component.  Stacked systems: spectra
// [sys][comp][Ns], tpo tiles per system, partials [sys][tpo]; tiles are
// taken through xcd_tile (chunk).
template <typename T, int NF, int C>
__global__ __launch_bounds__(kFwdResThreads) void k_gal_fwd_resid(Plan plan, const cpx<T>* __restrict__ tw, Geo g,
                                      Sym<T> sym, unsigned mbits, const cpx<T>* __restrict__ w_all,
                                      cpx<T>* __restrict__ r_all, long long inner, long long es,
                                      int TL_rt, int tpo, int chunk,
                                      double* __restrict__ partials,
                                      const KrylovCtl* __restrict__ ctl_all) {
  constexpr bool FIX = NF > 0;
  constexpr int NT = FIX ? kFwdResThreads : FFT_THREADS;
  constexpr int TLF = FIX ? fr_tile<T>(NF, C) : 1;
  __shared__ cpx<T> buf[FIX ? C * TLF * NF : LDS_ELEMS];
  static_assert(sizeof(buf) >= NT * sizeof(double), "reduction scratch aliases the tile");
  const long long tile = xcd_tile(blockIdx.x, gridDim.x, chunk);
  const long long sys = tile / tpo;
  const KrylovCtl* ctl = ctl_all + sys;
  if (ctl->done) return;
  const int n = FIX ? NF : plan.n;
  const int TL = FIX ? TLF : TL_rt;
  const int ld = C * TL;
  const int l = threadIdx.x % TL, t0 = threadIdx.x / TL, dt = NT / TL;
  const long long L = (tile % tpo) * TL + l;  // line of a component slab
  const bool live = L < inner;
  const cpx<T>* __restrict__ w = w_all + sys * C * g.Ns;
  cpx<T>* __restrict__ r = r_all + sys * C * g.Ns;
  for (int t = t0; t < n; t += dt)
#pragma unroll
    for (int j = 0; j < C; ++j)
      buf[t * ld + j * TL + l] = live ? w[j * g.Ns + L + t * es] : mk(T(0), T(0));
  // FP64: the first point's residual loaded before the transform, so that
  // its loads overlap the transform (measured at 128^3: 77.5 -> 70.7 us; in
  // FP32 the same made the pass slower, 40.5 -> 50.7 us)
  constexpr int PF = FIX && sizeof(T) == 8 ? C : 0;
  cpx<T> rp[PF > 0 ? PF : 1];
  if constexpr (PF > 0) {
    if (live && t0 < n)
#pragma unroll
      for (int j = 0; j < PF; ++j) rp[j] = r[j * g.Ns + L + t0 * es];
  }
  __syncthreads();
  if constexpr (FIX)
    lds_fft_c<T, true, true, NF, C * TLF, C * TLF, NT>(buf, tw);
  else
    lds_fft<T, true, true>(buf, plan, ld, ld, tw);
  const T alpha = (T)ctl->alpha;
  const bool zouter = g.ndim == 3;
  const int kx = live ? (int)(L % g.n1h) : 0, lky = live ? (int)(L / g.n1h) : 0;
  const double wt = live ? hweight(kx, g.n1h) : 0.0;
  double acc = 0.0;
  if (live)
    for (int t = t0; t < n; t += dt) {
      const long long gi = L + t * es;
      cpx<T> v[C];
#pragma unroll
      for (int j = 0; j < C; ++j) v[j] = buf[t * ld + j * TL + l];
      if (gi == 0) {
#pragma unroll
        for (int j = 0; j < C; ++j)
          if (!((mbits >> j) & 1u)) v[j] = mk(T(0), T(0));
      } else {
        T q[3];
        qvec(sym, false, kx, zouter ? lky : t, zouter ? t : 0, q);
        project_point<T, C>(q, v);
      }
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const cpx<T> ro = (j < PF && t == t0) ? rp[j < PF ? j : 0] : r[j * g.Ns + gi];
        const cpx<T> rn = ro - scale(v[j], alpha);
        r[j * g.Ns + gi] = rn;
        acc += wt * ((double)rn.x * (double)rn.x + (double)rn.y * (double)rn.y);
      }
    }
  const double s = block_sum<NT>(acc, reinterpret_cast<double*>(buf));
  if (threadIdx.x == 0) partials[tile] = s;
}

// Newton right-hand side b = -G*(sigma - Sbar) from the FP64 stress spectrum;
// partials: [0] weighted |b|^2, [1] weighted |sigma_hat|^2.
// Stacked systems: blockIdx.y is the system; Sb_sys (when given) holds the
// mean stress targets [sys][6]; partials [sys][2][gridDim.x].
template <typename T, int C>
FFTG_KERNEL void k_gal_rhs(Geo g, Sym<double> sym, unsigned char mk0, unsigned char mk1,
                           unsigned char mk2, unsigned char mk3, unsigned char mk4,
                           unsigned char mk5, double s0, double s1, double s2, double s3,
                           double s4, double s5, const cpx<double>* __restrict__ sh_all,
                           cpx<T>* __restrict__ r_all, double* __restrict__ partials_all,
                           const double* __restrict__ Sb_sys) {
  __shared__ double red[FFT_THREADS];
  const unsigned char mask[6] = {mk0, mk1, mk2, mk3, mk4, mk5};
  const long long so = (long long)blockIdx.y * C * g.Ns;
  const cpx<double>* __restrict__ sh = sh_all + so;
  cpx<T>* __restrict__ r = r_all + so;
  double* partials = partials_all + (long long)blockIdx.y * 2 * gridDim.x;
  double Sb[6] = {s0, s1, s2, s3, s4, s5};
  if (Sb_sys)
    for (int i = 0; i < 6; ++i) Sb[i] = Sb_sys[6 * blockIdx.y + i];
  double accb = 0.0, accs = 0.0;
  for (long long gi = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; gi < g.Ns;
       gi += (long long)gridDim.x * FFT_THREADS) {
    int kx, ky, kz;
    decode(g, gi, kx, ky, kz);
    const double wt = hweight(kx, g.n1h);
    cpx<double> v[C];
    for (int i = 0; i < C; ++i) {
      v[i] = sh[i * g.Ns + gi];
      accs += wt * (v[i].x * v[i].x + v[i].y * v[i].y);
    }
    if (gi == 0) {
      for (int i = 0; i < C; ++i)
        v[i] = mask[i] ? mk(v[i].x - (double)g.N * Sb[i], v[i].y) : mk(0.0, 0.0);
    } else {
      double q[3];
      qvec(sym, false, kx, ky, kz, q);
      project_point<double, C>(q, v);
    }
    for (int i = 0; i < C; ++i) {
      const cpx<double> b = mk(-v[i].x, -v[i].y);
      r[i * g.Ns + gi] = mk((T)b.x, (T)b.y);
      accb += wt * (b.x * b.x + b.y * b.y);
    }
  }
  double s = block_sum(accb, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  s = block_sum(accs, red);
  if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = s;
}

// In-place projection of a c-component spectrum (zero frequency: mask).
template <typename T, int C>
FFTG_KERNEL void k_project(Geo g, Sym<T> sym, unsigned char mk0, unsigned char mk1,
                           unsigned char mk2, unsigned char mk3, unsigned char mk4,
                           unsigned char mk5, cpx<T>* __restrict__ d) {
  const unsigned char mask[6] = {mk0, mk1, mk2, mk3, mk4, mk5};
  for (long long gi = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; gi < g.Ns;
       gi += (long long)gridDim.x * FFT_THREADS) {
    int kx, ky, kz;
    decode(g, gi, kx, ky, kz);
    cpx<T> v[C];
    for (int i = 0; i < C; ++i) v[i] = d[i * g.Ns + gi];
    if (gi == 0) {
      for (int i = 0; i < C; ++i)
        if (!mask[i]) v[i] = mk(T(0), T(0));
    } else {
      T q[3];
      qvec(sym, false, kx, ky, kz, q);
      project_point<T, C>(q, v);
    }
    for (int i = 0; i < C; ++i) d[i * g.Ns + gi] = v[i];
  }
}

// Helmholtz residual update (init: r = b - Ap; else r -= alpha Ap), with
// partials [0] weighted r.Mr and [1] weighted r.r.
// Stacked systems: blockIdx.y is the system (spectra [sys][Ns]); its
// partials are [r.Mr | r.r] at sys * 2 * gridDim.x.
template <typename T>
FFTG_KERNEL void k_h_resid(Geo g, Sym<T> sym, int init, cpx<T>* __restrict__ r,
                           const cpx<T>* __restrict__ b, const cpx<T>* __restrict__ Ap,
                           double* __restrict__ partials, const KrylovCtl* __restrict__ ctl_all) {
  const KrylovCtl* ctl = ctl_all + blockIdx.y;
  if (!init && ctl->done) return;
  __shared__ double red[FFT_THREADS];
  const T alpha = init ? T(0) : (T)ctl->alpha;
  const T l2 = (T)ctl->ell2ref;
  const long long off = (long long)blockIdx.y * g.Ns;
  double arz = 0.0, arr = 0.0;
  for (long long gi = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; gi < g.Ns;
       gi += (long long)gridDim.x * FFT_THREADS) {
    int kx, ky, kz;
    decode(g, gi, kx, ky, kz);
    T q[3];
    qvec(sym, true, kx, ky, kz, q);
    const T minv = T(1) / (T(1) + l2 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]));
    const long long e = off + gi;
    const cpx<T> rn = init ? b[e] - Ap[e] : r[e] - scale(Ap[e], alpha);
    r[e] = rn;
    const double wt = hweight(kx, g.n1h);
    const double rr = (double)rn.x * (double)rn.x + (double)rn.y * (double)rn.y;
    arr += wt * rr;
    arz += wt * rr * (double)minv;
  }
  double* pt = partials + (long long)blockIdx.y * 2 * gridDim.x;
  double s = block_sum(arz, red);
  if (threadIdx.x == 0) pt[blockIdx.x] = s;
  s = block_sum(arr, red);
  if (threadIdx.x == 0) pt[gridDim.x + blockIdx.x] = s;
}

// Exact Hermitian symmetry on the planes kx = 0 and kx = n1/2, where both
// members of a conjugate pair (ky, kz) <-> (-ky, -kz) are stored: replace the
// pair by (a + conj b)/2 and its conjugate.  Rounding in the y/z transforms of
// real data leaves an anti-Hermitian part there that no real field carries and
// that the half-spectrum operator maps to zero.  One thread per pair: the
// member with the smaller flat (kz, ky) index writes both.
template <typename T>
FFTG_KERNEL void k_hermitize(Geo g, int ncomp, cpx<T>* __restrict__ d) {
  const long long plane = (long long)g.n2 * g.n3;
  const long long total = plane * 2 * ncomp;
  for (long long e = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; e < total;
       e += (long long)gridDim.x * FFT_THREADS) {
    const long long yz = e % plane;
    const int side = (int)((e / plane) % 2);
    const long long comp = e / (2 * plane);
    const int kx = side ? g.n1h - 1 : 0;
    const int ky = (int)(yz % g.n2), kz = (int)(yz / g.n2);
    const int my = (g.n2 - ky) % g.n2, mz = (g.n3 - kz) % g.n3;
    const long long myz = (long long)mz * g.n2 + my;
    if (myz < yz) continue;
    const long long ia = comp * g.Ns + yz * g.n1h + kx;
    const long long ib = comp * g.Ns + myz * g.n1h + kx;
    const cpx<T> a = d[ia], b = d[ib];
    const cpx<T> avg = mk(T(0.5) * (a.x + b.x), T(0.5) * (a.y - b.y));
    d[ia] = avg;
    d[ib] = mk(avg.x, -avg.y);
  }
}

// Deferred last update x <- x + alpha p.
// Stacked systems: n / nsys elements each, blockIdx.y the system.
template <typename T>
FFTG_KERNEL void k_xfinal(cpx<T>* __restrict__ x, const cpx<T>* __restrict__ p, long long n,
                          const KrylovCtl* __restrict__ ctl) {
  const T alpha = (T)ctl[blockIdx.y].alpha;
  if (alpha == T(0)) return;
  const long long off = (long long)blockIdx.y * n;
  for (long long i = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; i < n;
       i += (long long)gridDim.x * FFT_THREADS)
    x[off + i] = x[off + i] + scale(p[off + i], alpha);
}

// Weighted |a|^2 of ncomp spectra per system; blockIdx.y is the system, its
// partials at blockIdx.y * gridDim.x.
template <typename T>
FFTG_KERNEL void k_wnorm2(Geo g, int ncomp, const cpx<T>* __restrict__ a,
                          double* __restrict__ partials) {
  __shared__ double red[FFT_THREADS];
  double acc = 0.0;
  const long long n = g.Ns * ncomp;
  const cpx<T>* as = a + (long long)blockIdx.y * n;
  for (long long i = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; i < n;
       i += (long long)gridDim.x * FFT_THREADS) {
    const cpx<T> v = as[i];
    acc += hweight((int)(i % g.n1h), g.n1h) * ((double)v.x * (double)v.x + (double)v.y * (double)v.y);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[(long long)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// ============================================================ scalars
__device__ double ordered_sum(const double* __restrict__ p, int nb, double* red) {
  double acc = 0.0;
  // unrolled so that several loads are in flight; the additions keep their order
#pragma unroll 8
  for (int i = threadIdx.x; i < nb; i += FFT_THREADS) acc += p[i];
  return block_sum(acc, red);
}

// One workgroup per system: partials of system s from s * nb, ctl[s].
FFTG_KERNEL void k_fin_alpha(const double* __restrict__ partials, int nb, KrylovCtl* ctl_all) {
  KrylovCtl* ctl = ctl_all + blockIdx.x;
  if (ctl->done) return;
  __shared__ double red[FFT_THREADS];
  const double pAp = ordered_sum(partials + (long long)blockIdx.x * nb, nb, red);
  if (threadIdx.x == 0) {
    ctl->pAp = pAp;
    if (!isfinite(pAp) || !isfinite(ctl->rz)) {
      ctl->alpha = 0.0;
      ctl->done = 4;
    } else if (!(pAp > 0.0)) {
      ctl->alpha = 0.0;
      ctl->done = 3;
    } else {
      ctl->alpha = ctl->rz / pAp;
    }
  }
}

// p.Ap as the sum of two sets of partial sums (system s: pa + s * na and
// pb + s * nb); otherwise as k_fin_alpha.
FFTG_KERNEL void k_fin_alpha2(const double* __restrict__ pa, int na,
                              const double* __restrict__ pb, int nb, KrylovCtl* ctl_all) {
  KrylovCtl* ctl = ctl_all + blockIdx.x;
  if (ctl->done) return;
  __shared__ double red[FFT_THREADS];
  const double sa = ordered_sum(pa + (long long)blockIdx.x * na, na, red);
  const double sb = ordered_sum(pb + (long long)blockIdx.x * nb, nb, red);
  if (threadIdx.x == 0) {
    const double pAp = sa + sb;
    ctl->pAp = pAp;
    if (!isfinite(pAp) || !isfinite(ctl->rz)) {
      ctl->alpha = 0.0;
      ctl->done = 4;
    } else if (!(pAp > 0.0)) {
      ctl->alpha = 0.0;
      ctl->done = 3;
    } else {
      ctl->alpha = ctl->rz / pAp;
    }
  }
}

// nred = 1 (CG: partials = r.r) or 2 (PCG: partials = [r.Mr | r.r]).
FFTG_KERNEL void k_fin_beta(const double* __restrict__ partials, int nb, int nred,
                            KrylovCtl* ctl_all) {
  KrylovCtl* ctl = ctl_all + blockIdx.x;
  if (ctl->done) return;
  __shared__ double red[FFT_THREADS];
  const double* ps = partials + (long long)blockIdx.x * nred * nb;
  const double rz = ordered_sum(ps, nb, red);
  const double rr = nred == 2 ? ordered_sum(ps + nb, nb, red) : rz;
  if (threadIdx.x == 0) {
    ctl->iters += 1;
    ctl->beta = rz / ctl->rz;
    ctl->rz = rz;
    ctl->rr = rr;
    if (rr < ctl->rrmin) {
      ctl->rrmin = rr;
      ctl->itmin = ctl->iters;
    }
    if (!isfinite(rr) || !isfinite(rz))
      ctl->done = 4;
    else if (rr <= ctl->tol2)
      ctl->done = 1;
    else if (ctl->iters >= ctl->maxit)
      ctl->done = 2;
    else if (ctl->window > 0 && ctl->iters - ctl->itmin >= ctl->window)
      ctl->done = 5;
  }
}

FFTG_KERNEL void k_fin_sums(const double* __restrict__ partials, int nb, int nred,
                            double* __restrict__ out) {
  __shared__ double red[FFT_THREADS];
  for (int k = 0; k < nred; ++k) {
    const double s = ordered_sum(partials + (long long)k * nb, nb, red);
    if (threadIdx.x == 0) out[k] = s;
  }
}

// ============================================================ constitutive
// Principal values of a symmetric 3x3 tensor (Mandel input) by the closed-form
// trigonometric solution of the characteristic cubic (Smith 1961).
__device__ void principal3(const double e[6], double lam[3]) {
  const double r2 = 0.70710678118654752440084436210485;
  const double a11 = e[0], a22 = e[1], a33 = e[2];
  const double a23 = e[3] * r2, a13 = e[4] * r2, a12 = e[5] * r2;
  const double p1 = a12 * a12 + a13 * a13 + a23 * a23;
  const double qm = (a11 + a22 + a33) / 3.0;
  const double d1 = a11 - qm, d2 = a22 - qm, d3 = a33 - qm;
  const double p2 = d1 * d1 + d2 * d2 + d3 * d3 + 2.0 * p1;
  if (p2 <= 0.0) {
    lam[0] = lam[1] = lam[2] = qm;
    return;
  }
  const double p = sqrt(p2 / 6.0);
  const double ip = 1.0 / p;
  const double b11 = d1 * ip, b22 = d2 * ip, b33 = d3 * ip;
  const double b12 = a12 * ip, b13 = a13 * ip, b23 = a23 * ip;
  const double detb = b11 * (b22 * b33 - b23 * b23) - b12 * (b12 * b33 - b23 * b13) +
                      b13 * (b12 * b23 - b22 * b13);
  double rr = 0.5 * detb;
  rr = rr < -1.0 ? -1.0 : (rr > 1.0 ? 1.0 : rr);
  const double phi = acos(rr) / 3.0;
  lam[0] = qm + 2.0 * p * cos(phi);
  lam[2] = qm + 2.0 * p * cos(phi + 2.0943951023931954923084289221863);
  lam[1] = 3.0 * qm - lam[0] - lam[2];
}

// ============================================================ Gurson (GTN)
// Aravas hardening s0/sy = (s0/sy + 3 mu e0/sy)^n.  y = s0/sy is the root of
// y - (y + c e0)^n, c = 3 mu/sy; Newton from y = 1 + c e0, where that function
// is positive, increasing and convex, so the iterates fall monotonically onto
// the root.  Returns s0 and ds0/de0 (differentiating the law).
__device__ void gtn_flow(const Mat& m, double e0, double& s0, double& h) {
  const double ce = 3.0 * m.mu / m.sy * e0;
  // (1 + 2 ce)^n lies between the root and 1 + ce when n <= 1/2, so the
  // monotone descent starts much closer to the root
  double y = m.n <= 0.5 ? pow(1.0 + 2.0 * ce, m.n) : 1.0 + ce;
  for (int it = 0; it < 60; ++it) {
    const double z = y + ce;
    const double zn = pow(z, m.n);
    const double step = (y - zn) / (1.0 - m.n * zn / z);
    y -= step;
    if (fabs(step) <= 1e-15 * y) break;
  }
  const double zn1 = m.n * pow(y + ce, m.n - 1.0);
  s0 = m.sy * y;
  h = 3.0 * m.mu * zn1 / (1.0 - zn1);
}

// Effective porosity: f below fC, linear from fC to fV on [fC, fF), fV beyond;
// capped at fu.
__device__ double gtn_fstar(const Mat& m, double f) {
  const double fs =
      f < m.fC ? f : (f < m.fF ? m.fC + (m.fV - m.fC) / (m.fF - m.fC) * (f - m.fC) : m.fV);
  return fs < m.fu ? fs : m.fu;
}

// Yield function in the Mises stress q and the mean stress sm.
__device__ double gtn_phi(const Mat& m, double q, double sm, double s0, double fs) {
  const double r = q / s0;
  return r * r + 2.0 * m.q1 * fs * cosh(1.5 * m.q2 * sm / s0) - (1.0 + m.q3 * fs * fs);
}

// Porosity at the end of the increment from the non-local fields e (matrix
// plastic strain) and t (trace of the plastic strain) at n+1 and n: backward
// Euler of the non-local porosity rate, Chu-Needleman nucleation taken at the
// end-of-step e; clamped at 0.
__device__ double gtn_porosity(const Mat& m, double fn, double e, double en, double t,
                               double tn) {
  const double z = (e - m.eN) / m.sN;
  const double An = m.fN / (m.sN * 2.5066282746310002) * exp(-0.5 * z * z);
  const double dt = t - tn;
  const double f = (fn + An * (e - en) + dt) / (1.0 + dt);
  return f > 0.0 ? f : 0.0;
}

// Root of fun on the bracket [a, b] (fa fb <= 0): regula falsi with the
// Illinois modification (Dowell & Jarratt 1971), bisecting whenever the
// secant point leaves the bracket; stops at an exact zero or a bracket a few
// ulps wide.
template <typename F>
__device__ double bracket_root(F fun, double a, double b, double fa, double fb) {
  if (fb == 0.0) return b;
  if (fa == 0.0 || a == b) return a;
  bool kept_a = false;  // the previous step kept a (replaced b)
  for (int it = 0; it < 200; ++it) {
    const double den = fb - fa;
    double c = den != 0.0 ? b - fb * (b - a) / den : 0.5 * (a + b);
    if (!(c > fmin(a, b) && c < fmax(a, b))) c = 0.5 * (a + b);
    const double fc = fun(c);
    if (fc == 0.0) return c;
    if ((fc > 0.0) == (fb > 0.0)) {
      if (kept_a) fa *= 0.5;
      kept_a = true;
    } else {
      a = b;
      fa = fb;
      kept_a = false;
    }
    b = c;
    fb = fc;
    if (fabs(b - a) <= 8.881784197001252e-16 * fmax(fabs(b), 1e-300)) return b;
  }
  return b;
}

// Return onto the yield surface of flow stress s0 with fixed f*: the point
// (q(sm), sm) of the surface where the plastic strain increment
// u N + v I/3, u = (q_tr - q)/(3 mu), v = (sm_tr - sm)/K, is normal to it.
// Outside the surface the normality residual changes sign between sm = 0 and
// sm_tr (clamped to the apex |sm| = acosh((1 + q3 f*^2)/(2 q1 f*))/kap, where
// q = 0); a surface that contains the trial point returns it unchanged.
__device__ void gtn_project(const Mat& m, double q_tr, double sm_tr, double s0, double fs,
                            double& q, double& sm) {
  if (gtn_phi(m, q_tr, sm_tr, s0, fs) <= 0.0) {
    q = q_tr;
    sm = sm_tr;
    return;
  }
  const double kap = 1.5 * m.q2 / s0;
  const double b2 = 2.0 * m.q1 * fs, a1 = 1.0 + m.q3 * fs * fs;
  const double apex = b2 > 0.0 ? acosh(fmax(a1 / b2, 1.0)) / kap : INFINITY;
  const double K = m.K, mu3 = 3.0 * m.mu, is02 = 2.0 / (s0 * s0);
  auto qsurf = [=](double x) {
    const double g = a1 - b2 * cosh(kap * x);
    return g > 0.0 ? s0 * sqrt(g) : 0.0;
  };
  auto gfun = [=](double x) {
    const double qs = qsurf(x);
    return (q_tr - qs) / mu3 * b2 * kap * sinh(kap * x) - (sm_tr - x) / K * qs * is02;
  };
  const bool clamped = fabs(sm_tr) >= apex;
  const double end = clamped ? copysign(apex, sm_tr) : sm_tr;
  const double fend = clamped ? q_tr / mu3 * b2 * kap * sinh(kap * end) : gfun(end);
  sm = bracket_root(gfun, 0.0, end, gfun(0.0), fend);
  q = (clamped && sm == end) ? 0.0 : qsurf(sm);
}

// Local Gurson equations at x = (u, v, w) for a trial state (q_tr, sm_tr):
//   F1 = s0 (u dphi/dsm - v dphi/dq), F2 = phi, F3 = (1 - f) w - (q u + sm v)/s0
// with q = q_tr - 3 mu u, sm = sm_tr - K v, s0 = s0(e0_n + w); also
// J = dF/dx and R = -dF/d(q_tr, sm_tr).  Returns max(|F1|/xs, |F2|, |F3|/xs),
// xs the largest increment (F1 and F3 are strain-sized, F2 is O(1)).
__device__ double gtn_system(const Mat& m, double q_tr, double sm_tr, double e0n, double f,
                             double fs, double u, double v, double w, double F[3],
                             double J[3][3], double R[3][2], double& q, double& sm) {
  const double K = m.K, mu = m.mu, q1 = m.q1, q2 = m.q2;
  double s0, h;
  gtn_flow(m, e0n + w, s0, h);
  q = q_tr - 3.0 * mu * u;
  sm = sm_tr - K * v;
  const double t = 1.5 * q2 * sm / s0, tq = 1.5 * q2 / s0;
  const double sh = sinh(t), ch = cosh(t), A = 3.0 * q1 * q2 * fs;
  const double is0 = 1.0 / s0;
  F[0] = A * u * sh - 2.0 * v * q * is0;
  F[1] = q * q * is0 * is0 + 2.0 * q1 * fs * ch - (1.0 + m.q3 * fs * fs);
  F[2] = (1.0 - f) * w - (q * u + sm * v) * is0;
  // partial derivatives: in (u, v, w) held directly, then in q, sm, s0
  const double d[3][6] = {
      {A * sh, -2.0 * q * is0, 0.0, -2.0 * v * is0, A * u * ch * tq,
       -A * u * ch * t * is0 + 2.0 * v * q * is0 * is0},
      {0.0, 0.0, 0.0, 2.0 * q * is0 * is0, 2.0 * q1 * fs * sh * tq,
       -2.0 * q * q * is0 * is0 * is0 - 2.0 * q1 * fs * sh * t * is0},
      {-q * is0, -sm * is0, 1.0 - f, -u * is0, -v * is0, (q * u + sm * v) * is0 * is0}};
  for (int i = 0; i < 3; ++i) {
    J[i][0] = d[i][0] - 3.0 * mu * d[i][3];
    J[i][1] = d[i][1] - K * d[i][4];
    J[i][2] = d[i][2] + h * d[i][5];
    R[i][0] = -d[i][3];
    R[i][1] = -d[i][4];
  }
  const double xs = fmax(fmax(fabs(u), fabs(v)), fmax(fabs(w), 1e-12));
  return fmax(fmax(fabs(F[0]) / xs, fabs(F[1])), fabs(F[2]) / xs);
}

// Solve the 3x3 system J y = b by cofactors; false when J is singular.
__device__ bool solve3(const double J[3][3], const double b[3], double y[3]) {
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  if (!(det != 0.0) || !isfinite(det)) return false;
  const double id = 1.0 / det;
  const double inv[3][3] = {
      {c00, J[0][2] * J[2][1] - J[0][1] * J[2][2], J[0][1] * J[1][2] - J[0][2] * J[1][1]},
      {c01, J[0][0] * J[2][2] - J[0][2] * J[2][0], J[0][2] * J[1][0] - J[0][0] * J[1][2]},
      {c02, J[0][1] * J[2][0] - J[0][0] * J[2][1], J[0][0] * J[1][1] - J[0][1] * J[1][0]}};
  for (int r = 0; r < 3; ++r) y[r] = id * (inv[r][0] * b[0] + inv[r][1] * b[1] + inv[r][2] * b[2]);
  return true;
}

// Backward-Euler Gurson update at frozen porosity f for one voxel.  The
// plastic strain increment is u N + v I/3 (N = 3 s_tr/(2 q_tr)), the matrix
// plastic strain grows by w with (1 - f) s0(e0_n + w) w = q u + sm v (plastic
// work).
//
// Fast path: damped Newton on (F1, F2, F3) = 0 from the J2-like estimate,
// accepted only when it converges to an admissible point (u >= 0, w >= 0,
// q >= 0, v of the sign of sm, i.e. a non-negative plastic multiplier):
// the return is unique there, so that point is the solution.
// Fallback (any other case): nested bracketed roots.  For a given w the stress
// is the normal return onto the surface of s0(e0_n + w); the work residual is
// negative at w = 0 and non-negative at
// w_hi = (q u + sm v)|_{w=0} / ((1 - f) s0(e0_n)).
//
// The compact tangent [a, b, m] (K:e = a tr(e) I + b dev(e) - (m.e) m) is the
// consistent one from the linearised local equations in (q_tr, sm_tr): with
// A_q = du/dq_tr, B_q = du/dsm_tr, A_v = dv/dq_tr, B_v = dv/dsm_tr and
// theta = q/q_tr,
//   K_t = 2 mu theta I_dev + K (1 - K B_v) I(x)I
//         + 4 mu/3 (1 - 3 mu A_q - theta) N(x)N - mu K (A_v + B_q)(N(x)I + I(x)N)
// (symmetrised), written as a I(x)I + b I_dev - m(x)m with m = alpha N + beta I.
// Where the N(x)N coefficient is not negative (trial stress many times the
// flow stress), or the volumetric-deviatoric coupling would need an
// ill-conditioned beta, the tangent drops those terms: Newton then converges
// more slowly to the same solution.
__device__ void gtn_update(const Mat& m, const double e[6], double ep[6], double& e0,
                           double f, double s[6], double& ta, double& tb, double tm[6]) {
  const double K = m.K, mu = m.mu;
  double ee[6];
  for (int i = 0; i < 6; ++i) ee[i] = e[i] - ep[i];
  const double tr = ee[0] + ee[1] + ee[2];
  double st[6], ss = 0.0;
  for (int i = 0; i < 6; ++i) {
    st[i] = 2.0 * mu * (ee[i] - (i < 3 ? tr / 3.0 : 0.0));
    ss += st[i] * st[i];
  }
  const double q_tr = sqrt(1.5 * ss), sm_tr = K * tr;
  const double fs = gtn_fstar(m, f);
  double s0n, hn;
  gtn_flow(m, e0, s0n, hn);
  ta = K;
  tb = 2.0 * mu;
  for (int i = 0; i < 6; ++i) tm[i] = 0.0;
  if (!(gtn_phi(m, q_tr, sm_tr, s0n, fs) > 0.0)) {
    for (int i = 0; i < 6; ++i) s[i] = st[i] + (i < 3 ? sm_tr : 0.0);
    return;
  }
  const double e0n = e0, w1f = 1.0 - f;
  double F[3], J[3][3], R[3][2], q, sm;
  // ---- fast path
  double u = fmax(q_tr - s0n, 0.0) / (3.0 * mu + hn), v = 0.0, w = u / w1f;
  bool ok = false;
  double r = gtn_system(m, q_tr, sm_tr, e0n, f, fs, u, v, w, F, J, R, q, sm);
  for (int it = 0; it < 16 && !ok; ++it) {
    double dx[3];
    const double nb[3] = {-F[0], -F[1], -F[2]};
    if (!solve3(J, nb, dx)) break;
    double lam = 1.0, un = u, vn = v, wn = w, rn = r;
    double Fn[3], Jn[3][3], Rn[3][2], qn, smn;
    bool dec = false;
    for (int k = 0; k < 8; ++k) {
      un = fmin(fmax(u + lam * dx[0], 0.0), q_tr / (3.0 * mu));
      vn = v + lam * dx[1];
      wn = fmax(w + lam * dx[2], 0.0);
      rn = gtn_system(m, q_tr, sm_tr, e0n, f, fs, un, vn, wn, Fn, Jn, Rn, qn, smn);
      if (rn < r) {
        dec = true;
        break;
      }
      lam *= 0.5;
    }
    if (!dec) break;
    u = un;
    v = vn;
    w = wn;
    r = rn;
    q = qn;
    sm = smn;
    for (int i = 0; i < 3; ++i) {
      F[i] = Fn[i];
      R[i][0] = Rn[i][0];
      R[i][1] = Rn[i][1];
      for (int k = 0; k < 3; ++k) J[i][k] = Jn[i][k];
    }
    ok = r <= 1e-14;
  }
  // a plastic multiplier of the wrong sign shows as v opposite to sm (beyond
  // the rounding left in v when f* = 0 and the flow is deviatoric)
  ok = ok && u >= 0.0 && w >= 0.0 && q >= 0.0 &&
       !(v * sm < 0.0 && fabs(v) > 1e-12 * fmax(u, w));
  if (!ok) {
    // ---- fallback: nested bracketed roots
    auto work = [&](double ww) {
      double s0, h, qq, ss2;
      gtn_flow(m, e0n + ww, s0, h);
      gtn_project(m, q_tr, sm_tr, s0, fs, qq, ss2);
      return w1f * s0 * ww - (qq * (q_tr - qq) / (3.0 * mu) + ss2 * (sm_tr - ss2) / K);
    };
    const double f0 = work(0.0);
    const double whi = -f0 / (w1f * s0n);
    w = bracket_root(work, 0.0, whi, f0, work(whi));
    double s0, h;
    gtn_flow(m, e0n + w, s0, h);
    gtn_project(m, q_tr, sm_tr, s0, fs, q, sm);
    u = (q_tr - q) / (3.0 * mu);
    v = (sm_tr - sm) / K;
    gtn_system(m, q_tr, sm_tr, e0n, f, fs, u, v, w, F, J, R, q, sm);
  }
  double N[6];
  for (int i = 0; i < 6; ++i) N[i] = q_tr > 0.0 ? 1.5 * st[i] / q_tr : 0.0;
  for (int i = 0; i < 6; ++i) {
    ep[i] += u * N[i] + (i < 3 ? v / 3.0 : 0.0);
    s[i] = st[i] - 2.0 * mu * u * N[i] + (i < 3 ? sm : 0.0);
  }
  e0 = e0n + w;
  // tangent: X = J^-1 R, rows (u, v), columns (q_tr, sm_tr)
  double X[2][2];
  bool okj = true;
  for (int k = 0; k < 2; ++k) {
    const double b[3] = {R[0][k], R[1][k], R[2][k]};
    double y[3];
    okj = okj && solve3(J, b, y);
    X[0][k] = y[0];
    X[1][k] = y[1];
  }
  if (!okj) return;  // elastic tangent
  const double th = q_tr > 0.0 ? q / q_tr : 1.0;
  const double Avol = K * (1.0 - K * X[1][1]);
  const double Cnn = 4.0 * mu / 3.0 * (1.0 - 3.0 * mu * X[0][0] - th);
  const double Cni = -mu * K * (X[1][0] + X[0][1]);
  tb = 2.0 * mu * th;
  ta = Avol;
  if (Cnn < 0.0) {
    const double al = sqrt(-Cnn);
    double be = -Cni / al;
    if (!(be * be <= 1e3 * Avol)) be = 0.0;
    ta = Avol + be * be;
    for (int i = 0; i < 6; ++i) tm[i] = al * N[i] + (i < 3 ? be : 0.0);
  }
}

// Per voxel: backward-Euler J2 radial return on the effective stress with
// linear hardening, frozen damage, sigma = (1-D) sigma_eff, compact consistent
// tangent (1-D){K, 2 mu theta, 2 mu theta_bar, n} stored as
// [a, b, m0..m5] with K:e = a tr(e) I + b dev(e) - (m.e) m, m = sqrt(c) n;
// local sources per field.  Elastic phases: sigma = (1-D) C:e.  With GTN set,
// Gurson phases take gtn_update at the frozen porosity D[dfield] (no stress
// scaling) and feed fields dfield (matrix plastic strain) and dfield + 1
// (trace of the plastic strain).
template <typename TT, bool GTN>
FFTG_KERNEL void k_constitutive(MatTable tab, Geo g, int c, int J,
                                const unsigned char* __restrict__ phase,
                                const double* __restrict__ eps, const double* __restrict__ st_n,
                                const double* __restrict__ D, double* __restrict__ sigma,
                                double* __restrict__ st_np1, double* __restrict__ alpha,
                                TT* __restrict__ tan) {
  const long long N = g.N;
  const double sq32 = 1.2247448713915890490986420373529;  // sqrt(3/2)
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS) {
    const int ph = phase[v];
    const Mat m = tab.m[ph < tab.nphase ? ph : 0];
    double e[6];
    if (c == 6) {
      for (int i = 0; i < 6; ++i) e[i] = eps[i * N + v];
    } else {
      e[0] = eps[v];
      e[1] = eps[N + v];
      e[2] = 0.0;
      e[3] = 0.0;
      e[4] = 0.0;
      e[5] = eps[2 * N + v];
    }
    double ep[6];
    for (int i = 0; i < 6; ++i) ep[i] = st_n[i * N + v];
    double kap = st_n[6 * N + v];
    const double K = m.K, mu = m.mu;
    double s[6], tb = 2.0 * mu, tc = 0.0, nv[6] = {0, 0, 0, 0, 0, 0};
    double ta_g = 0.0, tm_g[6];
    const bool gtn = GTN && m.model == 3;
    if (gtn) {
      gtn_update(m, e, ep, kap, D[(long long)m.dfield * N + v], s, ta_g, tb, tm_g);
    } else if (m.model == 1) {
      double ee[6];
      for (int i = 0; i < 6; ++i) ee[i] = e[i] - ep[i];
      const double tr = ee[0] + ee[1] + ee[2];
      double dev[6];
      for (int i = 0; i < 6; ++i) dev[i] = 2.0 * mu * ee[i];
      for (int i = 0; i < 3; ++i) dev[i] -= 2.0 * mu * tr / 3.0;
      double ns2 = 0.0;
      for (int i = 0; i < 6; ++i) ns2 += dev[i] * dev[i];
      const double ns = sqrt(ns2);
      const double f = sq32 * ns - (m.sy + m.H * kap);
      if (f > 0.0) {
        const double dk = f / (3.0 * mu + m.H);
        for (int i = 0; i < 6; ++i) nv[i] = dev[i] / ns;
        const double gam = sq32 * dk;
        for (int i = 0; i < 6; ++i) {
          ep[i] += gam * nv[i];
          dev[i] -= 2.0 * mu * gam * nv[i];
        }
        kap += dk;
        const double theta = 1.0 - 2.0 * mu * gam / ns;
        const double thetab = 1.0 / (1.0 + m.H / (3.0 * mu)) - (1.0 - theta);
        tb = 2.0 * mu * theta;
        tc = 2.0 * mu * thetab;
      }
      for (int i = 0; i < 6; ++i) s[i] = dev[i];
      for (int i = 0; i < 3; ++i) s[i] += K * tr;
    } else {
      const double tr = e[0] + e[1] + e[2];
      for (int i = 0; i < 6; ++i) s[i] = 2.0 * mu * e[i];
      for (int i = 0; i < 3; ++i) s[i] += (K - 2.0 * mu / 3.0) * tr;
    }
    double dmg = 0.0;
    if (!gtn && m.model != 0 && m.dfield >= 0 && m.dfield < J)
      dmg = D[(long long)m.dfield * N + v];
    const double w1 = 1.0 - dmg;
    if (c == 6) {
      for (int i = 0; i < 6; ++i) sigma[i * N + v] = w1 * s[i];
    } else {
      sigma[v] = w1 * s[0];
      sigma[N + v] = w1 * s[1];
      sigma[2 * N + v] = w1 * s[5];
    }
    for (int i = 0; i < 6; ++i) st_np1[i * N + v] = ep[i];
    st_np1[6 * N + v] = kap;
    TT* tv = tan + 8 * v;  // [a, b, m0..m5] of the voxel, contiguous
    if (gtn) {
      tv[0] = (TT)ta_g;
      tv[1] = (TT)tb;
      for (int i = 0; i < 6; ++i) tv[2 + i] = (TT)tm_g[i];
    } else {
      tv[0] = (TT)(w1 * K);
      tv[1] = (TT)(w1 * tb);
      const double sc = sqrt(w1 * tc);
      for (int i = 0; i < 6; ++i) tv[2 + i] = (TT)(sc * nv[i]);
    }
    for (int j = 0; j < J; ++j) {
      double a = 0.0;
      if (gtn) {
        if (j == m.dfield) a = kap;
        else if (j == m.dfield + 1) a = ep[0] + ep[1] + ep[2];
      } else if (j == m.dfield) {
        if (m.model == 1) {
          a = kap;
        } else if (m.model == 2) {
          double lam[3];
          principal3(e, lam);
          double s2 = 0.0;
          for (int i = 0; i < 3; ++i)
            if (lam[i] > 0.0) s2 += lam[i] * lam[i];
          a = sqrt(s2);
        }
      }
      alpha[(long long)j * N + v] = a;
    }
  }
}

// D_j(x) from the non-local fields (damage laws of the phase models).  A
// Gurson phase takes the porosity f_{n+1} from the fields abar (n+1) and
// abar_n (n) of its two fields and the committed porosity hist[dfield].
FFTG_KERNEL void k_damage(MatTable tab, long long N, int J, const unsigned char* __restrict__ phase,
                          const double* __restrict__ abar, const double* __restrict__ hist,
                          const double* __restrict__ abar_n, double* __restrict__ D) {
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS) {
    const int ph = phase[v];
    const Mat m = tab.m[ph < tab.nphase ? ph : 0];
    for (int j = 0; j < J; ++j) {
      double d = 0.0;
      if (m.model == 3) {
        if (j == m.dfield) {
          const long long i0 = (long long)j * N + v, i1 = i0 + N;
          d = gtn_porosity(m, hist[i0], abar[i0], abar_n[i0], abar[i1], abar_n[i1]);
        }
      } else if (m.model != 0 && m.dfield == j) {
        double a = abar[(long long)j * N + v];
        if (m.model == 2) {
          const double hv = hist[(long long)j * N + v];
          a = hv > a ? hv : a;
        }
        d = (a - m.dC) / (m.dR - m.dC);
        d = d < 0.0 ? 0.0 : (d > m.dmax ? m.dmax : d);
      }
      D[(long long)j * N + v] = d;
    }
  }
}

// End of an increment: hist <- max(hist, abar) (cracking irreversibility),
// except the porosity slot of a Gurson phase, which takes f_{n+1} of the final
// fields (read before it is overwritten: the same element).
FFTG_KERNEL void k_commit_hist(MatTable tab, long long N, int J,
                               const unsigned char* __restrict__ phase,
                               const double* __restrict__ abar, const double* __restrict__ abar_n,
                               double* __restrict__ hist) {
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS) {
    const int ph = phase[v];
    const Mat m = tab.m[ph < tab.nphase ? ph : 0];
    for (int j = 0; j < J; ++j) {
      const long long i0 = (long long)j * N + v;
      if (m.model == 3 && j == m.dfield) {
        const long long i1 = i0 + N;
        hist[i0] = gtn_porosity(m, hist[i0], abar[i0], abar_n[i0], abar[i1], abar_n[i1]);
      } else {
        const double a = abar[i0];
        if (a > hist[i0]) hist[i0] = a;
      }
    }
  }
}

// Positive part <A>_+ of a symmetric 3x3 tensor (Mandel in and out) from its
// eigenvalues l0 >= l1 >= l2 and the eigenprojection of the eigenvalue group
// that is separated by the sign change:
//   one positive (l0 > 0 >= l1):  <A>_+ = l0 (A - l1 I)(A - l2 I) / ((l0 - l1)(l0 - l2))
//   two positive (l1 > 0 >= l2):  <A>_+ = A - l2 (A - l0 I)(A - l1 I) / ((l2 - l0)(l2 - l1))
// The denominators are bounded below by l0^2 and l0 l1, so no gap between
// eigenvalues of the same sign enters.
__device__ void positive_part(const double e[6], const double lam[3], double out[6]) {
  const double r2 = 1.4142135623730950488016887242097, ir2 = 0.70710678118654752440084436210485;
  if (lam[2] >= 0.0) {
    for (int i = 0; i < 6; ++i) out[i] = e[i];
    return;
  }
  if (lam[0] <= 0.0) {
    for (int i = 0; i < 6; ++i) out[i] = 0.0;
    return;
  }
  const double A[3][3] = {{e[0], e[5] * ir2, e[4] * ir2},
                          {e[5] * ir2, e[1], e[3] * ir2},
                          {e[4] * ir2, e[3] * ir2, e[2]}};
  const bool one = !(lam[1] > 0.0);
  // product (A - a I)(A - b I) with the two other eigenvalues
  const double a = one ? lam[1] : lam[0], b = one ? lam[2] : lam[1];
  const double lk = one ? lam[0] : lam[2];
  double M[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double sum = 0.0;
      for (int k = 0; k < 3; ++k)
        sum += (A[i][k] - (i == k ? a : 0.0)) * (A[k][j] - (k == j ? b : 0.0));
      M[i][j] = sum;
    }
  const double f = lk / ((lk - a) * (lk - b));
  double P[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[i][j] = one ? f * M[i][j] : A[i][j] - f * M[i][j];
  out[0] = P[0][0];
  out[1] = P[1][1];
  out[2] = P[2][2];
  out[3] = r2 * 0.5 * (P[1][2] + P[2][1]);
  out[4] = r2 * 0.5 * (P[0][2] + P[2][0]);
  out[5] = r2 * 0.5 * (P[0][1] + P[1][0]);
}

// Transposed source derivative: out = sum_j lam_j (d alpha_j / d eps) at the
// converged strain, [c][N].  For a J2 damage phase driven by field j the
// source is kappa_n + dk with dk = (sqrt(3/2) ||s_tr|| - sy - H kappa_n)/(3 mu + H)
// where plastic, so d alpha_j / d eps = sqrt(3/2) 2 mu s_tr / ((3 mu + H) ||s_tr||)
// (0 where elastic).  For a cracking phase the source is the Mazars
// equivalent strain alpha = ||<eps>_+||, with gradient <eps>_+ / alpha (0 where
// alpha = 0).  Other phases contribute nothing.
FFTG_KERNEL void k_source_adj(MatTable tab, long long N, int c, int J,
                              const unsigned char* __restrict__ phase,
                              const double* __restrict__ eps, const double* __restrict__ st_n,
                              const double* __restrict__ lam, double* __restrict__ out) {
  const double sq32 = 1.2247448713915890490986420373529;
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS) {
    const int ph = phase[v];
    const Mat m = tab.m[ph < tab.nphase ? ph : 0];
    double o[6] = {0, 0, 0, 0, 0, 0};
    if (m.model == 2 && m.dfield >= 0 && m.dfield < J) {
      double e[6];
      if (c == 6) {
        for (int i = 0; i < 6; ++i) e[i] = eps[i * N + v];
      } else {
        e[0] = eps[v];
        e[1] = eps[N + v];
        e[2] = e[3] = e[4] = 0.0;
        e[5] = eps[2 * N + v];
      }
      double lam3[3], pp[6];
      principal3(e, lam3);
      double s2 = 0.0;
      for (int i = 0; i < 3; ++i)
        if (lam3[i] > 0.0) s2 += lam3[i] * lam3[i];
      if (s2 > 0.0) {
        positive_part(e, lam3, pp);
        const double gf = lam[(long long)m.dfield * N + v] / sqrt(s2);
        for (int i = 0; i < 6; ++i) o[i] = gf * pp[i];
      }
    } else if (m.model == 1 && m.dfield >= 0 && m.dfield < J) {
      double ee[6];
      if (c == 6) {
        for (int i = 0; i < 6; ++i) ee[i] = eps[i * N + v];
      } else {
        ee[0] = eps[v];
        ee[1] = eps[N + v];
        ee[2] = ee[3] = ee[4] = 0.0;
        ee[5] = eps[2 * N + v];
      }
      for (int i = 0; i < 6; ++i) ee[i] -= st_n[i * N + v];
      const double tr = ee[0] + ee[1] + ee[2];
      double sd[6], ns2 = 0.0;
      for (int i = 0; i < 6; ++i) {
        sd[i] = 2.0 * m.mu * (ee[i] - (i < 3 ? tr / 3.0 : 0.0));
        ns2 += sd[i] * sd[i];
      }
      const double ns = sqrt(ns2);
      if (sq32 * ns - (m.sy + m.H * st_n[6 * N + v]) > 0.0) {
        const double gf = lam[(long long)m.dfield * N + v] * sq32 * 2.0 * m.mu /
                          ((3.0 * m.mu + m.H) * ns);
        for (int i = 0; i < 6; ++i) o[i] = gf * sd[i];
      }
    }
    if (c == 6) {
      for (int i = 0; i < 6; ++i) out[i * N + v] = o[i];
    } else {
      out[v] = o[0];
      out[N + v] = o[1];
      out[2 * N + v] = o[5];
    }
  }
}

// Streaming copy of n16 16-byte words (the HBM reference rate): one 16-byte
// load and store per lane per step, grid-stride over the buffer.
FFTG_KERNEL void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                               long long n16) {
  for (long long i = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; i < n16;
       i += (long long)gridDim.x * FFT_THREADS)
    dst[i] = src[i];
}

// J2 return of one voxel (linear hardening) re-evaluated at the converged
// strain for the history adjoint: unit deviatoric trial direction n, plastic
// flag, and the scalars of the derivatives
//   d kappa/d eps = gk n,  d eps_p/d eps = a n(x)n + b (I_dev - n(x)n),
//   d kappa/d kappa_n = kk,  d eps_p/d kappa_n = pk n,  d sigma_eff/d kappa_n = sk n,
//   C_eff = K I(x)I + 2 mu theta I_dev - 2 mu theta_bar n(x)n.
struct HistJ2 {
  double n[6];
  bool plastic;
  double gk, a, b, kk, pk, sk, th, thb;
};

__device__ HistJ2 hist_j2(const Mat& m, const double e[6], const double* st_n, long long N,
                          long long v) {
  const double sq32 = 1.2247448713915890490986420373529;
  HistJ2 r{};
  double ee[6];
  for (int i = 0; i < 6; ++i) ee[i] = e[i] - st_n[i * N + v];
  const double tr = ee[0] + ee[1] + ee[2];
  double ns2 = 0.0;
  for (int i = 0; i < 6; ++i) {
    r.n[i] = 2.0 * m.mu * (ee[i] - (i < 3 ? tr / 3.0 : 0.0));
    ns2 += r.n[i] * r.n[i];
  }
  const double ns = sqrt(ns2);
  const double f = sq32 * ns - (m.sy + m.H * st_n[6 * N + v]);
  r.plastic = f > 0.0;
  r.kk = 1.0;
  r.th = 1.0;
  if (!r.plastic) return r;
  for (int i = 0; i < 6; ++i) r.n[i] /= ns;
  const double h3 = 3.0 * m.mu + m.H;
  const double dk = f / h3;
  r.gk = sq32 * 2.0 * m.mu / h3;
  r.a = 3.0 * m.mu / h3;
  r.b = sq32 * dk * 2.0 * m.mu / ns;
  r.kk = r.a;
  r.pk = -sq32 * m.H / h3;
  r.sk = 2.0 * m.mu * sq32 * m.H / h3;
  r.th = 1.0 - 2.0 * m.mu * sq32 * dk / ns;
  r.thb = 1.0 / (1.0 + m.H / (3.0 * m.mu)) - (1.0 - r.th);
  return r;
}

__device__ inline void load_strain6(const double* eps, int c, long long N, long long v,
                                    double e[6]) {
  if (c == 6) {
    for (int i = 0; i < 6; ++i) e[i] = eps[i * N + v];
  } else {
    e[0] = eps[v];
    e[1] = eps[N + v];
    e[2] = e[3] = e[4] = 0.0;
    e[5] = eps[2 * N + v];
  }
}

// (a n(x)n + b (I_dev - n(x)n)) g for a deviatoric unit n
__device__ inline void dep_apply(const HistJ2& h, const double g[6], double out[6]) {
  double ng = 0.0;
  for (int i = 0; i < 6; ++i) ng += h.n[i] * g[i];
  const double tg = (g[0] + g[1] + g[2]) / 3.0;
  for (int i = 0; i < 6; ++i)
    out[i] = h.a * ng * h.n[i] + h.b * (g[i] - (i < 3 ? tg : 0.0) - ng * h.n[i]);
}

// Strain cotangent from the cotangents of the committed plastic state of the
// J2 voxels: g_eps = (d eps_p/d eps)^T g_epsp + (d kappa/d eps) g_kappa
// (0 elsewhere).  g_epsp [6][N], g_kappa [N] may be null.
FFTG_KERNEL void k_hist_out_cot(MatTable tab, long long N, int c,
                                const unsigned char* __restrict__ phase,
                                const double* __restrict__ eps, const double* __restrict__ st_n,
                                const double* __restrict__ g_epsp,
                                const double* __restrict__ g_kappa, double* __restrict__ g_eps) {
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS) {
    const int ph = phase[v];
    const Mat m = tab.m[ph < tab.nphase ? ph : 0];
    double o[6] = {0, 0, 0, 0, 0, 0};
    if (m.model == 1) {
      double e[6];
      load_strain6(eps, c, N, v, e);
      const HistJ2 h = hist_j2(m, e, st_n, N, v);
      if (h.plastic) {
        if (g_epsp) {
          double g[6];
          for (int i = 0; i < 6; ++i) g[i] = g_epsp[i * N + v];
          dep_apply(h, g, o);
        }
        if (g_kappa)
          for (int i = 0; i < 6; ++i) o[i] += h.gk * h.n[i] * g_kappa[v];
      }
    }
    if (c == 6) {
      for (int i = 0; i < 6; ++i) g_eps[i * N + v] = o[i];
    } else {
      g_eps[v] = o[0];
      g_eps[N + v] = o[1];
      g_eps[2 * N + v] = o[5];
    }
  }
}

// Cotangents of the plastic history an increment started from, at its
// converged state: with w = mu - g_sig (mu the total mechanics adjoint) and
// lam the Helmholtz adjoint of the voxel's field,
//   g_epsp_n  = (1 - D) C_eff w - lam d kappa/d eps + g_epsp - (d eps_p/d eps)^T g_epsp
//               - (d kappa/d eps) g_kappa
//   g_kappa_n = -(1 - D) (d sigma_eff/d kappa_n) . w + lam d kappa/d kappa_n
//               + (d eps_p/d kappa_n) . g_epsp + (d kappa/d kappa_n) g_kappa
// on J2 damage voxels; other phases pass g_epsp, g_kappa through (their stress
// acts on the total strain).
FFTG_KERNEL void k_hist_in_cot(MatTable tab, long long N, int c, int J,
                               const unsigned char* __restrict__ phase,
                               const double* __restrict__ eps, const double* __restrict__ st_n,
                               const double* __restrict__ D, const double* __restrict__ mu,
                               const double* __restrict__ g_sig, const double* __restrict__ lam,
                               const double* __restrict__ g_epsp,
                               const double* __restrict__ g_kappa,
                               double* __restrict__ g_epsp_n, double* __restrict__ g_kappa_n) {
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS) {
    const int ph = phase[v];
    const Mat m = tab.m[ph < tab.nphase ? ph : 0];
    double gp[6], gpo[6];
    for (int i = 0; i < 6; ++i) gp[i] = g_epsp ? g_epsp[i * N + v] : 0.0;
    const double gkap = g_kappa ? g_kappa[v] : 0.0;
    for (int i = 0; i < 6; ++i) gpo[i] = gp[i];
    double gko = gkap;
    if (m.model == 1) {
      double e[6];
      load_strain6(eps, c, N, v, e);
      const HistJ2 h = hist_j2(m, e, st_n, N, v);
      double w[6] = {0, 0, 0, 0, 0, 0};
      const int idx[6] = {0, 1, 5, 2, 3, 4};
      for (int k = 0; k < c; ++k) {
        const int i = c == 6 ? k : idx[k];
        w[i] = mu[(long long)k * N + v] - (g_sig ? g_sig[(long long)k * N + v] : 0.0);
      }
      const bool fld = m.dfield >= 0 && m.dfield < J;
      const double w1 = fld ? 1.0 - D[(long long)m.dfield * N + v] : 1.0;
      const double lv = fld ? lam[(long long)m.dfield * N + v] : 0.0;
      // C_eff w
      const double trw = w[0] + w[1] + w[2];
      double nw = 0.0;
      for (int i = 0; i < 6; ++i) nw += h.n[i] * w[i];
      double cw[6];
      for (int i = 0; i < 6; ++i)
        cw[i] = (i < 3 ? m.K * trw : 0.0) + 2.0 * m.mu * h.th * (w[i] - (i < 3 ? trw / 3.0 : 0.0)) -
                2.0 * m.mu * h.thb * nw * h.n[i];
      double dg[6] = {0, 0, 0, 0, 0, 0};
      if (h.plastic) dep_apply(h, gp, dg);
      double ngp = 0.0;
      for (int i = 0; i < 6; ++i) ngp += h.n[i] * gp[i];
      for (int i = 0; i < 6; ++i)
        gpo[i] = w1 * cw[i] - lv * h.gk * h.n[i] + gp[i] - dg[i] - h.gk * h.n[i] * gkap;
      gko = -w1 * h.sk * nw + lv * h.kk + h.pk * ngp + h.kk * gkap;
    }
    for (int i = 0; i < 6; ++i) g_epsp_n[i * N + v] = gpo[i];
    g_kappa_n[v] = gko;
  }
}

// partials [0][block] = sum (a - b)^2, [1][block] = sum a^2
FFTG_KERNEL void k_diff2(long long n, const double* __restrict__ a, const double* __restrict__ b,
                         double* __restrict__ partials) {
  __shared__ double red[FFT_THREADS];
  double d2 = 0.0, a2 = 0.0;
  for (long long i = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; i < n;
       i += (long long)gridDim.x * FFT_THREADS) {
    const double d = a[i] - b[i];
    d2 += d * d;
    a2 += a[i] * a[i];
  }
  double s = block_sum(d2, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  s = block_sum(a2, red);
  if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = s;
}

FFTG_KERNEL void k_axpby(long long n, double a, const double* __restrict__ x, double b,
                         const double* __restrict__ y, double* __restrict__ out) {
  for (long long i = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; i < n;
       i += (long long)gridDim.x * FFT_THREADS)
    out[i] = a * x[i] + b * y[i];
}

template <typename TL>
FFTG_KERNEL void k_ell2(MatTable tab, long long N, int j, const unsigned char* __restrict__ phase,
                        TL* __restrict__ ell2) {
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS) {
    const int ph = phase[v];
    ell2[v] = (TL)tab.m[ph < tab.nphase ? ph : 0].ell2[j];
  }
}

// Adjoint of k_damage: gabar_j(x) = gD_j(x) dD_j/dabar_j(x).  The law is
// linear with slope 1 / (dR - dC) strictly inside (dC, dR) while below the
// cap; elsewhere (and where the cracking history, not abar, drives D) the
// derivative is 0 (one-sided at the kinks).
FFTG_KERNEL void k_damage_adj(MatTable tab, long long N, int J,
                              const unsigned char* __restrict__ phase,
                              const double* __restrict__ abar, const double* __restrict__ hist,
                              const double* __restrict__ gD, double* __restrict__ gabar) {
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS) {
    const int ph = phase[v];
    const Mat m = tab.m[ph < tab.nphase ? ph : 0];
    for (int j = 0; j < J; ++j) {
      double gv = 0.0;
      if (m.model != 0 && m.dfield == j) {
        const double a = abar[(long long)j * N + v];
        const bool by_abar = m.model != 2 || !(hist[(long long)j * N + v] > a);
        const double d = (a - m.dC) / (m.dR - m.dC);
        if (by_abar && d > 0.0 && d < m.dmax)
          gv = gD[(long long)j * N + v] / (m.dR - m.dC);
      }
      gabar[(long long)j * N + v] = gv;
    }
  }
}

// Damage-history cotangents of an increment (hist_{n+1} = max(hist_n, abar),
// read back by the cracking law through the same max).  With the history the
// max (hist_n > abar, the damage law's tie convention):
//   g_abar  = g_hist where abar is the max, 0 elsewhere            (k_hist_split)
//   g_hist_n = g_hist where hist_n is the max, plus zeta / (dR - dC) on a
//              cracking voxel of the field whose history drives D inside the
//              slope band                                           (k_hist_damage_cot)
// zeta: the total damage cotangent [J][N].  g_hist may be null (zero).
FFTG_KERNEL void k_hist_split(long long n, const double* __restrict__ abar,
                              const double* __restrict__ hist_n,
                              const double* __restrict__ g_hist, double* __restrict__ g_abar) {
  for (long long i = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; i < n;
       i += (long long)gridDim.x * FFT_THREADS)
    g_abar[i] = hist_n[i] > abar[i] ? 0.0 : g_hist[i];
}

FFTG_KERNEL void k_hist_damage_cot(MatTable tab, long long N, int J,
                                   const unsigned char* __restrict__ phase,
                                   const double* __restrict__ abar,
                                   const double* __restrict__ hist_n,
                                   const double* __restrict__ zeta,
                                   const double* __restrict__ g_hist,
                                   double* __restrict__ g_hist_n) {
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS) {
    const int ph = phase[v];
    const Mat m = tab.m[ph < tab.nphase ? ph : 0];
    for (int j = 0; j < J; ++j) {
      const long long i = (long long)j * N + v;
      const double h = hist_n[i];
      const bool by_hist = h > abar[i];
      double gv = by_hist && g_hist ? g_hist[i] : 0.0;
      if (m.model == 2 && m.dfield == j && by_hist) {
        const double d = (h - m.dC) / (m.dR - m.dC);
        if (d > 0.0 && d < m.dmax) gv += zeta[i] / (m.dR - m.dC);
      }
      g_hist_n[i] = gv;
    }
  }
}

// Per-phase sums of a real field [N] -> partials [nphase][gridDim].
FFTG_KERNEL void k_phase_sums(long long N, int nphase, const unsigned char* __restrict__ phase,
                              const double* __restrict__ f, double* __restrict__ partials) {
  __shared__ double red[FFT_THREADS];
  for (int q = 0; q < nphase; ++q) {
    double acc = 0.0;
    for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
         v += (long long)gridDim.x * FFT_THREADS)
      if (phase[v] == q) acc += f[v];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[(long long)q * gridDim.x + blockIdx.x] = s;
  }
}

// Number of voxels whose phase id is >= nphase -> partials [gridDim] (exact:
// counts stay far below 2^53).
FFTG_KERNEL void k_count_bad_phase(long long N, int nphase,
                                   const unsigned char* __restrict__ phase,
                                   double* __restrict__ partials) {
  __shared__ double red[FFT_THREADS];
  double acc = 0.0;
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS)
    acc += phase[v] >= nphase ? 1.0 : 0.0;
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Per-component sums of a real field [ncomp][N] -> partials [ncomp][gridDim].
FFTG_KERNEL void k_comp_sums(long long N, int ncomp, const double* __restrict__ f,
                             double* __restrict__ partials) {
  __shared__ double red[FFT_THREADS];
  for (int k = 0; k < ncomp; ++k) {
    double acc = 0.0;
    for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
         v += (long long)gridDim.x * FFT_THREADS)
      acc += f[k * N + v];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[(long long)k * gridDim.x + blockIdx.x] = s;
  }
}

struct Vec6 {
  double v[6];
};

FFTG_KERNEL void k_add_const(long long N, int ncomp, double* __restrict__ f, Vec6 d) {
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS)
    for (int k = 0; k < ncomp; ++k)
      if (d.v[k] != 0.0) f[k * N + v] += d.v[k];
}

// Staggered error terms: partials [0] max_x ||eps_new - eps_old||^2,
// [1 + 2j] sum (abar_new - abar_old)^2, [2 + 2j] sum abar_new^2.
FFTG_KERNEL void k_stagger_err(long long N, int c, int J, const double* __restrict__ en,
                               const double* __restrict__ eo, const double* __restrict__ an,
                               const double* __restrict__ ao, double* __restrict__ partials) {
  __shared__ double red[FFT_THREADS];
  double mx = 0.0;
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS) {
    double s = 0.0;
    for (int k = 0; k < c; ++k) {
      const double d = en[k * N + v] - eo[k * N + v];
      s += d * d;
    }
    mx = s > mx ? s : mx;
  }
  // max reduction
  __syncthreads();
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = FFT_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s && red[threadIdx.x + s] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
  for (int j = 0; j < J; ++j) {
    double a1 = 0.0, a2 = 0.0;
    for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
         v += (long long)gridDim.x * FFT_THREADS) {
      const double x = an[j * N + v], d = x - ao[j * N + v];
      a1 += d * d;
      a2 += x * x;
    }
    double s = block_sum(a1, red);
    if (threadIdx.x == 0) partials[(long long)(1 + 2 * j) * gridDim.x + blockIdx.x] = s;
    s = block_sum(a2, red);
    if (threadIdx.x == 0) partials[(long long)(2 + 2 * j) * gridDim.x + blockIdx.x] = s;
  }
}

FFTG_KERNEL void k_vmax(long long n, double* __restrict__ a, const double* __restrict__ b) {
  for (long long i = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; i < n;
       i += (long long)gridDim.x * FFT_THREADS)
    a[i] = b[i] > a[i] ? b[i] : a[i];
}

template <typename TA, typename TB>
FFTG_KERNEL void k_convert(long long n, const TA* __restrict__ a, TB* __restrict__ b) {
  for (long long i = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; i < n;
       i += (long long)gridDim.x * FFT_THREADS)
    b[i] = (TB)a[i];
}

// b <- b + a, widening a to FP64 (the FP64 accumulation of an FP32 correction).
template <typename TA>
FFTG_KERNEL void k_acc_wide(long long n, const TA* __restrict__ a, double* __restrict__ b) {
  for (long long i = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; i < n;
       i += (long long)gridDim.x * FFT_THREADS)
    b[i] += (double)a[i];
}

// FP64 residual of an iterative-refinement sweep of the Helmholtz solve:
// r = b - Ap on the half spectrum, stored rounded to FP32 as the right-hand
// side of the next FP32 correction solve; partials: weighted |r|^2 in FP64.
FFTG_KERNEL void k_h_refine_resid(Geo g, const cpx<double>* __restrict__ b,
                                  const cpx<double>* __restrict__ Ap, cpx<float>* __restrict__ r32,
                                  double* __restrict__ partials) {
  __shared__ double red[FFT_THREADS];
  double acc = 0.0;
  const long long off = (long long)blockIdx.y * g.Ns;  // system blockIdx.y
  for (long long gi = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; gi < g.Ns;
       gi += (long long)gridDim.x * FFT_THREADS) {
    const cpx<double> r = b[off + gi] - Ap[off + gi];
    r32[off + gi] = mk((float)r.x, (float)r.y);
    acc += hweight((int)(gi % g.n1h), g.n1h) * (r.x * r.x + r.y * r.y);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[(long long)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// Sum of ell2 over N voxels for each system blockIdx.y (ell2 [sys][N]).
template <typename T>
FFTG_KERNEL void k_sum_ell2(long long N, const T* __restrict__ e, double* __restrict__ partials) {
  __shared__ double red[FFT_THREADS];
  double acc = 0.0;
  const T* es = e + (long long)blockIdx.y * N;
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS)
    acc += (double)es[v];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[(long long)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// ============================================================ adjoint helpers
// out = i q~_j in: gradient component j of the Helmholtz operator's symbol.
template <typename T>
FFTG_KERNEL void k_grad_comp(Geo g, Sym<T> sym, int j, const cpx<T>* __restrict__ in,
                             cpx<T>* __restrict__ out) {
  for (long long gi = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; gi < g.Ns;
       gi += (long long)gridDim.x * FFT_THREADS) {
    int kx, ky, kz;
    decode(g, gi, kx, ky, kz);
    T q[3];
    qvec(sym, true, kx, ky, kz, q);
    out[gi] = mul_i(scale(in[gi], q[j]));
  }
}

// gout = gin + K : gsig per voxel with the compact tangent (a, b, m) of the
// constitutive update: K:e = a tr(e) I + b dev(e) - (m.e) m (plane strain: the
// in-plane components, e33 = 0).  gin may be null.
template <typename TT>
FFTG_KERNEL void k_tangent_apply(long long N, int c, const TT* __restrict__ tan,
                                 const double* __restrict__ gsig, const double* __restrict__ gin,
                                 double* __restrict__ gout) {
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS) {
    const TT* tv = tan + 8 * v;
    const double a = (double)tv[0], b = (double)tv[1];
    double m[6], e[6], o[6];
    for (int i = 0; i < 6; ++i) m[i] = (double)tv[2 + i];
    for (int i = 0; i < c; ++i) e[i] = gsig[(long long)i * N + v];
    if (c == 6) {
      const double tr = e[0] + e[1] + e[2];
      const double md = m[0] * e[0] + m[1] * e[1] + m[2] * e[2] + m[3] * e[3] + m[4] * e[4] +
                        m[5] * e[5];
      for (int i = 0; i < 3; ++i) o[i] = a * tr + b * (e[i] - tr / 3.0) - md * m[i];
      for (int i = 3; i < 6; ++i) o[i] = b * e[i] - md * m[i];
    } else {
      const double tr = e[0] + e[1];
      const double md = m[0] * e[0] + m[1] * e[1] + m[5] * e[2];
      o[0] = a * tr + b * (e[0] - tr / 3.0) - md * m[0];
      o[1] = a * tr + b * (e[1] - tr / 3.0) - md * m[1];
      o[2] = b * e[2] - md * m[5];
    }
    for (int i = 0; i < c; ++i)
      gout[(long long)i * N + v] = (gin ? gin[(long long)i * N + v] : 0.0) + o[i];
  }
}

// out = (acc ? out : 0) - a b
FFTG_KERNEL void k_sub_prod(long long n, const double* __restrict__ a,
                            const double* __restrict__ b, double* __restrict__ out, int acc) {
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < n;
       v += (long long)gridDim.x * FFT_THREADS)
    out[v] = (acc ? out[v] : 0.0) - a[v] * b[v];
}

// y = s x
FFTG_KERNEL void k_scale(long long n, double s, const double* __restrict__ x,
                         double* __restrict__ y) {
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < n;
       v += (long long)gridDim.x * FFT_THREADS)
    y[v] = s * x[v];
}

// dJ/dD_j(x) = (mu(x) - gsig(x)) : sigma(x) / (1 - D_j(x)) where the voxel's
// phase has a damage law driven by field j (sigma / (1 - D) is the effective
// stress, and d sigma / dD = -sigma_eff); 0 elsewhere.  gsig may be null.
FFTG_KERNEL void k_adj_damage(MatTable tab, long long N, int c, int J,
                              const unsigned char* __restrict__ phase,
                              const double* __restrict__ D, const double* __restrict__ sigma,
                              const double* __restrict__ mu, const double* __restrict__ gsig,
                              double* __restrict__ dD) {
  for (long long v = (long long)blockIdx.x * FFT_THREADS + threadIdx.x; v < N;
       v += (long long)gridDim.x * FFT_THREADS) {
    const int ph = phase[v];
    const Mat m = tab.m[ph < tab.nphase ? ph : 0];
    double dot = 0.0;
    for (int i = 0; i < c; ++i)
      dot += (mu[(long long)i * N + v] - (gsig ? gsig[(long long)i * N + v] : 0.0)) *
             sigma[(long long)i * N + v];
    for (int j = 0; j < J; ++j) {
      double d = 0.0;
      if (m.model != 0 && m.dfield == j) d = dot / (1.0 - D[(long long)j * N + v]);
      dD[(long long)j * N + v] = d;
    }
  }
}

// ============================================================ launchers
static inline int grid_for(long long n) {
  long long b = (n + FFT_THREADS - 1) / FFT_THREADS;
  if (b > RED_BLOCKS) b = RED_BLOCKS;
  if (b < 1) b = 1;
  return (int)b;
}

// Runs the statement with NF set to the compile-time length matching n
// (0 = run-time path).
#define FFTG_DISPATCH_N(n, ...)     \
  switch (n) {                      \
    case 16: {                      \
      constexpr int NF = 16;        \
      __VA_ARGS__;                  \
    } break;                        \
    case 32: {                      \
      constexpr int NF = 32;        \
      __VA_ARGS__;                  \
    } break;                        \
    case 48: {                      \
      constexpr int NF = 48;        \
      __VA_ARGS__;                  \
    } break;                        \
    case 64: {                      \
      constexpr int NF = 64;        \
      __VA_ARGS__;                  \
    } break;                        \
    case 96: {                      \
      constexpr int NF = 96;        \
      __VA_ARGS__;                  \
    } break;                        \
    case 128: {                     \
      constexpr int NF = 128;       \
      __VA_ARGS__;                  \
    } break;                        \
    case 256: {                     \
      constexpr int NF = 256;       \
      __VA_ARGS__;                  \
    } break;                        \
    default: {                      \
      constexpr int NF = 0;         \
      __VA_ARGS__;                  \
    } break;                        \
  }

static inline void require(bool ok, const char* what) {
  if (!ok) throw std::runtime_error(what);
}

template <typename T>
void launch_x_r2c(const Plan& p, const cpx<T>* tw, const T* in, cpx<T>* out, long long S,
                  int n1, int n1h, hipStream_t st) {
  FFTG_DISPATCH_N(n1, {
    const int P = NF ? fx_pairs<T>(NF) : LDS_ELEMS / n1;
    const long long nb = (S + 2 * P - 1) / (2 * P);
    hipLaunchKernelGGL((k_x_r2c<T, NF>), dim3((unsigned)nb), dim3(FFT_THREADS), 0, st, p, tw, in,
                       out, S, n1, n1h, P);
  })
}

template <typename T, typename TO>
void launch_x_c2r(const Plan& p, const cpx<T>* tw, const cpx<T>* in, TO* out, long long S,
                  int n1, int n1h, T scl, bool acc, hipStream_t st) {
  FFTG_DISPATCH_N(n1, {
    const int P = NF ? fx_pairs<T>(NF) : LDS_ELEMS / n1;
    const long long nb = (S + 2 * P - 1) / (2 * P);
    hipLaunchKernelGGL((k_x_c2r<T, TO, NF>), dim3((unsigned)nb), dim3(FFT_THREADS), 0, st, p, tw,
                       in, out, S, n1, n1h, P, scl, acc ? 1 : 0);
  })
}

// Lines per tile of the run-time path: the largest power of two that fits
// (at most FFT_THREADS), so that it divides the block size.
static inline int tile_lines(int n, int ncomp) {
  const int cap = LDS_ELEMS / (n * ncomp);
  if (cap < 1) throw std::runtime_error("strided pass: line does not fit in LDS");
  int tl = 1;
  while (2 * tl <= cap && 2 * tl <= FFT_THREADS) tl *= 2;
  return tl;
}

// tile-budget code of the fixed-length strided kernels (0..3, tile_budget)
#define FFTG_DISPATCH_SH(sh, ...)   \
  switch (sh) {                     \
    case 1: {                       \
      constexpr int SH = 1;         \
      __VA_ARGS__;                  \
    } break;                        \
    case 2: {                       \
      constexpr int SH = 2;         \
      __VA_ARGS__;                  \
    } break;                        \
    case 3: {                       \
      constexpr int SH = 3;         \
      __VA_ARGS__;                  \
    } break;                        \
    default: {                      \
      constexpr int SH = 0;         \
      __VA_ARGS__;                  \
    }                               \
  }

// XCD run length for lines of several stacked systems, lps lines each, in
// tiles of TL lines: runs of up to 16 tiles, at least 8 runs per system, so
// that every system keeps all eight XCDs busy when others have converged; 0
// (one contiguous run per XCD) for a single system.
static inline int xcd_chunk(long long nlines, long long lps, int TL) {
  if (lps >= nlines) return 0;
  const long long per = lps / TL / 8;
  return (int)(per < 1 ? 1 : per > 16 ? 16 : per);
}

template <typename T>
void launch_strided(const Plan& p, const cpx<T>* tw, cpx<T>* data, long long nlines,
                    long long inner, long long ostride, long long es, bool fwd,
                    const KrylovCtl* ctl, hipStream_t st, int sh, long long lps) {
  if (lps <= 0) lps = nlines;
  FFTG_DISPATCH_N(p.n, FFTG_DISPATCH_SH(NF ? sh : 0, {
    const int TL = NF ? fs_tile<T, tile_budget<SH>()>(NF) : tile_lines(p.n, 1);
    const int NT = NF ? kStridedThreads : FFT_THREADS;
    const long long nb = (nlines + TL - 1) / TL;
    // One FP64 system, inverse: runs of 16 tiles handed to the XCDs in turn
    // rather than one contiguous run each.  Part of the spectrum this pass
    // reads (just written by the outer inverse pass) is still in the
    // Infinity Cache, unevenly over the tile range; with contiguous runs the
    // XCDs holding the uncached runs set the pass's time (measured in the CG
    // loop at 128^3: 46.9 -> 42.4 us; the forward pass and FP32 are faster
    // with contiguous runs).
    const int chunk = lps < nlines ? xcd_chunk(nlines, lps, TL) : (!fwd && sizeof(T) == 8 ? 16 : 0);
    if (fwd)
      hipLaunchKernelGGL((k_strided<T, true, NF, SH>), dim3((unsigned)nb), dim3(NT), 0, st, p, tw,
                         data, nlines, inner, ostride, es, TL, ctl, lps, chunk);
    else
      hipLaunchKernelGGL((k_strided<T, false, NF, SH>), dim3((unsigned)nb), dim3(NT), 0, st, p,
                         tw, data, nlines, inner, ostride, es, TL, ctl, lps, chunk);
  }))
}

// tiles per slab of an outer-axis pass (TL lines each, no tile across two
// slabs: systems, or components of a system)
static inline int tiles_per_sys(long long inner, int TL) { return (int)((inner + TL - 1) / TL); }

// outer axis line geometry for a c-component spectrum
static inline void outer_lines(const Geo& g, int ncomp, bool zouter, long long& nlines,
                               long long& inner, long long& ostride, long long& es) {
  if (zouter) {
    inner = (long long)g.n2 * g.n1h;
    nlines = inner * ncomp;
    ostride = g.Ns;
    es = inner;
  } else {  // 2D: y is the outer axis, n3 == 1
    inner = g.n1h;
    nlines = inner * ncomp;
    ostride = g.Ns;
    es = g.n1h;
  }
}

template <typename T>
int launch_gal_dir_inv(const Plan& p, const cpx<T>* tw, const Geo& g, int c, bool zouter,
                       cpx<T>* r, cpx<T>* pp, cpx<T>* x, cpx<T>* w, KrylovCtl* ctl,
                       hipStream_t st, int sh, int nsys, int parity, const double* rpart,
                       int nbr) {
  long long nl, inner, os, es;
  outer_lines(g, c, zouter, nl, inner, os, es);
  long long nb = 0;
  FFTG_DISPATCH_N(p.n, FFTG_DISPATCH_SH(NF ? sh : 0, {
    const int TL = NF ? fs_tile<T, tile_budget<SH>()>(NF) : tile_lines(p.n, 1);
    const int NT = NF ? kStridedThreads : FFT_THREADS;
    const int tpo = tiles_per_sys(inner, TL);
    nb = (long long)tpo * c * nsys;
    hipLaunchKernelGGL((k_gal_dir_inv<T, NF, SH>), dim3((unsigned)nb), dim3(NT), 0, st, p, tw, r,
                       pp, x, w, inner, os, es, TL, tpo, c, ctl, parity, rpart, nbr);
  }))
  return (int)nb;
}

template <typename T>
int launch_gal_dot_fwd(const Plan& p, const cpx<T>* tw, const Geo& g, int c, bool zouter,
                       const cpx<T>* pp, cpx<T>* w, double* partials, const KrylovCtl* ctl,
                       hipStream_t st, int nsys) {
  long long nl, inner, os, es;
  outer_lines(g, c, zouter, nl, inner, os, es);
  long long nb = 0;
  FFTG_DISPATCH_N(p.n, {
    const int TL = NF ? fs_tile<T, kDotBytes<T>>(NF) : tile_lines(p.n, 1);
    const int tpo = tiles_per_sys(inner, TL);
    nb = (long long)tpo * c * nsys;
    hipLaunchKernelGGL((k_gal_dot_fwd<T, NF>), dim3((unsigned)nb), dim3(NF ? kDotThreads<T> : FFT_THREADS), 0, st, p,
                       tw, pp, w, inner, os, es, TL, tpo, c, g.n1h, partials, ctl);
  })
  return (int)(nb / nsys);  // partials per system
}

template <typename T>
int gal_dot_count(const Plan& p, const Geo& g, int c, bool zouter) {
  long long nl, inner, os, es;
  outer_lines(g, c, zouter, nl, inner, os, es);
  int cnt = 0;
  FFTG_DISPATCH_N(p.n, {
    const int TL = NF ? fs_tile<T, kDotBytes<T>>(NF) : tile_lines(p.n, 1);
    cnt = tiles_per_sys(inner, TL) * c;
  })
  return cnt;
}
int gal_resid_count(const Geo& g) { return grid_for(g.Ns); }

static inline int fused_lines_rt(int n1, int c) {
  int NL = (2 * LDS_ELEMS) / (c * n1);
  NL -= NL % 2;
  if (NL < 2) NL = 2;
  require((c * NL / 2) * n1 <= LDS_ELEMS, "x pass: line batch does not fit in LDS");
  return NL;
}

template <typename T>
int gal_xdot_count(const Geo& g, int c) {
  const long long nlines = (long long)g.n2 * g.n3;
  int cnt = 0;
  FFTG_DISPATCH_N(g.n1, {
    const int NL = c == 6 ? (NF ? fx_fused_lines<T>(NF, 6) : fused_lines_rt(g.n1, 6))
                          : (NF ? fx_fused_lines<T>(NF, 3) : fused_lines_rt(g.n1, 3));
    cnt = (int)((nlines + NL - 1) / NL);
  })
  return cnt;
}

template <typename T, typename TT>
int launch_x_fused_gal(const Plan& p, const cpx<T>* tw, const Geo& g, int c, cpx<T>* w,
                       const TT* tan, T scl, const KrylovCtl* ctl, hipStream_t st, int nsys,
                       double* partials) {
  const long long nlines = (long long)g.n2 * g.n3;
  long long bps = 0;
  FFTG_DISPATCH_N(g.n1, {
    if (c == 6) {
      const int NL = NF ? fx_fused_lines<T>(NF, 6) : fused_lines_rt(g.n1, 6);
      bps = (nlines + NL - 1) / NL;
      hipLaunchKernelGGL((k_x_fused_gal<T, TT, NF, 6>), dim3((unsigned)(bps * nsys)),
                         dim3(NF ? kFusedThreads : FFT_THREADS), 0,
                         st, p, tw, g, NL, w, tan, scl, ctl, partials);
    } else {
      const int NL = NF ? fx_fused_lines<T>(NF, 3) : fused_lines_rt(g.n1, 3);
      bps = (nlines + NL - 1) / NL;
      hipLaunchKernelGGL((k_x_fused_gal<T, TT, NF, 3>), dim3((unsigned)(bps * nsys)),
                         dim3(NF ? kFusedThreads : FFT_THREADS), 0,
                         st, p, tw, g, NL, w, tan, scl, ctl, partials);
    }
  })
  return (int)bps;  // partials per system
}

template <typename T, typename TL>
int launch_x_fused_helm(const Plan& p, const cpx<T>* tw, const Geo& g, cpx<T>* w,
                        const TL* ell2, T scl, const KrylovCtl* ctl, hipStream_t st, int nsys,
                        const unsigned char* phase, const TL* ptab, double* partials) {
  const long long lpsys = (long long)g.n2 * g.n3;
  const long long ws = (long long)nsys * g.Ns;
  long long bps = 0;
  FFTG_DISPATCH_N(g.n1, {
    if (g.ndim == 3) {
      const int NL = NF ? fx_helm_lines<T>(NF, 3) : fused_lines_rt(g.n1, 3);
      bps = (lpsys + NL - 1) / NL;
      hipLaunchKernelGGL((k_x_fused_helm<T, TL, NF, 3>), dim3((unsigned)(bps * nsys)),
                         dim3(NF ? kFusedThreads : FFT_THREADS), 0,
                         st, p, tw, g, NL, w, ell2, scl, nsys, ws, ctl, phase, ptab, partials);
    } else {
      const int NL = NF ? fx_helm_lines<T>(NF, 2) : fused_lines_rt(g.n1, 2);
      bps = (lpsys + NL - 1) / NL;
      hipLaunchKernelGGL((k_x_fused_helm<T, TL, NF, 2>), dim3((unsigned)(bps * nsys)),
                         dim3(NF ? kFusedThreads : FFT_THREADS), 0,
                         st, p, tw, g, NL, w, ell2, scl, nsys, ws, ctl, phase, ptab, partials);
    }
  })
  return (int)bps;  // partials per system
}

template <typename T>
int launch_gal_resid(const Geo& g, int c, const Sym<T>& sym, const unsigned char* m,
                     cpx<T>* r, const cpx<T>* w, double* partials, KrylovCtl* ctl,
                     hipStream_t st, int nsys, int parity, const double* dpart, int nbd) {
  const int nb = grid_for(g.Ns);
  if (c == 6)
    hipLaunchKernelGGL((k_gal_resid<T, 6>), dim3(nb, nsys), dim3(FFT_THREADS), 0, st, g, sym, m[0], m[1],
                       m[2], m[3], m[4], m[5], r, w, partials, ctl, parity, dpart, nbd);
  else
    hipLaunchKernelGGL((k_gal_resid<T, 3>), dim3(nb, nsys), dim3(FFT_THREADS), 0, st, g, sym, m[0], m[1],
                       m[2], m[3], m[4], m[5], r, w, partials, ctl, parity, dpart, nbd);
  return nb;
}

template <typename T>
int launch_gal_fwd_resid(const Plan& p, const cpx<T>* tw, const Geo& g, int c, bool zouter,
                         const Sym<T>& sym, const unsigned char* m, const cpx<T>* w, cpx<T>* r,
                         double* partials, const KrylovCtl* ctl, hipStream_t st, int nsys) {
  long long nl, inner, os, es;
  outer_lines(g, 1, zouter, nl, inner, os, es);
  unsigned mb = 0;
  for (int i = 0; i < 6; ++i)
    if (m[i]) mb |= 1u << i;
  int tpo = 0;
  FFTG_DISPATCH_N(p.n, {
    if (c == 6) {
      const int TL = NF ? fr_tile<T>(NF, 6) : tile_lines(p.n, 6);
      tpo = tiles_per_sys(inner, TL);
      const long long nb = (long long)tpo * nsys;
      const int chunk = xcd_chunk(nb * TL, (long long)tpo * TL, TL);
      hipLaunchKernelGGL((k_gal_fwd_resid<T, NF, 6>), dim3((unsigned)nb),
                         dim3(NF ? kFwdResThreads : FFT_THREADS), 0, st, p, tw, g, sym, mb, w, r,
                         inner, es, TL, tpo, chunk, partials, ctl);
    } else {
      const int TL = NF ? fr_tile<T>(NF, 3) : tile_lines(p.n, 3);
      tpo = tiles_per_sys(inner, TL);
      const long long nb = (long long)tpo * nsys;
      const int chunk = xcd_chunk(nb * TL, (long long)tpo * TL, TL);
      hipLaunchKernelGGL((k_gal_fwd_resid<T, NF, 3>), dim3((unsigned)nb),
                         dim3(NF ? kFwdResThreads : FFT_THREADS), 0, st, p, tw, g, sym, mb, w, r,
                         inner, es, TL, tpo, chunk, partials, ctl);
    }
  })
  return tpo;  // partials per system
}

template <typename T>
int gal_fwd_resid_count(const Plan& p, const Geo& g, int c, bool zouter) {
  long long nl, inner, os, es;
  outer_lines(g, 1, zouter, nl, inner, os, es);
  int cnt = 0;
  FFTG_DISPATCH_N(p.n, {
    const int TL = c == 6 ? (NF ? fr_tile<T>(NF, 6) : tile_lines(p.n, 6))
                          : (NF ? fr_tile<T>(NF, 3) : tile_lines(p.n, 3));
    cnt = tiles_per_sys(inner, TL);
  })
  return cnt;
}

template <typename T>
int launch_gal_rhs(const Geo& g, int c, const Sym<double>& sym, const unsigned char* m,
                   const double* S, const cpx<double>* sh, cpx<T>* r, double* partials,
                   hipStream_t st, int nsys, const double* S_sys) {
  const int nb = grid_for(g.Ns);
  if (c == 6)
    hipLaunchKernelGGL((k_gal_rhs<T, 6>), dim3(nb, nsys), dim3(FFT_THREADS), 0, st, g, sym, m[0],
                       m[1], m[2], m[3], m[4], m[5], S[0], S[1], S[2], S[3], S[4], S[5], sh, r,
                       partials, S_sys);
  else
    hipLaunchKernelGGL((k_gal_rhs<T, 3>), dim3(nb, nsys), dim3(FFT_THREADS), 0, st, g, sym, m[0],
                       m[1], m[2], m[3], m[4], m[5], S[0], S[1], S[2], S[3], S[4], S[5], sh, r,
                       partials, S_sys);
  return nb;
}

template <typename T>
void launch_project(const Geo& g, int c, const Sym<T>& sym, const unsigned char* m,
                    cpx<T>* data, hipStream_t st) {
  const int nb = grid_for(g.Ns);
  if (c == 6)
    hipLaunchKernelGGL((k_project<T, 6>), dim3(nb), dim3(FFT_THREADS), 0, st, g, sym, m[0], m[1],
                       m[2], m[3], m[4], m[5], data);
  else
    hipLaunchKernelGGL((k_project<T, 3>), dim3(nb), dim3(FFT_THREADS), 0, st, g, sym, m[0], m[1],
                       m[2], m[3], m[4], m[5], data);
}


template <typename T>
int launch_h_dir_inv(const Plan& p, const cpx<T>* tw, const Geo& g, bool zouter,
                     const Sym<T>& sym, bool update, const cpx<T>* r, cpx<T>* pp, cpx<T>* x,
                     cpx<T>* w, const KrylovCtl* ctl, hipStream_t st, int nsys, double* ppart) {
  long long nl, inner, os, es;
  outer_lines(g, 1, zouter, nl, inner, os, es);
  const long long ws = (long long)nsys * g.Ns;
  int tpo = 0;
  FFTG_DISPATCH_N(p.n, {
    if (helm_split(g)) {
      const int TL = NF ? fs_tile_wide<T>(NF, 2) : tile_lines(p.n, 2);
      tpo = tiles_per_sys(inner, TL);
      hipLaunchKernelGGL((k_h_dir_inv<T, NF, 3, true>), dim3((unsigned)(tpo * nsys)), dim3(NF ? kWideThreads : FFT_THREADS), 0, st, p,
                         tw, g, sym, update ? 1 : 0, r, pp, x, w, inner, os, es, TL, tpo, ws, ctl,
                         ppart);
    } else if (g.ndim == 3) {
      const int TL = NF ? fs_tile_wide<T>(NF, 3) : tile_lines(p.n, 3);
      tpo = tiles_per_sys(inner, TL);
      hipLaunchKernelGGL((k_h_dir_inv<T, NF, 3, false>), dim3((unsigned)(tpo * nsys)), dim3(NF ? kWideThreads : FFT_THREADS), 0, st, p,
                         tw, g, sym, update ? 1 : 0, r, pp, x, w, inner, os, es, TL, tpo, ws, ctl,
                         ppart);
    } else {
      const int TL = NF ? fs_tile_wide<T>(NF, 2) : tile_lines(p.n, 2);
      tpo = tiles_per_sys(inner, TL);
      hipLaunchKernelGGL((k_h_dir_inv<T, NF, 2, false>), dim3((unsigned)(tpo * nsys)), dim3(NF ? kWideThreads : FFT_THREADS), 0, st, p,
                         tw, g, sym, update ? 1 : 0, r, pp, x, w, inner, os, es, TL, tpo, ws, ctl,
                         ppart);
    }
  })
  return tpo;
}

template <typename T>
void launch_h_y_split(const Plan& p, const cpx<T>* tw, const Geo& g, const Sym<T>& sym,
                      cpx<T>* w, bool fwd, const KrylovCtl* ctl, hipStream_t st, int nsys) {
  require(helm_split(g), "split Helmholtz y pass: 3D grids with n2 > 1 only");
  const long long nl = (long long)nsys * g.n3 * g.n1h;
  const long long ws = (long long)nsys * g.Ns;
  FFTG_DISPATCH_N(p.n, {
    const int TL = NF ? fs_tile_wide<T>(NF, 3) : tile_lines(p.n, 3);
    const long long nb = (nl + TL - 1) / TL;
    const int chunk = xcd_chunk(nl, (long long)g.n3 * g.n1h, TL);
    if (fwd)
      hipLaunchKernelGGL((k_h_y_split<T, true, NF>), dim3((unsigned)nb),
                         dim3(NF ? kWideThreads : FFT_THREADS), 0, st, p, tw, g, sym, w, nl, TL,
                         ws, ctl, chunk);
    else
      hipLaunchKernelGGL((k_h_y_split<T, false, NF>), dim3((unsigned)nb),
                         dim3(NF ? kWideThreads : FFT_THREADS), 0, st, p, tw, g, sym, w, nl, TL,
                         ws, ctl, chunk);
  })
}

template <typename T>
int launch_h_div_fwd(const Plan& p, const cpx<T>* tw, const Geo& g, bool zouter,
                     const Sym<T>& sym, const cpx<T>* pp, cpx<T>* w, cpx<T>* Ap,
                     double* partials, const KrylovCtl* ctl, hipStream_t st, int nsys) {
  long long nl, inner, os, es;
  outer_lines(g, 1, zouter, nl, inner, os, es);
  const long long ws = (long long)nsys * g.Ns;
  int tpo = 0;
  FFTG_DISPATCH_N(p.n, {
    if (helm_split(g)) {
      const int TL = NF ? fs_tile_wide<T>(NF, 2) : tile_lines(p.n, 2);
      tpo = tiles_per_sys(inner, TL);
      hipLaunchKernelGGL((k_h_div_fwd<T, NF, 3, true>), dim3((unsigned)(tpo * nsys)), dim3(NF ? kWideThreads : FFT_THREADS), 0, st, p,
                         tw, g, sym, pp, w, Ap, inner, os, es, TL, tpo, ws, partials, ctl);
    } else if (g.ndim == 3) {
      const int TL = NF ? fs_tile_wide<T>(NF, 3) : tile_lines(p.n, 3);
      tpo = tiles_per_sys(inner, TL);
      hipLaunchKernelGGL((k_h_div_fwd<T, NF, 3, false>), dim3((unsigned)(tpo * nsys)), dim3(NF ? kWideThreads : FFT_THREADS), 0, st, p,
                         tw, g, sym, pp, w, Ap, inner, os, es, TL, tpo, ws, partials, ctl);
    } else {
      const int TL = NF ? fs_tile_wide<T>(NF, 2) : tile_lines(p.n, 2);
      tpo = tiles_per_sys(inner, TL);
      hipLaunchKernelGGL((k_h_div_fwd<T, NF, 2, false>), dim3((unsigned)(tpo * nsys)), dim3(NF ? kWideThreads : FFT_THREADS), 0, st, p,
                         tw, g, sym, pp, w, Ap, inner, os, es, TL, tpo, ws, partials, ctl);
    }
  })
  return tpo;
}

template <typename T>
int launch_h_fwd_resid(const Plan& p, const cpx<T>* tw, const Geo& g, bool zouter,
                       const Sym<T>& sym, const cpx<T>* pp, cpx<T>* w, cpx<T>* r,
                       double* partials, const KrylovCtl* ctl, hipStream_t st, int nsys) {
  long long nl, inner, os, es;
  outer_lines(g, 1, zouter, nl, inner, os, es);
  const long long ws = (long long)nsys * g.Ns;
  int tpo = 0;
  FFTG_DISPATCH_N(p.n, {
    if (helm_split(g)) {
      const int TL = NF ? fs_tile_wide<T>(NF, 2) : tile_lines(p.n, 2);
      tpo = tiles_per_sys(inner, TL);
      hipLaunchKernelGGL((k_h_fwd_resid<T, NF, 3, true>), dim3((unsigned)(tpo * nsys)),
                         dim3(NF ? kWideThreads : FFT_THREADS), 0, st, p, tw, g, sym, pp, w, r,
                         inner, os, es, TL, tpo, ws, partials, ctl);
    } else if (g.ndim == 3) {
      const int TL = NF ? fs_tile_wide<T>(NF, 3) : tile_lines(p.n, 3);
      tpo = tiles_per_sys(inner, TL);
      hipLaunchKernelGGL((k_h_fwd_resid<T, NF, 3, false>), dim3((unsigned)(tpo * nsys)),
                         dim3(NF ? kWideThreads : FFT_THREADS), 0, st, p, tw, g, sym, pp, w, r,
                         inner, os, es, TL, tpo, ws, partials, ctl);
    } else {
      const int TL = NF ? fs_tile_wide<T>(NF, 2) : tile_lines(p.n, 2);
      tpo = tiles_per_sys(inner, TL);
      hipLaunchKernelGGL((k_h_fwd_resid<T, NF, 2, false>), dim3((unsigned)(tpo * nsys)),
                         dim3(NF ? kWideThreads : FFT_THREADS), 0, st, p, tw, g, sym, pp, w, r,
                         inner, os, es, TL, tpo, ws, partials, ctl);
    }
  })
  return tpo;  // [sys][2][tpo] partials
}

template <typename T>
int launch_h_resid(const Geo& g, const Sym<T>& sym, bool init, cpx<T>* r, const cpx<T>* b,
                   const cpx<T>* Ap, double* partials, const KrylovCtl* ctl, hipStream_t st,
                   int nsys) {
  const int nb = grid_for(g.Ns);
  hipLaunchKernelGGL(k_h_resid<T>, dim3(nb, nsys), dim3(FFT_THREADS), 0, st, g, sym, init ? 1 : 0,
                     r, b, Ap, partials, ctl);
  return nb;
}

template <typename T>
void launch_grad_comp(const Geo& g, const Sym<T>& sym, int j, const cpx<T>* in, cpx<T>* out,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_grad_comp<T>, dim3(grid_for(g.Ns)), dim3(FFT_THREADS), 0, st, g, sym, j,
                     in, out);
}
void launch_sub_prod(long long n, const double* a, const double* b, double* out, bool acc,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_sub_prod, dim3(grid_for(n)), dim3(FFT_THREADS), 0, st, n, a, b, out,
                     acc ? 1 : 0);
}
void launch_scale(long long n, double s, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(FFT_THREADS), 0, st, n, s, x, y);
}
void launch_damage_adj(const MatTable& tab, long long N, int J, const unsigned char* phase,
                       const double* abar, const double* hist, const double* gD, double* gabar,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_damage_adj, dim3(grid_for(N)), dim3(FFT_THREADS), 0, st, tab, N, J, phase,
                     abar, hist, gD, gabar);
}
int launch_count_bad_phase(long long N, int nphase, const unsigned char* phase,
                           double* partials, hipStream_t st) {
  const int nb = grid_for(N);
  hipLaunchKernelGGL(k_count_bad_phase, dim3(nb), dim3(FFT_THREADS), 0, st, N, nphase, phase,
                     partials);
  return nb;
}
int launch_phase_sums(long long N, int nphase, const unsigned char* phase, const double* f,
                      double* partials, hipStream_t st) {
  const int nb = grid_for(N);
  hipLaunchKernelGGL(k_phase_sums, dim3(nb), dim3(FFT_THREADS), 0, st, N, nphase, phase, f,
                     partials);
  return nb;
}
void launch_adj_damage(const MatTable& tab, long long N, int c, int J,
                       const unsigned char* phase, const double* D, const double* sigma,
                       const double* mu, const double* gsig, double* dD, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_damage, dim3(grid_for(N)), dim3(FFT_THREADS), 0, st, tab, N, c, J,
                     phase, D, sigma, mu, gsig, dD);
}
template <typename TT>
void launch_tangent_apply(long long N, int c, const TT* tan, const double* gsig,
                          const double* gin, double* gout, hipStream_t st) {
  hipLaunchKernelGGL(k_tangent_apply<TT>, dim3(grid_for(N)), dim3(FFT_THREADS), 0, st, N, c, tan,
                     gsig, gin, gout);
}

void launch_fin_alpha(double* partials, int nb, KrylovCtl* ctl, hipStream_t st, int nsys) {
  hipLaunchKernelGGL(k_fin_alpha, dim3(nsys), dim3(FFT_THREADS), 0, st, partials, nb, ctl);
}
void launch_fin_alpha2(const double* pa, int na, const double* pb, int nb, KrylovCtl* ctl,
                       hipStream_t st, int nsys) {
  hipLaunchKernelGGL(k_fin_alpha2, dim3(nsys), dim3(FFT_THREADS), 0, st, pa, na, pb, nb, ctl);
}
void launch_fin_beta(double* partials, int nb, int nred, KrylovCtl* ctl, hipStream_t st,
                     int nsys) {
  hipLaunchKernelGGL(k_fin_beta, dim3(nsys), dim3(FFT_THREADS), 0, st, partials, nb, nred, ctl);
}
void launch_fin_sums(const double* partials, int nb, int nred, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_fin_sums, dim3(1), dim3(FFT_THREADS), 0, st, partials, nb, nred, out);
}

template <typename T>
void launch_xfinal(cpx<T>* x, const cpx<T>* p, long long n, const KrylovCtl* ctl,
                   hipStream_t st, int nsys) {
  hipLaunchKernelGGL(k_xfinal<T>, dim3(grid_for(n), nsys), dim3(FFT_THREADS), 0, st, x, p, n,
                     ctl);
}

template <typename T>
void launch_hermitize(const Geo& g, int ncomp, cpx<T>* d, hipStream_t st) {
  hipLaunchKernelGGL(k_hermitize<T>, dim3(grid_for(2LL * g.n2 * g.n3 * ncomp)), dim3(FFT_THREADS), 0,
                     st, g, ncomp, d);
}

template <typename T>
int launch_wnorm2(const Geo& g, int ncomp, const cpx<T>* a, double* partials, hipStream_t st,
                  int nsys) {
  const int nb = grid_for(g.Ns * ncomp);
  hipLaunchKernelGGL(k_wnorm2<T>, dim3(nb, nsys), dim3(FFT_THREADS), 0, st, g, ncomp, a, partials);
  return nb;
}

template <typename TT>
void launch_constitutive(const MatTable& tab, const Geo& g, int c, int J,
                         const unsigned char* phase, const double* eps, const double* st_n,
                         const double* D, double* sigma, double* st_np1, double* alpha, TT* tan,
                         hipStream_t st) {
  if (tab.gtn)
    hipLaunchKernelGGL((k_constitutive<TT, true>), dim3(grid_for(g.N)), dim3(FFT_THREADS), 0, st,
                       tab, g, c, J, phase, eps, st_n, D, sigma, st_np1, alpha, tan);
  else
    hipLaunchKernelGGL((k_constitutive<TT, false>), dim3(grid_for(g.N)), dim3(FFT_THREADS), 0, st,
                       tab, g, c, J, phase, eps, st_n, D, sigma, st_np1, alpha, tan);
}

void launch_damage(const MatTable& tab, long long N, int J, const unsigned char* phase,
                   const double* abar, const double* hist, const double* abar_n, double* D,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_damage, dim3(grid_for(N)), dim3(FFT_THREADS), 0, st, tab, N, J, phase, abar,
                     hist, abar_n, D);
}

void launch_source_adj(const MatTable& tab, long long N, int c, int J, const unsigned char* phase,
                       const double* eps, const double* state_n, const double* lam, double* out,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_source_adj, dim3(grid_for(N)), dim3(FFT_THREADS), 0, st, tab, N, c, J,
                     phase, eps, state_n, lam, out);
}

void launch_hist_out_cot(const MatTable& tab, long long N, int c, const unsigned char* phase,
                         const double* eps, const double* state_n, const double* g_epsp,
                         const double* g_kappa, double* g_eps, hipStream_t st) {
  hipLaunchKernelGGL(k_hist_out_cot, dim3(grid_for(N)), dim3(FFT_THREADS), 0, st, tab, N, c,
                     phase, eps, state_n, g_epsp, g_kappa, g_eps);
}

void launch_hist_in_cot(const MatTable& tab, long long N, int c, int J, const unsigned char* phase,
                        const double* eps, const double* state_n, const double* D,
                        const double* mu, const double* g_sig, const double* lam,
                        const double* g_epsp, const double* g_kappa, double* g_epsp_n,
                        double* g_kappa_n, hipStream_t st) {
  hipLaunchKernelGGL(k_hist_in_cot, dim3(grid_for(N)), dim3(FFT_THREADS), 0, st, tab, N, c, J,
                     phase, eps, state_n, D, mu, g_sig, lam, g_epsp, g_kappa, g_epsp_n,
                     g_kappa_n);
}

void launch_hist_split(long long n, const double* abar, const double* hist_n,
                       const double* g_hist, double* g_abar, hipStream_t st) {
  hipLaunchKernelGGL(k_hist_split, dim3(grid_for(n)), dim3(FFT_THREADS), 0, st, n, abar, hist_n,
                     g_hist, g_abar);
}

void launch_hist_damage_cot(const MatTable& tab, long long N, int J, const unsigned char* phase,
                            const double* abar, const double* hist_n, const double* zeta,
                            const double* g_hist, double* g_hist_n, hipStream_t st) {
  hipLaunchKernelGGL(k_hist_damage_cot, dim3(grid_for(N)), dim3(FFT_THREADS), 0, st, tab, N, J,
                     phase, abar, hist_n, zeta, g_hist, g_hist_n);
}

void launch_stream_copy(const void* src, void* dst, long long n16, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(FFT_THREADS), 0, st,
                     reinterpret_cast<const uint4*>(src), reinterpret_cast<uint4*>(dst), n16);
}

int launch_diff2(long long n, const double* a, const double* b, double* partials, hipStream_t st) {
  const int nb = grid_for(n);
  hipLaunchKernelGGL(k_diff2, dim3(nb), dim3(FFT_THREADS), 0, st, n, a, b, partials);
  return nb;
}

void launch_axpby(long long n, double a, const double* x, double b, const double* y, double* out,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(FFT_THREADS), 0, st, n, a, x, b, y, out);
}

void launch_commit_hist(const MatTable& tab, long long N, int J, const unsigned char* phase,
                        const double* abar, const double* abar_n, double* hist, hipStream_t st) {
  hipLaunchKernelGGL(k_commit_hist, dim3(grid_for(N)), dim3(FFT_THREADS), 0, st, tab, N, J, phase,
                     abar, abar_n, hist);
}

template <typename TL>
void launch_ell2(const MatTable& tab, long long N, int j, const unsigned char* phase, TL* ell2,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_ell2<TL>, dim3(grid_for(N)), dim3(FFT_THREADS), 0, st, tab, N, j, phase,
                     ell2);
}

int launch_comp_sums(long long N, int ncomp, const double* f, double* partials,
                     hipStream_t st) {
  const int nb = grid_for(N);
  hipLaunchKernelGGL(k_comp_sums, dim3(nb), dim3(FFT_THREADS), 0, st, N, ncomp, f, partials);
  return nb;
}

void launch_add_const(long long N, int ncomp, double* f, const double* delta6, hipStream_t st) {
  Vec6 d;
  for (int i = 0; i < 6; ++i) d.v[i] = i < ncomp ? delta6[i] : 0.0;
  hipLaunchKernelGGL(k_add_const, dim3(grid_for(N)), dim3(FFT_THREADS), 0, st, N, ncomp, f, d);
}

int launch_stagger_err(long long N, int c, int J, const double* en, const double* eo,
                       const double* an, const double* ao, double* partials, hipStream_t st) {
  const int nb = grid_for(N);
  hipLaunchKernelGGL(k_stagger_err, dim3(nb), dim3(FFT_THREADS), 0, st, N, c, J, en, eo, an, ao,
                     partials);
  return nb;
}

void launch_vmax(long long n, double* a, const double* b, hipStream_t st) {
  hipLaunchKernelGGL(k_vmax, dim3(grid_for(n)), dim3(FFT_THREADS), 0, st, n, a, b);
}

template <typename TA, typename TB>
void launch_convert(long long n, const TA* a, TB* b, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<TA, TB>), dim3(grid_for(n)), dim3(FFT_THREADS), 0, st, n, a, b);
}

template <typename TA>
void launch_acc_wide(long long n, const TA* a, double* b, hipStream_t st) {
  hipLaunchKernelGGL((k_acc_wide<TA>), dim3(grid_for(n)), dim3(FFT_THREADS), 0, st, n, a, b);
}
template void launch_acc_wide<float>(long long, const float*, double*, hipStream_t);

int launch_h_refine_resid(const Geo& g, const cpx<double>* b, const cpx<double>* Ap,
                          cpx<float>* r32, double* partials, hipStream_t st, int nsys) {
  const int nb = grid_for(g.Ns);
  hipLaunchKernelGGL(k_h_refine_resid, dim3(nb, nsys), dim3(FFT_THREADS), 0, st, g, b, Ap, r32,
                     partials);
  return nb;
}

template <typename T>
int launch_sum_ell2(long long N, const T* e, double* partials, hipStream_t st, int nsys) {
  const int nb = grid_for(N);
  hipLaunchKernelGGL(k_sum_ell2<T>, dim3(nb, nsys), dim3(FFT_THREADS), 0, st, N, e, partials);
  return nb;
}

// ------------------------------------------------------------ instantiations
#define INST_T(T)                                                                               \
  template void launch_x_r2c<T>(const Plan&, const cpx<T>*, const T*, cpx<T>*, long long, int,  \
                                int, hipStream_t);                                               \
  template void launch_strided<T>(const Plan&, const cpx<T>*, cpx<T>*, long long, long long,     \
                                  long long, long long, bool, const KrylovCtl*, hipStream_t,     \
                                  int, long long);                                               \
  template int launch_gal_dir_inv<T>(const Plan&, const cpx<T>*, const Geo&, int, bool, cpx<T>*, \
                                     cpx<T>*, cpx<T>*, cpx<T>*, KrylovCtl*, hipStream_t, int,    \
                                     int, int, const double*, int);                              \
  template int gal_dot_count<T>(const Plan&, const Geo&, int, bool);                            \
  template int launch_gal_dot_fwd<T>(const Plan&, const cpx<T>*, const Geo&, int, bool,          \
                                     const cpx<T>*, cpx<T>*, double*, const KrylovCtl*,          \
                                     hipStream_t, int);                                          \
  template int launch_gal_resid<T>(const Geo&, int, const Sym<T>&, const unsigned char*,        \
                                    cpx<T>*, const cpx<T>*, double*, KrylovCtl*, hipStream_t,   \
                                    int, int, const double*, int);                               \
  template int launch_gal_rhs<T>(const Geo&, int, const Sym<double>&, const unsigned char*,     \
                                  const double*, const cpx<double>*, cpx<T>*, double*,           \
                                  hipStream_t, int, const double*);                              \
  template void launch_project<T>(const Geo&, int, const Sym<T>&, const unsigned char*, cpx<T>*, \
                                  hipStream_t);                                                  \
  template int launch_h_dir_inv<T>(const Plan&, const cpx<T>*, const Geo&, bool, const Sym<T>&,  \
                                   bool, const cpx<T>*, cpx<T>*, cpx<T>*, cpx<T>*,               \
                                   const KrylovCtl*, hipStream_t, int, double*);                 \
  template int launch_h_fwd_resid<T>(const Plan&, const cpx<T>*, const Geo&, bool,              \
                                     const Sym<T>&, const cpx<T>*, cpx<T>*, cpx<T>*, double*,    \
                                     const KrylovCtl*, hipStream_t, int);                        \
  template int launch_h_div_fwd<T>(const Plan&, const cpx<T>*, const Geo&, bool, const Sym<T>&,  \
                                   const cpx<T>*, cpx<T>*, cpx<T>*, double*, const KrylovCtl*,   \
                                   hipStream_t, int);                                            \
  template void launch_h_y_split<T>(const Plan&, const cpx<T>*, const Geo&, const Sym<T>&,      \
                                    cpx<T>*, bool, const KrylovCtl*, hipStream_t, int);          \
  template int launch_h_resid<T>(const Geo&, const Sym<T>&, bool, cpx<T>*, const cpx<T>*,       \
                                  const cpx<T>*, double*, const KrylovCtl*, hipStream_t, int);   \
  template void launch_xfinal<T>(cpx<T>*, const cpx<T>*, long long, const KrylovCtl*,            \
                                 hipStream_t, int);                                              \
  template void launch_hermitize<T>(const Geo&, int, cpx<T>*, hipStream_t);                     \
  template int launch_wnorm2<T>(const Geo&, int, const cpx<T>*, double*, hipStream_t, int);     \
  template int launch_x_fused_gal<T, T>(const Plan&, const cpx<T>*, const Geo&, int, cpx<T>*,    \
                                        const T*, T, const KrylovCtl*, hipStream_t, int,         \
                                        double*);                                                \
  template int gal_xdot_count<T>(const Geo&, int);                                               \
  template int launch_gal_fwd_resid<T>(const Plan&, const cpx<T>*, const Geo&, int, bool,       \
                                       const Sym<T>&, const unsigned char*, const cpx<T>*,       \
                                       cpx<T>*, double*, const KrylovCtl*, hipStream_t, int);    \
  template int gal_fwd_resid_count<T>(const Plan&, const Geo&, int, bool);                     \
  template int launch_x_fused_helm<T, T>(const Plan&, const cpx<T>*, const Geo&, cpx<T>*,        \
                                         const T*, T, const KrylovCtl*, hipStream_t, int,        \
                                         const unsigned char*, const T*, double*);               \
  template void launch_constitutive<T>(const MatTable&, const Geo&, int, int,                    \
                                       const unsigned char*, const double*, const double*,       \
                                       const double*, double*, double*, double*, T*,             \
                                       hipStream_t);                                             \
  template void launch_ell2<T>(const MatTable&, long long, int, const unsigned char*, T*,        \
                               hipStream_t);                                                     \
  template int launch_sum_ell2<T>(long long, const T*, double*, hipStream_t, int);

INST_T(double)
INST_T(float)

template void launch_x_c2r<double, double>(const Plan&, const cpx<double>*, const cpx<double>*,
                                           double*, long long, int, int, double, bool,
                                           hipStream_t);
template void launch_x_c2r<float, double>(const Plan&, const cpx<float>*, const cpx<float>*,
                                          double*, long long, int, int, float, bool, hipStream_t);
template void launch_x_c2r<float, float>(const Plan&, const cpx<float>*, const cpx<float>*,
                                         float*, long long, int, int, float, bool, hipStream_t);
template void launch_convert<double, float>(long long, const double*, float*, hipStream_t);
template void launch_convert<float, double>(long long, const float*, double*, hipStream_t);

template void launch_grad_comp<double>(const Geo&, const Sym<double>&, int,
                                       const cpx<double>*, cpx<double>*, hipStream_t);
template void launch_tangent_apply<double>(long long, int, const double*, const double*,
                                           const double*, double*, hipStream_t);
template void launch_tangent_apply<float>(long long, int, const float*, const double*,
                                          const double*, double*, hipStream_t);

}  // namespace fftg
