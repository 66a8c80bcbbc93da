// Line-transform kernels shared by the translation units that instantiate
// them: the register-resident radix-8 transforms of one grid axis, as a
// cosine transform (homogeneous Neumann condition, Eq. 7) or as a packed
// real Fourier transform (periodic axis), and the argument block of every
// transform launch.  Included by pc_solve.hip (Neumann axes) and
// pc_solve_per.hip (periodic axes), which each instantiate rad_launch for
// their own boundary condition.
#pragma once

#include <type_traits>

#include "pc_internal.h"

namespace pc {

constexpr int XCDS = 8;
// Workgroup -> tile map that gives each XCD (own L2) a contiguous range of
// tiles, so tiles that share cache lines meet in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  if (nb % XCDS != 0) return b;
  return (b % XCDS) * (nb / XCDS) + b / XCDS;
}

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {  // a * conj(b)
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> conj_(cplx<T> a) { return {a.re, -a.im}; }

// Position of x[n] in Makhoul's reordering v: v[m] = x[2m], v[N-1-m] = x[2m+1].
__device__ __forceinline__ int mk_pos(int n, int N) { return (n & 1) ? (N - 1 - (n >> 1)) : (n >> 1); }

enum { OP_FWD = 0, OP_INV = 1, OP_FDI = 2 };
enum { LD_PLAIN = 0, LD_RESID = 1 };
enum { ST_PLAIN = 0, ST_ACCUM = 1 };

template <typename TC>
struct LineArgs {
  const void* in;       // TI*
  void* out;            // TO*
  const double* rb;     // residual loader: b
  const double* rphi;   // residual loader / accumulating store: phi
  const double* sub;    // nullable: float64 scalar subtracted on load
  const int32_t* skip;  // nullable: the launch does nothing when *skip != 0
  const int32_t* tiles; // nullable: workgroup b transforms tile tiles[b]
  int N, logH;
  int nrad;             // generic kernel: the radices of the half length H
  int rad[24];
  int pad;              // LDS line padding in reals (0 or 2)
  int C;                // lines per tile
  int tx;               // tiles along x (strided axes)
  int axis;             // 0, 1, 2
  int d;
  int perm;             // bit a set: axis a is periodic (residual wrap-around)
  int own_table;        // pseudo-spectral eigenvalues: the generic kernels read
                        // them from tab.lam by slot, the register kernel's FDI
                        // computes lams * m^2 for the slot's mode m
  int32_t n0, n1, n2;
  int64_t lines;        // lines along this axis (vertex-grid kernel: masking)
  double ih2[3];        // 1/h^2 (residual)
  int64_t stride;       // element stride along the axis
  AxisTables<TC> tab;   // tables of this axis
  const TC* lam0;       // FDI: eigenvalues of axis 0 (indexed by i)
  const TC* lam1;       // FDI in 3D: eigenvalues of axis 1 (indexed by j)
  TC outscale;          // store scale
  TC lscale;            // FDI: eigenvalues are multiplied by this (sigma)
  TC lamc;              // FDI: -4 / h^2 of this axis
  TC lams;              // FDI, pseudo-spectral: -(pi / L)^2 (cosine axis) or
                        // -(2 pi / L)^2 (periodic axis), L = n h
  double rscale;        // residual: r = b - rscale * lap_h phi
  double* bmean;        // FDI: receives X(0)/prod(2N_a) from the zero line
  double meannorm;
};

// Global offset of element n of line c in tile t.
template <typename TC>
__device__ __forceinline__ int64_t line_base(const LineArgs<TC>& A, int t, int c, int* i_out,
                                             int* o_out) {
  if (A.axis == 0) {
    int64_t l = (int64_t)t * A.C + c;
    *i_out = 0;
    *o_out = (int)l;
    return l * A.N;
  }
  int i = (t % A.tx) * A.C + c;
  int o = t / A.tx;
  *i_out = i;
  *o_out = o;
  if (A.axis == 1) return (int64_t)i + (int64_t)o * A.n0 * A.n1;  // o = k
  return (int64_t)i + (int64_t)o * A.n0;                          // axis 2: o = j
}

// The float64 residual r = b - rscale * lap_h phi at cell (i, j, k) of flat
// index p.  Neumann axes take the mirror ghost (phi_{-1} = phi_0; on a vertex
// grid, VERTEX, the mirror about the end vertex phi_{-1} = phi_1), periodic
// axes (bit a of perm) wrap around.  Each neighbour's address is selected
// first (the ghost re-reads a point of the line), so all loads are
// unconditional and in flight together.
template <bool VERTEX = false>
__device__ __forceinline__ double resid_ijk(const double* __restrict__ b,
                                            const double* __restrict__ phi, int64_t p, int i,
                                            int j, int k, int d, int32_t n0, int32_t n1,
                                            int32_t n2, int perm, const double* ih2,
                                            double rscale) {
  const int64_t s1 = n0, s2 = (int64_t)n0 * n1;
  constexpr int64_t vx = VERTEX ? 1 : 0;
  const int64_t pxm = i > 0 ? p - 1 : ((perm & 1) ? p + (n0 - 1) : p + vx);
  const int64_t pxp = i < n0 - 1 ? p + 1 : ((perm & 1) ? p - (n0 - 1) : p - vx);
  const int64_t pym = j > 0 ? p - s1 : ((perm & 2) ? p + (n1 - 1) * s1 : p + vx * s1);
  const int64_t pyp = j < n1 - 1 ? p + s1 : ((perm & 2) ? p - (n1 - 1) * s1 : p - vx * s1);
  const double c = phi[p];
  const double xm = phi[pxm], xp = phi[pxp], ym = phi[pym], yp = phi[pyp];
  double lap = ((xp - c) - (c - xm)) * ih2[0] + ((yp - c) - (c - ym)) * ih2[1];
  if (d == 3) {
    const int64_t pzm = k > 0 ? p - s2 : ((perm & 4) ? p + (n2 - 1) * s2 : p + vx * s2);
    const int64_t pzp = k < n2 - 1 ? p + s2 : ((perm & 4) ? p - (n2 - 1) * s2 : p - vx * s2);
    const double zm = phi[pzm], zp = phi[pzp];
    lap += ((zp - c) - (c - zm)) * ih2[2];
  }
  return b[p] - rscale * lap;
}

// The residuals, less sb, of RB points of one line along x (cell grid), at
// x = n + q dn (q < RB) of line c of a tile of C lines whose phi is staged
// in LDS (ph0: line cc at ph0 + cc n0); the line is at (j, k) and starts at
// flat index lb.  The arithmetic of resid_ijk: x neighbours, and y
// neighbours whose line is in the tile, come from LDS; z neighbours, b and
// y neighbours outside the tile from memory.  The dimension is a template
// argument and the y and z offsets are the line's own, so a batch's memory
// loads are issued before the first is used.
template <int D, int RB>
__device__ __forceinline__ void resid_row(const double* __restrict__ b,
                                          const double* __restrict__ phi, const double* ph0,
                                          int c, int C, int64_t lb, int n, int dn, int j, int k,
                                          int32_t n0, int32_t n1, int32_t n2, int perm,
                                          const double* ih2, double rscale, double sb, double* r) {
  const int64_t s1 = n0, s2 = (int64_t)n0 * n1;
  // y neighbour lines as line offsets: -1 / +1 inside, the mirror (0) or the
  // wrap-around at the ends
  const int dym = j > 0 ? -1 : ((perm & 2) ? n1 - 1 : 0);
  const int dyp = j < n1 - 1 ? 1 : ((perm & 2) ? -(n1 - 1) : 0);
  int64_t ozm = 0, ozp = 0;
  if (D == 3) {
    ozm = k > 0 ? -s2 : ((perm & 4) ? (int64_t)(n2 - 1) * s2 : 0);
    ozp = k < n2 - 1 ? s2 : ((perm & 4) ? -(int64_t)(n2 - 1) * s2 : 0);
  }
  const double* ph = ph0 + (int64_t)c * n0;
  const bool in_m = (unsigned)(c + dym) < (unsigned)C, in_p = (unsigned)(c + dyp) < (unsigned)C;
  double cv[RB], xm[RB], xp[RB], ym[RB], yp[RB], zm[RB], zp[RB], bb[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q) {
    const int64_t p = lb + n + q * dn;
    if (D == 3) {
      zm[q] = phi[p + ozm];
      zp[q] = phi[p + ozp];
    }
    bb[q] = b[p];
  }
  if (in_m) {
#pragma unroll
    for (int q = 0; q < RB; ++q) ym[q] = ph[(int64_t)dym * n0 + n + q * dn];
  } else {
#pragma unroll
    for (int q = 0; q < RB; ++q) ym[q] = phi[lb + n + q * dn + dym * s1];
  }
  if (in_p) {
#pragma unroll
    for (int q = 0; q < RB; ++q) yp[q] = ph[(int64_t)dyp * n0 + n + q * dn];
  } else {
#pragma unroll
    for (int q = 0; q < RB; ++q) yp[q] = phi[lb + n + q * dn + dyp * s1];
  }
#pragma unroll
  for (int q = 0; q < RB; ++q) {
    const int i = n + q * dn;
    cv[q] = ph[i];
    xm[q] = ph[i > 0 ? i - 1 : ((perm & 1) ? n0 - 1 : i)];
    xp[q] = ph[i < n0 - 1 ? i + 1 : ((perm & 1) ? 0 : i)];
  }
#pragma unroll
  for (int q = 0; q < RB; ++q) {
    double lap = ((xp[q] - cv[q]) - (cv[q] - xm[q])) * ih2[0] +
                 ((yp[q] - cv[q]) - (cv[q] - ym[q])) * ih2[1];
    if (D == 3) lap += ((zp[q] - cv[q]) - (cv[q] - zm[q])) * ih2[2];
    r[q] = (bb[q] - rscale * lap) - sb;
  }
}

// The same residual at flat index p (coordinates by division).
template <bool VERTEX = false>
__device__ __forceinline__ double resid_at(const double* __restrict__ b,
                                           const double* __restrict__ phi, int64_t p, int d,
                                           int32_t n0, int32_t n1, int32_t n2, int perm,
                                           const double* ih2, double rscale) {
  const int i = (int)(p % n0);
  const int j = (int)((p / n0) % n1);
  const int k = d == 3 ? (int)(p / ((int64_t)n0 * n1)) : 0;
  return resid_ijk<VERTEX>(b, phi, p, i, j, k, d, n0, n1, n2, perm, ih2, rscale);
}

// ---- register-resident radix-8 line transform --------------------------------
// For H = N/2 >= 16, every line is handled by T = H/RT threads (RT = 8
// values per thread); thread t holds the RT complex values a[q] =
// z[t + T q] of the half-length FFT input.  The Stockham stages are radix 8
// followed by one stage of the remaining radix: every stage reads only the
// thread's own values and scatters its outputs through LDS (the last stage
// is in place), so a radix-8 FFT of 1024 points costs three LDS exchanges.
// The real-FFT split needs Z[H-k] next to Z[k] (one exchange); the fused
// forward/divide/inverse exchanges the divided spectrum once more for the
// inverse split, which needs slots H-k and H+k next to k and N-k.

template <typename TC, bool INV>
__device__ __forceinline__ void dft4(cplx<TC>& a0, cplx<TC>& a1, cplx<TC>& a2, cplx<TC>& a3) {
  cplx<TC> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
  cplx<TC> it3 = INV ? cplx<TC>{-t3.im, t3.re} : cplx<TC>{t3.im, -t3.re};
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, it3);
  a3 = csub(t1, it3);
}

// multiply by exp(-+ 2 pi i m / 16) for the constant m (sign by INV)
template <typename TC, bool INV, int m>
__device__ __forceinline__ cplx<TC> w16(cplx<TC> a) {
  constexpr double C1 = 0.92387953251128675613;  // cos(pi/8)
  constexpr double S1 = 0.38268343236508977173;  // sin(pi/8)
  constexpr double R2 = 0.70710678118654752440;  // sqrt(1/2)
  double c, s;  // w = c - i s (forward)
  if (m == 0) return a;
  if (m == 1) { c = C1; s = S1; }
  if (m == 2) { c = R2; s = R2; }
  if (m == 3) { c = S1; s = C1; }
  if (m == 4) {  // -i (forward) / +i (inverse)
    return INV ? cplx<TC>{-a.im, a.re} : cplx<TC>{a.im, -a.re};
  }
  if (m == 6) { c = -R2; s = R2; }
  if (m == 9) { c = -C1; s = -S1; }
  cplx<TC> w = {(TC)c, INV ? (TC)s : (TC)-s};
  return cmul(a, w);
}

template <typename TC, bool INV>
__device__ __forceinline__ void dft8(cplx<TC>* a) {  // a[0..7], natural order in and out
  dft4<TC, INV>(a[0], a[2], a[4], a[6]);
  dft4<TC, INV>(a[1], a[3], a[5], a[7]);
  // B1[k1] at a[2 k1 + 1] times W8^k1
  a[3] = w16<TC, INV, 2>(a[3]);
  a[5] = w16<TC, INV, 4>(a[5]);
  a[7] = w16<TC, INV, 6>(a[7]);
  cplx<TC> o[8];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    o[k1] = cadd(a[2 * k1], a[2 * k1 + 1]);
    o[k1 + 4] = csub(a[2 * k1], a[2 * k1 + 1]);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = o[i];
}

// DFT of length 3 and 5 (forward exp(-2 pi i / r), inverse the conjugate).
template <typename TC, bool INV>
__device__ __forceinline__ void dft3(cplx<TC>* v) {
  constexpr double S3 = 0.86602540378443864676;  // sin(2 pi / 3)
  const cplx<TC> t = cadd(v[1], v[2]);
  const cplx<TC> m = {v[0].re - TC(0.5) * t.re, v[0].im - TC(0.5) * t.im};
  const cplx<TC> d = {TC(S3) * (v[1].re - v[2].re), TC(S3) * (v[1].im - v[2].im)};
  const cplx<TC> id = INV ? cplx<TC>{-d.im, d.re} : cplx<TC>{d.im, -d.re};  // -+ i d
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, id);
  v[2] = csub(m, id);
}

template <typename TC, bool INV>
__device__ __forceinline__ void dft5(cplx<TC>* v) {
  constexpr double C1 = 0.30901699437494742410;   // cos(2 pi / 5)
  constexpr double C2 = -0.80901699437494742410;  // cos(4 pi / 5)
  constexpr double S1 = 0.95105651629515357212;   // sin(2 pi / 5)
  constexpr double S2 = 0.58778525229247312917;   // sin(4 pi / 5)
  const cplx<TC> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  const cplx<TC> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  const cplx<TC> a1 = {v[0].re + TC(C1) * t1.re + TC(C2) * t2.re,
                       v[0].im + TC(C1) * t1.im + TC(C2) * t2.im};
  const cplx<TC> a2 = {v[0].re + TC(C2) * t1.re + TC(C1) * t2.re,
                       v[0].im + TC(C2) * t1.im + TC(C1) * t2.im};
  const cplx<TC> b1 = {TC(S1) * t3.re + TC(S2) * t4.re, TC(S1) * t3.im + TC(S2) * t4.im};
  const cplx<TC> b2 = {TC(S2) * t3.re - TC(S1) * t4.re, TC(S2) * t3.im - TC(S1) * t4.im};
  // -+ i b
  const cplx<TC> ib1 = INV ? cplx<TC>{-b1.im, b1.re} : cplx<TC>{b1.im, -b1.re};
  const cplx<TC> ib2 = INV ? cplx<TC>{-b2.im, b2.re} : cplx<TC>{b2.im, -b2.re};
  v[0] = cadd(v[0], cadd(t1, t2));
  v[1] = cadd(a1, ib1);
  v[4] = csub(a1, ib1);
  v[2] = cadd(a2, ib2);
  v[3] = csub(a2, ib2);
}

// DFT of length 10 (natural order in and out) as two of length 5: E and O
// over the even and odd inputs, X[k] = E[k] + W10^k O[k] and
// X[k+5] = E[k] - W10^k O[k], W10 = exp(-+2 pi i / 10).
template <typename TC, bool INV>
__device__ __forceinline__ void dft10(cplx<TC>* a) {
  constexpr double C1 = 0.80901699437494742410;  // cos(pi/5)
  constexpr double S1 = 0.58778525229247312917;  // sin(pi/5)
  constexpr double C2 = 0.30901699437494742410;  // cos(2 pi/5)
  constexpr double S2 = 0.95105651629515357212;  // sin(2 pi/5)
  cplx<TC> e[5], o[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    e[i] = a[2 * i];
    o[i] = a[2 * i + 1];
  }
  dft5<TC, INV>(e);
  dft5<TC, INV>(o);
  // W10^k = c_k -+ i s_k for k = 1..4 (s_k >= 0)
  const TC sg = INV ? TC(1) : TC(-1);
  const cplx<TC> w1 = {(TC)C1, sg * (TC)S1}, w2 = {(TC)C2, sg * (TC)S2},
                 w3 = {(TC)-C2, sg * (TC)S2}, w4 = {(TC)-C1, sg * (TC)S1};
  o[1] = cmul(o[1], w1);
  o[2] = cmul(o[2], w2);
  o[3] = cmul(o[3], w3);
  o[4] = cmul(o[4], w4);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    a[k] = cadd(e[k], o[k]);
    a[k + 5] = csub(e[k], o[k]);
  }
}

template <typename TC, bool INV, int R>
__device__ __forceinline__ void dftR(cplx<TC>* a) {
  if (R == 10) dft10<TC, INV>(a);
  if (R == 5) dft5<TC, INV>(a);
  if (R == 8) dft8<TC, INV>(a);
  if (R == 4) dft4<TC, INV>(a[0], a[1], a[2], a[3]);
  if (R == 2) {
    cplx<TC> x0 = a[0], x1 = a[1];
    a[0] = cadd(x0, x1);
    a[1] = csub(x0, x1);
  }
}

// Load of a table entry whose address is the same in every lane, through
// the scalar data cache (read only): the value lands in scalar registers
// instead of occupying vector registers and a vector memory slot.
template <typename TC>
__device__ __forceinline__ cplx<TC> ldu(const cplx<TC>* p) {
  const __attribute__((address_space(4))) TC* q = (const __attribute__((address_space(4))) TC*)(p);
  return {q[0], q[1]};
}

// LDS index of complex element i of a line (one pad slot per 16).
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
// lpad(t + T q) from lt = lpad(t): linear in q when T is a multiple of 16
template <int T>
__device__ __forceinline__ int lpad_tq(int t, int lt, int q) {
  if constexpr (T % 16 == 0)
    return lt + q * (T + T / 16);
  else
    return lpad(t + T * q);
}
// lpad(base + r L) from lb = lpad(base), for the Stockham scatter of the
// register kernels: base mod 16 plus r L mod 16 stays below 16 there
// (L = 1 with base a multiple of the radix, or k < 8 with L = 8, or L a
// multiple of 16), so the pad of base + r L is the pad of base plus that
// of r L.
__device__ __forceinline__ int lpad_scatter(int lb, int rl) { return lb + rl + (rl >> 4); }

// Synchronisation of the threads of one line.  When T divides 64 a line
// lies inside one wavefront, whose LDS accesses execute in issue order, so
// wavefront-scope fences (compiler ordering only) are enough; longer lines,
// and lines of a T that does not divide 64 (the radix-10 plan), span
// several wavefronts and need the workgroup barrier.
template <int T>
__device__ __forceinline__ void line_sync() {
  if (T <= 64 && 64 % T == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// ---- radix-8 plan (8 values per thread, T = H/8 threads per line) -------------
// Radix-8 Stockham stages (the values of a stage are the thread's own; the
// outputs scatter through LDS) and one final stage of radix 2 or 4.  A
// radix-16 plan (half the threads per line, fewer stages) was measured no
// faster in float64 and slower in the mixed mode, where its residual pass
// held twice the registers.

// Twiddle state of the radix-8 plan: the stage bases w = exp(-+2 pi i k/(8L))
// for the stages with L = 8 and L = 64 (k = t mod L), and twH[t] for the
// final stage; loaded once per launch.
template <typename TC>
struct R8Tw {
  cplx<TC> s1, s2, fin;
};

// v[r] *= w^r, r = 1..7, with the powers built by squaring (each power is at
// most three products away from w).
template <typename TC, bool INV>
__device__ __forceinline__ void twiddle_r8(cplx<TC>* v, cplx<TC> w) {
  const cplx<TC> w2 = cmul(w, w);
  const cplx<TC> w4 = cmul(w2, w2);
  const cplx<TC> w3 = cmul(w2, w);
  cplx<TC> p[8];
  p[1] = w;
  p[2] = w2;
  p[3] = w3;
  p[4] = w4;
  p[5] = cmul(w4, w);
  p[6] = cmul(w4, w2);
  p[7] = cmul(w4, w3);
#pragma unroll
  for (int r = 1; r < 8; ++r) v[r] = INV ? cmulc(v[r], p[r]) : cmul(v[r], p[r]);
}

// One radix-8 Stockham stage with sub-transform length L on the thread's 8
// values: butterfly j = t, k = t mod L, inputs at j + T r (the thread's own
// values), twiddles w^(k r), an 8-point DFT, outputs to (j - k) 8 + k + r L
// through LDS and back as the next stage's inputs (in place for the last).
template <typename TC, bool INV, bool LAST, int T>
__device__ __forceinline__ void r8_stage(cplx<TC>* a, int t, int L, cplx<TC> w, cplx<TC>* z) {
  cplx<TC> v[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = a[r];
  if (L > 1) twiddle_r8<TC, INV>(v, w);
  dft8<TC, INV>(v);
  if (LAST) {
#pragma unroll
    for (int r = 0; r < 8; ++r) a[r] = v[r];
  } else {
    const int k = t & (L - 1);
    const int lb = lpad((t - k) * 8 + k);
#pragma unroll
    for (int r = 0; r < 8; ++r) z[lpad_scatter(lb, r * L)] = v[r];
    line_sync<T>();
    const int lt = lpad(t);
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = z[lpad_tq<T>(t, lt, q)];
    line_sync<T>();
  }
}

// The final stage of radix R < RT on a thread holding RT values (always in
// place: butterflies j = t + T b, b < RT/R, with k = j).
template <typename TC, bool INV, int RT, int R>
__device__ __forceinline__ void rad_final(cplx<TC>* a, int T, cplx<TC> fin,
                                          const cplx<TC>* __restrict__ twH) {
  constexpr int NB = RT / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    cplx<TC> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a[b + NB * r];
    const cplx<TC> w = b ? cmul(fin, ldu(twH + T * b)) : fin;  // twH[t + T b]
    cplx<TC> wr = w;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      v[r] = INV ? cmulc(v[r], wr) : cmul(v[r], wr);
      if (r + 1 < R) wr = cmul(wr, w);
    }
    dftR<TC, INV, R>(v);
#pragma unroll
    for (int r = 0; r < R; ++r) a[b + NB * r] = v[r];
  }
}

template <typename TC, bool INV, int LOGH>
__device__ __forceinline__ void r8_fft(cplx<TC>* a, int t, const R8Tw<TC>& tw,
                                       const cplx<TC>* __restrict__ twH, cplx<TC>* z) {
  constexpr int H = 1 << LOGH;
  constexpr int T = H / 8;
  constexpr int S8 = LOGH / 3;         // radix-8 stages (1 to 3 for 16 <= H <= 2048)
  constexpr int RR = 1 << (LOGH % 3);  // final radix (1: none)
  static_assert(S8 >= 1 && S8 <= 3, "radix-8 plan covers 16 <= H <= 2048");
  r8_stage<TC, INV, (S8 == 1 && RR == 1), T>(a, t, 1, tw.s1, z);
  if (S8 >= 2) r8_stage<TC, INV, (S8 == 2 && RR == 1), T>(a, t, 8, tw.s1, z);
  if (S8 >= 3) r8_stage<TC, INV, (RR == 1), T>(a, t, 64, tw.s2, z);
  if (RR == 4) rad_final<TC, INV, 8, 4>(a, T, tw.fin, twH);
  if (RR == 2) rad_final<TC, INV, 8, 2>(a, T, tw.fin, twH);
}

// ---- radix-10 plan (10 values per thread, T = H/10 threads per line) ----------
// For H = 10^s f with f = 1, 2 or 5 (the n/2 = 200 and 1000 of the 400 and
// 2000 point grids of Sec. 3): s radix-10 Stockham stages (L = 1, 10, 100),
// then, for f > 1, a final in-place stage of radix f.  The twiddle state
// (R8Tw) holds the stage bases for L = 10 (s1) and L = 100 (s2) and twH[t]
// (fin).  LDS indices carry one pad slot per 16 complex values (lpad).

template <int H>
struct R10Plan {
  static constexpr int S = H % 1000 == 0 ? 3 : (H % 100 == 0 ? 2 : 1);  // radix-10 stages
  static constexpr int F = H / (S == 3 ? 1000 : (S == 2 ? 100 : 10));    // final radix
  static_assert(F == 1 || F == 2 || F == 5, "H = 10^s f with f in {1, 2, 5}");
};

// v[r] *= w^r, r = 1..9, the powers by products of at most four factors.
template <typename TC, bool INV>
__device__ __forceinline__ void twiddle_r10(cplx<TC>* v, cplx<TC> w) {
  cplx<TC> p[10];
  p[1] = w;
  p[2] = cmul(w, w);
  p[3] = cmul(p[2], w);
  p[4] = cmul(p[2], p[2]);
  p[5] = cmul(p[4], w);
  p[6] = cmul(p[3], p[3]);
  p[7] = cmul(p[6], w);
  p[8] = cmul(p[4], p[4]);
  p[9] = cmul(p[8], w);
#pragma unroll
  for (int r = 1; r < 10; ++r) v[r] = INV ? cmulc(v[r], p[r]) : cmul(v[r], p[r]);
}

// One radix-10 Stockham stage of sub-transform length L: butterfly j = t,
// k = t mod L, inputs the thread's own values (j + T r), twiddles w^(k r),
// a 10-point DFT, outputs to (j - k) 10 + k + r L through LDS and back as
// the next stage's inputs t + T q (in place for the last stage).
template <typename TC, bool INV, bool LAST, int T, int L>
__device__ __forceinline__ void r10_stage(cplx<TC>* a, int t, cplx<TC> w, cplx<TC>* z) {
  cplx<TC> v[10];
#pragma unroll
  for (int r = 0; r < 10; ++r) v[r] = a[r];
  if (L > 1) twiddle_r10<TC, INV>(v, w);
  dft10<TC, INV>(v);
  if (LAST) {
#pragma unroll
    for (int r = 0; r < 10; ++r) a[r] = v[r];
  } else {
    const int k = t % L;
    const int b = (t - k) * 10 + k;
#pragma unroll
    for (int r = 0; r < 10; ++r) z[lpad(b + r * L)] = v[r];
    line_sync<T>();
#pragma unroll
    for (int q = 0; q < 10; ++q) a[q] = z[lpad(t + T * q)];
    line_sync<T>();
  }
}

template <typename TC, bool INV, int H>
__device__ __forceinline__ void r10_fft(cplx<TC>* a, int t, const R8Tw<TC>& tw,
                                        const cplx<TC>* __restrict__ twH, cplx<TC>* z) {
  constexpr int T = H / 10;
  constexpr int S = R10Plan<H>::S, F = R10Plan<H>::F;
  r10_stage<TC, INV, (S == 1 && F == 1), T, 1>(a, t, tw.s1, z);
  if constexpr (S >= 2) r10_stage<TC, INV, (S == 2 && F == 1), T, 10>(a, t, tw.s1, z);
  if constexpr (S >= 3) r10_stage<TC, INV, (F == 1), T, 100>(a, t, tw.s2, z);
  if constexpr (F == 2) rad_final<TC, INV, 10, 2>(a, T, tw.fin, twH);
  if constexpr (F == 5) rad_final<TC, INV, 10, 5>(a, T, tw.fin, twH);
}

// The register kernels' half-length H from the length code HL of their
// template: log2(H) for the radix-8 plan, H itself for the radix-10 plan.
template <int HL, int RT>
struct RadLen {
  static constexpr int H = RT == 8 ? (1 << HL) : HL;
};

// Twiddle state of either plan for thread t of a line.
template <typename TC, int H, int RT>
__device__ __forceinline__ R8Tw<TC> rad_twiddles(const cplx<TC>* __restrict__ twH, int t) {
  R8Tw<TC> tw;
  if constexpr (RT == 8) {
    if (H >= 64) tw.s1 = twH[(H / 64) * (t & 7)];
    if (H >= 512) tw.s2 = twH[(H / 512) * (t & 63)];
    if (__builtin_ctz(H) % 3) tw.fin = twH[t];
  } else {
    constexpr int S = R10Plan<H>::S, F = R10Plan<H>::F;
    if (S >= 2) tw.s1 = twH[(H / 100) * (t % 10)];
    if (S >= 3) tw.s2 = twH[(H / 1000) * (t % 100)];
    if (F > 1) tw.fin = twH[t];
  }
  return tw;
}

template <typename TC, bool INV, int H, int RT>
__device__ __forceinline__ void rad_fft(cplx<TC>* a, int t, const R8Tw<TC>& tw8,
                                        const cplx<TC>* __restrict__ twH, cplx<TC>* z) {
  static_assert(RT == 8 || RT == 10, "the register kernels run radix-8 or radix-10 plans");
  if constexpr (RT == 8)
    r8_fft<TC, INV, __builtin_ctz(H)>(a, t, tw8, twH, z);
  else
    r10_fft<TC, INV, H>(a, t, tw8, twH, z);
}

// exp(-i pi (H-k) / (2N)) = exp(-i pi / 4) conj(exp(-i pi k / (2N))), N = 2H
template <typename TC>
__device__ __forceinline__ cplx<TC> t4n_mirror(cplx<TC> w) {
  const TC r = (TC)0.70710678118654752440;
  return {r * (w.re - w.im), -r * (w.re + w.im)};
}

// Inverse pre-processing of the own index k (see pre_pair): from X[k],
// X[N-k], X[H-k], X[H+k] and the shift twiddles of k, returns Z[k].
template <typename TC>
__device__ __forceinline__ cplx<TC> pre_own(TC xk, TC xnk, TC xhk, TC xhpk, cplx<TC> w4, cplx<TC> wN) {
  cplx<TC> Yk = {xk * TC(0.5), -xnk * TC(0.5)};
  cplx<TC> Yj = {xhk * TC(0.5), -xhpk * TC(0.5)};
  cplx<TC> Vk = cmulc(Yk, w4);
  cplx<TC> Vj = cmulc(Yj, t4n_mirror(w4));
  cplx<TC> Vjc = conj_(Vj);
  cplx<TC> E = {(Vk.re + Vjc.re) * TC(0.5), (Vk.im + Vjc.im) * TC(0.5)};
  cplx<TC> D = {(Vk.re - Vjc.re) * TC(0.5), (Vk.im - Vjc.im) * TC(0.5)};
  cplx<TC> O = cmulc(D, wN);
  return {E.re - O.im, E.im + O.re};
}

// Inverse pre-processing of the packed real DFT for the own index k: from
// slots k, N-k (Re, Im of X_k), H-k and H+k (Re, Im of X_{H-k}) returns
// Z[k] of the half-length inverse FFT, whose unscaled output z[m] holds
// H (x[2m] + i x[2m+1]).  For k = 0 the caller passes slot 0, 0, slot H, 0
// (X_0 and X_H are real).
template <typename TC>
__device__ __forceinline__ cplx<TC> pre_own_per(TC xk, TC xnk, TC xhk, TC xhpk, cplx<TC> wN) {
  // Z[k] = E + i O with E = (X_k + conj X_{H-k}) / 2 and
  // O = (X_k - conj X_{H-k}) conj(w_N^k) / 2, the even/odd split of X
  cplx<TC> E = {(xk + xhk) * TC(0.5), (xnk - xhpk) * TC(0.5)};
  cplx<TC> D = {(xk - xhk) * TC(0.5), (xnk + xhpk) * TC(0.5)};
  cplx<TC> O = cmulc(D, wN);
  return {E.re - O.im, E.im + O.re};
}

// pre_own and pre_own_per without their halvings: 4 Z[k] (cosine) and
// 2 Z[k] (real DFT); the register kernel folds the factor into its output
// scale (a power of two, so exact), with eight (four) multiplies fewer per
// value.
template <typename TC>
__device__ __forceinline__ cplx<TC> pre_own_x4(TC xk, TC xnk, TC xhk, TC xhpk, cplx<TC> w4,
                                               cplx<TC> wN) {
  cplx<TC> Yk = {xk, -xnk};
  cplx<TC> Yj = {xhk, -xhpk};
  cplx<TC> Vk = cmulc(Yk, w4);
  cplx<TC> Vj = cmulc(Yj, t4n_mirror(w4));
  cplx<TC> Vjc = conj_(Vj);
  cplx<TC> E = {Vk.re + Vjc.re, Vk.im + Vjc.im};
  cplx<TC> D = {Vk.re - Vjc.re, Vk.im - Vjc.im};
  cplx<TC> O = cmulc(D, wN);
  return {E.re - O.im, E.im + O.re};
}

template <typename TC>
__device__ __forceinline__ cplx<TC> pre_own_per_x2(TC xk, TC xnk, TC xhk, TC xhpk, cplx<TC> wN) {
  cplx<TC> E = {xk + xhk, xnk - xhpk};
  cplx<TC> D = {xk - xhk, xnk + xhpk};
  cplx<TC> O = cmulc(D, wN);
  return {E.re - O.im, E.im + O.re};
}

// Position of the line's element n in the half-length FFT input (reals):
// Makhoul's order for the cosine transform, the natural order for the real
// DFT (z[m] = x[2m] + i x[2m+1]).
template <bool PER>
__device__ __forceinline__ int line_pos(int n, int N) { return PER ? n : mk_pos(n, N); }

// Position of real v[p] (Makhoul order) in the line: x[2p] or x[2(N-1-p)+1].
__device__ __forceinline__ int mk_src(int p, int N) { return p < N / 2 ? 2 * p : 2 * (N - 1 - p) + 1; }
// LDS real index of v[p] (complex slot lpad(p/2), component p&1).
__device__ __forceinline__ int vpad(int p) { return 2 * lpad(p >> 1) + (p & 1); }
// LDS real index of X[r] (two pad slots per 32 reals).
__device__ __forceinline__ int xpad(int r) { return r + 2 * (r >> 5); }

// One pass of the line transforms over a tile of C lines: forward (OP_FWD),
// inverse (OP_INV), or forward, division by the eigenvalues and inverse
// along the last axis (OP_FDI).  RT = 8 (radix-8 plan) or 10 (radix-10
// plan) complex values per thread, T = H / RT threads per line.
//   PER = false: DCT-II forward, DCT-III / (2N) inverse (Neumann axis).
//   PER = true:  packed real DFT of a periodic axis, in the same slots:
//                slot k = Re X_k (k < H), slot N-k = Im X_k (0 < k < H),
//                slot H = X_H; the inverse is the exact inverse.
// Both leave the line's modes in slots whose 1D eigenvalue is a function of
// the slot index (see the FDI step), so the passes of different axes
// combine freely.
// The kernel asks for four wavefronts per SIMD (at most 128 VGPRs), which
// the float64 fused pass would otherwise exceed by a few registers.
template <typename TC, typename TI, typename TO, int OP, int LD, int ST, int HL, int RT,
          bool PER>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
dct_rad(LineArgs<TC> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (A.skip && *A.skip) return;
  constexpr int H = RadLen<HL, RT>::H;
  constexpr int N = 2 * H;
  constexpr int T = H / RT;
  constexpr int NV = 2 * RT;  // reals per thread
  constexpr int RB = NV % 8 == 0 ? 8 : 10;  // points per batch of the residual loader
  static_assert(NV % RB == 0, "residual batches cover the thread's points");
  const int LS = H + H / 16 + 1;  // complex slots per line in LDS
  const int C = A.C;
  const bool rows = A.axis == 0;
  const int tile = A.tiles ? A.tiles[blockIdx.x] : (rows ? blockIdx.x : xcd_tile(blockIdx.x, gridDim.x));
  // the T threads of a line are consecutive (one wavefront for T <= 64)
  const int c = threadIdx.x / T;
  const int t = threadIdx.x - c * T;
  cplx<TC>* z = reinterpret_cast<cplx<TC>*>(smem_raw) + c * LS;
  TC* const zr0 = reinterpret_cast<TC*>(smem_raw);  // line cc at zr0 + 2 * cc * LS
  // Strided passes move the C-line tile cooperatively: element e of the
  // tile is line e % C, position e / C, so each access covers C adjacent
  // lines (C * sizeof element contiguous bytes).
  int64_t lbase[1];
  {
    int li0, lo0;
    lbase[0] = line_base(A, tile, 0, &li0, &lo0);  // line cc is at lbase + cc (x-adjacent)
  }
  TC* zr = reinterpret_cast<TC*>(z);
  int li, lo;
  const int64_t lb = line_base(A, tile, c, &li, &lo);
  const int64_t st = A.stride;
  const TI* __restrict__ in = reinterpret_cast<const TI*>(A.in);
  TO* __restrict__ out = reinterpret_cast<TO*>(A.out);
  const AxisTables<TC>& Tb = A.tab;

  // twiddle state (issued first; in flight with the data loads)
  R8Tw<TC> tw8 = rad_twiddles<TC, H, RT>(Tb.twH, t);
  const cplx<TC> tNb = Tb.tN[t];
  const cplx<TC> t4b = Tb.t4N[t];

  // coordinates of this line's cells for the residual (rows: x varies)
  const int lj = rows ? lo % A.n1 : 0, lk = rows ? lo / A.n1 : 0;
  auto load = [&](int n) -> TC {
    int64_t p = lb + (int64_t)n * st;
    if (LD == LD_RESID) {
      double r = resid_ijk(A.rb, A.rphi, p, n, lj, lk, A.d, A.n0, A.n1, A.n2, A.perm, A.ih2, A.rscale);
      if (A.sub) r -= *A.sub;
      return (TC)r;
    } else if (A.sub) {
      return (TC)((double)in[p] - *A.sub);
    }
    return (TC)in[p];
  };

  // Strided passes move the tile cooperatively.  Thread x takes line
  // cc = x % C at positions n = x / C + r T, r < NV (C T threads, N = NV T
  // positions per line), so each access covers C adjacent lines; all NV
  // loads are issued before the first is used.
  const int tcc = threadIdx.x & (C - 1);
  const int tn0 = threadIdx.x >> __builtin_ctz(C);
  // value of position n of line tcc goes to real index pos(n) of its LDS region
  auto tile_load = [&](auto pos) {
    const int64_t p0 = lbase[0] + tcc + (int64_t)tn0 * st;
    int ti_x = 0, to = 0;
    if (LD == LD_RESID) line_base(A, tile, tcc, &ti_x, &to);
    const int64_t dp = (int64_t)T * st;
    TC* zl = zr0 + 2 * tcc * LS;
    if (LD == LD_RESID) {
      // the residual reads 5-7 values per point: batches of RB points (RB
      // divides NV), the batch loop kept rolled so that the kernel stays small
#pragma unroll 1
      for (int r0 = 0; r0 < NV; r0 += RB) {
        TC v[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          // strided line along axis 1 (y) or 2 (z) at x position ti_x, the
          // other coordinate to
          const int pn = tn0 + (r0 + r) * T;
          const int cj = A.axis == 1 ? pn : to, ck = A.axis == 1 ? to : pn;
          double x = resid_ijk(A.rb, A.rphi, p0 + (r0 + r) * dp, ti_x, cj, ck, A.d, A.n0, A.n1,
                               A.n2, A.perm, A.ih2, A.rscale);
          if (A.sub) x -= *A.sub;
          v[r] = (TC)x;
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) zl[pos(tn0 + (r0 + r) * T)] = v[r];
      }
    } else {
      TC v[NV];
      const TI* src = in + p0;
      if (A.sub) {
        const double sb = *A.sub;
#pragma unroll
        for (int r = 0; r < NV; ++r) v[r] = (TC)((double)src[r * dp] - sb);
      } else {
#pragma unroll
        for (int r = 0; r < NV; ++r) v[r] = (TC)src[r * dp];
      }
#pragma unroll
      for (int r = 0; r < NV; ++r) zl[pos(tn0 + r * T)] = v[r];
    }
    __syncthreads();
  };

  cplx<TC> a[RT];
  if (OP != OP_INV) {
    if (rows && LD == LD_RESID) {
      // phi of the tile's C lines (C N contiguous doubles) is staged in LDS
      // once, so that a point reads 3-5 values from memory instead of 6-8;
      // the float residuals stay in registers until every thread is done
      // with the staged lines, which the transform's LDS area overlaps
      double* const ph0 = reinterpret_cast<double*>(smem_raw);
      {
        const int CT = C * T;
        const double* src = A.rphi + lbase[0];
#pragma unroll
        for (int r = 0; r < NV; ++r) ph0[threadIdx.x + r * CT] = src[threadIdx.x + r * CT];
      }
      __syncthreads();
      const double sb = A.sub ? *A.sub : 0.0;  // r - 0 is r exactly
      TC rv[NV];
      auto rows_resid = [&](auto dim) {
        constexpr int D = decltype(dim)::value;
        constexpr int RR = 4;
        static_assert(NV % RR == 0, "residual batches cover the thread's points");
#pragma unroll
        for (int i0 = 0; i0 < NV; i0 += RR) {
          double rb4[RR];
          resid_row<D, RR>(A.rb, A.rphi, ph0, c, C, lb, t + T * i0, T, lj, lk, A.n0, A.n1, A.n2,
                           A.perm, A.ih2, A.rscale, sb, rb4);
#pragma unroll
          for (int i = 0; i < RR; ++i) rv[i0 + i] = (TC)rb4[i];
        }
      };
      if (A.d == 3)
        rows_resid(std::integral_constant<int, 3>{});
      else
        rows_resid(std::integral_constant<int, 2>{});
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NV; ++i) zr[vpad(line_pos<PER>(t + T * i, N))] = rv[i];
      line_sync<T>();
    } else if (rows) {
      // coalesced loads, reordered into Makhoul order through LDS
      TC xv[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) xv[i] = load(t + T * i);
#pragma unroll
      for (int i = 0; i < NV; ++i) zr[vpad(line_pos<PER>(t + T * i, N))] = xv[i];
      line_sync<T>();
    } else {
      tile_load([&](int n) { return vpad(line_pos<PER>(n, N)); });
    }
#pragma unroll
    for (int q = 0; q < RT; ++q) a[q] = z[lpad_tq<T>(t, lpad(t), q)];
    line_sync<T>();
    rad_fft<TC, false, H, RT>(a, t, tw8, Tb.twH, z);
    // partner exchange: Z[H-k] next to Z[k]
#pragma unroll
    for (int q = 0; q < RT; ++q) z[lpad_tq<T>(t, lpad(t), q)] = a[q];
    line_sync<T>();
    TC rest = TC(0), x0 = TC(0);
    if (OP == OP_FDI) {
      rest = A.lam0[li];
      if (A.lam1) rest += A.lam1[lo];
    }
    const TC lc = A.lamc, ls_ = A.lscale;
    TC ya[RT], yb[RT];  // own X[k] and X[N-k] (X[H] for k = 0), divided in FDI
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      const int k = t + T * q;
      cplx<TC> Zk = a[q];
      cplx<TC> Zc = conj_(z[lpad(RT == 8 ? (H - k) & (H - 1) : (k ? H - k : 0))]);
      // twice the even/odd split E, D (and O = -i D): the cosine transform's
      // factor 2 absorbs the halving (scaling by powers of two is exact; the
      // results differ from halving first only where the compiler fuses
      // multiply-adds differently), with multiplies fewer
      cplx<TC> E2 = {Zk.re + Zc.re, Zk.im + Zc.im};
      cplx<TC> D2 = {Zk.re - Zc.re, Zk.im - Zc.im};
      cplx<TC> O2 = {D2.im, -D2.re};
      const cplx<TC> wN = q ? cmul(tNb, ldu(Tb.tN + T * q)) : tNb;   // tN[k]
      const cplx<TC> w4 = q ? cmul(t4b, ldu(Tb.t4N + T * q)) : t4b;  // t4N[k]
      cplx<TC> WO2 = cmul(wN, O2);
      TC xa, xb;  // slots k and N-k; for k = 0 slots 0 and H
      if (PER) {
        // X_k = E + w_N^k O; X_H = E_0 - O_0
        cplx<TC> V2 = cadd(E2, WO2);
        xa = TC(0.5) * V2.re;
        xb = TC(0.5) * (k ? V2.im : csub(E2, WO2).re);
      } else {
        // X[k] = 2 Re Y, X[N-k] = -2 Im Y with Y = t4N[k] (E + w_N^k O)
        cplx<TC> Y2 = cmul(w4, cadd(E2, WO2));
        xa = Y2.re;
        xb = -Y2.im;  // X[N-k]; for k = 0 replaced by X[H]
        if (k == 0) {
          cplx<TC> Yh2 = cmul(t4n_mirror(w4), conj_(csub(E2, WO2)));
          xb = Yh2.re;
        }
      }
      if (OP == OP_FWD) {
        ya[q] = xa;
        yb[q] = xb;
      } else {
        // divide by the summed eigenvalues.  Cosine transform: the 1D
        // eigenvalue of slot j is -(4/h^2) sin^2(pi j / (2N)), with
        // sin(pi k/2N) = -Im w4, cos = Re w4, and slot H (k = 0) has
        // sin^2 = 1/2.  Real DFT: slots k and N-k both hold mode k, of
        // eigenvalue -(4/h^2) sin^2(pi k / N) = -(4/h^2) 4 sin^2 cos^2 of
        // pi k / (2N), and slot H (k = 0) has sin^2 = 1.  Pseudo-spectral:
        // lams m^2 for the slot's mode m (slot k: mode k; slot N-k: mode N-k
        // on a cosine axis, k on a periodic one; slot H: mode H).  Both are
        // scale * s^2 with per-slot s, picked by selects: a branch per slot
        // (or per-slot table loads) costs the kernel half its occupancy.
        const bool own = A.own_table;
        TC sa, sb;
        if (PER) {
          sa = TC(2) * w4.re * w4.im;
          sb = sa;
        } else {
          sa = w4.im;
          sb = w4.re;
        }
        if (own) {
          sa = (TC)k;
          sb = (TC)(PER ? k : N - k);
        }
        const TC scale = own ? A.lams : lc;
        const TC e_a = scale * (sa * sa);
        TC e_b = scale * (sb * sb);
        if (k == 0) e_b = own ? A.lams * (TC(H) * TC(H)) : (PER ? lc : lc * TC(0.5));
        TC l_a = (rest + e_a) * ls_;
        TC l_b = (rest + e_b) * ls_;
        if (k == 0) x0 = xa;
        if constexpr (sizeof(TC) == 4) {
          // float32: the hardware reciprocal (1 ulp) instead of the
          // correctly rounded division sequence, about ten instructions
          // each; the quotient is within 2 ulp
          ya[q] = l_a != TC(0) ? xa * __builtin_amdgcn_rcpf(l_a) : TC(0);
          yb[q] = xb * __builtin_amdgcn_rcpf(l_b);
        } else {
          ya[q] = l_a != TC(0) ? xa / l_a : TC(0);
          yb[q] = xb / l_b;
        }
      }
    }
    if (OP == OP_FWD) {
      if (rows) {
#pragma unroll
        for (int q = 0; q < RT; ++q) {
          const int k = t + T * q;
          out[lb + (int64_t)k * st] = (TO)ya[q];
          out[lb + (int64_t)(k ? N - k : H) * st] = (TO)yb[q];
        }
      } else {
        line_sync<T>();
#pragma unroll
        for (int q = 0; q < RT; ++q) {
          const int k = t + T * q;
          zr[xpad(k)] = ya[q];
          zr[xpad(k ? N - k : H)] = yb[q];
        }
        __syncthreads();
        TO* dst = out + lbase[0] + tcc + (int64_t)tn0 * st;
        const TC* zl = zr0 + 2 * tcc * LS;
#pragma unroll
        for (int r = 0; r < NV; ++r) dst[(int64_t)r * T * st] = (TO)zl[xpad(tn0 + r * T)];
      }
      return;
    }
    // the zero line's mode 0 is sum(b) * prod(c_a N_a) (c_a = 2 for a cosine
    // axis, 1 for a periodic axis): the compatibility defect
    if (t == 0 && rest == TC(0) && A.bmean) *A.bmean = (double)x0 * A.meannorm;
    line_sync<T>();
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      const int k = t + T * q;
      zr[xpad(k)] = ya[q];
      zr[xpad(k ? N - k : H)] = yb[q];
    }
    line_sync<T>();
    // opaque copies of the base twiddles: the compiler would otherwise keep
    // the forward split's 2 RT twiddle products live through the division
    // and exchange (twice the registers of the data) instead of redoing them
    cplx<TC> tNi = tNb, t4i = t4b;
    asm volatile("" : "+v"(tNi.re), "+v"(tNi.im), "+v"(t4i.re), "+v"(t4i.im));
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      const int k = t + T * q;
      const cplx<TC> wN = q ? cmul(tNi, ldu(Tb.tN + T * q)) : tNi;
      const cplx<TC> w4 = q ? cmul(t4i, ldu(Tb.t4N + T * q)) : t4i;
      TC xhk = zr[xpad(H - k)];
      TC xhpk = zr[xpad(H + k)];
      if (PER)
        a[q] = pre_own_per_x2(ya[q], k ? yb[q] : TC(0), xhk, k ? xhpk : TC(0), wN);
      else
        a[q] = pre_own_x4(ya[q], k ? yb[q] : TC(0), xhk, xhpk, w4, wN);
    }
    line_sync<T>();
  } else {
    // X in natural order: own X[k], X[N-k] and the partners' via LDS
    TC xk[RT], xn[RT];
    if (rows) {
#pragma unroll
      for (int q = 0; q < RT; ++q) {
        int k = t + T * q;
        xk[q] = load(k);
        xn[q] = load(k ? N - k : H);
      }
#pragma unroll
      for (int q = 0; q < RT; ++q) {
        int k = t + T * q;
        zr[xpad(k)] = xk[q];
        zr[xpad(k ? N - k : H)] = xn[q];
      }
      line_sync<T>();
    } else {
      tile_load([&](int n) { return xpad(n); });
#pragma unroll
      for (int q = 0; q < RT; ++q) {
        int k = t + T * q;
        xk[q] = zr[xpad(k)];
        xn[q] = zr[xpad(k ? N - k : H)];
      }
    }
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      const int k = t + T * q;
      const cplx<TC> wN = q ? cmul(tNb, ldu(Tb.tN + T * q)) : tNb;
      const cplx<TC> w4 = q ? cmul(t4b, ldu(Tb.t4N + T * q)) : t4b;
      TC xhk = zr[xpad(H - k)];
      TC xhpk = zr[xpad(H + k)];
      if (PER)
        a[q] = pre_own_per_x2(xk[q], k ? xn[q] : TC(0), xhk, k ? xhpk : TC(0), wN);
      else
        a[q] = pre_own_x4(xk[q], k ? xn[q] : TC(0), xhk, xhpk, w4, wN);
    }
    line_sync<T>();
  }

  // inverse half-length FFT, then unpack v -> x.  Opaque copies of the
  // thread index and LDS base keep the compiler from carrying the forward
  // FFT's address arithmetic live into this second FFT.
  if constexpr (OP == OP_FDI) {
    // opaque twiddle state: otherwise the forward FFT's twiddle powers stay
    // live through the division for reuse (as conjugates) in the inverse,
    // which halves the occupancy
    asm volatile("" : "+v"(tw8.s1.re), "+v"(tw8.s1.im), "+v"(tw8.s2.re), "+v"(tw8.s2.im));
    asm volatile("" : "+v"(tw8.fin.re), "+v"(tw8.fin.im));
  }
  int ti = t, zoff = c * LS;
  asm volatile("" : "+v"(ti));
  asm volatile("" : "+v"(zoff));
  // from the LDS base itself, so that the accesses stay LDS instructions
  cplx<TC>* zi = reinterpret_cast<cplx<TC>*>(smem_raw) + zoff;
  rad_fft<TC, true, H, RT>(a, ti, tw8, Tb.twH, zi);
  const TC sc = A.outscale * (PER ? TC(0.5) : TC(0.25));  // undoes pre_own*_x2/_x4
  // The stores hit the same addresses as the loads; opaque copies of the
  // line base and stride make the compiler recompute them here instead of
  // keeping them live through the whole kernel.
  int64_t lb2 = lb, st2 = st;
  int t2 = t;
  asm volatile("" : "+v"(lb2));
  asm volatile("" : "+s"(st2));
  asm volatile("" : "+v"(t2));
  auto put = [&](int64_t p, TC v) {
    if (ST == ST_ACCUM) {
      double* o = reinterpret_cast<double*>(A.out);
      o[p] = A.rphi[p] + (double)v;
    } else {
      out[p] = (TO)v;
    }
  };
#pragma unroll
  for (int q = 0; q < RT; ++q) zi[lpad_tq<T>(ti, lpad(ti), q)] = {a[q].re * sc, a[q].im * sc};
  if (rows) {
    // back to natural order through LDS, then coalesced stores
    line_sync<T>();
    TC* zri = reinterpret_cast<TC*>(zi);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int n = t2 + T * i;
      put(lb2 + (int64_t)n * st2, zri[vpad(line_pos<PER>(n, N))]);
    }
  } else {
    __syncthreads();
    const int64_t p0 = lbase[0] + tcc + (int64_t)tn0 * st2;
    const TC* zl = zr0 + 2 * tcc * LS;
#pragma unroll
    for (int r = 0; r < NV; ++r)
      put(p0 + (int64_t)r * T * st2, zl[vpad(line_pos<PER>(tn0 + r * T, N))]);
  }
}

// Launches dct_rad<..., PER> for the transform length and radix of `key`
// (HL * 32 + RT, HL = log2(H) for RT = 8 and H for RT = 10) on `grid`
// workgroups of `block` threads.
template <typename TC, typename TI, typename TO, int OP, int LD, int ST, bool PER>
int rad_launch(const LineArgs<TC>& A, int key, dim3 grid, dim3 block, size_t lds,
               hipStream_t s) {
  const void* fn = nullptr;
  switch (key) {
#define PC_RAD_CASE(LH, R) \
    case LH * 32 + R: fn = (const void*)dct_rad<TC, TI, TO, OP, LD, ST, LH, R, PER>; break;
    PC_RAD_CASE(4, 8) PC_RAD_CASE(5, 8) PC_RAD_CASE(6, 8) PC_RAD_CASE(7, 8)
    PC_RAD_CASE(8, 8) PC_RAD_CASE(9, 8) PC_RAD_CASE(10, 8) PC_RAD_CASE(11, 8)
    PC_RAD_CASE(100, 10) PC_RAD_CASE(200, 10) PC_RAD_CASE(500, 10) PC_RAD_CASE(1000, 10)
#undef PC_RAD_CASE
    default: return fail(PC_ERR_UNSUPPORTED_SIZE, "transform length");
  }
  if (lds > 65536)
    PC_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  switch (key) {
#define PC_RAD_LAUNCH(LH, R) \
    case LH * 32 + R: \
      hipLaunchKernelGGL((dct_rad<TC, TI, TO, OP, LD, ST, LH, R, PER>), grid, block, lds, s, A); \
      break;
    PC_RAD_LAUNCH(4, 8) PC_RAD_LAUNCH(5, 8) PC_RAD_LAUNCH(6, 8) PC_RAD_LAUNCH(7, 8)
    PC_RAD_LAUNCH(8, 8) PC_RAD_LAUNCH(9, 8) PC_RAD_LAUNCH(10, 8) PC_RAD_LAUNCH(11, 8)
    PC_RAD_LAUNCH(100, 10) PC_RAD_LAUNCH(200, 10) PC_RAD_LAUNCH(500, 10) PC_RAD_LAUNCH(1000, 10)
#undef PC_RAD_LAUNCH
  }
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

// The (compute, input, output, operation, loader, store) combinations the
// solves launch: float64; float32; float32 transforms between float64
// fields (defect correction: plain and residual loads, plain and
// accumulating stores).
#define PC_RAD_COMBOS(X)                                  \
  X(double, double, double, OP_FWD, LD_PLAIN, ST_PLAIN)   \
  X(double, double, double, OP_FDI, LD_PLAIN, ST_PLAIN)   \
  X(double, double, double, OP_INV, LD_PLAIN, ST_PLAIN)   \
  X(float, float, float, OP_FWD, LD_PLAIN, ST_PLAIN)      \
  X(float, float, float, OP_FDI, LD_PLAIN, ST_PLAIN)      \
  X(float, float, float, OP_INV, LD_PLAIN, ST_PLAIN)      \
  X(float, double, float, OP_FWD, LD_PLAIN, ST_PLAIN)     \
  X(float, float, double, OP_INV, LD_PLAIN, ST_PLAIN)     \
  X(float, double, float, OP_FWD, LD_RESID, ST_PLAIN)     \
  X(float, float, double, OP_INV, LD_PLAIN, ST_ACCUM)

// Declares (EXTERN) or instantiates (INST) the periodic-axis launchers,
// which live in their own translation unit.
#define PC_RAD_EXTERN_PER(TC, TI, TO, OP, LD, ST)                                    \
  extern template int rad_launch<TC, TI, TO, OP, LD, ST, true>(                      \
      const LineArgs<TC>&, int, dim3, dim3, size_t, hipStream_t);
#define PC_RAD_INST_PER(TC, TI, TO, OP, LD, ST)                                      \
  template int rad_launch<TC, TI, TO, OP, LD, ST, true>(const LineArgs<TC>&, int, dim3, \
                                                        dim3, size_t, hipStream_t);

}  // namespace pc
