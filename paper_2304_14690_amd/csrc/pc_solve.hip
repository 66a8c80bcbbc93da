// Neumann-box Poisson solve by cosine transforms (Sec. 2.3, three-step
// transform algorithm; homogeneous Neumann condition of Eq. 7 on every box
// face, cell-centred grid, central-difference eigenvalues).
//
// Each 1D cosine transform of length N is computed through a complex FFT of
// length H = N/2 (Makhoul's even/odd reordering, the real-FFT split and a
// quarter-sample shift), staged in LDS:
//   DCT-II   X[k] = 2 sum_n x[n] cos(pi k (2n+1) / (2N))
//   inverse  x = DCT-III(X) / (2N), the exact inverse of the above.
// One kernel launch transforms every line of the grid along one axis.  A
// workgroup holds C lines; along x the lines are whole rows, along y/z the C
// lines are adjacent in x so that each global access touches C contiguous
// elements.  The last axis fuses forward transform, division by the summed
// eigenvalues and inverse transform in registers, so a 2D solve is three
// passes over the grid and a 3D solve five.
#include <cmath>

#include "pc_internal.h"

namespace pc {

namespace {

constexpr int XCDS = 8;
// Radix-16 transform tiles: threads per workgroup for contiguous rows, and
// the thread cap for the strided (column/pencil) passes.
constexpr int ROW_THREADS = 256;
constexpr int COL_MAX_THREADS = 512;

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
  int pad;              // LDS line padding in reals (0 or 2)
  int C;                // lines per tile
  int tx;               // tiles along x (strided axes)
  int axis;             // 0, 1, 2
  int d;
  int32_t n0, n1, n2;
  double ih2[3];        // 1/h^2 (residual)
  int64_t stride;       // element stride along the axis
  AxisTables<TC> tab;   // tables of this axis
  const TC* lam0;       // FDI: eigenvalues of axis 0 (indexed by i)
  const TC* lam1;       // FDI in 3D: eigenvalues of axis 1 (indexed by j)
  TC outscale;          // store scale
  TC lscale;            // FDI: eigenvalues are multiplied by this (sigma)
  TC lamc;              // FDI: -4 / h^2 of this axis
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

// Residual r = b - lap_h phi at flat index p (mirror ghosts), float64.
__device__ __forceinline__ double resid_at(const double* __restrict__ b,
                                           const double* __restrict__ phi, int64_t p, int d,
                                           int32_t n0, int32_t n1, int32_t n2, const double* ih2,
                                           double rscale) {
  int64_t s1 = n0, s2 = (int64_t)n0 * n1;
  int i = (int)(p % n0);
  int j = (int)((p / n0) % n1);
  int k = d == 3 ? (int)(p / s2) : 0;
  double c = phi[p];
  double xm = i > 0 ? phi[p - 1] : c;
  double xp = i < n0 - 1 ? phi[p + 1] : c;
  double ym = j > 0 ? phi[p - s1] : c;
  double yp = j < n1 - 1 ? phi[p + s1] : c;
  double lap = ((xp - c) - (c - xm)) * ih2[0] + ((yp - c) - (c - ym)) * ih2[1];
  if (d == 3) {
    double zm = k > 0 ? phi[p - s2] : c;
    double zp = k < n2 - 1 ? phi[p + s2] : c;
    lap += ((zp - c) - (c - zm)) * ih2[2];
  }
  return b[p] - rscale * lap;
}

// The same residual at cell (i, j, k) of flat index p, with the coordinates
// known to the caller (no divisions).
__device__ __forceinline__ double resid_ijk(const double* __restrict__ b,
                                            const double* __restrict__ phi, int64_t p, int i,
                                            int j, int k, int d, int32_t n0, int32_t n1,
                                            int32_t n2, const double* ih2, double rscale) {
  const int64_t s1 = n0, s2 = (int64_t)n0 * n1;
  double c = phi[p];
  double xm = i > 0 ? phi[p - 1] : c;
  double xp = i < n0 - 1 ? phi[p + 1] : c;
  double ym = j > 0 ? phi[p - s1] : c;
  double yp = j < n1 - 1 ? phi[p + s1] : c;
  double lap = ((xp - c) - (c - xm)) * ih2[0] + ((yp - c) - (c - ym)) * ih2[1];
  if (d == 3) {
    double zm = k > 0 ? phi[p - s2] : c;
    double zp = k < n2 - 1 ? phi[p + s2] : c;
    lap += ((zp - c) - (c - zm)) * ih2[2];
  }
  return b[p] - rscale * lap;
}

// Radix-4 / radix-2 Stockham FFT of the C lines held in LDS (complex view,
// line c at zc + c*ls).  B butterflies per thread per radix-4 stage.
template <typename TC, int B, bool INV>
__device__ __forceinline__ void fft_lds(cplx<TC>* zc, int ls, int C, int H, int logH,
                                        const cplx<TC>* __restrict__ twH, int tid, int nthr) {
  int L = 1;
  int rem = logH;
  while (rem > 0) {
    if (rem >= 2) {
      const int nb = H >> 2;  // butterflies per line
      cplx<TC> a[B][4];
      int pos[B];
      int lc[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        int bi = tid + b * nthr;
        lc[b] = -1;
        if (bi < C * nb) {
          int c = bi / nb;
          int j = bi - c * nb;
          int k = j & (L - 1);
          cplx<TC>* z = zc + c * ls;
          int tstep = (H / (L * 4)) * k;
#pragma unroll
          for (int r = 0; r < 4; ++r) a[b][r] = z[j + r * nb];
#pragma unroll
          for (int r = 1; r < 4; ++r) {
            cplx<TC> w = twH[tstep * r];
            a[b][r] = INV ? cmulc(a[b][r], w) : cmul(a[b][r], w);
          }
          cplx<TC> t0 = cadd(a[b][0], a[b][2]), t1 = csub(a[b][0], a[b][2]);
          cplx<TC> t2 = cadd(a[b][1], a[b][3]), t3 = csub(a[b][1], a[b][3]);
          // -i*t3 (forward) or +i*t3 (inverse)
          cplx<TC> it3 = INV ? cplx<TC>{-t3.im, t3.re} : cplx<TC>{t3.im, -t3.re};
          a[b][0] = cadd(t0, t2);
          a[b][2] = csub(t0, t2);
          a[b][1] = cadd(t1, it3);
          a[b][3] = csub(t1, it3);
          lc[b] = c;
          pos[b] = (j - k) * 4 + k;
        }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if (lc[b] >= 0) {
          cplx<TC>* z = zc + lc[b] * ls;
#pragma unroll
          for (int r = 0; r < 4; ++r) z[pos[b] + r * L] = a[b][r];
        }
      }
      __syncthreads();
      L <<= 2;
      rem -= 2;
    } else {
      const int nb = H >> 1;
      cplx<TC> a[2 * B][2];
      int pos[2 * B];
      int lc[2 * B];
#pragma unroll
      for (int b = 0; b < 2 * B; ++b) {
        int bi = tid + b * nthr;
        lc[b] = -1;
        if (bi < C * nb) {
          int c = bi / nb;
          int j = bi - c * nb;
          int k = j & (L - 1);
          cplx<TC>* z = zc + c * ls;
          cplx<TC> x0 = z[j], x1 = z[j + nb];
          cplx<TC> w = twH[(H / (L * 2)) * k];
          x1 = INV ? cmulc(x1, w) : cmul(x1, w);
          a[b][0] = cadd(x0, x1);
          a[b][1] = csub(x0, x1);
          lc[b] = c;
          pos[b] = (j - k) * 2 + k;
        }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < 2 * B; ++b) {
        if (lc[b] >= 0) {
          cplx<TC>* z = zc + lc[b] * ls;
          z[pos[b]] = a[b][0];
          z[pos[b] + L] = a[b][1];
        }
      }
      __syncthreads();
      L <<= 1;
      rem -= 1;
    }
  }
}

// Forward post-processing of pair k (0 <= k <= H/2) of one line: from the
// half-length FFT Z produce X[k], X[N-k], X[H-k], X[H+k].
template <typename TC>
__device__ __forceinline__ void post_pair(const cplx<TC>* z, int k, int N, int H,
                                          const AxisTables<TC>& T, TC* xk, TC* xnk, TC* xhk,
                                          TC* xhpk) {
  cplx<TC> Zk = z[k];
  cplx<TC> Zc = conj_(z[(H - k) & (H - 1)]);
  cplx<TC> E = {(Zk.re + Zc.re) * TC(0.5), (Zk.im + Zc.im) * TC(0.5)};
  cplx<TC> D = {(Zk.re - Zc.re) * TC(0.5), (Zk.im - Zc.im) * TC(0.5)};
  cplx<TC> O = {D.im, -D.re};  // -i * D
  cplx<TC> WO = cmul(T.tN[k], O);
  cplx<TC> Vk = cadd(E, WO);
  cplx<TC> Vj = conj_(csub(E, WO));  // V[H-k]
  cplx<TC> Y = cmul(T.t4N[k], Vk);
  cplx<TC> Yj = cmul(T.t4N[H - k], Vj);
  *xk = TC(2) * Y.re;
  *xnk = TC(-2) * Y.im;   // X[N-k] (meaningless for k = 0)
  *xhk = TC(2) * Yj.re;   // X[H-k]
  *xhpk = TC(-2) * Yj.im; // X[H+k] = X[N-(H-k)]
}

// Inverse pre-processing of pair k: from X[k], X[N-k], X[H-k], X[H+k]
// (X[N] = 0) produce Z[k] and Z[H-k] of the half-length inverse FFT.
template <typename TC>
__device__ __forceinline__ void pre_pair(TC xk, TC xnk, TC xhk, TC xhpk, int k, int H,
                                         const AxisTables<TC>& T, cplx<TC>* Zk, cplx<TC>* Zhk) {
  cplx<TC> Yk = {xk * TC(0.5), -xnk * TC(0.5)};
  cplx<TC> Yj = {xhk * TC(0.5), -xhpk * TC(0.5)};
  cplx<TC> Vk = cmulc(Yk, T.t4N[k]);
  cplx<TC> Vj = cmulc(Yj, T.t4N[H - k]);
  cplx<TC> Vjc = conj_(Vj);
  cplx<TC> E = {(Vk.re + Vjc.re) * TC(0.5), (Vk.im + Vjc.im) * TC(0.5)};
  cplx<TC> D = {(Vk.re - Vjc.re) * TC(0.5), (Vk.im - Vjc.im) * TC(0.5)};
  cplx<TC> O = cmulc(D, T.tN[k]);
  *Zk = {E.re - O.im, E.im + O.re};      // E + i O
  *Zhk = {E.re + O.im, -E.im + O.re};    // conj(E) + i conj(O)
}

template <typename TC, typename TI, typename TO, int OP, int LD, int ST, int B>
__global__ void __launch_bounds__(1024) dct_lines(LineArgs<TC> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (A.skip && *A.skip) return;
  TC* s = reinterpret_cast<TC*>(smem_raw);
  const int N = A.N, H = N >> 1, C = A.C;
  const int ls = N + A.pad;  // line stride in LDS (reals)
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int t = A.axis == 0 ? blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
  const TI* __restrict__ in = reinterpret_cast<const TI*>(A.in);
  TO* __restrict__ out = reinterpret_cast<TO*>(A.out);

  // ---- load ----------------------------------------------------------------
  for (int e = tid; e < C * N; e += nthr) {
    int c, n;
    if (A.axis == 0) { c = e / N; n = e - c * N; } else { n = e / C; c = e - n * C; }
    int i, o;
    int64_t p = line_base(A, t, c, &i, &o) + (int64_t)n * A.stride;
    TC v;
    if (LD == LD_RESID) {
      double r = resid_at(A.rb, A.rphi, p, A.d, A.n0, A.n1, A.n2, A.ih2, A.rscale);
      if (A.sub) r -= *A.sub;
      v = (TC)r;
    } else if (A.sub) {
      v = (TC)((double)in[p] - *A.sub);
    } else {
      v = (TC)in[p];
    }
    int q = (OP == OP_INV) ? n : mk_pos(n, N);
    s[c * ls + q] = v;
  }
  __syncthreads();

  cplx<TC>* zc = reinterpret_cast<cplx<TC>*>(s);
  const int lsc = ls >> 1;
  const int npair = H / 2 + 1;

  if (OP == OP_INV) {
    // pre-process pairs into Z (in place through registers)
    constexpr int PB = 2 * B + 1;  // pairs per thread: C*(H/2+1) <= (2B+1)*nthr
    cplx<TC> zk[PB], zh[PB];
    int ck[PB], kk[PB];
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      int w = tid + b * nthr;
      ck[b] = -1;
      if (w < C * npair) {
        int c = w / npair, k = w - c * npair;
        const TC* x = s + c * ls;
        TC xk = x[k], xnk = k ? x[N - k] : TC(0), xhk = x[H - k], xhpk = x[H + k];
        pre_pair(xk, xnk, xhk, xhpk, k, H, A.tab, &zk[b], &zh[b]);
        ck[b] = c;
        kk[b] = k;
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      if (ck[b] >= 0) {
        cplx<TC>* z = zc + ck[b] * lsc;
        int k = kk[b];
        z[k] = zk[b];
        if (k != 0 && k != H - k) z[H - k] = zh[b];
      }
    }
    __syncthreads();
    fft_lds<TC, B, true>(zc, lsc, C, H, A.logH, A.tab.twH, tid, nthr);
  } else {
    fft_lds<TC, B, false>(zc, lsc, C, H, A.logH, A.tab.twH, tid, nthr);
    constexpr int PB = 2 * B + 1;
    TC xa[PB], xb[PB], xc[PB], xd[PB];
    int ck[PB], kk[PB];
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      int w = tid + b * nthr;
      ck[b] = -1;
      if (w < C * npair) {
        int c = w / npair, k = w - c * npair;
        post_pair(zc + c * lsc, k, N, H, A.tab, &xa[b], &xb[b], &xc[b], &xd[b]);
        ck[b] = c;
        kk[b] = k;
      }
    }
    if (OP == OP_FDI) {
      // divide by the summed eigenvalues, then inverse pre-processing
      cplx<TC> zk[PB], zh[PB];
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        if (ck[b] >= 0) {
          int c = ck[b], k = kk[b];
          int i, o;
          (void)line_base(A, t, c, &i, &o);
          TC rest = A.lam0[i];
          if (A.lam1) rest += A.lam1[o];
          const TC* lam = A.tab.lam;
          const TC ls_ = A.lscale;
          TC l0 = (rest + lam[k]) * ls_, l1 = (rest + lam[(N - k) & (N - 1)]) * ls_,
             l2 = (rest + lam[H - k]) * ls_, l3 = (rest + lam[H + k]) * ls_;
          if (k == 0) {
            if (rest == TC(0) && A.bmean) *A.bmean = (double)xa[b] * A.meannorm;
            l1 = TC(1);
          }
          TC y0 = l0 != TC(0) ? xa[b] / l0 : TC(0);
          TC y1 = xb[b] / l1;
          TC y2 = xc[b] / l2;
          TC y3 = xd[b] / l3;
          if (k == 0) y1 = TC(0);
          pre_pair(y0, y1, y2, y3, k, H, A.tab, &zk[b], &zh[b]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        if (ck[b] >= 0) {
          cplx<TC>* z = zc + ck[b] * lsc;
          int k = kk[b];
          z[k] = zk[b];
          if (k != 0 && k != H - k) z[H - k] = zh[b];
        }
      }
      __syncthreads();
      fft_lds<TC, B, true>(zc, lsc, C, H, A.logH, A.tab.twH, tid, nthr);
    } else {
      __syncthreads();
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        if (ck[b] >= 0) {
          TC* x = s + ck[b] * ls;
          int k = kk[b];
          x[k] = xa[b];
          if (k != 0) x[N - k] = xb[b];
          if (k != H / 2 || H == 1) x[H - k] = xc[b];
          if (k != 0 && k != H / 2) x[H + k] = xd[b];
        }
      }
      __syncthreads();
    }
  }

  // ---- store ----------------------------------------------------------------
  for (int e = tid; e < C * N; e += nthr) {
    int c, n;
    if (A.axis == 0) { c = e / N; n = e - c * N; } else { n = e / C; c = e - n * C; }
    int i, o;
    int64_t p = line_base(A, t, c, &i, &o) + (int64_t)n * A.stride;
    int q = (OP == OP_FWD) ? n : mk_pos(n, N);
    TC v = s[c * ls + q] * A.outscale;
    if (ST == ST_ACCUM) {
      reinterpret_cast<double*>(A.out)[p] = A.rphi[p] + (double)v;
    } else {
      out[p] = (TO)v;
    }
  }
}

// ---- register-resident radix-16 line transform ------------------------------
// For H = N/2 >= 16, every line is handled by T = H/16 threads; thread t holds
// the 16 complex values a[q] = z[t + T q] of the half-length FFT input.  The
// Stockham stages are radix 16 followed by one stage of radix 2^(log2 H mod
// 4): every stage reads only the thread's own values, scatters its outputs
// through LDS (the last stage is in place), so an FFT of 1024 points costs
// two LDS exchanges.  The cosine-transform split needs Z[H-k] next to Z[k]
// (one exchange); the fused forward/divide/inverse then recomputes the
// partner's outputs instead of exchanging them again.

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
__device__ __forceinline__ void dft16(cplx<TC>* a) {
  // n = 4 n1 + n2, k = k1 + 4 k2
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<TC, INV>(a[n2], a[4 + n2], a[8 + n2], a[12 + n2]);
  // a[4 k1 + n2] *= W16^(n2 k1)
  a[5] = w16<TC, INV, 1>(a[5]);
  a[6] = w16<TC, INV, 2>(a[6]);
  a[7] = w16<TC, INV, 3>(a[7]);
  a[9] = w16<TC, INV, 2>(a[9]);
  a[10] = w16<TC, INV, 4>(a[10]);
  a[11] = w16<TC, INV, 6>(a[11]);
  a[13] = w16<TC, INV, 3>(a[13]);
  a[14] = w16<TC, INV, 6>(a[14]);
  a[15] = w16<TC, INV, 9>(a[15]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<TC, INV>(a[4 * k1], a[4 * k1 + 1], a[4 * k1 + 2], a[4 * k1 + 3]);
  // a[4 k1 + k2] = A[k1 + 4 k2]: transpose to natural order
  cplx<TC> o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = a[4 * k1 + k2];
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = o[i];
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

template <typename TC, bool INV, int R>
__device__ __forceinline__ void dftR(cplx<TC>* a) {
  if (R == 16) dft16<TC, INV>(a);
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

// Synchronisation of the threads of one line.  A line of T <= 64 threads
// lies inside one wavefront, whose LDS accesses execute in issue order, so
// wavefront-scope fences (compiler ordering only) are enough; longer lines
// span several wavefronts and need the workgroup barrier.
template <int T>
__device__ __forceinline__ void line_sync() {
  if (T <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Per-thread twiddle state of the radix-16 FFT, loaded once per launch so
// that no table load sits on the critical path of a stage:
//   the radix-16 stage with L = 16: butterfly j = t, k = t mod 16; the
//   factors w^(r k) come from w^k and w^(4k) by at most two products;
//   the final stage of radix R < 16: butterflies j = t + T b with k = j, and
//   w^k = w^t w^(T b) where w^(T b) is the same for the whole wavefront.
template <typename TC>
struct R16Tw {
  cplx<TC> w1, w4;  // radix-16 stage with L = 16
  cplx<TC> fin;     // final stage: twH[t]
};

template <typename TC>
__device__ __forceinline__ void twiddle_r16(cplx<TC>* v, cplx<TC> w1, cplx<TC> w4, bool inv) {
  cplx<TC> p[4], q4[4];
  p[0] = {TC(1), TC(0)};
  p[1] = w1;
  p[2] = cmul(w1, w1);
  p[3] = cmul(p[2], w1);
  q4[0] = {TC(1), TC(0)};
  q4[1] = w4;
  q4[2] = cmul(w4, w4);
  q4[3] = cmul(q4[2], w4);
#pragma unroll
  for (int r = 1; r < 16; ++r) {
    cplx<TC> w = (r >> 2) == 0 ? p[r & 3] : ((r & 3) == 0 ? q4[r >> 2] : cmul(q4[r >> 2], p[r & 3]));
    v[r] = inv ? cmulc(v[r], w) : cmul(v[r], w);
  }
}

// One radix-16 Stockham stage (L = 1 or 16) on the thread's 16 values.
// LAST: outputs stay in the thread's own slots; otherwise they go through
// the line's LDS region z and come back in the z[t + T q] layout.
template <typename TC, bool INV, bool LAST, int T>
__device__ __forceinline__ void r16_stage16(cplx<TC>* a, int t, int L, const R16Tw<TC>& tw,
                                            cplx<TC>* z) {
  cplx<TC> v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = a[r];
  if (L > 1) twiddle_r16(v, tw.w1, tw.w4, INV);
  dft16<TC, INV>(v);
  if (LAST) {
#pragma unroll
    for (int r = 0; r < 16; ++r) a[r] = v[r];
  } else {
    const int k = t & (L - 1);
    const int base = (t - k) * 16 + k;
#pragma unroll
    for (int r = 0; r < 16; ++r) z[lpad(base + r * L)] = v[r];
    line_sync<T>();
#pragma unroll
    for (int q = 0; q < 16; ++q) a[q] = z[lpad(t + T * q)];
    line_sync<T>();
  }
}

// The final stage of radix R < 16 (always in place: L = H / R > j).
template <typename TC, bool INV, int R>
__device__ __forceinline__ void r16_final(cplx<TC>* a, int T, const R16Tw<TC>& tw,
                                          const cplx<TC>* __restrict__ twH) {
  constexpr int NB = 16 / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    cplx<TC> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a[b + NB * r];
    const cplx<TC> w = b ? cmul(tw.fin, ldu(twH + T * b)) : tw.fin;  // twH[t + T b]
    cplx<TC> wr = w;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      v[r] = INV ? cmulc(v[r], wr) : cmul(v[r], wr);
      if (r + 1 < R) wr = cmul(wr, w);  // w^(r+1)
    }
    dftR<TC, INV, R>(v);
#pragma unroll
    for (int r = 0; r < R; ++r) a[b + NB * r] = v[r];
  }
}

template <typename TC, bool INV, int LOGH>
__device__ __forceinline__ void r16_fft(cplx<TC>* a, int t, const R16Tw<TC>& tw,
                                        const cplx<TC>* __restrict__ twH, cplx<TC>* z) {
  constexpr int H = 1 << LOGH;
  constexpr int T = H / 16;
  constexpr int S16 = LOGH / 4;        // radix-16 stages (1 or 2 for H <= 2048)
  constexpr int RR = 1 << (LOGH % 4);  // final radix (1: none)
  static_assert(S16 >= 1 && S16 <= 2, "radix-16 plan covers 16 <= H <= 2048");
  r16_stage16<TC, INV, (S16 == 1 && RR == 1), T>(a, t, 1, tw, z);
  if (S16 == 2) r16_stage16<TC, INV, (RR == 1), T>(a, t, 16, tw, z);
  if (RR == 8) r16_final<TC, INV, 8>(a, T, tw, twH);
  if (RR == 4) r16_final<TC, INV, 4>(a, T, tw, twH);
  if (RR == 2) r16_final<TC, INV, 2>(a, T, tw, twH);
}

// ---- radix-8 plan (8 values per thread, T = H/8 threads per line) -------------
// Used where a pass has few lines (a 2D grid): twice the threads per line of
// the radix-16 plan, so twice the wavefronts to hide latency with.

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
// values (butterfly j = t, k = t mod L, inputs at j + T r, outputs at
// (j - k) 8 + k + r L); see r16_stage16.
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
    const int base = (t - k) * 8 + k;
#pragma unroll
    for (int r = 0; r < 8; ++r) z[lpad(base + r * L)] = v[r];
    line_sync<T>();
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = z[lpad(t + T * q)];
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

template <typename TC, bool INV, int LOGH, int RT>
__device__ __forceinline__ void rad_fft(cplx<TC>* a, int t, const R16Tw<TC>& tw,
                                        const R8Tw<TC>& tw8, const cplx<TC>* __restrict__ twH,
                                        cplx<TC>* z) {
  if constexpr (RT == 16)
    r16_fft<TC, INV, LOGH>(a, t, tw, twH, z);
  else
    r8_fft<TC, INV, LOGH>(a, t, tw8, twH, z);
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

// Position of real v[p] (Makhoul order) in the line: x[2p] or x[2(N-1-p)+1].
__device__ __forceinline__ int mk_src(int p, int N) { return p < N / 2 ? 2 * p : 2 * (N - 1 - p) + 1; }
// LDS real index of v[p] (complex slot lpad(p/2), component p&1).
__device__ __forceinline__ int vpad(int p) { return 2 * lpad(p >> 1) + (p & 1); }
// LDS real index of X[r] (two pad slots per 32 reals).
__device__ __forceinline__ int xpad(int r) { return r + 2 * (r >> 5); }

// One pass of the cosine transforms over a tile of C lines: forward DCT-II
// (OP_FWD), inverse DCT-III (OP_INV), or forward, division by the
// eigenvalues and inverse along the last axis (OP_FDI).  RT complex values
// per thread (16 or 8), T = H / RT threads per line.
template <typename TC, typename TI, typename TO, int OP, int LD, int ST, int LOGH, int RT>
__global__ void __launch_bounds__(512) dct_rad(LineArgs<TC> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (A.skip && *A.skip) return;
  constexpr int H = 1 << LOGH;
  constexpr int N = 2 * H;
  constexpr int T = H / RT;
  constexpr int NV = 2 * RT;  // reals per thread
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
  R16Tw<TC> tw;
  R8Tw<TC> tw8;
  if constexpr (RT == 16) {
    if (LOGH >= 8) {
      const int step = (H / 256) * (t & 15);
      tw.w1 = Tb.twH[step];
      tw.w4 = Tb.twH[4 * step];
    }
    if (LOGH % 4) tw.fin = Tb.twH[t];
  } else {
    if (LOGH >= 6) tw8.s1 = Tb.twH[(H / 64) * (t & 7)];
    if (LOGH >= 9) tw8.s2 = Tb.twH[(H / 512) * (t & 63)];
    if (LOGH % 3) tw8.fin = Tb.twH[t];
  }
  const cplx<TC> tNb = Tb.tN[t];
  const cplx<TC> t4b = Tb.t4N[t];

  // coordinates of this line's cells for the residual (rows: x varies)
  const int lj = rows ? lo % A.n1 : 0, lk = rows ? lo / A.n1 : 0;
  auto load = [&](int n) -> TC {
    int64_t p = lb + (int64_t)n * st;
    if (LD == LD_RESID) {
      double r = resid_ijk(A.rb, A.rphi, p, n, lj, lk, A.d, A.n0, A.n1, A.n2, A.ih2, A.rscale);
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
      // the residual reads 5-7 values per point: batches of 8 points, the
      // batch loop kept rolled so that the kernel stays small
#pragma unroll 1
      for (int r0 = 0; r0 < NV; r0 += 8) {
        TC v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          // strided line along axis 1 (y) or 2 (z) at x position ti_x, the
          // other coordinate to
          const int pn = tn0 + (r0 + r) * T;
          const int cj = A.axis == 1 ? pn : to, ck = A.axis == 1 ? to : pn;
          double x = resid_ijk(A.rb, A.rphi, p0 + (r0 + r) * dp, ti_x, cj, ck, A.d, A.n0, A.n1,
                               A.n2, A.ih2, A.rscale);
          if (A.sub) x -= *A.sub;
          v[r] = (TC)x;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) zl[pos(tn0 + (r0 + r) * T)] = v[r];
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
      // the residual reads 5-7 values per point: batches of 8 points, the
      // batch loop kept rolled so that the kernel stays small
#pragma unroll 1
      for (int i0 = 0; i0 < NV; i0 += 8) {
        TC xv[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) xv[i] = load(t + T * (i0 + i));
#pragma unroll
        for (int i = 0; i < 8; ++i) zr[vpad(mk_pos(t + T * (i0 + i), N))] = xv[i];
      }
      line_sync<T>();
    } else if (rows) {
      // coalesced loads, reordered into Makhoul order through LDS
      TC xv[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) xv[i] = load(t + T * i);
#pragma unroll
      for (int i = 0; i < NV; ++i) zr[vpad(mk_pos(t + T * i, N))] = xv[i];
      line_sync<T>();
    } else {
      tile_load([&](int n) { return vpad(mk_pos(n, N)); });
    }
#pragma unroll
    for (int q = 0; q < RT; ++q) a[q] = z[lpad(t + T * q)];
    line_sync<T>();
    rad_fft<TC, false, LOGH, RT>(a, t, tw, tw8, Tb.twH, z);
    // partner exchange: Z[H-k] next to Z[k]
#pragma unroll
    for (int q = 0; q < RT; ++q) z[lpad(t + T * q)] = a[q];
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
      cplx<TC> Zc = conj_(z[lpad((H - k) & (H - 1))]);
      cplx<TC> E = {(Zk.re + Zc.re) * TC(0.5), (Zk.im + Zc.im) * TC(0.5)};
      cplx<TC> D = {(Zk.re - Zc.re) * TC(0.5), (Zk.im - Zc.im) * TC(0.5)};
      cplx<TC> O = {D.im, -D.re};
      const cplx<TC> wN = q ? cmul(tNb, ldu(Tb.tN + T * q)) : tNb;   // tN[k]
      const cplx<TC> w4 = q ? cmul(t4b, ldu(Tb.t4N + T * q)) : t4b;  // t4N[k]
      cplx<TC> WO = cmul(wN, O);
      cplx<TC> Y = cmul(w4, cadd(E, WO));
      TC xa = TC(2) * Y.re;   // X[k]
      TC xb = TC(-2) * Y.im;  // X[N-k]; for k = 0 replaced by X[H]
      if (k == 0) {
        cplx<TC> Yh = cmul(t4n_mirror(w4), conj_(csub(E, WO)));
        xb = TC(2) * Yh.re;
      }
      if (OP == OP_FWD) {
        ya[q] = xa;
        yb[q] = xb;
      } else {
        // divide by the summed eigenvalues; the 1D eigenvalue of index j is
        // -(4/h^2) sin^2(pi j / (2N)): sin(pi k/2N) = -Im w4, cos = Re w4,
        // and index H (k = 0) has sin^2 = 1/2
        TC s_a = w4.im * w4.im;
        TC s_b = k ? w4.re * w4.re : TC(0.5);
        TC l_a = (rest + lc * s_a) * ls_;
        TC l_b = (rest + lc * s_b) * ls_;
        if (k == 0) x0 = xa;
        ya[q] = l_a != TC(0) ? xa / l_a : TC(0);
        yb[q] = xb / l_b;
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
    // the zero line's mode 0 is sum(b) * prod(2 N_a): the compatibility defect
    if (t == 0 && rest == TC(0) && A.bmean) *A.bmean = (double)x0 * A.meannorm;
    line_sync<T>();
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      const int k = t + T * q;
      zr[xpad(k)] = ya[q];
      zr[xpad(k ? N - k : H)] = yb[q];
    }
    line_sync<T>();
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      const int k = t + T * q;
      const cplx<TC> wN = q ? cmul(tNb, ldu(Tb.tN + T * q)) : tNb;
      const cplx<TC> w4 = q ? cmul(t4b, ldu(Tb.t4N + T * q)) : t4b;
      TC xhk = zr[xpad(H - k)];
      TC xhpk = zr[xpad(H + k)];
      a[q] = pre_own(ya[q], k ? yb[q] : TC(0), xhk, xhpk, w4, wN);
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
      a[q] = pre_own(xk[q], k ? xn[q] : TC(0), xhk, xhpk, w4, wN);
    }
    line_sync<T>();
  }

  // inverse half-length FFT, then unpack v -> x.  Opaque copies of the
  // thread index and LDS base keep the compiler from carrying the forward
  // FFT's address arithmetic live into this second FFT.
  int ti = t;
  cplx<TC>* zi = z;
  asm volatile("" : "+v"(ti));
  asm volatile("" : "+v"(zi));
  rad_fft<TC, true, LOGH, RT>(a, ti, tw, tw8, Tb.twH, zi);
  const TC sc = A.outscale;
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
  for (int q = 0; q < RT; ++q) zi[lpad(ti + T * q)] = {a[q].re * sc, a[q].im * sc};
  if (rows) {
    // back to natural order through LDS, then coalesced stores
    line_sync<T>();
    TC* zri = reinterpret_cast<TC*>(zi);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int n = t2 + T * i;
      put(lb2 + (int64_t)n * st2, zri[vpad(mk_pos(n, N))]);
    }
  } else {
    __syncthreads();
    const int64_t p0 = lbase[0] + tcc + (int64_t)tn0 * st2;
    const TC* zl = zr0 + 2 * tcc * LS;
#pragma unroll
    for (int r = 0; r < NV; ++r)
      put(p0 + (int64_t)r * T * st2, zl[vpad(mk_pos(tn0 + r * T, N))]);
  }
}

// ---- deterministic mean ----------------------------------------------------
__global__ void __launch_bounds__(256) partial_sum_f64(const double* __restrict__ x, int64_t n,
                                                       double* __restrict__ part,
                                                       const int32_t* __restrict__ skip) {
  __shared__ double red[256];
  if (skip && *skip) return;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    acc += x[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) finish_mean(const double* __restrict__ part, int nblk,
                                                   double scale, double* __restrict__ out,
                                                   const int32_t* __restrict__ skip) {
  __shared__ double red[256];
  if (skip && *skip) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * scale;
}

__global__ void __launch_bounds__(256) sub_scalar_f64(double* __restrict__ x, int64_t n,
                                                      const double* __restrict__ m,
                                                      const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  double mv = m[0];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    x[i] -= mv;
}

__global__ void __launch_bounds__(256) zero_bytes(uint32_t* __restrict__ p, int64_t nwords) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nwords;
       i += (int64_t)gridDim.x * 256)
    p[i] = 0u;
}

int g_lds_limit = 0;

int lds_limit() {
  if (g_lds_limit == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v <= 0)
      v = 65536;
    g_lds_limit = v;
  }
  return g_lds_limit;
}

// Chooses lines per tile and threads for one pass.
template <typename TC>
void tile_shape(int axis, int N, int lines_x, int* C, int* nthr, int* B) {
  const int H = N / 2;
  const int lim = lds_limit();
  int c;
  if (axis == 0) {
    c = 1024 / H;  // aim for C*H/4 = 256 threads
    if (c < 1) c = 1;
    while (c > lines_x) c >>= 1;
  } else {
    c = (int)(128 / sizeof(TC));  // 128-byte row segments
    while (c > 1 && (size_t)c * N * sizeof(TC) > (size_t)lim / 2) c >>= 1;
    while (c > lines_x) c >>= 1;
  }
  while (c > 1 && (size_t)c * N * sizeof(TC) > (size_t)lim) c >>= 1;
  int want = c * H / 4;
  if (want < 64) want = 64;
  int t = want > 1024 ? 1024 : want;
  int b = (c * H / 4 + t - 1) / t;
  if (b < 1) b = 1;
  *C = c;
  *nthr = t;
  *B = b;
}

}  // namespace

// Complex values per thread of the transforms along `axis`: 16, or 8 when
// the pass has too few lines to give the device four wavefronts per SIMD
// with 16 (a 2D grid; small 3D grids), which doubles the wavefronts.
int pass_radix(const pc_plan* P, int axis) {
  const int64_t N = P->n[axis];
  const int64_t lines = P->G / N;
  const int64_t t16 = N / 32;  // threads per line with 16 values each
  const int64_t waves16 = (lines * t16 + 63) / 64;
  return waves16 < 4 * 1024 ? 8 : 16;
}

// Lines per workgroup tile of the radix-16/8 transform along `axis` (0 when
// the axis uses the generic kernel, N < 32).
int r16_tile_lines(const pc_plan* P, int axis, size_t elem) {
  const int N = P->n[axis];
  if (N < 32) return 0;
  const int H = N / 2, T = H / pass_radix(P, axis), LS = H + H / 16 + 1;
  const int64_t lines = P->G / N;
  int C;
  if (axis == 0) {
    C = std::max(1, ROW_THREADS / T);
    while (C > 1 && (int64_t)C > lines) C >>= 1;
  } else {
    C = (int)(128 / elem);
    while (C > 1 && (C * T > COL_MAX_THREADS || C > P->n[0])) C >>= 1;
  }
  while (C > 1 && (size_t)C * LS * 2 * elem > (size_t)lds_limit()) C >>= 1;
  return C;
}

namespace {

template <typename TC, typename TI, typename TO, int OP, int LD, int ST>
int launch_pass(const pc_plan* P, int axis, const TI* in, TO* out, const AxisTables<TC>* tabs,
                const double* rb, const double* rphi, double* bmean, hipStream_t s,
                const double* sub = nullptr, double sigma = 1.0, const int32_t* skip = nullptr,
                const int32_t* tiles = nullptr, int ntiles = -1) {
  LineArgs<TC> A{};
  A.sub = sub;
  A.skip = skip;
  A.tiles = tiles;
  A.lscale = (TC)sigma;
  A.rscale = sigma;
  A.lamc = (TC)(-4.0 / (P->h[axis] * P->h[axis]));
  A.in = in;
  A.out = out;
  A.rb = rb;
  A.rphi = rphi;
  A.N = P->n[axis];
  int H = A.N / 2;
  int logH = 0;
  while ((1 << logH) < H) ++logH;
  A.logH = logH;
  A.axis = axis;
  A.d = P->d;
  A.n0 = P->n[0];
  A.n1 = P->n[1];
  A.n2 = P->d == 3 ? P->n[2] : 1;
  for (int a = 0; a < 3; ++a) A.ih2[a] = a < P->d ? 1.0 / (P->h[a] * P->h[a]) : 0.0;
  A.stride = axis == 0 ? 1 : (axis == 1 ? (int64_t)P->n[0] : (int64_t)P->n[0] * P->n[1]);
  A.tab = tabs[axis];
  A.lam0 = tabs[0].lam;
  A.lam1 = (P->d == 3 && axis == 2) ? tabs[1].lam : nullptr;
  A.outscale = (OP == OP_FWD) ? TC(1) : TC(1.0 / (double)H);
  A.bmean = bmean;
  double norm = 1.0;
  for (int a = 0; a < P->d; ++a) norm *= 2.0 * P->n[a];
  A.meannorm = 1.0 / norm;
  int64_t lines = P->G / A.N;
  if (A.N >= 32) {
    // register kernel: T = H/RT threads per line, C lines per group
    const int RT = pass_radix(P, axis);
    const int T = H / RT;
    const int LS = H + H / 16 + 1;
    const int C = r16_tile_lines(P, axis, sizeof(TC));
    if ((size_t)C * LS * 2 * sizeof(TC) > (size_t)lds_limit())
      return fail(PC_ERR_UNSUPPORTED_SIZE, "transform line does not fit in LDS");
    A.C = C;
    int ntile;
    if (axis == 0) {
      if (lines % C) return fail(PC_ERR_UNSUPPORTED_SIZE, "row count not a multiple of the tile");
      ntile = (int)(lines / C);
    } else {
      A.tx = P->n[0] / C;
      ntile = (int)(lines / C);
    }
    if (tiles) {
      if (ntiles <= 0) return PC_OK;
      ntile = ntiles;
    }
    size_t lds = (size_t)C * LS * 2 * sizeof(TC);
    dim3 grid(ntile), block(C * T);
    const void* fn = nullptr;
    const int key = logH * 32 + RT;
    switch (key) {
#define PC_RAD_CASE(LH, R) \
      case LH * 32 + R: fn = (const void*)dct_rad<TC, TI, TO, OP, LD, ST, LH, R>; break;
      PC_RAD_CASE(4, 16) PC_RAD_CASE(5, 16) PC_RAD_CASE(6, 16) PC_RAD_CASE(7, 16)
      PC_RAD_CASE(8, 16) PC_RAD_CASE(9, 16) PC_RAD_CASE(10, 16) PC_RAD_CASE(11, 16)
      PC_RAD_CASE(4, 8) PC_RAD_CASE(5, 8) PC_RAD_CASE(6, 8) PC_RAD_CASE(7, 8)
      PC_RAD_CASE(8, 8) PC_RAD_CASE(9, 8) PC_RAD_CASE(10, 8) PC_RAD_CASE(11, 8)
#undef PC_RAD_CASE
      default: return fail(PC_ERR_UNSUPPORTED_SIZE, "transform length");
    }
    if (lds > 65536)
      PC_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    switch (key) {
#define PC_RAD_LAUNCH(LH, R) \
      case LH * 32 + R: \
        hipLaunchKernelGGL((dct_rad<TC, TI, TO, OP, LD, ST, LH, R>), grid, block, lds, s, A); break;
      PC_RAD_LAUNCH(4, 16) PC_RAD_LAUNCH(5, 16) PC_RAD_LAUNCH(6, 16) PC_RAD_LAUNCH(7, 16)
      PC_RAD_LAUNCH(8, 16) PC_RAD_LAUNCH(9, 16) PC_RAD_LAUNCH(10, 16) PC_RAD_LAUNCH(11, 16)
      PC_RAD_LAUNCH(4, 8) PC_RAD_LAUNCH(5, 8) PC_RAD_LAUNCH(6, 8) PC_RAD_LAUNCH(7, 8)
      PC_RAD_LAUNCH(8, 8) PC_RAD_LAUNCH(9, 8) PC_RAD_LAUNCH(10, 8) PC_RAD_LAUNCH(11, 8)
#undef PC_RAD_LAUNCH
    }
    PC_HIP_CHECK(hipGetLastError());
    return PC_OK;
  }
  int C, nthr, B;

  tile_shape<TC>(axis, A.N, axis == 0 ? (int)std::min<int64_t>(lines, 1 << 20) : P->n[0], &C,
                 &nthr, &B);
  A.C = C;
  if (C > nthr) return fail(PC_ERR_UNSUPPORTED_SIZE, "transform tile has more lines than threads");
  int ntile;
  if (axis == 0) {
    ntile = (int)((lines + C - 1) / C);
    if (lines % C) return fail(PC_ERR_UNSUPPORTED_SIZE, "row count not a multiple of the tile");
  } else {
    A.tx = P->n[0] / C;
    ntile = (int)(lines / C);
  }
  // pad each LDS line by one complex when it fits (fewer bank conflicts)
  A.pad = ((size_t)C * (A.N + 2) * sizeof(TC) <= (size_t)lds_limit()) ? 2 : 0;
  size_t lds = (size_t)C * (A.N + A.pad) * sizeof(TC);
  dim3 grid(ntile), block(nthr);
  const void* fn;
  switch (B) {
    case 1: fn = (const void*)dct_lines<TC, TI, TO, OP, LD, ST, 1>; break;
    case 2: fn = (const void*)dct_lines<TC, TI, TO, OP, LD, ST, 2>; break;
    case 4: fn = (const void*)dct_lines<TC, TI, TO, OP, LD, ST, 4>; break;
    default: return fail(PC_ERR_UNSUPPORTED_SIZE, "transform tile shape");
  }
  if (lds > 65536)
    PC_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  switch (B) {
    case 1:
      hipLaunchKernelGGL((dct_lines<TC, TI, TO, OP, LD, ST, 1>), grid, block, lds, s, A);
      break;
    case 2:
      hipLaunchKernelGGL((dct_lines<TC, TI, TO, OP, LD, ST, 2>), grid, block, lds, s, A);
      break;
    default:
      hipLaunchKernelGGL((dct_lines<TC, TI, TO, OP, LD, ST, 4>), grid, block, lds, s, A);
      break;
  }
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

// Full solve with compute type TC from TI input to TO output.  Forward
// along axes 0..d-2, fused forward/divide/inverse on axis d-1, inverse back.
// The first pass may compute the float64 residual on the fly (LD) and the
// last pass may accumulate into float64 phi (ST).
template <typename TC, typename TI, typename TO, int LD, int ST>
int solve_passes(const pc_plan* P, const AxisTables<TC>* tabs, const TI* in, TO* out,
                 TC* work, const double* rb, const double* rphi, double* bmean, hipStream_t s,
                 const double* sub = nullptr, double sigma = 1.0,
                 const int32_t* skip = nullptr) {
  if (P->d == 2) {
    PC_TRY((launch_pass<TC, TI, TC, OP_FWD, LD, ST_PLAIN>(P, 0, in, work, tabs, rb, rphi, nullptr, s,
                                                          sub, sigma, skip)));
    PC_TRY((launch_pass<TC, TC, TC, OP_FDI, LD_PLAIN, ST_PLAIN>(P, 1, work, work, tabs, nullptr,
                                                                nullptr, bmean, s, nullptr,
                                                                sigma, skip)));
    PC_TRY((launch_pass<TC, TC, TO, OP_INV, LD_PLAIN, ST>(P, 0, work, out, tabs, nullptr, rphi,
                                                          nullptr, s, nullptr, 1.0, skip)));
  } else {
    PC_TRY((launch_pass<TC, TI, TC, OP_FWD, LD, ST_PLAIN>(P, 0, in, work, tabs, rb, rphi, nullptr, s,
                                                          sub, sigma, skip)));
    PC_TRY((launch_pass<TC, TC, TC, OP_FWD, LD_PLAIN, ST_PLAIN>(P, 1, work, work, tabs, nullptr,
                                                                nullptr, nullptr, s, nullptr, 1.0,
                                                                skip)));
    PC_TRY((launch_pass<TC, TC, TC, OP_FDI, LD_PLAIN, ST_PLAIN>(P, 2, work, work, tabs, nullptr,
                                                                nullptr, bmean, s, nullptr,
                                                                sigma, skip)));
    PC_TRY((launch_pass<TC, TC, TC, OP_INV, LD_PLAIN, ST_PLAIN>(P, 1, work, work, tabs, nullptr,
                                                                nullptr, nullptr, s, nullptr, 1.0,
                                                                skip)));
    PC_TRY((launch_pass<TC, TC, TO, OP_INV, LD_PLAIN, ST>(P, 0, work, out, tabs, nullptr, rphi,
                                                          nullptr, s, nullptr, 1.0, skip)));
  }
  return PC_OK;
}

}  // namespace

int fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return PC_OK;
  if (bytes % 4) return fail(PC_ERR_INVALID_ARG, "fill_zero size");
  int64_t nw = (int64_t)(bytes / 4);
  int nb = (int)std::min<int64_t>(4096, (nw + 255) / 256);
  hipLaunchKernelGGL(zero_bytes, dim3(nb), dim3(256), 0, s, reinterpret_cast<uint32_t*>(p), nw);
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

int mean_f64(const double* x, int64_t n, double* partial, int nblk, double* out_dev,
             hipStream_t s, const int32_t* skip) {
  hipLaunchKernelGGL(partial_sum_f64, dim3(nblk), dim3(256), 0, s, x, n, partial, skip);
  hipLaunchKernelGGL(finish_mean, dim3(1), dim3(256), 0, s, partial, nblk, 1.0 / (double)n,
                     out_dev, skip);
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

int solve_f64(const pc_plan* P, const double* b, double* phi, double* bmean_dev, pc_workspace*,
              hipStream_t s, double sigma, const int32_t* skip) {
  return solve_passes<double, double, double, LD_PLAIN, ST_PLAIN>(
      P, P->ax64, b, phi, phi, nullptr, nullptr, bmean_dev, s, nullptr, sigma, skip);
}

int solve_f32(const pc_plan* P, const float* b, float* phi, double* bmean_dev, pc_workspace*,
              hipStream_t s, double sigma, const int32_t* skip) {
  return solve_passes<float, float, float, LD_PLAIN, ST_PLAIN>(
      P, P->ax32, b, phi, phi, nullptr, nullptr, bmean_dev, s, nullptr, sigma, skip);
}

// Defect correction: bbar = mean(b) in float64; phi0 = S32(b - bbar); then
// `sweeps` times r = (b - bbar) - lap_h phi (float64, fused into the first
// pass), phi += S32(r) (accumulated in float64 in the last pass); finally
// mean(phi) is removed in float64.  The mean is taken out in float64 before
// each conversion to float32: left in, the compatibility defect would
// dominate the float32 rounding of the much smaller residual.
int solve_mixed(const pc_plan* P, const double* b, double* phi, int sweeps, double* bmean_dev,
                pc_workspace* ws, hipStream_t s, double sigma, const int32_t* skip) {
  if (!ws || !ws->w32) return fail(PC_ERR_INVALID_ARG, "mixed solve needs a MIXED workspace");
  float* w = ws->w32;
  double* bm = bmean_dev ? bmean_dev : ws->scal;
  PC_TRY(mean_f64(b, P->G, ws->partial, ws->nblk, bm, s, skip));
  PC_TRY((solve_passes<float, double, double, LD_PLAIN, ST_PLAIN>(
      P, P->ax32, b, phi, w, nullptr, nullptr, nullptr, s, bm, sigma, skip)));
  for (int it = 0; it < sweeps; ++it) {
    PC_TRY((solve_passes<float, double, double, LD_RESID, ST_ACCUM>(
        P, P->ax32, b, phi, w, b, phi, nullptr, s, bm, sigma, skip)));
  }
  PC_TRY(mean_f64(phi, P->G, ws->partial, ws->nblk, ws->scal + 3, s, skip));
  int nb = (int)std::min<int64_t>(8192, (P->G + 255) / 256);
  hipLaunchKernelGGL(sub_scalar_f64, dim3(nb), dim3(256), 0, s, phi, P->G,
                     (const double*)(ws->scal + 3), skip);
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}


// ---- resident transforms of the IB iteration -----------------------------------
// After the first IB iteration the right-hand side changes only at the
// near-IB grid points (Sec. 2.3), and each 1D transform acts on its own line,
// so the forward transforms of the lines without near-IB points carry over
// unchanged from iteration to iteration.  The iteration itself reads the
// solution only through the gradient at the B+V nodes, so the inverse
// transforms can stop at the lines that gradient reads; the other lines are
// completed once, after the last iteration.  Every line that is transformed
// is transformed exactly as in the full solve, so the result is the same
// bit for bit.

bool resident_ok(const pc_plan* P, const pc_geom* g, int mode) {
  if (!g || g->n_ib == 0 || (mode != PC_F64 && mode != PC_F32)) return false;
  for (int a = 0; a < P->d; ++a)
    if (P->n[a] < 32) return false;
  return true;
}

int64_t resident_tiles_max(const pc_plan* P, size_t elem) {
  const int C0 = r16_tile_lines(P, 0, elem);
  int64_t t0 = C0 > 0 ? P->G / P->n[0] / C0 : 0;
  int64_t t1 = 0;
  if (P->d == 3) {
    const int C1 = r16_tile_lines(P, 1, elem);
    t1 = C1 > 0 ? P->G / P->n[1] / C1 : 0;
  }
  return 3 * (t0 + t1);
}

void resident_tiles(const pc_plan* P, size_t elem, const std::vector<int32_t>& near_pts,
                    const std::vector<int32_t>& ib_base, int m, std::vector<int32_t> out[6]) {
  for (int l = 0; l < 6; ++l) out[l].clear();
  const int64_t n0 = P->n[0], n1 = P->n[1], n2 = P->d == 3 ? P->n[2] : 1;
  const int C0 = r16_tile_lines(P, 0, elem);
  const int64_t t0 = n1 * n2 / C0;  // x-line tiles: line j + n1 k, tile line / C0
  std::vector<char> f0(t0, 0), i0(t0, 0);
  for (int32_t q : near_pts) f0[(q / n0) / C0] = 1;
  // lines read by the B+V gradient: the m x m (x m) block at each corner
  std::vector<char> ibplane(n2, 0);
  for (int32_t q : ib_base) {
    const int64_t j0 = (q / n0) % n1, k0 = q / (n0 * n1);
    const int kn = P->d == 3 ? m : 1;
    for (int kk = 0; kk < kn; ++kk) {
      ibplane[k0 + kk] = 1;
      for (int jj = 0; jj < m; ++jj) i0[((j0 + jj) + n1 * (k0 + kk)) / C0] = 1;
    }
  }
  for (int64_t t = 0; t < t0; ++t) {
    if (f0[t]) out[TL_FWD0].push_back((int32_t)t);
    out[i0[t] ? TL_INV0_IB : TL_INV0_REST].push_back((int32_t)t);
    // the x-inverse runs in place on whole tiles, whose lines may reach into
    // further planes (C0 > n1): those planes need their y-inverse first
    if (i0[t])
      for (int64_t l = t * C0; l < (t + 1) * C0; ++l) ibplane[l / n1] = 1;
  }
  if (P->d == 3) {
    // y-line tiles: C1 adjacent x positions of one plane k, tile = k * tx + i / C1
    const int C1 = r16_tile_lines(P, 1, elem);
    const int64_t tx = n0 / C1;
    std::vector<char> nearplane(n2, 0);
    for (int32_t q : near_pts) nearplane[q / (n0 * n1)] = 1;
    for (int64_t k = 0; k < n2; ++k)
      for (int64_t t = k * tx; t < (k + 1) * tx; ++t) {
        if (nearplane[k]) out[TL_FWD1].push_back((int32_t)t);
        out[ibplane[k] ? TL_INV1_IB : TL_INV1_REST].push_back((int32_t)t);
      }
  }
}

namespace {

template <typename TC>
int solve_resident(const pc_plan* P, const AxisTables<TC>* tabs, const TC* b, TC* p,
                   double* bmean, pc_workspace* W, hipStream_t s, double sigma,
                   const int32_t* skip, int phase) {
  if (!W || !W->resident) return fail(PC_ERR_INVALID_ARG, "resident solve without its workspace");
  TC* w1 = reinterpret_cast<TC*>(W->phi);
  TC* w1b = reinterpret_cast<TC*>(W->w1b);
  auto tl = [&](int l) { return W->tl[l]; };
  auto nt = [&](int l) { return W->ntl[l]; };
  if (phase < 2) {
    const bool later = phase == 1;
    PC_TRY((launch_pass<TC, TC, TC, OP_FWD, LD_PLAIN, ST_PLAIN>(
        P, 0, b, w1, tabs, nullptr, nullptr, nullptr, s, nullptr, sigma, skip,
        later ? tl(TL_FWD0) : nullptr, later ? nt(TL_FWD0) : -1)));
    const TC* last_in = w1;
    if (P->d == 3) {
      PC_TRY((launch_pass<TC, TC, TC, OP_FWD, LD_PLAIN, ST_PLAIN>(
          P, 1, w1, w1b, tabs, nullptr, nullptr, nullptr, s, nullptr, 1.0, skip,
          later ? tl(TL_FWD1) : nullptr, later ? nt(TL_FWD1) : -1)));
      last_in = w1b;
    }
    PC_TRY((launch_pass<TC, TC, TC, OP_FDI, LD_PLAIN, ST_PLAIN>(
        P, P->d - 1, last_in, p, tabs, nullptr, nullptr, bmean, s, nullptr, sigma, skip)));
    if (P->d == 3)
      PC_TRY((launch_pass<TC, TC, TC, OP_INV, LD_PLAIN, ST_PLAIN>(
          P, 1, p, p, tabs, nullptr, nullptr, nullptr, s, nullptr, 1.0, skip, tl(TL_INV1_IB),
          nt(TL_INV1_IB))));
    PC_TRY((launch_pass<TC, TC, TC, OP_INV, LD_PLAIN, ST_PLAIN>(
        P, 0, p, p, tabs, nullptr, nullptr, nullptr, s, nullptr, 1.0, skip, tl(TL_INV0_IB),
        nt(TL_INV0_IB))));
  } else {
    if (P->d == 3)
      PC_TRY((launch_pass<TC, TC, TC, OP_INV, LD_PLAIN, ST_PLAIN>(
          P, 1, p, p, tabs, nullptr, nullptr, nullptr, s, nullptr, 1.0, skip, tl(TL_INV1_REST),
          nt(TL_INV1_REST))));
    PC_TRY((launch_pass<TC, TC, TC, OP_INV, LD_PLAIN, ST_PLAIN>(
        P, 0, p, p, tabs, nullptr, nullptr, nullptr, s, nullptr, 1.0, skip, tl(TL_INV0_REST),
        nt(TL_INV0_REST))));
  }
  return PC_OK;
}

}  // namespace

int solve_resident_f64(const pc_plan* P, const double* b, double* p, double* bmean_dev,
                       pc_workspace* ws, hipStream_t s, double sigma, const int32_t* skip,
                       int phase) {
  return solve_resident<double>(P, P->ax64, b, p, bmean_dev, ws, s, sigma, skip, phase);
}

int solve_resident_f32(const pc_plan* P, const float* b, float* p, double* bmean_dev,
                       pc_workspace* ws, hipStream_t s, double sigma, const int32_t* skip,
                       int phase) {
  return solve_resident<float>(P, P->ax32, b, p, bmean_dev, ws, s, sigma, skip, phase);
}

}  // namespace pc
