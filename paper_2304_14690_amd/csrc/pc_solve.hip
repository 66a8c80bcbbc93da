// Poisson solve by line transforms (Sec. 2.3, three-step transform
// algorithm; cell-centred grid, central-difference eigenvalues).  Each axis
// carries the homogeneous Neumann condition of Eq. 7 or is periodic (the
// lateral condition of the verification cases of Sec. 3).
//
// Each 1D transform of length N is computed through a complex FFT of length
// H = N/2, staged in LDS and registers:
//   Neumann axis   DCT-II   X[k] = 2 sum_n x[n] cos(pi k (2n+1) / (2N)) by
//                  Makhoul's even/odd reordering, the real-FFT split and a
//                  quarter-sample shift; inverse x = DCT-III(X) / (2N);
//   periodic axis  the real DFT X_k = sum_n x[n] exp(-2 pi i k n / N) by the
//                  real-FFT split alone, packed into N reals; its exact
//                  inverse.
// One kernel launch transforms every line of the grid along one axis.  A
// workgroup holds C lines; along x the lines are whole rows, along y/z the C
// lines are adjacent in x so that each global access touches C contiguous
// elements.  The last axis fuses forward transform, division by the summed
// eigenvalues and inverse transform in registers, so a 2D solve is three
// passes over the grid and a 3D solve five.
#include <cmath>

#include "pc_transform.h"

namespace pc {
PC_RAD_COMBOS(PC_RAD_EXTERN_PER)
}  // namespace pc

namespace pc {

namespace {

// Register-transform tiles: threads per workgroup for contiguous rows, and
// the thread cap for the strided (column/pencil) passes.
constexpr int ROW_THREADS = 256;
constexpr int COL_MAX_THREADS = 512;

// n / d for 0 <= n < 2^17 and 0 < d <= 2^16, with rinv = 1.0f / d: the
// float32 product is within one of the quotient, and one correction step
// makes it exact (integer division by a runtime divisor costs far more).
__device__ __forceinline__ int div_small(int n, int d, float rinv) {
  int q = (int)((float)n * rinv);
  const int r = n - q * d;
  if (r < 0) --q;
  else if (r >= d) ++q;
  return q;
}

// One Stockham butterfly of compile-time radix R: inputs x[g + nb s],
// twiddles w^(k s) = twH[tstep k s] (w = exp(-+2 pi i / (L R))), a length-R
// DFT, outputs y[s' L] (y already offset by (g - k) R + k).
template <typename TC, bool INV, int R>
__device__ __forceinline__ void mixed_bfly(const cplx<TC>* x, cplx<TC>* y, int g, int nb, int k,
                                           int L, int tstep, const cplx<TC>* __restrict__ twH) {
  cplx<TC> v[R], w[R];
#pragma unroll
  for (int s = 0; s < R; ++s) v[s] = x[g + nb * s];
#pragma unroll
  for (int s = 1; s < R; ++s) w[s] = twH[tstep * k * s];
#pragma unroll
  for (int s = 1; s < R; ++s) v[s] = INV ? cmulc(v[s], w[s]) : cmul(v[s], w[s]);
  if constexpr (R == 3)
    dft3<TC, INV>(v);
  else if constexpr (R == 5)
    dft5<TC, INV>(v);
  else
    dftR<TC, INV, R>(v);
#pragma unroll
  for (int s = 0; s < R; ++s) y[s * L] = v[s];
}

// Mixed-radix Stockham FFT of the C lines held in LDS, for any H whose
// factors are listed in A.rad (complex view, line c at a + c*lsc; b is a
// second buffer of the same shape).  The stage of radix r after the stages
// of combined length L takes butterfly g (k = g mod L) of each line:
//   v_s = in[g + (H/r) s] w^(k s),  w = exp(-+2 pi i / (L r)),
//   out[(g - k) r + k + s' L] = sum_{s<r} v_s exp(-+2 pi i s s' / r),
// with w^e = twH[(H / (L r)) e]; radices 2, 3, 4, 5 and 8 have their own
// butterflies, any other prime factor (7, 67, ...) a direct sum of r terms
// per output.  Returns the buffer holding the result (the stages alternate
// between a and b).
template <typename TC, bool INV>
__device__ cplx<TC>* fft_lds_mixed(cplx<TC>* a, cplx<TC>* b, int lsc, int C, int H,
                                   const LineArgs<TC>& A, int tid, int nthr) {
  const cplx<TC>* __restrict__ twH = A.tab.twH;
  int L = 1;
  for (int st = 0; st < A.nrad; ++st) {
    const int r = A.rad[st];
    const int nb = H / r;
    const int Lr = L * r;
    const int tstep = H / Lr;
    const float rnb = 1.0f / (float)nb, rL = 1.0f / (float)L;
    for (int e = tid; e < C * nb; e += nthr) {
      const int c = div_small(e, nb, rnb);
      const int g = e - c * nb;
      const int k = g - L * div_small(g, L, rL);
      const cplx<TC>* x = a + c * lsc;
      cplx<TC>* y = b + c * lsc + (g - k) * r + k;
      switch (r) {
        case 2: mixed_bfly<TC, INV, 2>(x, y, g, nb, k, L, tstep, twH); break;
        case 3: mixed_bfly<TC, INV, 3>(x, y, g, nb, k, L, tstep, twH); break;
        case 4: mixed_bfly<TC, INV, 4>(x, y, g, nb, k, L, tstep, twH); break;
        case 5: mixed_bfly<TC, INV, 5>(x, y, g, nb, k, L, tstep, twH); break;
        case 8: mixed_bfly<TC, INV, 8>(x, y, g, nb, k, L, tstep, twH); break;
        default: {
          // direct sum: output s' takes v_s W_r^(s s'), W_r^m = twH[nb (m mod r)]
          for (int sp = 0; sp < r; ++sp) {
            cplx<TC> acc = x[g];
            int ex = 0;            // (k + L s') s mod Lr, as in the twiddled DFT
            const int q = k + L * sp;
            for (int sidx = 1; sidx < r; ++sidx) {
              ex += q;
              if (ex >= Lr) ex -= Lr;
              const cplx<TC> w = twH[tstep * ex];
              const cplx<TC> v = x[g + nb * sidx];
              acc = cadd(acc, INV ? cmulc(v, w) : cmul(v, w));
            }
            y[sp * L] = acc;
          }
        }
      }
    }
    __syncthreads();
    cplx<TC>* t = a;
    a = b;
    b = t;
    L = Lr;
  }
  return a;
}

// Forward post-processing of pair k (0 <= k <= H/2) of one line: from the
// half-length FFT Z produce X[k], X[N-k], X[H-k], X[H+k].
template <typename TC>
__device__ __forceinline__ void post_pair(const cplx<TC>* z, int k, int N, int H,
                                          const AxisTables<TC>& T, TC* xk, TC* xnk, TC* xhk,
                                          TC* xhpk) {
  cplx<TC> Zk = z[k];
  cplx<TC> Zc = conj_(z[k ? H - k : 0]);
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

// The generic line transform (cosine transforms of Neumann axes of any even
// length N, short or not a power of two): C lines per workgroup staged in
// LDS, the mixed-radix FFT above, pairs (k, H-k) of the real-FFT split per
// thread.  Two LDS buffers of C lines each.  With H odd no pair is its own
// partner; with H even the pair k = H/2 is.
template <typename TC, typename TI, typename TO, int OP, int LD, int ST, int B>
__global__ void __launch_bounds__(1024) dct_lines(LineArgs<TC> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (A.skip && *A.skip) return;
  TC* s = reinterpret_cast<TC*>(smem_raw);
  const int N = A.N, H = N >> 1, C = A.C;
  const int ls = N + A.pad;  // line stride in LDS (reals)
  TC* s2 = s + (size_t)C * ls;  // second buffer
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int t = A.tiles ? A.tiles[blockIdx.x]
                        : (A.axis == 0 ? blockIdx.x : xcd_tile(blockIdx.x, gridDim.x));
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
      double r = resid_at(A.rb, A.rphi, p, A.d, A.n0, A.n1, A.n2, A.perm, A.ih2, A.rscale);
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
  cplx<TC>* zc2 = reinterpret_cast<cplx<TC>*>(s2);
  const int lsc = ls >> 1;
  const int npair = H / 2 + 1;
  const TC* res = s;  // reals of the final result (natural or Makhoul order)

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
    res = reinterpret_cast<const TC*>(fft_lds_mixed<TC, true>(zc, zc2, lsc, C, H, A, tid, nthr));
  } else {
    const cplx<TC>* zf = fft_lds_mixed<TC, false>(zc, zc2, lsc, C, H, A, tid, nthr);
    constexpr int PB = 2 * B + 1;
    TC xa[PB], xb[PB], xc[PB], xd[PB];
    int ck[PB], kk[PB];
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      int w = tid + b * nthr;
      ck[b] = -1;
      if (w < C * npair) {
        int c = w / npair, k = w - c * npair;
        post_pair(zf + c * lsc, k, N, H, A.tab, &xa[b], &xb[b], &xc[b], &xd[b]);
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
          TC l0 = (rest + lam[k]) * ls_, l1 = (rest + lam[k ? N - k : 0]) * ls_,
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
      res = reinterpret_cast<const TC*>(fft_lds_mixed<TC, true>(zc, zc2, lsc, C, H, A, tid, nthr));
    } else {
      __syncthreads();
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        if (ck[b] >= 0) {
          TC* x = s + ck[b] * ls;
          int k = kk[b];
          // the pair k = H/2 (H even) is its own partner: X[H-k] = X[k] and
          // X[H+k] = X[N-k] are written once
          x[k] = xa[b];
          if (k != 0) x[N - k] = xb[b];
          if (2 * k != H || H == 1) x[H - k] = xc[b];
          if (k != 0 && 2 * k != H) x[H + k] = xd[b];
        }
      }
      __syncthreads();
      res = s;
    }
  }

  // ---- store ----------------------------------------------------------------
  for (int e = tid; e < C * N; e += nthr) {
    int c, n;
    if (A.axis == 0) { c = e / N; n = e - c * N; } else { n = e / C; c = e - n * C; }
    int i, o;
    int64_t p = line_base(A, t, c, &i, &o) + (int64_t)n * A.stride;
    int q = (OP == OP_FWD) ? n : mk_pos(n, N);
    TC v = res[c * ls + q] * A.outscale;
    if (ST == ST_ACCUM) {
      reinterpret_cast<double*>(A.out)[p] = A.rphi[p] + (double)v;
    } else {
      out[p] = (TO)v;
    }
  }
}

// DCT-I of the lines of a vertex axis (n points, mirror about the end
// vertices): the real DFT of the even extension e of length NS = 2(n-1)
// (e[i] = x[i], e[NS-i] = x[i]) through the half-length complex FFT of
// z[m] = e[2m] + i e[2m+1] (length H = n - 1) and the real-FFT split
// X_k = Re(E_k + w^k O_k), w = exp(-2 pi i / NS), X_H = E_0 - O_0 (the
// spectrum of an even sequence is real); the inverse builds Z from the real
// spectrum with the same split, runs the inverse FFT and scales by 1/H.
// C lines per workgroup in three LDS regions (two FFT buffers and the
// spectra); lines past the end of a partial tile are masked.
template <typename TC, typename TI, typename TO, int OP, int LD, int ST>
__global__ void __launch_bounds__(1024) dct1_lines(LineArgs<TC> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (A.skip && *A.skip) return;
  const int n = A.N, H = n - 1, NS = 2 * H, C = A.C;
  const int ls = NS + A.pad;  // reals per line per region
  const int lsc = ls >> 1;
  TC* s0 = reinterpret_cast<TC*>(smem_raw);
  TC* s1 = s0 + (size_t)C * ls;
  TC* xs = s1 + (size_t)C * ls;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int t = A.axis == 0 ? blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
  const TI* __restrict__ in = reinterpret_cast<const TI*>(A.in);
  TO* __restrict__ out = reinterpret_cast<TO*>(A.out);
  const AxisTables<TC>& Tb = A.tab;
  // global index of point i of line c (or -1 past the end of the tile)
  auto gidx = [&](int c, int i) -> int64_t {
    int li, lo;
    const int64_t b = line_base(A, t, c, &li, &lo);
    if (A.axis == 0 ? (int64_t)t * C + c >= A.lines : li >= A.n0) return -1;
    return b + (int64_t)i * A.stride;
  };
  // element e of the tile's points: line c, point i (rows: points of a line
  // adjacent; strided: lines adjacent)
  auto split_e = [&](int e, int* c, int* i) {
    if (A.axis == 0) { *c = e / n; *i = e - *c * n; } else { *i = e / C; *c = e - *i * C; }
  };

  if (OP != OP_INV) {
    for (int e = tid; e < C * n; e += nthr) {
      int c, i;
      split_e(e, &c, &i);
      const int64_t p = gidx(c, i);
      TC v = TC(0);
      if (p >= 0) {
        if (LD == LD_RESID) {
          double r = resid_at<true>(A.rb, A.rphi, p, A.d, A.n0, A.n1, A.n2, A.perm, A.ih2, A.rscale);
          if (A.sub) r -= *A.sub;
          v = (TC)r;
        } else if (A.sub) {
          v = (TC)((double)in[p] - *A.sub);
        } else {
          v = (TC)in[p];
        }
      }
      s0[c * ls + i] = v;
      if (i > 0 && i < n - 1) s0[c * ls + NS - i] = v;
    }
    __syncthreads();
    const cplx<TC>* zf = fft_lds_mixed<TC, false>(reinterpret_cast<cplx<TC>*>(s0),
                                                  reinterpret_cast<cplx<TC>*>(s1), lsc, C, H, A,
                                                  tid, nthr);
    for (int e = tid; e < C * n; e += nthr) {
      const int c = e / n, k = e - c * n;
      const cplx<TC>* z = zf + c * lsc;
      const int kk = k < H ? k : 0;
      const cplx<TC> Zk = z[kk];
      const cplx<TC> Zc = conj_(z[kk ? H - kk : 0]);
      const cplx<TC> E = {(Zk.re + Zc.re) * TC(0.5), (Zk.im + Zc.im) * TC(0.5)};
      const cplx<TC> D = {(Zk.re - Zc.re) * TC(0.5), (Zk.im - Zc.im) * TC(0.5)};
      const cplx<TC> O = {D.im, -D.re};  // -i D
      TC X;
      if (k < H) {
        const cplx<TC> WO = cmul(Tb.tN[k], O);
        X = E.re + WO.re;
      } else {
        X = E.re - O.re;  // X_H = E_0 - O_0
      }
      xs[c * ls + k] = X;
    }
    __syncthreads();
    if (OP == OP_FWD) {
      for (int e = tid; e < C * n; e += nthr) {
        int c, i;
        split_e(e, &c, &i);
        const int64_t p = gidx(c, i);
        if (p >= 0) out[p] = (TO)(xs[c * ls + i] * A.outscale);
      }
      return;
    }
    // FDI: divide by the summed eigenvalues (slot k of this axis)
    for (int e = tid; e < C * n; e += nthr) {
      const int c = e / n, k = e - c * n;
      int li, lo;
      (void)line_base(A, t, c, &li, &lo);
      const bool valid = A.axis == 0 ? (int64_t)t * C + c < A.lines : li < A.n0;
      TC rest = TC(0);
      if (valid) {
        rest = A.lam0[li];
        if (A.lam1) rest += A.lam1[lo];
      }
      const TC l = (rest + Tb.lam[k]) * A.lscale;
      const TC X = xs[c * ls + k];
      if (valid && k == 0 && rest == TC(0) && A.bmean) *A.bmean = (double)X * A.meannorm;
      xs[c * ls + k] = l != TC(0) ? X / l : TC(0);
    }
    __syncthreads();
  } else {
    for (int e = tid; e < C * n; e += nthr) {
      int c, i;
      split_e(e, &c, &i);
      const int64_t p = gidx(c, i);
      xs[c * ls + i] = p >= 0 ? (TC)in[p] : TC(0);
    }
    __syncthreads();
  }
  // inverse: Z[k] from the real spectrum (imaginary parts zero)
  cplx<TC>* za = reinterpret_cast<cplx<TC>*>(s0);
  for (int e = tid; e < C * H; e += nthr) {
    const int c = e / H, k = e - c * H;
    const TC xk = xs[c * ls + k], xhk = xs[c * ls + H - k];
    za[c * lsc + k] = pre_own_per(xk, TC(0), xhk, TC(0), Tb.tN[k]);
  }
  __syncthreads();
  const TC* er = reinterpret_cast<const TC*>(
      fft_lds_mixed<TC, true>(za, reinterpret_cast<cplx<TC>*>(s1), lsc, C, H, A, tid, nthr));
  for (int e = tid; e < C * n; e += nthr) {
    int c, i;
    split_e(e, &c, &i);
    const int64_t p = gidx(c, i);
    if (p < 0) continue;
    const TC v = er[c * ls + i] * A.outscale;
    if (ST == ST_ACCUM)
      reinterpret_cast<double*>(A.out)[p] = A.rphi[p] + (double)v;
    else
      out[p] = (TO)v;
  }
}

// The packed real DFT of the lines of a periodic axis of any even length N
// (the generic counterpart of the periodic register kernel, same slots:
// slot k = Re X_k, slot N-k = Im X_k, slot H = X_H): the half-length complex
// FFT of z[m] = x[2m] + i x[2m+1] (mixed radix, H = N/2) and the real-FFT
// split X_k = E_k + w^k O_k, w = exp(-2 pi i / N); the inverse runs the same
// steps backwards and scales by 1/H.  C lines per workgroup in three LDS
// regions; lines past the end of a partial tile are masked.
template <typename TC, typename TI, typename TO, int OP, int LD, int ST>
__global__ void __launch_bounds__(1024) rdft_lines(LineArgs<TC> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (A.skip && *A.skip) return;
  const int N = A.N, H = N / 2, C = A.C;
  const int ls = N + A.pad;
  const int lsc = ls >> 1;
  TC* s0 = reinterpret_cast<TC*>(smem_raw);
  TC* s1 = s0 + (size_t)C * ls;
  TC* xs = s1 + (size_t)C * ls;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int t = A.tiles ? A.tiles[blockIdx.x]
                        : (A.axis == 0 ? blockIdx.x : xcd_tile(blockIdx.x, gridDim.x));
  const TI* __restrict__ in = reinterpret_cast<const TI*>(A.in);
  TO* __restrict__ out = reinterpret_cast<TO*>(A.out);
  const AxisTables<TC>& Tb = A.tab;
  auto gidx = [&](int c, int i) -> int64_t {
    int li, lo;
    const int64_t b = line_base(A, t, c, &li, &lo);
    if (A.axis == 0 ? (int64_t)t * C + c >= A.lines : li >= A.n0) return -1;
    return b + (int64_t)i * A.stride;
  };
  auto split_e = [&](int e, int* c, int* i) {
    if (A.axis == 0) { *c = e / N; *i = e - *c * N; } else { *i = e / C; *c = e - *i * C; }
  };

  if (OP != OP_INV) {
    for (int e = tid; e < C * N; e += nthr) {
      int c, i;
      split_e(e, &c, &i);
      const int64_t p = gidx(c, i);
      TC v = TC(0);
      if (p >= 0) {
        if (LD == LD_RESID) {
          double r = resid_at(A.rb, A.rphi, p, A.d, A.n0, A.n1, A.n2, A.perm, A.ih2, A.rscale);
          if (A.sub) r -= *A.sub;
          v = (TC)r;
        } else if (A.sub) {
          v = (TC)((double)in[p] - *A.sub);
        } else {
          v = (TC)in[p];
        }
      }
      s0[c * ls + i] = v;
    }
    __syncthreads();
    const cplx<TC>* zf = fft_lds_mixed<TC, false>(reinterpret_cast<cplx<TC>*>(s0),
                                                  reinterpret_cast<cplx<TC>*>(s1), lsc, C, H, A,
                                                  tid, nthr);
    // split: slots k and N-k from the own index k (k < H), slot H from k = 0
    for (int e = tid; e < C * H; e += nthr) {
      const int c = e / H, k = e - c * H;
      const cplx<TC>* z = zf + c * lsc;
      const cplx<TC> Zk = z[k];
      const cplx<TC> Zc = conj_(z[k ? H - k : 0]);
      const cplx<TC> E = {(Zk.re + Zc.re) * TC(0.5), (Zk.im + Zc.im) * TC(0.5)};
      const cplx<TC> D = {(Zk.re - Zc.re) * TC(0.5), (Zk.im - Zc.im) * TC(0.5)};
      const cplx<TC> O = {D.im, -D.re};  // -i D
      const cplx<TC> WO = cmul(Tb.tN[k], O);
      xs[c * ls + k] = E.re + WO.re;
      if (k)
        xs[c * ls + N - k] = E.im + WO.im;
      else
        xs[c * ls + H] = E.re - WO.re;  // X_H = E_0 - O_0 (w^0 = 1)
    }
    __syncthreads();
    if (OP == OP_FWD) {
      for (int e = tid; e < C * N; e += nthr) {
        int c, i;
        split_e(e, &c, &i);
        const int64_t p = gidx(c, i);
        if (p >= 0) out[p] = (TO)(xs[c * ls + i] * A.outscale);
      }
      return;
    }
    for (int e = tid; e < C * N; e += nthr) {
      const int c = e / N, k = e - c * N;
      int li, lo;
      (void)line_base(A, t, c, &li, &lo);
      const bool valid = A.axis == 0 ? (int64_t)t * C + c < A.lines : li < A.n0;
      TC rest = TC(0);
      if (valid) {
        rest = A.lam0[li];
        if (A.lam1) rest += A.lam1[lo];
      }
      const TC l = (rest + Tb.lam[k]) * A.lscale;  // the table is by slot
      const TC X = xs[c * ls + k];
      if (valid && k == 0 && rest == TC(0) && A.bmean) *A.bmean = (double)X * A.meannorm;
      xs[c * ls + k] = l != TC(0) ? X / l : TC(0);
    }
    __syncthreads();
  } else {
    for (int e = tid; e < C * N; e += nthr) {
      int c, i;
      split_e(e, &c, &i);
      const int64_t p = gidx(c, i);
      xs[c * ls + i] = p >= 0 ? (TC)in[p] : TC(0);
    }
    __syncthreads();
  }
  cplx<TC>* za = reinterpret_cast<cplx<TC>*>(s0);
  for (int e = tid; e < C * H; e += nthr) {
    const int c = e / H, k = e - c * H;
    const TC* x = xs + c * ls;
    // X_k = (slot k, slot N-k); X_{H-k} = (slot H-k, slot H+k); k = 0: X_0, X_H real
    za[c * lsc + k] = pre_own_per(x[k], k ? x[N - k] : TC(0), x[H - k], k ? x[H + k] : TC(0),
                                  Tb.tN[k]);
  }
  __syncthreads();
  const TC* er = reinterpret_cast<const TC*>(
      fft_lds_mixed<TC, true>(za, reinterpret_cast<cplx<TC>*>(s1), lsc, C, H, A, tid, nthr));
  for (int e = tid; e < C * N; e += nthr) {
    int c, i;
    split_e(e, &c, &i);
    const int64_t p = gidx(c, i);
    if (p < 0) continue;
    const TC v = er[c * ls + i] * A.outscale;
    if (ST == ST_ACCUM)
      reinterpret_cast<double*>(A.out)[p] = A.rphi[p] + (double)v;
    else
      out[p] = (TO)v;
  }
}

// ---- deterministic mean ----------------------------------------------------
__global__ void __launch_bounds__(256) partial_sum_f64(const double* __restrict__ x, int64_t n,
                                                       double* __restrict__ part,
                                                       const int32_t* __restrict__ skip) {
  __shared__ double red[256];
  if (skip && *skip) return;
  // four partial sums per thread, so that four loads are in flight
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (; i + 3 * stride < n; i += 4 * stride) {
    a0 += x[i];
    a1 += x[i + stride];
    a2 += x[i + 2 * stride];
    a3 += x[i + 3 * stride];
  }
  for (; i < n; i += stride) a0 += x[i];
  red[threadIdx.x] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// The same partial sums with the trapezoid weights of a vertex grid: each
// axis weighs its two end points by 1/2 (the zero mode of the DCT-I).
__global__ void __launch_bounds__(256) partial_wsum_f64(const double* __restrict__ x, int64_t n,
                                                        int32_t n0, int32_t n1, int32_t n2,
                                                        double* __restrict__ part,
                                                        const int32_t* __restrict__ skip) {
  __shared__ double red[256];
  if (skip && *skip) return;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t r = i / n0;
    const int a = (int)(i - r * n0), b = (int)(r % n1), c = (int)(r / n1);
    double w = 1.0;
    if (a == 0 || a == n0 - 1) w *= 0.5;
    if (b == 0 || b == n1 - 1) w *= 0.5;
    if (n2 > 1 && (c == 0 || c == n2 - 1)) w *= 0.5;
    acc += w * x[i];
  }
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
  const double mv = m[0];
  // four elements per thread and step, their loads in flight together
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const double v0 = x[i], v1 = x[i + stride], v2 = x[i + 2 * stride], v3 = x[i + 3 * stride];
    x[i] = v0 - mv;
    x[i + stride] = v1 - mv;
    x[i + 2 * stride] = v2 - mv;
    x[i + 3 * stride] = v3 - mv;
  }
  for (; i < n; i += stride) x[i] -= mv;
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

int g_cu_count = 0;

int cu_count() {
  if (g_cu_count == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        v <= 0)
      v = 256;
    g_cu_count = v;
  }
  return g_cu_count;
}

// Halves the lines per tile of a generic-kernel pass while the pass would
// give the device fewer than two workgroups per compute unit: on small grids
// (the 400 x 400 grids of Sec. 3) one or two lines per group fill the device
// better than 128-byte row segments, and their data sits in the caches.
// `tiles` is the tile count at C; halving C keeps C a divisor of the counts.
int fill_device(int C, int64_t tiles) {
  const int64_t want = 2 * (int64_t)cu_count();
  while (C > 1 && tiles < want) {
    C >>= 1;
    tiles *= 2;
  }
  return C;
}

// Chooses lines per tile and threads for one pass of the generic kernel
// (two LDS buffers of C lines; C a power of two that divides lines_x, the
// row count or the x extent).
template <typename TC>
void tile_shape(int axis, int N, int lines_x, int64_t groups, int* C, int* nthr, int* B) {
  const int H = N / 2;
  const int lim = lds_limit();
  int c;
  if (axis == 0) {
    c = 1;
    while (2 * c <= 1024 / H) c <<= 1;  // aim for C*H/4 = 256 threads
  } else {
    c = (int)(128 / sizeof(TC));  // 128-byte row segments
    while (c > 1 && (size_t)c * N * sizeof(TC) * 2 > (size_t)lim / 2) c >>= 1;
  }
  while (c > 1 && (c > lines_x || lines_x % c)) c >>= 1;
  while (c > 1 && (size_t)c * N * sizeof(TC) * 2 > (size_t)lim) c >>= 1;
  c = fill_device(c, (int64_t)(lines_x / c) * groups);
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

// Radices of the generic kernel's FFT of half length H: eights, then a four
// or a two, then the odd primes.
int generic_radices(int H, int* rad) {
  int n = 0;
  for (int r : {8, 4, 2}) {
    while (H % r == 0 && H > 1 && n < 24) {
      rad[n++] = r;
      H /= r;
    }
  }
  for (int p = 3; H > 1 && n < 24; p += 2) {
    while (H % p == 0 && n < 24) {
      rad[n++] = p;
      H /= p;
    }
  }
  return H == 1 ? n : -1;
}

bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int rad_values(int N) {
  if (N >= 32 && N <= 4096 && pow2(N)) return 8;
  if (N == 200 || N == 400 || N == 1000 || N == 2000) return 10;
  return 0;
}

namespace {
// Largest power of two not above v (v >= 1).
int floor_pow2(int v) {
  int c = 1;
  while (2 * c <= v) c <<= 1;
  return c;
}
}  // namespace

// Lines per workgroup tile of the register transform along `axis` (0 when
// the axis uses the generic kernel: N < 32 or not a power of two).
int rad_tile_lines(const pc_plan* P, int axis, size_t elem) {
  const int N = P->n[axis];
  const int RT = rad_values(N);
  if (!RT) return 0;
  const int H = N / 2, T = H / RT, LS = H + H / 16 + 1;
  const int64_t lines = P->G / N;
  int C;
  // C (a power of two) divides the row count (rows) or the x extent
  // (strided lines), which need not be powers of two when another axis is
  // not
  if (axis == 0) {
    C = floor_pow2(std::max(1, ROW_THREADS / T));
    while (C > 1 && ((int64_t)C > lines || lines % C)) C >>= 1;
  } else {
    C = (int)(128 / elem);
    while (C > 1 && (C * T > COL_MAX_THREADS || C > P->n[0] || P->n[0] % C)) C >>= 1;
  }
  while (C > 1 && (size_t)C * LS * 2 * elem > (size_t)lds_limit()) C >>= 1;
  // small grids (the 400 x 400 grid of Sec. 3): fewer lines per group, so
  // that every compute unit gets work
  return fill_device(C, lines / C);
}

// Lines per workgroup tile of the generic kernel for a Neumann axis (the
// choice of tile_shape) and for a periodic axis (rdft_lines), for elements
// of `elem` bytes.
static int generic_tile_lines(const pc_plan* P, int axis, size_t elem, int* nthr, int* B) {
  const int N = P->n[axis];
  const int64_t lines = P->G / N;
  int C = 1, t = 64, b = 1;
  if (P->bc[axis] == PC_BC_PERIODIC) {
    const size_t per_line = (size_t)3 * (N + 2) * elem;
    const int cmax = (int)std::max<size_t>(1, (size_t)lds_limit() / per_line);
    const int want = axis == 0 ? std::max(1, 2048 / N) : (int)(128 / elem);
    while (2 * C <= std::min(want, cmax)) C <<= 1;
    C = fill_device(C, axis == 0 ? (lines + C - 1) / C
                                 : (int64_t)((P->n[0] + C - 1) / C) * (lines / P->n[0]));
  } else if (elem == 8) {
    tile_shape<double>(axis, N, axis == 0 ? (int)lines : P->n[0], axis == 0 ? 1 : lines / P->n[0],
                       &C, &t, &b);
  } else {
    tile_shape<float>(axis, N, axis == 0 ? (int)lines : P->n[0], axis == 0 ? 1 : lines / P->n[0],
                      &C, &t, &b);
  }
  if (nthr) *nthr = t;
  if (B) *B = b;
  return C;
}

// Tile geometry of a pass along `axis` as the tile lists of the resident
// transforms number the tiles: C lines per tile, tx tiles along x (strided
// passes: tile = o * tx + i / C), ntile tiles in all.  Register kernels take
// whole tiles; the periodic generic kernel masks a partial last tile.
PassTiles pass_tiles(const pc_plan* P, int axis, size_t elem) {
  PassTiles pt{};
  const int N = P->n[axis];
  const int64_t lines = P->G / N;
  const bool reg = rad_values(N) != 0;
  const bool masked = !reg && P->bc[axis] == PC_BC_PERIODIC;
  pt.C = reg ? rad_tile_lines(P, axis, elem) : generic_tile_lines(P, axis, elem, nullptr, nullptr);
  if (axis == 0) {
    pt.tx = 1;
    pt.ntile = masked ? (lines + pt.C - 1) / pt.C : lines / pt.C;
  } else {
    pt.tx = masked ? (P->n[0] + pt.C - 1) / pt.C : P->n[0] / pt.C;
    pt.ntile = pt.tx * (lines / P->n[0]);
  }
  return pt;
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
  {
    const double L = (double)P->n[axis] * P->h[axis];
    const double w = (P->bc[axis] == PC_BC_PERIODIC ? 2.0 : 1.0) * 3.14159265358979323846 / L;
    A.lams = (TC)(-(w * w));
  }
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
  // mode 0 of a line is 2 sum (cosine transform), sum (real DFT) or twice
  // the trapezoid sum (DCT-I of a vertex axis)
  double norm = 1.0;
  for (int a = 0; a < P->d; ++a)
    norm *= P->vertex ? 2.0 * (P->n[a] - 1)
                      : (P->bc[a] == PC_BC_PERIODIC ? 1.0 : 2.0) * P->n[a];
  A.meannorm = 1.0 / norm;
  A.own_table = P->eig == PC_EIG_SPECTRAL;
  A.perm = 0;
  for (int a = 0; a < P->d; ++a)
    if (P->bc[a] == PC_BC_PERIODIC) A.perm |= 1 << a;
  int64_t lines = P->G / A.N;
  A.lines = lines;
  if (P->vertex) {
    // DCT-I kernel: C lines of the even extension (NS reals) in three LDS
    // regions; partial tiles are masked, so C need not divide the counts
    const int Hv = A.N - 1, NS = 2 * Hv;
    A.nrad = generic_radices(Hv, A.rad);
    if (A.nrad < 0) return fail(PC_ERR_UNSUPPORTED_SIZE, "transform length has too many factors");
    A.outscale = (OP == OP_FWD) ? TC(1) : TC(1.0 / (double)Hv);
    A.pad = 2;
    const size_t per_line = (size_t)3 * (NS + A.pad) * sizeof(TC);
    const int cmax = (int)std::max<size_t>(1, (size_t)lds_limit() / per_line);
    int C = 1;
    const int want = axis == 0 ? std::max(1, 2048 / NS) : (int)(128 / sizeof(TC));
    while (2 * C <= std::min(want, cmax)) C <<= 1;
    C = fill_device(C, axis == 0 ? (lines + C - 1) / C
                                 : (int64_t)((P->n[0] + C - 1) / C) * (lines / P->n[0]));
    if ((size_t)C * per_line > (size_t)lds_limit())
      return fail(PC_ERR_UNSUPPORTED_SIZE, "transform line does not fit in LDS");
    if ((int64_t)C * NS >= (1 << 17))  // div_small's range (butterfly indices)
      return fail(PC_ERR_UNSUPPORTED_SIZE, "transform tile too large");
    A.C = C;
    int64_t ntile;
    if (axis == 0) {
      ntile = (lines + C - 1) / C;
    } else {
      A.tx = (P->n[0] + C - 1) / C;
      ntile = (int64_t)A.tx * (lines / P->n[0]);
    }
    int nthr = std::min(1024, std::max(64, C * Hv / 2));
    nthr = (nthr + 63) / 64 * 64;
    const size_t lds = (size_t)C * per_line;
    const void* fn = (const void*)dct1_lines<TC, TI, TO, OP, LD, ST>;
    if (lds > 65536)
      PC_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((dct1_lines<TC, TI, TO, OP, LD, ST>), dim3((unsigned)ntile), dim3(nthr), lds,
                       s, A);
    PC_HIP_CHECK(hipGetLastError());
    return PC_OK;
  }
  if (const int RT = rad_values(A.N)) {
    // register kernel: T = H/RT threads per line, C lines per group
    const int T = H / RT;
    const int LS = H + H / 16 + 1;
    const int C = rad_tile_lines(P, axis, sizeof(TC));
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
    // the row residual loader stages the tile's float64 phi in the same LDS
    if (LD == LD_RESID && axis == 0) lds = std::max(lds, (size_t)C * A.N * sizeof(double));
    if (lds > (size_t)lds_limit()) return fail(PC_ERR_UNSUPPORTED_SIZE, "transform tile does not fit in LDS");
    const int key = (RT == 8 ? logH : H) * 32 + RT;
    if (P->bc[axis] == PC_BC_PERIODIC)
      return rad_launch<TC, TI, TO, OP, LD, ST, true>(A, key, dim3(ntile), dim3(C * T), lds, s);
    return rad_launch<TC, TI, TO, OP, LD, ST, false>(A, key, dim3(ntile), dim3(C * T), lds, s);
  }
  if (P->bc[axis] == PC_BC_PERIODIC) {
    // packed real DFT on the mixed-radix kernel (short or not a power of two)
    A.nrad = generic_radices(H, A.rad);
    if (A.nrad < 0) return fail(PC_ERR_UNSUPPORTED_SIZE, "transform length has too many factors");
    A.pad = 2;
    const size_t per_line = (size_t)3 * (A.N + A.pad) * sizeof(TC);
    const int C = generic_tile_lines(P, axis, sizeof(TC), nullptr, nullptr);
    if ((size_t)C * per_line > (size_t)lds_limit())
      return fail(PC_ERR_UNSUPPORTED_SIZE, "transform line does not fit in LDS");
    if ((int64_t)C * A.N >= (1 << 17))  // div_small's range (butterfly indices)
      return fail(PC_ERR_UNSUPPORTED_SIZE, "transform tile too large");
    A.C = C;
    int64_t ntile;
    if (axis == 0) {
      ntile = (lines + C - 1) / C;
    } else {
      A.tx = (P->n[0] + C - 1) / C;
      ntile = (int64_t)A.tx * (lines / P->n[0]);
    }
    if (tiles) {
      if (ntiles <= 0) return PC_OK;
      ntile = ntiles;
    }
    int nthr = std::min(1024, std::max(64, C * H / 2));
    nthr = (nthr + 63) / 64 * 64;
    const size_t lds = (size_t)C * per_line;
    const void* fn = (const void*)rdft_lines<TC, TI, TO, OP, LD, ST>;
    if (lds > 65536)
      PC_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((rdft_lines<TC, TI, TO, OP, LD, ST>), dim3((unsigned)ntile), dim3(nthr), lds,
                       s, A);
    PC_HIP_CHECK(hipGetLastError());
    return PC_OK;
  }
  A.nrad = generic_radices(H, A.rad);
  if (A.nrad < 0) return fail(PC_ERR_UNSUPPORTED_SIZE, "transform length has too many factors");
  int nthr, B;
  const int C = generic_tile_lines(P, axis, sizeof(TC), &nthr, &B);
  A.C = C;
  if (C > nthr) return fail(PC_ERR_UNSUPPORTED_SIZE, "transform tile has more lines than threads");
  if ((int64_t)C * A.N >= (1 << 17))  // div_small's range (butterfly indices)
    return fail(PC_ERR_UNSUPPORTED_SIZE, "transform tile too large");
  int ntile;
  if (axis == 0) {
    ntile = (int)((lines + C - 1) / C);
    if (lines % C) return fail(PC_ERR_UNSUPPORTED_SIZE, "row count not a multiple of the tile");
  } else {
    A.tx = P->n[0] / C;
    ntile = (int)(lines / C);
  }
  if (tiles) {
    if (ntiles <= 0) return PC_OK;
    ntile = ntiles;
  }
  // pad each LDS line by one complex when it fits (fewer bank conflicts)
  A.pad = ((size_t)C * (A.N + 2) * sizeof(TC) * 2 <= (size_t)lds_limit()) ? 2 : 0;
  size_t lds = (size_t)C * (A.N + A.pad) * sizeof(TC) * 2;
  if (lds > (size_t)lds_limit()) return fail(PC_ERR_UNSUPPORTED_SIZE, "transform line too long");
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

// Mean of a grid field: plain on a cell-centred grid, trapezoid-weighted
// (the DCT-I zero mode) on a vertex grid.
int grid_mean_f64(const pc_plan* P, const double* x, double* partial, int nblk, double* out_dev,
                  hipStream_t s, const int32_t* skip) {
  if (!P->vertex) return mean_f64(x, P->G, partial, nblk, out_dev, s, skip);
  double wsum = 1.0;
  for (int a = 0; a < P->d; ++a) wsum *= (double)(P->n[a] - 1);
  hipLaunchKernelGGL(partial_wsum_f64, dim3(nblk), dim3(256), 0, s, x, P->G, P->n[0], P->n[1],
                     P->d == 3 ? P->n[2] : 1, partial, skip);
  hipLaunchKernelGGL(finish_mean, dim3(1), dim3(256), 0, s, partial, nblk, 1.0 / wsum, out_dev,
                     skip);
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

// Defect correction (means trapezoid-weighted on a vertex grid): bbar =
// mean(b) in float64; phi0 = S32(b - bbar) (warm: phi0 = the phi passed in,
// the solution of a nearby right-hand side); then
// `sweeps` times r = (b - bbar) - lap_h phi (float64, fused into the first
// pass), phi += S32(r) (accumulated in float64 in the last pass); finally
// (remove_mean) mean(phi) is removed in float64.  The mean is taken out in float64 before
// each conversion to float32: left in, the compatibility defect would
// dominate the float32 rounding of the much smaller residual.
int solve_mixed(const pc_plan* P, const double* b, double* phi, int sweeps, double* bmean_dev,
                pc_workspace* ws, hipStream_t s, double sigma, const int32_t* skip, bool warm,
                bool remove_mean, bool bmean_given, bool delta) {
  if (!ws || !ws->w32) return fail(PC_ERR_INVALID_ARG, "mixed solve needs a MIXED workspace");
  float* w = ws->w32;
  double* bm = bmean_dev ? bmean_dev : ws->scal;
  if (!bmean_given) PC_TRY(grid_mean_f64(P, b, ws->partial, ws->nblk, bm, s, skip));
  if (!warm)
    PC_TRY((solve_passes<float, double, double, LD_PLAIN, ST_PLAIN>(
        P, P->ax32, b, phi, w, nullptr, nullptr, nullptr, s, bm, sigma, skip)));
  int first = 0;
  if (warm && delta && ws->delta) {
    // First sweep of a warm start: the residual of the previous solution is
    // the change of the right-hand side (the previous residual left after
    // its sweeps is below the float32 solve's own error), nonzero only at
    // the near-IB points, so only the lines holding them are transformed
    // forward; the division drops the mean (mode 0).  The inverse runs on
    // every line and adds the correction to phi.
    const int d = P->d;
    PC_TRY((launch_pass<float, double, float, OP_FWD, LD_PLAIN, ST_PLAIN>(
        P, 0, ws->dgrid, ws->dspec[0], P->ax32, nullptr, nullptr, nullptr, s, nullptr, 1.0, skip,
        ws->tl[TL_FWD0], ws->ntl[TL_FWD0])));
    const float* spec = ws->dspec[0];
    if (d == 3) {
      PC_TRY((launch_pass<float, float, float, OP_FWD, LD_PLAIN, ST_PLAIN>(
          P, 1, ws->dspec[0], ws->dspec[1], P->ax32, nullptr, nullptr, nullptr, s, nullptr, 1.0,
          skip, ws->tl[TL_FWD1], ws->ntl[TL_FWD1])));
      spec = ws->dspec[1];
    }
    PC_TRY((launch_pass<float, float, float, OP_FDI, LD_PLAIN, ST_PLAIN>(
        P, d - 1, spec, w, P->ax32, nullptr, nullptr, nullptr, s, nullptr, sigma, skip)));
    if (d == 3)
      PC_TRY((launch_pass<float, float, float, OP_INV, LD_PLAIN, ST_PLAIN>(
          P, 1, w, w, P->ax32, nullptr, nullptr, nullptr, s, nullptr, 1.0, skip)));
    PC_TRY((launch_pass<float, float, double, OP_INV, LD_PLAIN, ST_ACCUM>(
        P, 0, w, phi, P->ax32, nullptr, phi, nullptr, s, nullptr, 1.0, skip)));
    first = 1;
  }
  for (int it = first; it < sweeps; ++it) {
    PC_TRY((solve_passes<float, double, double, LD_RESID, ST_ACCUM>(
        P, P->ax32, b, phi, w, b, phi, nullptr, s, bm, sigma, skip)));
  }
  if (remove_mean) PC_TRY(remove_mean_f64(P, phi, ws, s, skip));
  return PC_OK;
}

int remove_mean_f64(const pc_plan* P, double* phi, pc_workspace* ws, hipStream_t s,
                    const int32_t* skip) {
  PC_TRY(grid_mean_f64(P, phi, ws->partial, ws->nblk, ws->scal + 3, s, skip));
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

// Every kernel of a cell-centred grid takes tile lists (the register
// kernels, and the generic ones for lengths that are short or not powers of
// two); the vertex grid's DCT-I kernel does not.
bool resident_possible(const pc_plan* P, int64_t n_ib, int mode) {
  if (n_ib == 0 || (mode != PC_F64 && mode != PC_F32)) return false;
  return !P->vertex;
}

bool delta_possible(const pc_plan* P, int64_t n_ib, int mode) {
  return mode == PC_MIXED && n_ib > 0 && !P->vertex;
}

bool resident_ok(const pc_plan* P, const pc_geom* g, int mode) {
  return g && resident_possible(P, g->n_ib, mode);
}

int64_t resident_tiles_max(const pc_plan* P, size_t elem) {
  const int64_t t0 = pass_tiles(P, 0, elem).ntile;
  const int64_t t1 = P->d == 3 ? pass_tiles(P, 1, elem).ntile : 0;
  return 3 * (t0 + t1);
}

void resident_tiles(const pc_plan* P, size_t elem, const std::vector<int32_t>& near_pts,
                    const std::vector<int32_t>& ib_base, int m, std::vector<int32_t> out[6]) {
  for (int l = 0; l < 6; ++l) out[l].clear();
  const int64_t n0 = P->n[0], n1 = P->n[1], n2 = P->d == 3 ? P->n[2] : 1;
  const PassTiles p0 = pass_tiles(P, 0, elem);
  const int C0 = p0.C;
  const int64_t t0 = p0.ntile;  // x-line tiles: line j + n1 k, tile line / C0
  std::vector<char> f0(t0, 0), i0(t0, 0);
  for (int32_t q : near_pts) f0[(q / n0) / C0] = 1;
  // lines read by the B+V gradient: the m x m (x m) block at each corner
  std::vector<char> ibplane(n2, 0);
  for (int32_t qb : ib_base) {
    // a negative base marks a block that wraps around a periodic axis
    const int64_t q = qb >= 0 ? qb : ~qb;
    const int64_t j0 = (q / n0) % n1, k0 = q / (n0 * n1);
    const int kn = P->d == 3 ? m : 1;
    for (int kk = 0; kk < kn; ++kk) {
      const int64_t kw = (k0 + kk) % n2;
      ibplane[kw] = 1;
      for (int jj = 0; jj < m; ++jj) i0[((j0 + jj) % n1 + n1 * kw) / C0] = 1;
    }
  }
  for (int64_t t = 0; t < t0; ++t) {
    if (f0[t]) out[TL_FWD0].push_back((int32_t)t);
    out[i0[t] ? TL_INV0_IB : TL_INV0_REST].push_back((int32_t)t);
    // the x-inverse runs in place on whole tiles, whose lines may reach into
    // further planes (C0 > n1): those planes need their y-inverse first
    if (i0[t])
      for (int64_t l = t * C0; l < std::min((t + 1) * C0, n1 * n2); ++l) ibplane[l / n1] = 1;
  }
  if (P->d == 3) {
    // y-line tiles: C1 adjacent x positions of one plane k, tile = k * tx + i / C1
    const PassTiles p1 = pass_tiles(P, 1, elem);
    const int64_t tx = p1.tx;
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
