// Transfers between nodes and grid and the whole pressure-correction
// sub-step (Sec. 2.3).
//
//   div_to_grid   b_p = sum_a sum_i c^a_{p,i} v_a[idx_{p,i}]      (RHS of Eq. 20)
//   grad_to_nodes G_a(n) = sum_j c^a_{n,j} phi[src_{n,j}]          (Eqs. 18-19)
//   ib_update     g = -u* + G at the B+V nodes, criterion sums      (Eq. 19)
//   project       u^{n+1} = u* - G on F, exactly 0 on B+V          (Eq. 18)
//
// The gathers are one thread per target.  Stencil arrays are laid out
// [entry][target] so that a wavefront reads 64 consecutive targets of one
// entry in one coalesced access; they are streamed with non-temporal loads so
// that the gathered field values (re-read by neighbouring targets) keep the
// caches.  In float32 mode the sums are taken relative to the value at the
// first stencil entry: the derivative rows annihilate constants, and the
// differences avoid the cancellation of sum_i c_i v_i (|c| ~ 1/h) in float32.
#include <cmath>
#include <cstring>

#include <chrono>
#include <mutex>

#include "pc_internal.h"

namespace pc {
namespace {

constexpr int XCDS = 8;

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  if (nb % XCDS != 0) return b;
  return (b % XCDS) * (nb / XCDS) + b / XCDS;
}

template <typename T>
__device__ __forceinline__ T ldnt(const T* p) {
  return __builtin_nontemporal_load(p);
}

constexpr int TPB = 256;
constexpr int IBT = 64;  // threads per block of the IB iteration kernel (one wavefront)

// ---- div_to_grid (all grid points) -------------------------------------------
// Order of the grid points over the workgroups of a 3D launch.  A workgroup
// takes TPB consecutive points of one x row (coalesced stencil streams);
// with `on`, the workgroups that one XCD runs in a row cover blocks of
// SY rows x SZ planes (all of each row), swept along y within slabs of SZ
// planes, so that the node values gathered for a block (the stencils reach
// one or two lines beyond it in every direction) are fetched into that
// XCD's L2 about once instead of once per plane that needs them.
struct DivMap {
  int on;
  int segs;       // TPB-point segments per row (n0 / TPB)
  int tiles_y;    // n1 / SY
  int64_t n0, n1;
};
constexpr int DIV_SY = 8, DIV_SZ = 16;

__device__ __forceinline__ int64_t div_point(int64_t blk, const DivMap& m) {
  if (!m.on) return blk * TPB + threadIdx.x;
  const int64_t per = (int64_t)m.segs * DIV_SY * DIV_SZ;
  const int64_t st = blk / per;
  const int64_t r = blk - st * per;
  const int64_t seg = r % m.segs;
  const int64_t zz = (r / m.segs) % DIV_SZ;
  const int64_t yy = r / ((int64_t)m.segs * DIV_SZ);
  const int64_t ty = st % m.tiles_y, tz = st / m.tiles_y;
  const int64_t y = ty * DIV_SY + yy, z = tz * DIV_SZ + zz;
  return (z * m.n1 + y) * m.n0 + seg * TPB + threadIdx.x;
}

template <typename T, int D, int K, bool LOCALREF>
__global__ void __launch_bounds__(TPB) k_div_all(const int32_t* __restrict__ gidx,
                                                 const T* __restrict__ gcoef, int64_t G, int krt,
                                                 const T* __restrict__ v, int64_t M,
                                                 T* __restrict__ b, DivMap dm) {
  const int k = K > 0 ? K : krt;
  const int64_t p = div_point(xcd_block(blockIdx.x, gridDim.x), dm);
  if (p >= G) return;
  T acc = T(0);
  T ref[D];
  if (LOCALREF) {
    int j0 = ldnt(gidx + p);
#pragma unroll
    for (int a = 0; a < D; ++a) ref[a] = v[a * M + j0];
  }
  // four entries at a time (a full unroll of the 27 entries, every index
  // load issued up front, was 2.6% slower at 512^3)
#pragma unroll 4
  for (int i = 0; i < k; ++i) {
    int j = ldnt(gidx + (int64_t)i * G + p);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T c = ldnt(gcoef + ((int64_t)a * k + i) * G + p);
      T val = v[a * M + j];
      if (LOCALREF) val -= ref[a];
      acc += c * val;
    }
  }
  b[p] = acc;
}

// ---- criterion of the IB iteration (Sec. 2.3) ------------------------------------
// The partial sums of k_ib_step's blocks, added in block order by one
// workgroup of TPB threads, give sums[0..1], the converged flag conv[0], the
// iteration count conv[1], conv[4] = 1 - converged (the guard of work queued
// for the converged case) and, if given, the flag and sums in coherent
// pinned host memory that the host polls.  Every thread of the block gets
// the converged flag; only a block with `write` set stores anything, so
// several blocks can evaluate the same criterion and agree on it.
struct IbClose {
  const double* part;  // [2 nblk] partial sums (numerator, denominator)
  int nblk;
  double tol;
  double* sums;
  int32_t* conv;
  int32_t* host_flag;  // nullable
  double* host_sums;
};

__device__ int ib_close_block(const IbClose& C, bool write) {
  __shared__ double rn[TPB / 64], rd[TPB / 64];
  __shared__ int cvs;
  double num = 0.0, den = 0.0;
  for (int i = threadIdx.x; i < C.nblk; i += TPB) {
    num += C.part[2 * i];
    den += C.part[2 * i + 1];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    num += __shfl_down(num, off, 64);
    den += __shfl_down(den, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    rn[threadIdx.x >> 6] = num;
    rd[threadIdx.x >> 6] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    num = rn[0];
    den = rd[0];
#pragma unroll
    for (int w = 1; w < TPB / 64; ++w) {
      num += rn[w];
      den += rd[w];
    }
    const int32_t cv = (num < C.tol * den || num == 0.0) ? 1 : 0;
    cvs = cv;
    if (write) {
      C.sums[0] = num;
      C.sums[1] = den;
      C.conv[0] = cv;
      C.conv[1] += 1;
      C.conv[4] = 1 - cv;
      if (C.host_flag) {
        // the sums first, then the flag that says they are there
        C.host_sums[0] = num;
        C.host_sums[1] = den;
        __threadfence_system();
        *C.host_flag = cv;
        __threadfence_system();
      }
    }
  }
  __syncthreads();
  return cvs;
}

// ---- div_to_grid near the IB: b[near[q]] = base[q] (or b) + D(g) -----------
// g lives on the B+V nodes only, so each near point sums over its B+V
// entries (ELL layout, coalesced over q).
// With CLOSE the launch first evaluates the criterion of the iteration that
// produced g (every block, identically; block 0 stores it), which saves the
// criterion its own launch, and updates b only if that iteration has not
// converged.
// b[near[q]] = base[q] (or b, ADD) + D(g) at near point q; returns D(g).
template <typename T, int D, bool ADD, int WT>
__device__ __forceinline__ T near_update(const int32_t* __restrict__ near, int64_t q, int64_t nns,
                                         const int32_t* __restrict__ nslot,
                                         const T* __restrict__ ncoef, const T* __restrict__ gib,
                                         int64_t nib, const T* __restrict__ base,
                                         T* __restrict__ b, T* __restrict__ dgrid) {
  // WT is the table width itself (padding entries have slot -1 and
  // coefficient exactly 0), so every load is unconditional and all of them
  // are in flight together
  int s[WT];
#pragma unroll
  for (int e = 0; e < WT; ++e) s[e] = max(nslot[(int64_t)e * nns + q], 0);
  T acc = T(0);
#pragma unroll
  for (int e = 0; e < WT; ++e) {
#pragma unroll
    for (int a = 0; a < D; ++a) acc += ncoef[((int64_t)a * WT + e) * nns + q] * gib[a * nib + s[e]];
  }
  int64_t p = near[q];
  if (ADD) {
    b[p] += acc;
  } else if (dgrid) {
    // the change of b at this point, for the float32 correction of PC_MIXED
    const T nb = base[q] + acc;
    dgrid[p] = nb - b[p];
    b[p] = nb;
  } else {
    b[p] = base[q] + acc;
  }
  return acc;
}

// With MEAN each block also adds up its D(g) values (fixed order) into
// part[blockIdx.x]: b changes only at the near points, so the mean of b is
// the mean of b_u plus their sum over the grid size (k_mean_near).
template <typename T, int D, bool ADD, int WT, bool CLOSE, bool MEAN>
__global__ void __launch_bounds__(TPB) k_div_near(const int32_t* __restrict__ near, int64_t nnear,
                                                  int64_t nns, const int32_t* __restrict__ nslot,
                                                  const T* __restrict__ ncoef,
                                                  const T* __restrict__ gib, int64_t nib,
                                                  const T* __restrict__ base, T* __restrict__ b,
                                                  const int32_t* __restrict__ skip, IbClose close,
                                                  double* __restrict__ part,
                                                  T* __restrict__ dgrid) {
  if (CLOSE) {
    // block 0 may set the flag while other blocks start: read it once per
    // block, so that no thread leaves before the criterion's barriers
    __shared__ int sk;
    if (threadIdx.x == 0) sk = skip ? *skip : 0;
    __syncthreads();
    if (sk || ib_close_block(close, blockIdx.x == 0)) return;
  } else if (skip && *skip) {
    return;
  }
  int64_t q = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (MEAN) {
    // every thread of the block reaches the reduction
    T acc = T(0);
    if (q < nnear) acc = near_update<T, D, ADD, WT>(near, q, nns, nslot, ncoef, gib, nib, base, b, dgrid);
    __shared__ double red[TPB / 64];
    double v = (double)acc;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = red[0];
#pragma unroll
      for (int w = 1; w < TPB / 64; ++w) t += red[w];
      part[blockIdx.x] = t;
    }
    return;
  }
  if (q >= nnear) return;
  (void)near_update<T, D, ADD, WT>(near, q, nns, nslot, ncoef, gib, nib, base, b, dgrid);
}

// out[0] = mean_u[0] + (sum of part[0..nb)) * inv_g, the sum in a fixed order.
__global__ void __launch_bounds__(TPB) k_mean_near(const double* __restrict__ part, int nb,
                                                   const double* __restrict__ mean_u,
                                                   double inv_g, double* __restrict__ out,
                                                   const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double red[TPB / 64];
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += TPB) v += part[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
#pragma unroll
    for (int w = 1; w < TPB / 64; ++w) t += red[w];
    out[0] = mean_u[0] + t * inv_g;
  }
}

// ---- grad_to_nodes (all nodes), optionally fused with the projection ---------
struct BlockOffsets {
  int32_t off[PC_MAX_K_NODE];  // flat offset of block entry o from the low corner
  int32_t n0, n1, n2, m;       // grid and block shape, for blocks that wrap
  int32_t l0, l1;              // log2 n0, log2 n1, or -1 when n0 or n1 is not a power of two
  int32_t per;                 // bit a set: axis a is periodic
};

// Wrap thresholds of one node's block on a grid with periodic axes: block
// entry o with offsets (ox, oy, oz) from the low corner c0 runs past the last
// line along x when ox >= tx (and so on); its source is then one box length
// back along that axis.  A Neumann axis never wraps (threshold m).
struct BlockWrap {
  int tx, ty, tz;
};

__device__ __forceinline__ BlockWrap block_wrap(int64_t c0, const BlockOffsets& bo) {
  int i0, j0, k0;
  if (bo.l0 >= 0) {
    i0 = (int)(c0 & (bo.n0 - 1));
    j0 = (int)((c0 >> bo.l0) & (bo.n1 - 1));
    k0 = (int)(c0 >> (bo.l0 + bo.l1));
  } else {
    const int64_t r = c0 / bo.n0;
    i0 = (int)(c0 - r * bo.n0);
    k0 = (int)(r / bo.n1);
    j0 = (int)(r - (int64_t)k0 * bo.n1);
  }
  BlockWrap w;
  w.tx = (bo.per & 1) ? bo.n0 - i0 : bo.m;
  w.ty = (bo.per & 2) ? bo.n1 - j0 : bo.m;
  w.tz = (bo.per & 4) ? bo.n2 - k0 : bo.m;
  return w;
}

__device__ __forceinline__ int64_t wrap_adjust(int64_t src, int ox, int oy, int oz,
                                               const BlockWrap& w, const BlockOffsets& bo) {
  const int64_t plane = (int64_t)bo.n0 * bo.n1;
  if (ox >= w.tx) src -= bo.n0;
  if (oy >= w.ty) src -= plane;
  if (oz >= w.tz) src -= plane * bo.n2;
  return src;
}

// WRAP: the grid has periodic axes, and blocks next to a periodic face wrap
// around it (their base is marked by a one's complement); every lane then
// applies its own wrap thresholds, so such blocks cost no divergence.
template <typename T, int D, int BN, bool LOCALREF, bool PROJECT, bool WRAP>
__global__ void __launch_bounds__(TPB) k_grad_all(const int32_t* __restrict__ nbase,
                                                  const T* __restrict__ ncoef, int64_t M,
                                                  int64_t ms, int bnrt, BlockOffsets bo,
                                                  const T* __restrict__ phi, T scale,
                                                  const T* __restrict__ u,
                                                  T* __restrict__ out,
                                                  const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int bn = BN > 0 ? BN : bnrt;
  // block lines per axis (16 = 4^2 in 2D, 27 = 3^3 in 3D)
  constexpr int MB = BN == 16 && D == 2 ? 4 : (BN == 27 && D == 3 ? 3 : 0);
  const int m = MB > 0 ? MB : bo.m;
  const int64_t n = xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
  if (n >= M) return;
  const int32_t b32 = ldnt(nbase + n);
  const int64_t base = WRAP ? (b32 >= 0 ? b32 : ~b32) : b32;
  BlockWrap w = {0, 0, 0};
  if (WRAP) w = block_wrap(base, bo);
  T acc[D];
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = T(0);
  // u* first (in flight during the gather); u^{n+1} is stored non-temporally
  T uu[D];
  if (PROJECT) {
#pragma unroll
    for (int a = 0; a < D; ++a) uu[a] = ldnt(u + a * M + n);
  }
  T ref = LOCALREF ? phi[base + bo.off[0]] : T(0);
#pragma unroll 9
  for (int o = 0; o < bn; ++o) {
    int64_t src = base + bo.off[o];
    if (WRAP) src = wrap_adjust(src, o % m, (o / m) % m, o / (m * m), w, bo);
    T f = phi[src];
    if (LOCALREF) f -= ref;
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] += ldnt(ncoef + ((int64_t)a * bn + o) * ms + n) * f;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (PROJECT)
      __builtin_nontemporal_store(uu[a] - scale * acc[a], out + a * M + n);
    else
      out[a * M + n] = scale * acc[a];
  }
}

// ---- grad at the B+V nodes (compact stencils) ---------------------------------
template <typename T, int D, bool LOCALREF>
__global__ void __launch_bounds__(TPB) k_grad_ib(const int32_t* __restrict__ ibbase,
                                                 const T* __restrict__ ibcoef, int64_t nib,
                                                 int64_t ibs, int bn,
                                                 BlockOffsets bo, const T* __restrict__ phi,
                                                 T scale, T* __restrict__ out,
                                                 const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (s >= nib) return;
  const int32_t b32 = ibbase[s];
  const int64_t base = b32 >= 0 ? b32 : ~b32;  // ~corner: the block wraps
  const BlockWrap w = block_wrap(base, bo);
  T acc[D];
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = T(0);
  T ref = LOCALREF ? phi[base] : T(0);
  const int m = bo.m;
  for (int o = 0; o < bn; ++o) {
    T f = phi[wrap_adjust(base + bo.off[o], o % m, (o / m) % m, o / (m * m), w, bo)];
    if (LOCALREF) f -= ref;
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] += ibcoef[((int64_t)a * bn + o) * ibs + s] * f;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) out[a * nib + s] = scale * acc[a];
}

// ---- gathers / scatters on the IB list ------------------------------------------
template <typename T>
__global__ void __launch_bounds__(TPB) k_gather_ib(const int32_t* __restrict__ ib, int64_t nib,
                                                   int d, const T* __restrict__ u, int64_t M,
                                                   T* __restrict__ uib) {
  int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (s >= nib) return;
  int64_t n = ib[s];
  for (int a = 0; a < d; ++a) uib[a * nib + s] = u[a * M + n];
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_zero_ib(const int32_t* __restrict__ ib, int64_t nib,
                                                 int d, int64_t M, T* __restrict__ out,
                                                 const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (s >= nib) return;
  int64_t n = ib[s];
  for (int a = 0; a < d; ++a) out[a * M + n] = T(0);
}

// The work after the last iteration at the B+V nodes, in one launch:
// u^{n+1} = 0 there (Eqs. 18 and 19 cancel), the final force to the caller
// (g_out, nullable) and, with hs, the statistics into pinned host memory
// (bmean, criterion sums, flags).
template <typename T>
__global__ void __launch_bounds__(TPB) k_finish_ib(const int32_t* __restrict__ ib, int64_t nib,
                                                   int d, int64_t M, T* __restrict__ out,
                                                   const T* __restrict__ gib, T* __restrict__ g_out,
                                                   const double* __restrict__ scal,
                                                   const int32_t* __restrict__ flag, double* hs,
                                                   int32_t* hf, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  if (hs && blockIdx.x == 0 && threadIdx.x < 64) {
    if (threadIdx.x < 3) hs[threadIdx.x] = scal[threadIdx.x];
    if (threadIdx.x < 2) hf[threadIdx.x + 2] = flag[threadIdx.x];
    __threadfence_system();
  }
  int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (s >= nib) return;
  int64_t n = ib[s];
  for (int a = 0; a < d; ++a) {
    out[a * M + n] = T(0);
    if (g_out) g_out[a * nib + s] = gib[a * nib + s];
  }
}

// ---- IB-force update with deterministic criterion sums ----------------------------
constexpr int IB_BLOCKS = 256;

template <typename T, int D>
__global__ void __launch_bounds__(TPB) k_ib_update(const T* __restrict__ uib,
                                                   const T* __restrict__ grad, T* __restrict__ g,
                                                   int64_t nib, double* __restrict__ part,
                                                   const int32_t* __restrict__ skip) {
  __shared__ double rn[TPB], rd[TPB];
  if (skip && *skip) return;
  double num = 0.0, den = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x; s < nib;
       s += (int64_t)gridDim.x * TPB) {
    double mn = 0.0, mo = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T gn = -uib[a * nib + s] + grad[a * nib + s];
      T go = g[a * nib + s];
      mn += (double)gn * (double)gn;
      mo += (double)go * (double)go;
      g[a * nib + s] = gn;
    }
    double dm = sqrt(mn) - sqrt(mo);
    num += dm * dm;
    den += mo;
  }
  rn[threadIdx.x] = num;
  rd[threadIdx.x] = den;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rn[threadIdx.x] += rn[threadIdx.x + w];
      rd[threadIdx.x] += rd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = rn[0];
    part[2 * blockIdx.x + 1] = rd[0];
  }
}

// conv[0]: converged flag (also the skip flag of later iterations);
// conv[1]: number of iterations run.
__global__ void __launch_bounds__(TPB) k_ib_finish(const double* __restrict__ part, int nblk,
                                                   double tol, double* __restrict__ sums,
                                                   int32_t* __restrict__ conv, int count) {
  __shared__ double rn[TPB], rd[TPB];
  if (count && conv[0]) return;
  double num = 0.0, den = 0.0;
  for (int i = threadIdx.x; i < nblk; i += TPB) {
    num += part[2 * i];
    den += part[2 * i + 1];
  }
  rn[threadIdx.x] = num;
  rd[threadIdx.x] = den;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rn[threadIdx.x] += rn[threadIdx.x + w];
      rd[threadIdx.x] += rd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sums[0] = rn[0];
    sums[1] = rd[0];
    conv[0] = (rn[0] < tol * rd[0] || rn[0] == 0.0) ? 1 : 0;
    if (count) conv[1] += 1;
  }
}

// ---- fused IB step: gradient at the B+V nodes, force update, criterion ----------
// Every thread takes one B+V node, computes grad phi there (sigma * grad p),
// g_new = -u* + grad and the two criterion terms, and overwrites g.  Each
// block (one wavefront) writes its partial sums to part[]; the criterion
// (ib_close_block) adds them in the next launch: k_ib_close, or the next
// iteration's RHS update near the IB.  (A last-block-finishes scheme needs a
// device-scope fence and an atomic per block, which cost more than a second
// launch here.)
template <typename T, int D, int BN>
__global__ void __launch_bounds__(IBT) k_ib_step(const int32_t* __restrict__ ibbase,
                                                 const T* __restrict__ ibcoef, int64_t nib,
                                                 int64_t ibs, int bnrt,
                                                 BlockOffsets bo, const T* __restrict__ phi,
                                                 T scale, const T* __restrict__ uib,
                                                 T* __restrict__ g, double* __restrict__ part,
                                                 const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int bn = BN > 0 ? BN : bnrt;
  const int64_t s = (int64_t)blockIdx.x * IBT + threadIdx.x;
  double num = 0.0, den = 0.0;
  if (s < nib) {
    const int32_t b32 = ibbase[s];
    const int64_t base = b32 >= 0 ? b32 : ~b32;  // ~corner: the block wraps
    const BlockWrap w = block_wrap(base, bo);
    constexpr int MB = BN == 16 && D == 2 ? 4 : (BN == 27 && D == 3 ? 3 : 0);
    const int m = MB > 0 ? MB : bo.m;
    T acc[D];
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] = T(0);
    const bool lr = sizeof(T) == 4;
    T ref = lr ? phi[base + bo.off[0]] : T(0);
#pragma unroll
    for (int o = 0; o < (BN > 0 ? BN : PC_MAX_K_NODE); ++o) {
      if (o < bn) {
        T f = phi[wrap_adjust(base + bo.off[o], o % m, (o / m) % m, o / (m * m), w, bo)];
        if (lr) f -= ref;
#pragma unroll
        for (int a = 0; a < D; ++a) acc[a] += ibcoef[((int64_t)a * bn + o) * ibs + s] * f;
      }
    }
    double mn = 0.0, mo = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T gn = -uib[a * nib + s] + scale * acc[a];
      T go = g[a * nib + s];
      mn += (double)gn * (double)gn;
      mo += (double)go * (double)go;
      g[a * nib + s] = gn;
    }
    double dm = sqrt(mn) - sqrt(mo);
    num = dm * dm;
    den = mo;
  }
  // one wavefront per block: reduce in a fixed order (the result does not
  // depend on scheduling)
#pragma unroll
  for (int off = IBT / 2; off > 0; off >>= 1) {
    num += __shfl_down(num, off, IBT);
    den += __shfl_down(den, off, IBT);
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = num;
    part[2 * blockIdx.x + 1] = den;
  }
}

// Criterion of the IB iteration from k_ib_step's block partial sums, in a
// launch of its own (see ib_close_block).
__global__ void __launch_bounds__(TPB) k_ib_close(IbClose close, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  (void)ib_close_block(close, true);
}

// Prologue of a sub-step: u* at the B+V nodes, the initial IB force (zero or
// the caller's warm start) and the device flags, in one launch; the blocks
// past the first nbib copy b_u at the near-IB points (bnear[q] = b[near[q]]).
template <typename T>
__global__ void __launch_bounds__(TPB) k_prologue(const int32_t* __restrict__ ib, int64_t nib,
                                                  int d, const T* __restrict__ u, int64_t M,
                                                  T* __restrict__ uib, T* __restrict__ gib,
                                                  const T* __restrict__ g_in,
                                                  int32_t* __restrict__ flag, int nbib,
                                                  const int32_t* __restrict__ near, int64_t nnear,
                                                  const T* __restrict__ b, T* __restrict__ bnear) {
  if ((int)blockIdx.x >= nbib) {
    const int64_t q = (int64_t)(blockIdx.x - nbib) * TPB + threadIdx.x;
    if (q < nnear) bnear[q] = b[near[q]];
    return;
  }
  int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x < 16) flag[threadIdx.x] = 0;
  if (s >= nib) return;
  int64_t n = ib[s];
  for (int a = 0; a < d; ++a) {
    uib[a * nib + s] = u[a * M + n];
    gib[a * nib + s] = g_in ? g_in[a * nib + s] : T(0);
  }
}

// Statistics into pinned host memory: bmean, criterion sums, flags.
__global__ void __launch_bounds__(64) k_stats_out(const double* __restrict__ scal,
                                                  const int32_t* __restrict__ flag,
                                                  double* hs, int32_t* hf,
                                                  const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  if (threadIdx.x < 3) hs[threadIdx.x] = scal[threadIdx.x];
  if (threadIdx.x < 2) hf[threadIdx.x + 2] = flag[threadIdx.x];
  __threadfence_system();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_project(const T* __restrict__ u, const T* __restrict__ grad,
                                                 int64_t n, T* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < n) out[i] = u[i] - grad[i];
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_sub_first(T* __restrict__ x, int64_t n,
                                                   const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  // gauge: subtract the value at the first cell (read once per thread before
  // any write of this launch can reach it: element 0 is written last)
  T v0 = x[0];
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i > 0 && i < n) x[i] -= v0;
}

template <typename T>
__global__ void __launch_bounds__(1) k_zero_first(T* __restrict__ x,
                                                 const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  x[0] = T(0);
}

unsigned nblk(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

BlockOffsets block_offsets(const pc_geom* g) {
  BlockOffsets bo;
  std::memset(&bo, 0, sizeof(bo));
  const int m = g->m_node;
  for (int o = 0; o < g->bn; ++o) {
    int ox = o % m, oy = (o / m) % m, oz = o / (m * m);
    bo.off[o] = ox + g->n[0] * (oy + g->n[1] * (g->d == 3 ? oz : 0));
  }
  bo.n0 = g->n[0];
  bo.n1 = g->n[1];
  bo.n2 = g->d == 3 ? g->n[2] : 1;
  bo.m = m;
  const bool p2 = (bo.n0 & (bo.n0 - 1)) == 0 && (bo.n1 & (bo.n1 - 1)) == 0;
  bo.l0 = p2 ? __builtin_ctz((unsigned)bo.n0) : -1;
  bo.l1 = p2 ? __builtin_ctz((unsigned)bo.n1) : -1;
  bo.per = g->per;
  return bo;
}

int check_dtype(const pc_geom* g, int dtype) {
  if (dtype != PC_F64 && dtype != PC_F32)
    return fail(PC_ERR_INVALID_ARG, "dtype must be PC_F64 or PC_F32");
  if (dtype == PC_F32 && !g->has32)
    return fail(PC_ERR_INVALID_ARG, "geometry was built without float32 stencils");
  if (dtype == PC_F64 && !g->has64)
    return fail(PC_ERR_INVALID_ARG, "geometry holds float32 stencils only");
  return PC_OK;
}

// ---- launch helpers ---------------------------------------------------------------
// The block order of k_div_all (see DivMap): on 3D grids whose rows split
// into whole workgroups and whose y and z extents hold whole blocks.
DivMap div_map(const pc_geom* g) {
  DivMap m{};
  if (g->d == 3 && g->n[0] % TPB == 0 && g->n[1] % DIV_SY == 0 && g->n[2] % DIV_SZ == 0) {
    m.on = 1;
    m.segs = g->n[0] / TPB;
    m.tiles_y = g->n[1] / DIV_SY;
    m.n0 = g->n[0];
    m.n1 = g->n[1];
  }
  return m;
}

template <typename T>
int launch_div_all(const pc_geom* g, const T* gcoef, const T* v, T* b, hipStream_t s) {
  const bool lr = sizeof(T) == 4;
  dim3 grid(nblk(g->G)), block(TPB);
  const DivMap dm = div_map(g);
#define DIVL(D, K)                                                                           \
  do {                                                                                      \
    if (lr)                                                                                 \
      hipLaunchKernelGGL((k_div_all<T, D, K, true>), grid, block, 0, s, g->gidx, gcoef, g->G, \
                         g->k_grid, v, g->M, b, dm);                                       \
    else                                                                                    \
      hipLaunchKernelGGL((k_div_all<T, D, K, false>), grid, block, 0, s, g->gidx, gcoef, g->G, \
                         g->k_grid, v, g->M, b, dm);                                       \
  } while (0)
  if (g->d == 2) {
    if (g->k_grid == 16) DIVL(2, 16);
    else if (g->k_grid == 12) DIVL(2, 12);
    else DIVL(2, 0);
  } else {
    if (g->k_grid == 27) DIVL(3, 27);
    else DIVL(3, 0);
  }
#undef DIVL
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

// close (nullable): the criterion of the iteration that produced gib,
// evaluated in the same launch (needs n_near > 0).  mean_part (nullable):
// each block's sum of D(g) (k_div_near's MEAN), nblk(n_near) doubles.
template <typename T>
int launch_div_near(const pc_geom* g, const T* ncoefib, const T* gib, const T* base, T* b,
                    bool add, hipStream_t s, const int32_t* skip = nullptr,
                    const IbClose* close = nullptr, double* mean_part = nullptr,
                    T* dgrid = nullptr) {
  if (g->n_near == 0) return close ? fail(PC_ERR_INVALID_ARG, "criterion without near points")
                                   : PC_OK;
  dim3 grid(nblk(g->n_near)), block(TPB);
  const IbClose cl = close ? *close : IbClose{};
#define DNM(D, ADD, WT, CL)                                                                    \
  do {                                                                                         \
    if (mean_part)                                                                             \
      hipLaunchKernelGGL((k_div_near<T, D, ADD, WT, CL, true>), grid, block, 0, s, g->near,   \
                         g->n_near, g->nns, g->nslot, ncoefib, gib, g->n_ib, base, b, skip, cl, \
                         mean_part, dgrid);                                                    \
    else                                                                                       \
      hipLaunchKernelGGL((k_div_near<T, D, ADD, WT, CL, false>), grid, block, 0, s, g->near,  \
                         g->n_near, g->nns, g->nslot, ncoefib, gib, g->n_ib, base, b, skip, cl, \
                         mean_part, dgrid);                                                    \
  } while (0)
#define DNL(D, ADD, WT)                     \
  do {                                      \
    if (close) DNM(D, ADD, WT, true);       \
    else DNM(D, ADD, WT, false);            \
  } while (0)
#define DNW(D, ADD)                                 \
  do {                                              \
    if (g->near_w == 8) DNL(D, ADD, 8);             \
    else if (g->near_w == 16) DNL(D, ADD, 16);      \
    else if (D == 3 && g->near_w == 27) DNL(D, ADD, 27); \
    else DNL(D, ADD, 32);                           \
  } while (0)
  if (g->near_w != 8 && g->near_w != 16 && g->near_w != 32 && !(g->d == 3 && g->near_w == 27))
    return fail(PC_ERR_INVALID_ARG, "near-IB table width");
  if (g->d == 2) {
    if (add) DNW(2, true); else DNW(2, false);
  } else {
    if (add) DNW(3, true); else DNW(3, false);
  }
#undef DNW
#undef DNL
#undef DNM
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

template <typename T, bool PROJECT>
int launch_grad_all(const pc_geom* g, const T* ncoef, const T* phi, T scale, const T* u, T* out,
                    hipStream_t s, const int32_t* skip = nullptr) {
  const bool lr = sizeof(T) == 4;
  BlockOffsets bo = block_offsets(g);
  dim3 grid(nblk(g->M)), block(TPB);
#define GRW(D, BN, W)                                                                           \
  do {                                                                                          \
    if (lr)                                                                                     \
      hipLaunchKernelGGL((k_grad_all<T, D, BN, true, PROJECT, W>), grid, block, 0, s, g->nbase,  \
                         ncoef, g->M, g->ms, g->bn, bo, phi, scale, u, out, skip);              \
    else                                                                                        \
      hipLaunchKernelGGL((k_grad_all<T, D, BN, false, PROJECT, W>), grid, block, 0, s, g->nbase, \
                         ncoef, g->M, g->ms, g->bn, bo, phi, scale, u, out, skip);              \
  } while (0)
#define GRL(D, BN)                  \
  do {                              \
    if (g->per) GRW(D, BN, true);   \
    else GRW(D, BN, false);         \
  } while (0)
  if (g->d == 2) {
    if (g->bn == 16) GRL(2, 16);
    else GRL(2, 0);
  } else {
    if (g->bn == 27) GRL(3, 27);
    else GRL(3, 0);
  }
#undef GRL
#undef GRW
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

template <typename T>
int launch_grad_ib(const pc_geom* g, const T* ibcoef, const T* phi, T scale, T* out,
                   hipStream_t s, const int32_t* skip = nullptr) {
  if (g->n_ib == 0) return PC_OK;
  const bool lr = sizeof(T) == 4;
  BlockOffsets bo = block_offsets(g);
  dim3 grid(nblk(g->n_ib)), block(TPB);
  if (g->d == 2) {
    if (lr)
      hipLaunchKernelGGL((k_grad_ib<T, 2, true>), grid, block, 0, s, g->ibbase, ibcoef, g->n_ib,
                         g->ibs, g->bn, bo, phi, scale, out, skip);
    else
      hipLaunchKernelGGL((k_grad_ib<T, 2, false>), grid, block, 0, s, g->ibbase, ibcoef, g->n_ib,
                         g->ibs, g->bn, bo, phi, scale, out, skip);
  } else {
    if (lr)
      hipLaunchKernelGGL((k_grad_ib<T, 3, true>), grid, block, 0, s, g->ibbase, ibcoef, g->n_ib,
                         g->ibs, g->bn, bo, phi, scale, out, skip);
    else
      hipLaunchKernelGGL((k_grad_ib<T, 3, false>), grid, block, 0, s, g->ibbase, ibcoef, g->n_ib,
                         g->ibs, g->bn, bo, phi, scale, out, skip);
  }
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

template <typename T>
int launch_ib_update(const pc_geom* g, const T* uib, const T* grad, T* gib, double tol,
                     double* part, double* sums, int32_t* conv, hipStream_t s,
                     const int32_t* skip = nullptr, int count = 0) {
  int nb = (int)std::min<int64_t>(IB_BLOCKS, std::max<int64_t>(1, nblk(g->n_ib)));
  if (g->d == 2)
    hipLaunchKernelGGL((k_ib_update<T, 2>), dim3(nb), dim3(TPB), 0, s, uib, grad, gib, g->n_ib, part,
                       skip);
  else
    hipLaunchKernelGGL((k_ib_update<T, 3>), dim3(nb), dim3(TPB), 0, s, uib, grad, gib, g->n_ib, part,
                       skip);
  hipLaunchKernelGGL(k_ib_finish, dim3(1), dim3(TPB), 0, s, (const double*)part, nb, tol, sums,
                     conv, count);
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

// The criterion arguments of the IB step launched with these arguments.
inline IbClose ib_close_args(const pc_geom* g, double tol, double* part, int32_t* flag,
                             double* sums, int32_t* host_flag, double* host_sums) {
  return IbClose{part, (int)((g->n_ib + IBT - 1) / IBT), tol, sums, flag, host_flag, host_sums};
}

// The IB step; with `close` also its criterion in a launch of its own
// (otherwise the caller evaluates it, merged into the next RHS update).
template <typename T>
int launch_ib_step(const pc_geom* g, const T* ibcoef, const T* phi, T scale, const T* uib, T* gib,
                   double tol, double* part, int32_t* flag, double* sums, hipStream_t s,
                   const int32_t* skip, int32_t* host_flag, double* host_sums, bool close = true) {
  if (g->n_ib == 0) return PC_OK;
  BlockOffsets bo = block_offsets(g);
  dim3 grid((unsigned)((g->n_ib + IBT - 1) / IBT)), block(IBT);
  // flag[0]: converged, flag[1]: iterations
#define IBS(D, BN)                                                                              \
  hipLaunchKernelGGL((k_ib_step<T, D, BN>), grid, block, 0, s, g->ibbase, ibcoef, g->n_ib, g->ibs, \
                     g->bn, bo, phi, scale, uib, gib, part, skip)
  if (g->d == 2) {
    if (g->bn == 16) IBS(2, 16); else IBS(2, 0);
  } else {
    if (g->bn == 27) IBS(3, 27); else IBS(3, 0);
  }
#undef IBS
  if (close)
    hipLaunchKernelGGL(k_ib_close, dim3(1), dim3(TPB), 0, s,
                       ib_close_args(g, tol, part, flag, sums, host_flag, host_sums), skip);
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

template <typename T>
int launch_zero_ib(const pc_geom* g, T* out, hipStream_t s, const int32_t* skip = nullptr) {
  if (g->n_ib == 0) return PC_OK;
  hipLaunchKernelGGL(k_zero_ib<T>, dim3(nblk(g->n_ib)), dim3(TPB), 0, s, g->ib, g->n_ib, g->d,
                     g->M, out, skip);
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

template <typename T>
const T* gc(const pc_geom* g) {
  if constexpr (sizeof(T) == 8) return g->gcoef; else return g->gcoef32;
}
template <typename T>
const T* nc(const pc_geom* g) {
  if constexpr (sizeof(T) == 8) return g->ncoef; else return g->ncoef32;
}
template <typename T>
const T* nci(const pc_geom* g) {
  if constexpr (sizeof(T) == 8) return g->ncoefib; else return g->ncoefib32;
}
template <typename T>
const T* ibc(const pc_geom* g) {
  if constexpr (sizeof(T) == 8) return g->ibcoef; else return g->ibcoef32;
}

// Waits until the device has stored a value other than -1 into the coherent
// host flag *f.  The stream is not queried while the wait is short (a query
// places a marker in the stream, which stalls the device); after two
// seconds it is, so that a stream that drained without the store ends the
// wait with an error instead of spinning forever.
int wait_host_flag(volatile int32_t* f, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  for (int64_t spin = 0;; ++spin) {
    if (*f != -1) return PC_OK;
    if ((spin & 4095) == 4095 &&
        std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) {
        if (*f != -1) return PC_OK;
        return fail(PC_ERR_HIP, "IB convergence flag not written by the device");
      }
      if (e != hipErrorNotReady) return fail(PC_ERR_HIP, hipGetErrorString(e));
    }
  }
}

// ---- the sub-step ---------------------------------------------------------------------
template <typename T>
int pressure_correct_t(const pc_geom* g, const pc_plan* P, int mode, const T* u, double dt,
                       T* u_out, T* p_out, T* g_io, const pc_ib_opts* o, pc_stats* st,
                       pc_workspace* W, hipStream_t s) {
  const double tol = o && o->tol > 0.0 ? o->tol : 1e-3;
  const int max_it = o && o->max_it > 0 ? o->max_it : 50;
  const int fixed_it = o ? o->fixed_it : 0;
  const int sweeps = o && o->sweeps > 0 ? o->sweeps : 2;
  const int gauge = o ? o->gauge : 0;
  const bool resident = W->resident && !(o && (o->flags & PC_IB_FULL_TRANSFORMS)) &&
                        mode != PC_MIXED;
  // PC_MIXED: the first correction sweep of later iterations on the change
  // of the right-hand side (near-IB lines only)
  const bool delta = W->delta && mode == PC_MIXED && !(o && (o->flags & PC_IB_FULL_TRANSFORMS));
  // the solve returns p = phi / sigma directly; the gradient of phi is
  // sigma * grad p
  const double sigma = 1.5 * dt;
  T* b = reinterpret_cast<T*>(W->b);
  T* p = p_out;
  T* bnear = reinterpret_cast<T*>(W->bnear);
  T* uib = reinterpret_cast<T*>(W->uib);
  T* gib = reinterpret_cast<T*>(W->gib);
  T* gradib = reinterpret_cast<T*>(W->gradib);
  const int64_t nib = g->n_ib;

  // the long gather goes first so that the host queues the rest behind it
  PC_TRY(launch_div_all<T>(g, gc<T>(g), u, b, s));
  {
    const unsigned nbib = std::max<unsigned>(1, nblk(nib));
    hipLaunchKernelGGL(k_prologue<T>, dim3(nbib + nblk(g->n_near)), dim3(TPB), 0, s, g->ib, nib,
                       g->d, u, g->M, uib, gib, (const T*)g_io, W->flag, (int)nbib, g->near,
                       g->n_near, (const T*)b, bnear);
    PC_HIP_CHECK(hipGetLastError());
  }
  // PC_MIXED needs mean(b) before its first float32 pass in every
  // iteration.  b changes only at the near points, so it is mean(b_u) (one
  // pass, here) plus the near update's sum over G, which the update kernel
  // adds up per block (cell-centred grids; a vertex grid's mean is
  // weighted, and every iteration takes it over the grid).
  const bool inc_mean = mode == PC_MIXED && !P->vertex && g->n_near > 0 && W->part2;
  if (inc_mean) PC_TRY(grid_mean_f64(P, (const double*)b, W->partial, W->nblk, W->scal + 5, s));

  // One IB iteration (Sec. 2.3): RHS update near the IB, Poisson solve,
  // gradient at the B+V nodes, force update and criterion.  With `skip` set,
  // every launch of the iteration returns at once once the device flag says
  // an earlier iteration has converged.
  // With `defer` the iteration leaves its criterion to the caller (merged
  // into the next iteration's RHS update, or queued alone); `prev` is the
  // deferred criterion of iteration it - 1, evaluated in this iteration's
  // RHS update.
  auto iteration = [&](int it, const int32_t* skip, int32_t* host_flag, bool defer = false,
                       const IbClose* prev = nullptr) -> int {
    double* host_sums = host_flag ? W->hscal + 4 + 2 * (it & 1) : nullptr;
    const bool upd = it > 1 || g_io;
    if (upd)
      PC_TRY(launch_div_near<T>(g, nci<T>(g), gib, bnear, b, false, s, skip, prev,
                                inc_mean ? W->part2 : nullptr,
                                delta ? reinterpret_cast<T*>(W->dgrid) : nullptr));
    if (inc_mean) {
      hipLaunchKernelGGL(k_mean_near, dim3(1), dim3(TPB), 0, s, (const double*)W->part2,
                         upd ? (int)nblk(g->n_near) : 0, (const double*)(W->scal + 5),
                         1.0 / (double)P->G, W->scal, skip);
      PC_HIP_CHECK(hipGetLastError());
    }
    if (resident && mode == PC_F64)
      PC_TRY(solve_resident_f64(P, (const double*)b, (double*)p, W->scal, W, s, sigma, skip,
                                it > 1 ? 1 : 0));
    else if (resident)
      PC_TRY(solve_resident_f32(P, (const float*)b, (float*)p, W->scal, W, s, sigma, skip,
                                it > 1 ? 1 : 0));
    else if (mode == PC_F64)
      PC_TRY(solve_f64(P, (const double*)b, (double*)p, W->scal, W, s, sigma, skip));
    else if (mode == PC_F32)
      PC_TRY(solve_f32(P, (const float*)b, (float*)p, W->scal, W, s, sigma, skip));
    else
      // the corrections of later iterations start from the previous
      // iteration's pressure, whose right-hand side differs only near the
      // IB; the mean is removed once, after the last iteration
      PC_TRY(solve_mixed(P, (const double*)b, (double*)p, sweeps, W->scal, W, s, sigma, skip,
                         it > 1, false, inc_mean, delta));
    if (nib)
      PC_TRY(launch_ib_step<T>(g, ibc<T>(g), p, (T)sigma, uib, gib, tol, W->partial, W->flag,
                               W->scal + 1, s, skip, host_flag, host_sums, !defer));
    return PC_OK;
  };
  // the criterion of iteration it (host slot it % 2), deferred or alone
  auto close_args = [&](int it) {
    return ib_close_args(g, tol, W->partial, W->flag, W->scal + 1, W->hflag + (it & 1),
                         W->hscal + 4 + 2 * (it & 1));
  };
  auto close_alone = [&](int it) -> int {
    hipLaunchKernelGGL(k_ib_close, dim3(1), dim3(TPB), 0, s, close_args(it),
                       (const int32_t*)W->flag);
    PC_HIP_CHECK(hipGetLastError());
    return PC_OK;
  };

  // The work after the last iteration: complete the inverse transforms on
  // the lines the B+V gradient did not need, the gradient at every node
  // fused with the projection (Eq. 18), exactly 0 at B+V, the final force,
  // the gauge and the statistics.  With a guard it does nothing unless the
  // guarded iteration converged.
  auto final_work = [&](const int32_t* guard) -> int {
    if (mode == PC_MIXED) PC_TRY(remove_mean_f64(P, (double*)p, W, s, guard));
    if (resident && mode == PC_F64)
      PC_TRY(solve_resident_f64(P, (const double*)b, (double*)p, W->scal, W, s, sigma, guard, 2));
    else if (resident)
      PC_TRY(solve_resident_f32(P, (const float*)b, (float*)p, W->scal, W, s, sigma, guard, 2));
    PC_TRY((launch_grad_all<T, true>(g, nc<T>(g), p, (T)sigma, u, u_out, s, guard)));
    if (nib)
      hipLaunchKernelGGL(k_finish_ib<T>, dim3(nblk(nib)), dim3(TPB), 0, s, g->ib, nib, g->d, g->M,
                         u_out, (const T*)gib, g_io, (const double*)W->scal,
                         (const int32_t*)W->flag, st ? W->hscal : nullptr, W->hflag, guard);
    else if (st)
      hipLaunchKernelGGL(k_stats_out, dim3(1), dim3(64), 0, s, (const double*)W->scal,
                         (const int32_t*)W->flag, W->hscal, W->hflag, guard);
    if (gauge == 1) {
      hipLaunchKernelGGL(k_sub_first<T>, dim3(nblk(P->G)), dim3(TPB), 0, s, p, P->G, guard);
      hipLaunchKernelGGL(k_zero_first<T>, dim3(1), dim3(1), 0, s, p, guard);
    }
    PC_HIP_CHECK(hipGetLastError());
    return PC_OK;
  };

  int it = 0;
  bool converged = nib == 0;
  bool final_queued = false;
  if (nib == 0) {
    PC_TRY(iteration(1, nullptr, nullptr));
    it = 1;
  } else if (fixed_it > 0) {
    for (it = 1; it <= fixed_it; ++it) PC_TRY(iteration(it, nullptr, nullptr));
    it = fixed_it;
  } else {
    // Enqueue one iteration ahead of the convergence test: while the host
    // waits for iteration i, the device already runs i+1 (which does nothing
    // if i converged), so the device does not idle on the host.  The IB
    // kernels of iteration i store its flag (0/1) and criterion sums straight
    // into coherent pinned host slot i % 2, which the host resets to -1
    // before queueing the iteration that reuses it.
    // Where iteration i is predicted to meet the criterion, the final work
    // is queued behind it instead, guarded by the device's "not converged"
    // word: the ratio q = num/den of the criterion falls about
    // geometrically, q_i ~ q_{i-1}^2 / q_{i-2}, and the prediction must be
    // below 2/3 of the tolerance.  A wrong prediction costs a few launches
    // that return at once and a late enqueue; it never changes the result.
    // The criterion of iteration i runs in the first launch of iteration
    // i+1 (its RHS update near the IB) when that iteration is queued next,
    // and in a launch of its own otherwise.
    volatile int32_t* hf = W->hflag;
    volatile double* hs = W->hscal;
    double q1 = 0.0, q2 = 0.0;  // q of the two previous iterations (0: unknown)
    const bool merge = g->n_near > 0;
    hf[1] = -1;
    PC_TRY(iteration(1, W->flag, W->hflag + 1, merge));
    bool pending = merge;  // the criterion of iteration `it` is not queued yet
    for (it = 1;; ++it) {
      bool ahead = false;
      const bool likely = q1 > 0.0 && q2 > 0.0 && q1 * q1 < (2.0 / 3.0) * tol * q2;
      if (likely) {
        if (pending) PC_TRY(close_alone(it));
        pending = false;
        PC_TRY(final_work(W->flag + 4));
      } else if (it < max_it) {
        hf[(it + 1) & 1] = -1;
        const IbClose prev = close_args(it);
        PC_TRY(iteration(it + 1, W->flag, W->hflag + ((it + 1) & 1), merge,
                         pending ? &prev : nullptr));
        pending = merge;  // now the criterion of iteration it + 1
        ahead = true;
      } else if (pending) {
        PC_TRY(close_alone(it));
        pending = false;
      }
      PC_TRY(wait_host_flag(hf + (it & 1), s));
      if (hf[it & 1] == 1) {
        converged = true;
        final_queued = likely;
        break;
      }
      if (it >= max_it) break;
      const double num = hs[4 + 2 * (it & 1)], den = hs[5 + 2 * (it & 1)];
      q2 = q1;
      q1 = den > 0.0 ? num / den : 0.0;
      if (!ahead) {
        hf[(it + 1) & 1] = -1;
        PC_TRY(iteration(it + 1, W->flag, W->hflag + ((it + 1) & 1), merge));
        pending = merge;
      }
    }
  }
  if (!final_queued) PC_TRY(final_work(nullptr));
  if (st) {
    PC_HIP_CHECK(hipEventRecord(W->ev[0], s));
    PC_HIP_CHECK(hipEventSynchronize(W->ev[0]));
    volatile double* hs = W->hscal;
    volatile int32_t* hf = W->hflag;
    st->n_it = it;
    st->converged = (nib == 0 || hf[2]) ? 1 : 0;
    if (nib && fixed_it <= 0) st->converged = converged ? 1 : 0;
    st->bmean = hs[0];
    st->ib_num = hs[1];
    st->ib_den = hs[2];
    converged = st->converged;
  }
  if (fixed_it > 0) return PC_OK;
  return converged ? PC_OK : PC_WARN_IB_NOT_CONVERGED;
}

// ---- the first fractional step (Eq. 3) ---------------------------------------------
struct Force3 {
  double f[3];
};

// R = -u.grad u + nu lap u + F at every node from its node-to-node stencil
// (known-value WLS rows applied to u(x_i) - u(x)), and the Adams-Bashforth
// predictor u* = u + dt (3/2 R - 1/2 R_prev) (u + dt R when rprev is null).
// One thread per node; the stencil streams are coalesced over nodes.
template <typename T, int D, int K>
__global__ void __launch_bounds__(TPB) k_momentum(const int32_t* __restrict__ sidx,
                                                  const T* __restrict__ scoef, int64_t M,
                                                  int64_t ms, int krt, const T* __restrict__ u,
                                                  const T* __restrict__ rprev, T dt, T nu,
                                                  Force3 F, T* __restrict__ rout,
                                                  T* __restrict__ ustar) {
  const int k = K > 0 ? K : krt;
  const int64_t n = xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
  if (n >= M) return;
  T un[D], lp[D], gr[D][D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    un[c] = u[c * M + n];
    lp[c] = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) gr[a][c] = T(0);
  }
#pragma unroll 4
  for (int i = 0; i < k; ++i) {
    const int64_t j = ldnt(sidx + (int64_t)i * ms + n);
    T du[D];
#pragma unroll
    for (int c = 0; c < D; ++c) du[c] = u[c * M + j] - un[c];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const T cg = ldnt(scoef + ((int64_t)a * k + i) * ms + n);
#pragma unroll
      for (int c = 0; c < D; ++c) gr[a][c] += cg * du[c];
    }
    const T cl = ldnt(scoef + ((int64_t)D * k + i) * ms + n);
#pragma unroll
    for (int c = 0; c < D; ++c) lp[c] += cl * du[c];
  }
#pragma unroll
  for (int c = 0; c < D; ++c) {
    T conv = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) conv += un[a] * gr[a][c];
    const T R = -conv + nu * lp[c] + (T)F.f[c];
    const T rp = rprev ? rprev[c * M + n] : T(0);
    rout[c * M + n] = R;
    ustar[c * M + n] = un[c] + dt * (rprev ? (T(1.5) * R - T(0.5) * rp) : R);
  }
}

// R_prev = R - c (u* - u^{n+1}) over [d][M]; then R_prev -= c g at the B+V
// nodes (c = 2 / (3 dt): the pressure gradient of Eq. 18)
template <typename T>
__global__ void __launch_bounds__(TPB) k_rprev(const T* __restrict__ r, const T* __restrict__ us,
                                               const T* __restrict__ un, T c, int64_t n,
                                               T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < n) out[i] = r[i] - c * (us[i] - un[i]);
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_rprev_ib(const int32_t* __restrict__ ib, int64_t nib,
                                                  int d, int64_t M, const T* __restrict__ g, T c,
                                                  T* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (s >= nib) return;
  const int64_t n = ib[s];
  for (int a = 0; a < d; ++a) out[a * M + n] -= c * g[a * nib + s];
}

template <typename T>
int momentum_predict_t(const pc_geom* g, const T* u, const T* rprev, T dt, T nu, Force3 F,
                       T* r, T* ustar, const T* coef, hipStream_t s) {
  dim3 grid(nblk(g->M)), block(TPB);
#define MOM(D, K)                                                                          \
  hipLaunchKernelGGL((k_momentum<T, D, K>), grid, block, 0, s, g->sidx, coef, g->M, g->ms, \
                     g->k_self, u, rprev, dt, nu, F, r, ustar)
  if (g->d == 2) {
    if (g->k_self == 12) MOM(2, 12);
    else if (g->k_self == 16) MOM(2, 16);
    else MOM(2, 0);
  } else {
    if (g->k_self == 20) MOM(3, 20);
    else if (g->k_self == 27) MOM(3, 27);
    else MOM(3, 0);
  }
#undef MOM
  PC_HIP_CHECK(hipGetLastError());
  // virtual points: the frozen fluid inside the body (Sec. 2.3)
  if (g->n_v) {
    hipLaunchKernelGGL(k_zero_ib<T>, dim3(nblk(g->n_v)), dim3(TPB), 0, s, g->vlist, g->n_v, g->d,
                       g->M, ustar, (const int32_t*)nullptr);
    PC_HIP_CHECK(hipGetLastError());
  }
  return PC_OK;
}

template <typename T>
int momentum_pressure_t(const pc_geom* g, const T* r, const T* us, const T* un, const T* gib,
                        T dt, T* out, hipStream_t s) {
  const T c = T(2.0 / (3.0 * (double)dt));
  const int64_t n = (int64_t)g->d * g->M;
  hipLaunchKernelGGL(k_rprev<T>, dim3(nblk(n)), dim3(TPB), 0, s, r, us, un, c, n, out);
  if (gib && g->n_ib)
    hipLaunchKernelGGL(k_rprev_ib<T>, dim3(nblk(g->n_ib)), dim3(TPB), 0, s, g->ib, g->n_ib, g->d,
                       g->M, gib, c, out);
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

int check_fields(const void* a, const void* b = nullptr, const void* c = nullptr) {
  if (!a) return fail(PC_ERR_INVALID_ARG, "null field");
  for (const void* p : {a, b, c})
    if (p && !aligned16(p)) return fail(PC_ERR_ALIGN, "fields must be 16-byte aligned");
  return PC_OK;
}

// ---- one IB-force update (pc_ib_update and its allocation-free variant) ---------
int ib_update_check(const pc_geom* g, int dtype, const void* u, const void* grad_ib,
                    const void* gib, const double* sums, const int32_t* conv) {
  if (!g || !u || !grad_ib || !gib || !sums || !conv)
    return fail(PC_ERR_INVALID_ARG, "pc_ib_update: null argument");
  PC_TRY(check_dtype(g, dtype));
  PC_TRY(check_fields(u, grad_ib, gib));
  return PC_OK;
}

// Scratch of one update: the block partial sums, then u* gathered at the
// B+V nodes.
constexpr size_t IB_PART_BYTES = 2 * IB_BLOCKS * 8 + 256;

size_t ib_scratch_bytes(const pc_geom* g, int dtype) {
  const size_t es = dtype == PC_F64 ? 8 : 4;
  return IB_PART_BYTES + (size_t)g->d * g->n_ib * es;
}

int ib_update_with(const pc_geom* g, int dtype, const void* u, const void* grad_ib, void* gib,
                   double tol, double* sums, int32_t* conv, void* scratch, hipStream_t s) {
  double* part = reinterpret_cast<double*>(scratch);
  void* uib = reinterpret_cast<char*>(scratch) + IB_PART_BYTES;
  if (dtype == PC_F64) {
    hipLaunchKernelGGL(k_gather_ib<double>, dim3(nblk(g->n_ib)), dim3(TPB), 0, s, g->ib, g->n_ib,
                       g->d, (const double*)u, g->M, (double*)uib);
    return launch_ib_update<double>(g, (const double*)uib, (const double*)grad_ib, (double*)gib,
                                    tol, part, sums, conv, s);
  }
  hipLaunchKernelGGL(k_gather_ib<float>, dim3(nblk(g->n_ib)), dim3(TPB), 0, s, g->ib, g->n_ib,
                     g->d, (const float*)u, g->M, (float*)uib);
  return launch_ib_update<float>(g, (const float*)uib, (const float*)grad_ib, (float*)gib, tol,
                                 part, sums, conv, s);
}

// The static scratch of pc_ib_update_noalloc: one copy per device, held
// until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, once per device, with that device
// current.  The kernels write every partial sum and every gathered value
// they read afterwards, so nothing needs clearing between calls.
__device__ __align__(256) unsigned char scratch[PC_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

int noalloc_scratch(void** out) {
  int dev = 0;
  PC_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(PC_ERR_UNSUPPORTED_SIZE, "device ordinal above the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(PC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                  hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PC_OK;
}

}  // namespace
}  // namespace pc

using namespace pc;

extern "C" {

int pc_div_to_grid(const pc_geom* g, int dtype, const void* v, void* b, int subset,
                   void* stream) {
  if (!g || !v || !b) return fail(PC_ERR_INVALID_ARG, "pc_div_to_grid: null argument");
  PC_TRY(check_dtype(g, dtype));
  PC_TRY(check_fields(v, b));
  hipStream_t s = as_stream(stream);
  if (subset == PC_ALL) {
    if (dtype == PC_F64) return launch_div_all<double>(g, g->gcoef, (const double*)v, (double*)b, s);
    return launch_div_all<float>(g, g->gcoef32, (const float*)v, (float*)b, s);
  }
  if (subset == PC_NEAR_IB) {
    if (dtype == PC_F64)
      return launch_div_near<double>(g, g->ncoefib, (const double*)v, nullptr, (double*)b, true, s);
    return launch_div_near<float>(g, g->ncoefib32, (const float*)v, nullptr, (float*)b, true, s);
  }
  return fail(PC_ERR_INVALID_ARG, "subset must be PC_ALL or PC_NEAR_IB");
}

int pc_grad_to_nodes(const pc_geom* g, int dtype, const void* phi, void* grad, int subset,
                     void* stream) {
  if (!g || !phi || !grad) return fail(PC_ERR_INVALID_ARG, "pc_grad_to_nodes: null argument");
  PC_TRY(check_dtype(g, dtype));
  PC_TRY(check_fields(phi, grad));
  hipStream_t s = as_stream(stream);
  if (subset == PC_ALL) {
    if (dtype == PC_F64)
      return launch_grad_all<double, false>(g, g->ncoef, (const double*)phi, 1.0, nullptr,
                                            (double*)grad, s);
    return launch_grad_all<float, false>(g, g->ncoef32, (const float*)phi, 1.0f, nullptr,
                                         (float*)grad, s);
  }
  if (subset == PC_IB) {
    if (dtype == PC_F64)
      return launch_grad_ib<double>(g, g->ibcoef, (const double*)phi, 1.0, (double*)grad, s);
    return launch_grad_ib<float>(g, g->ibcoef32, (const float*)phi, 1.0f, (float*)grad, s);
  }
  return fail(PC_ERR_INVALID_ARG, "subset must be PC_ALL or PC_IB");
}

int pc_ib_update(const pc_geom* g, int dtype, const void* u, const void* grad_ib, void* gib,
                 double tol, double* sums, int32_t* conv, void* stream) {
  PC_TRY(ib_update_check(g, dtype, u, grad_ib, gib, sums, conv));
  if (g->n_ib == 0) return PC_OK;
  hipStream_t s = as_stream(stream);
  void* tmp = nullptr;
  PC_TRY(dev_alloc(&tmp, ib_scratch_bytes(g, dtype), "ib scratch"));
  const int rc = ib_update_with(g, dtype, u, grad_ib, gib, tol, sums, conv, tmp, s);
  (void)hipStreamSynchronize(s);
  dev_free(tmp);
  return rc;
}

int pc_ib_update_noalloc(const pc_geom* g, int dtype, const void* u, const void* grad_ib,
                         void* gib, double tol, double* sums, int32_t* conv, void* stream) {
  PC_TRY(ib_update_check(g, dtype, u, grad_ib, gib, sums, conv));
  if (g->n_ib == 0) return PC_OK;
  const size_t need = ib_scratch_bytes(g, dtype);
  if (need > (size_t)PC_NOALLOC_SCRATCH_BYTES)
    return fail(PC_ERR_UNSUPPORTED_SIZE,
                "pc_ib_update_noalloc: " + std::to_string(g->n_ib) +
                    " boundary/virtual nodes need " + std::to_string(need) +
                    " bytes of scratch, above the static " +
                    std::to_string((long long)PC_NOALLOC_SCRATCH_BYTES) +
                    " (PC_NOALLOC_MAX_IB; use pc_ib_update)");
  void* scr = nullptr;
  PC_TRY(noalloc_scratch(&scr));
  return ib_update_with(g, dtype, u, grad_ib, gib, tol, sums, conv, scr, as_stream(stream));
}

int pc_project(const pc_geom* g, int dtype, const void* u, const void* grad, void* u_out,
               void* stream) {
  if (!g || !u || !grad || !u_out) return fail(PC_ERR_INVALID_ARG, "pc_project: null argument");
  if (dtype != PC_F64 && dtype != PC_F32) return fail(PC_ERR_INVALID_ARG, "dtype");
  PC_TRY(check_fields(u, grad, u_out));
  hipStream_t s = as_stream(stream);
  // u_out = u - grad on every node, then exactly 0 on the B+V nodes
  int64_t n = (int64_t)g->d * g->M;
  if (dtype == PC_F64) {
    hipLaunchKernelGGL((k_project<double>), dim3(nblk(n)), dim3(TPB), 0, s, (const double*)u,
                       (const double*)grad, n, (double*)u_out);
    PC_HIP_CHECK(hipGetLastError());
    return launch_zero_ib<double>(g, (double*)u_out, s);
  }
  hipLaunchKernelGGL((k_project<float>), dim3(nblk(n)), dim3(TPB), 0, s, (const float*)u,
                     (const float*)grad, n, (float*)u_out);
  PC_HIP_CHECK(hipGetLastError());
  return launch_zero_ib<float>(g, (float*)u_out, s);
}

int pc_pressure_correct(const pc_geom* g, const pc_plan* P, int mode, const void* u, double dt,
                        void* u_out, void* p, void* g_io, const pc_ib_opts* o, pc_stats* st,
                        pc_workspace* ws, void* stream) {
  if (!g || !P || !u || !u_out || !p)
    return fail(PC_ERR_INVALID_ARG, "pc_pressure_correct: null argument");
  if (mode != PC_F64 && mode != PC_F32 && mode != PC_MIXED)
    return fail(PC_ERR_INVALID_ARG, "mode must be PC_F64, PC_F32 or PC_MIXED");
  if (!same_grid(P, g)) return fail(PC_ERR_INVALID_ARG, "plan and geometry differ");
  if (mode == PC_MIXED && P->eig != PC_EIG_FD2)
    return fail(PC_ERR_INVALID_ARG, "PC_MIXED needs the central-difference eigenvalues");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(PC_ERR_INVALID_ARG, "dt must be positive");
  if (mode == PC_F32 && !g->has32)
    return fail(PC_ERR_INVALID_ARG, "geometry was built without float32 stencils");
  if (mode != PC_F32 && !g->has64)
    return fail(PC_ERR_INVALID_ARG, "geometry holds float32 stencils only");
  PC_TRY(check_fields(u, u_out, p));
  if (g_io && !aligned16(g_io)) return fail(PC_ERR_ALIGN, "g must be 16-byte aligned");
  if (u == u_out) return fail(PC_ERR_INVALID_ARG, "u_out must not alias u");
  if (ws) {
    if (ws->mode != mode || ws->geom != g || ws->plan != P)
      return fail(PC_ERR_INVALID_ARG, "workspace was created for another mode/plan/geometry");
  } else {
    pc_geom* mg = const_cast<pc_geom*>(g);
    if (mg->own_ws && (mg->own_ws->mode != mode || mg->own_ws->plan != P)) {
      pc_workspace_destroy(mg->own_ws);
      mg->own_ws = nullptr;
    }
    if (!mg->own_ws) PC_TRY(pc_workspace_create(P, g, mode, &mg->own_ws));
    ws = mg->own_ws;
  }
  hipStream_t s = as_stream(stream);
  if (mode == PC_F32)
    return pressure_correct_t<float>(g, P, mode, (const float*)u, dt, (float*)u_out, (float*)p,
                                     (float*)g_io, o, st, ws, s);
  return pressure_correct_t<double>(g, P, mode, (const double*)u, dt, (double*)u_out, (double*)p,
                                    (double*)g_io, o, st, ws, s);
}

int pc_momentum_predict(const pc_geom* g, int dtype, const void* u, const void* r_prev,
                        double dt, double nu, const double* force, void* r, void* ustar,
                        void* stream) {
  if (!g || !u || !r || !ustar) return fail(PC_ERR_INVALID_ARG, "pc_momentum_predict: null argument");
  if (!g->k_self)
    return fail(PC_ERR_INVALID_ARG, "the geometry was built without node-to-node stencils");
  if (dtype != PC_F64 && dtype != PC_F32) return fail(PC_ERR_INVALID_ARG, "dtype");
  if (dtype == PC_F32 && !g->scoef32)
    return fail(PC_ERR_INVALID_ARG, "geometry was built without float32 stencils");
  if (dtype == PC_F64 && !g->scoef)
    return fail(PC_ERR_INVALID_ARG, "geometry holds float32 stencils only");
  if (!(dt > 0.0) || !std::isfinite(dt) || !(nu >= 0.0) || !std::isfinite(nu))
    return fail(PC_ERR_INVALID_ARG, "dt must be positive and nu non-negative");
  if (ustar == u) return fail(PC_ERR_INVALID_ARG, "ustar must not alias u");
  PC_TRY(check_fields(u, r, ustar));
  if (r_prev && !aligned16(r_prev)) return fail(PC_ERR_ALIGN, "fields must be 16-byte aligned");
  Force3 F{{0.0, 0.0, 0.0}};
  if (force)
    for (int a = 0; a < g->d; ++a) F.f[a] = force[a];
  hipStream_t s = as_stream(stream);
  if (dtype == PC_F64)
    return momentum_predict_t<double>(g, (const double*)u, (const double*)r_prev, dt, nu, F,
                                      (double*)r, (double*)ustar, g->scoef, s);
  return momentum_predict_t<float>(g, (const float*)u, (const float*)r_prev, (float)dt,
                                   (float)nu, F, (float*)r, (float*)ustar, g->scoef32, s);
}

int pc_momentum_pressure(const pc_geom* g, int dtype, const void* r, const void* ustar,
                         const void* unew, const void* g_ib, double dt, void* r_prev,
                         void* stream) {
  if (!g || !r || !ustar || !unew || !r_prev)
    return fail(PC_ERR_INVALID_ARG, "pc_momentum_pressure: null argument");
  if (dtype != PC_F64 && dtype != PC_F32) return fail(PC_ERR_INVALID_ARG, "dtype");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(PC_ERR_INVALID_ARG, "dt must be positive");
  PC_TRY(check_fields(r, ustar, unew));
  if (!aligned16(r_prev) || (g_ib && !aligned16(g_ib)))
    return fail(PC_ERR_ALIGN, "fields must be 16-byte aligned");
  hipStream_t s = as_stream(stream);
  if (dtype == PC_F64)
    return momentum_pressure_t<double>(g, (const double*)r, (const double*)ustar,
                                       (const double*)unew, (const double*)g_ib, dt,
                                       (double*)r_prev, s);
  return momentum_pressure_t<float>(g, (const float*)r, (const float*)ustar, (const float*)unew,
                                    (const float*)g_ib, (float)dt, (float*)r_prev, s);
}

}  // extern "C"
