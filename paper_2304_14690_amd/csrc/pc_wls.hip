// WLS stencils of one node cloud (Sec. 2.2), computed once per geometry
// ("the coefficients only need to be calculated once", last paragraph of
// Sec. 2.2):
//   * a cell list of the nodes over the pressure-grid cells (the paper's
//     linked-list neighbour search, here a counting sort);
//   * for every grid point, its k_grid nearest nodes by the key (d^2, node
//     index) with d^2 = ((dx*dx) + dy*dy) + dz*dz rounded term by term,
//     found by scanning rings of cells until no unscanned cell can hold a
//     closer node;
//   * for every node, the k_node nearest grid points by (d^2, flat index)
//     within the block of the m grid lines nearest to it along each axis
//     (block clamped inside the box, except along a periodic axis, where it
//     wraps around);
//   * along a periodic axis (the lateral condition of the verification
//     cases of Sec. 3) offsets are minimal images: t = x_s - x_t, then
//     t - L if t > L/2 or t + L if t < -L/2;
//   * per target, the Eq. 16 polynomial vector (10 terms in 3D) in
//     coordinates scaled by h_t = max(support*delta, r_k), the Gaussian
//     weights of Eq. 17, C = sum w q q^T (Eq. 14), its Cholesky factor, and
//     the first-derivative rows of C^-1 A (Eq. 13): c_{a,i} = w_i (C^-1 q_i)_a
//     / h_t, all in float64;
//   * the boundary/virtual node list, the grid points whose stencil holds
//     one of them, and compact copies of the stencils the IB iteration uses.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "pc_internal.h"

namespace pc {
namespace {

constexpr int KMAX = PC_MAX_K_GRID;   // grid-target stencil capacity
constexpr int BNMAX = PC_MAX_K_NODE;  // node block capacity
constexpr double SINGULAR_RATIO = 1e-12;

// ---- exact squared distance (no contraction) --------------------------------
__device__ __forceinline__ double sq_sum2(double dx, double dy) {
#pragma clang fp contract(off)
  double a = dx * dx;
  double b = dy * dy;
  return a + b;
}
__device__ __forceinline__ double sq_sum3(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  double a = dx * dx;
  double b = dy * dy;
  double c = dz * dz;
  return (a + b) + c;
}

__device__ __forceinline__ bool key_lt(double d1, int i1, double d2, int i2) {
  return d1 < d2 || (d1 == d2 && i1 < i2);
}

// Eq. 16 polynomial vector (2D: 6 terms; 3D: 10 terms) of scaled offsets.
template <int D>
__device__ __forceinline__ void basis(const double* xi, double* q) {
  if (D == 2) {
    q[0] = 1.0; q[1] = xi[0]; q[2] = xi[1];
    q[3] = 0.5 * xi[0] * xi[0]; q[4] = xi[0] * xi[1]; q[5] = 0.5 * xi[1] * xi[1];
  } else {
    q[0] = 1.0; q[1] = xi[0]; q[2] = xi[1]; q[3] = xi[2];
    q[4] = 0.5 * xi[0] * xi[0]; q[5] = xi[0] * xi[1]; q[6] = xi[0] * xi[2];
    q[7] = 0.5 * xi[1] * xi[1]; q[8] = xi[1] * xi[2]; q[9] = 0.5 * xi[2] * xi[2];
  }
}

// Packed lower-triangular index of (r, c), r >= c.
__host__ __device__ constexpr int tri(int r, int c) { return r * (r + 1) / 2 + c; }

// In-place Cholesky of the packed symmetric matrix A (m x m).  Returns the
// ratio min(L_jj^2) / max(L_jj^2) (0 if a pivot is not positive).
template <int MU>
__device__ __forceinline__ double cholesky(double* A) {
  double pmin = 1e300, pmax = 0.0;
#pragma unroll
  for (int j = 0; j < MU; ++j) {
    double s = A[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= A[tri(j, k)] * A[tri(j, k)];
    if (!(s > 0.0)) return 0.0;
    pmin = fmin(pmin, s);
    pmax = fmax(pmax, s);
    double l = sqrt(s);
    A[tri(j, j)] = l;
    double il = 1.0 / l;
#pragma unroll
    for (int r = j + 1; r < MU; ++r) {
      double t = A[tri(r, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= A[tri(r, k)] * A[tri(j, k)];
      A[tri(r, j)] = t * il;
    }
  }
  return pmin / pmax;
}

// Solves (L L^T) y = e_col for the Cholesky factor L (packed).
template <int MU>
__device__ __forceinline__ void chol_unit_solve(const double* L, int col, double* y) {
#pragma unroll
  for (int r = 0; r < MU; ++r) {
    double t = (r == col) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < r; ++k) t -= L[tri(r, k)] * y[k];
    y[r] = t / L[tri(r, r)];
  }
#pragma unroll
  for (int r = MU - 1; r >= 0; --r) {
    double t = y[r];
#pragma unroll
    for (int k = r + 1; k < MU; ++k) t -= L[tri(k, r)] * y[k];
    y[r] = t / L[tri(r, r)];
  }
}

struct GridDesc {
  int32_t n[3];
  double h[3];
  double L[3];  // box length n h per axis
  int per;      // bit a set: axis a is periodic
  double off;   // grid point i sits at (i + off) h: 1/2 (cell centres) or 0 (vertices)
  int64_t G;
};

// Offset x_s - x_t along axis a, as the minimal image on a periodic axis.
__device__ __forceinline__ double axis_diff(double xs, double xt, const GridDesc& g, int a) {
#pragma clang fp contract(off)
  double t = xs - xt;
  if ((g.per >> a) & 1) {
    const double hl = 0.5 * g.L[a];
    if (t > hl)
      t = t - g.L[a];
    else if (t < -hl)
      t = t + g.L[a];
  }
  return t;
}

// ---- cell list ------------------------------------------------------------
template <int D>
__device__ __forceinline__ int64_t cell_of(const double* __restrict__ xyz, int64_t M, int64_t n,
                                           const GridDesc& g) {
  int64_t c = 0, stride = 1;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    double t = floor(xyz[a * M + n] / g.h[a]);
    int64_t ci = (int64_t)fmin(fmax(t, 0.0), (double)(g.n[a] - 1));
    c += ci * stride;
    stride *= g.n[a];
  }
  return c;
}

template <int D>
__global__ void __launch_bounds__(256) k_cell_count(const double* __restrict__ xyz, int64_t M,
                                                    GridDesc g, int32_t* __restrict__ count,
                                                    int32_t* __restrict__ bad) {
  int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= M) return;
  // positions along a periodic axis must lie in the box [0, L)
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double x = xyz[a * M + n];
    if (((g.per >> a) & 1) && !(x >= 0.0 && x < g.L[a])) atomicOr(bad, 4);
  }
  atomicAdd(&count[cell_of<D>(xyz, M, n, g)], 1);
}

template <int D>
__global__ void __launch_bounds__(256) k_cell_fill(const double* __restrict__ xyz, int64_t M,
                                                   GridDesc g, const int32_t* __restrict__ start,
                                                   int32_t* __restrict__ cursor,
                                                   int32_t* __restrict__ sorted) {
  int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= M) return;
  int64_t c = cell_of<D>(xyz, M, n, g);
  int slot = atomicAdd(&cursor[c], 1);
  sorted[start[c] + slot] = (int32_t)n;
}

// Orders the nodes of every cell by position (x, then y, then z) and then
// by caller index (insertion sort of the cell's slice; cells hold a few
// nodes), so that the cell order of a node cloud does not depend on the
// order the caller lists it in.
template <int D>
__global__ void __launch_bounds__(256) k_cell_order(const double* __restrict__ xyz, int64_t M,
                                                    int64_t G, const int32_t* __restrict__ start,
                                                    int32_t* __restrict__ sorted) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= G) return;
  const int s0 = start[c], s1 = start[c + 1];
  auto less = [&](int a, int b) {
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      const double xa = xyz[ax * M + a], xb = xyz[ax * M + b];
      if (xa < xb) return true;
      if (xb < xa) return false;
    }
    return a < b;
  };
  for (int i = s0 + 1; i < s1; ++i) {
    const int v = sorted[i];
    int j = i - 1;
    while (j >= s0 && less(v, sorted[j])) {
      sorted[j + 1] = sorted[j];
      --j;
    }
    sorted[j + 1] = v;
  }
}

// Node positions and kinds in the internal order: node i is caller node
// perm[i].
__global__ void __launch_bounds__(256) k_gather_nodes(const int32_t* __restrict__ perm, int64_t M,
                                                      int d, const double* __restrict__ xyz,
                                                      const uint8_t* __restrict__ kind,
                                                      double* __restrict__ xo,
                                                      uint8_t* __restrict__ ko) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const int64_t n = perm[i];
  for (int a = 0; a < d; ++a) xo[a * M + i] = xyz[a * M + n];
  ko[i] = kind[n];
}

// [ncomp][M] node fields between the caller's order and the internal one.
template <typename T>
__global__ void __launch_bounds__(256) k_permute(const int32_t* __restrict__ perm, int64_t M,
                                                 int ncomp, int to_internal,
                                                 const T* __restrict__ src, T* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const int64_t n = perm[i];
  for (int c = 0; c < ncomp; ++c) {
    if (to_internal)
      dst[c * M + i] = src[c * M + n];
    else
      dst[c * M + n] = src[c * M + i];
  }
}

__global__ void __launch_bounds__(256) k_iota(int32_t* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = (int32_t)i;
}

// Exclusive scan of int32 counts (n elements) into out (n+1 elements), in
// three launches: block sums, a one-block scan of the sums, block rescans.
constexpr int SCAN_B = 1024;

__global__ void __launch_bounds__(SCAN_B) k_scan_blocksum(const int32_t* __restrict__ in,
                                                          int64_t n, int64_t* __restrict__ bsum) {
  __shared__ int64_t red[SCAN_B];
  int64_t i = (int64_t)blockIdx.x * SCAN_B + threadIdx.x;
  red[threadIdx.x] = i < n ? in[i] : 0;
  __syncthreads();
  for (int w = SCAN_B / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(SCAN_B) k_scan_sums(int64_t* __restrict__ bsum, int64_t nb) {
  __shared__ int64_t buf[SCAN_B];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += SCAN_B) {
    int64_t i = base + threadIdx.x;
    int64_t v = i < nb ? bsum[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_B; off <<= 1) {
      int64_t t = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + buf[threadIdx.x] - v;  // exclusive
    int64_t tot = buf[SCAN_B - 1];
    __syncthreads();
    carry += tot;
  }
}

__global__ void __launch_bounds__(SCAN_B) k_scan_apply(const int32_t* __restrict__ in, int64_t n,
                                                       const int64_t* __restrict__ boff,
                                                       int32_t* __restrict__ out) {
  __shared__ int64_t buf[SCAN_B];
  int64_t i = (int64_t)blockIdx.x * SCAN_B + threadIdx.x;
  int64_t v = i < n ? in[i] : 0;
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_B; off <<= 1) {
    int64_t t = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
    __syncthreads();
    buf[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t incl = boff[blockIdx.x] + buf[threadIdx.x];
  if (i < n) out[i] = (int32_t)(incl - v);
  if (i == n - 1) out[n] = (int32_t)incl;
}

// ---- k-nearest search over the cell list ------------------------------------------
struct RingArgs {
  const double* xyz;
  int64_t M;
  GridDesc g;
  const int32_t* start;   // [G+1]
  const int32_t* sorted;  // [M]
};

// The k nearest nodes of target xt (in cell ci) by the key (d^2, node index),
// skipping node `exclude` (-1: none), kept in ld/li in descending key order
// (ld[0] the worst kept).  Rings of cells at Chebyshev distance R = 0, 1, ...
// are scanned until every unscanned node lies at least (R + bound_off) hmin
// away: bound_off = 1/2 for a target at a cell centre, 0 for one anywhere in
// its cell.  Returns the number of nodes seen.
template <int D, bool EXCL>
__device__ __forceinline__ int knn_ring(const RingArgs& A, const double (&xt)[3], const int (&ci)[3],
                                        int k, int exclude, double bound_off, double (&ld)[KMAX],
                                        int (&li)[KMAX]) {
  double hmin = A.g.h[0];
#pragma unroll
  for (int a = 1; a < D; ++a) hmin = fmin(hmin, A.g.h[a]);
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    ld[j] = INFINITY;
    li[j] = 0x7fffffff;
  }
  int found = 0;
  int nmax = A.g.n[0];
#pragma unroll
  for (int a = 1; a < D; ++a) nmax = max(nmax, (int)A.g.n[a]);
  for (int R = 0; R <= nmax; ++R) {
    // cells at Chebyshev distance exactly R from the target's cell
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = a < D ? ci[a] - R : 0;
      hi[a] = a < D ? ci[a] + R : 0;
    }
    // A cell index c along axis a is scanned when it lies in the box (a
    // Neumann axis) or in the window of n cells centred on the target's
    // cell (a periodic axis; c then stands for its wrapped cell, each cell
    // once).
    auto cell_in = [&](int a, int c, int* w) -> bool {
      const int na = A.g.n[a];
      if ((A.g.per >> a) & 1) {
        const int lo_w = ci[a] - na / 2;
        if (c < lo_w || c >= lo_w + na) return false;
        *w = c < 0 ? c + na : (c >= na ? c - na : c);
        return true;
      }
      *w = c;
      return c >= 0 && c < na;
    };
    for (int cz = lo[2]; cz <= hi[2]; ++cz) {
      int wz = 0;
      if (D == 3 && !cell_in(2, cz, &wz)) continue;
      for (int cy = lo[1]; cy <= hi[1]; ++cy) {
        int wy;
        if (!cell_in(1, cy, &wy)) continue;
        bool yz_edge = (cy == lo[1] || cy == hi[1]) || (D == 3 && (cz == lo[2] || cz == hi[2]));
        int step = (yz_edge || R == 0) ? 1 : 2 * R;
        for (int cx = lo[0]; cx <= hi[0]; cx += step) {
          int wx;
          if (!cell_in(0, cx, &wx)) continue;
          int64_t c = wx + (int64_t)A.g.n[0] * (wy + (int64_t)A.g.n[1] * wz);
          int s0 = A.start[c], s1 = A.start[c + 1];
          for (int s = s0; s < s1; ++s) {
            int nid = A.sorted[s];
            if (EXCL && nid == exclude) continue;
            double dx = axis_diff(A.xyz[nid], xt[0], A.g, 0);
            double dy = axis_diff(A.xyz[A.M + nid], xt[1], A.g, 1);
            double d2 = D == 2 ? sq_sum2(dx, dy)
                               : sq_sum3(dx, dy, axis_diff(A.xyz[2 * A.M + nid], xt[2], A.g, 2));
            ++found;
            if (key_lt(d2, nid, ld[0], li[0])) {
              ld[0] = d2;
              li[0] = nid;
#pragma unroll
              for (int j = 0; j + 1 < KMAX; ++j) {
                if (j + 1 < k && key_lt(ld[j], li[j], ld[j + 1], li[j + 1])) {
                  double td = ld[j];
                  ld[j] = ld[j + 1];
                  ld[j + 1] = td;
                  int ti = li[j];
                  li[j] = li[j + 1];
                  li[j + 1] = ti;
                }
              }
            }
          }
        }
      }
    }
    // every unscanned node lies at least (R + bound_off) hmin away
    double bound = (R + bound_off) * hmin;
    if (found >= k && ld[0] < bound * bound * (1.0 - 1e-12)) break;
  }
  return found;
}

// ---- grid-target stencils ---------------------------------------------------
struct GridStencilArgs {
  RingArgs r;
  int k;
  double eps, hsup;       // hsup = support * delta
  int32_t* gidx;          // [k][G]
  double* gcoef;          // [d][k][G]
  float* gcoef32;
  int32_t* bad;           // singular flag
};

// The ring search is written out here rather than through knn_ring: the
// shared version costs this kernel its second wavefront per SIMD (register
// spills into accumulation registers), which doubles the build time.
template <int D>
__global__ void __launch_bounds__(64) k_grid_stencils(GridStencilArgs GA) {
  constexpr int MU = D == 2 ? 6 : 10;
  const RingArgs& A = GA.r;
  const int64_t p = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (p >= A.g.G) return;
  const int k = GA.k;
  int ci[3] = {0, 0, 0};
  {
    int64_t r = p;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      ci[a] = (int)(r % A.g.n[a]);
      r /= A.g.n[a];
    }
  }
  double xt[3];
#pragma unroll
  for (int a = 0; a < D; ++a) xt[a] = ((double)ci[a] + A.g.off) * A.g.h[a];
  double hmin = A.g.h[0];
#pragma unroll
  for (int a = 1; a < D; ++a) hmin = fmin(hmin, A.g.h[a]);

  // kept list in descending key order: L[0] is the worst kept
  double ld[KMAX];
  int li[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    ld[j] = INFINITY;
    li[j] = 0x7fffffff;
  }
  int found = 0;
  int nmax = A.g.n[0];
#pragma unroll
  for (int a = 1; a < D; ++a) nmax = max(nmax, (int)A.g.n[a]);
  for (int R = 0; R <= nmax; ++R) {
    // cells at Chebyshev distance exactly R from the target's cell
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = a < D ? ci[a] - R : 0;
      hi[a] = a < D ? ci[a] + R : 0;
    }
    // A cell index c along axis a is scanned when it lies in the box (a
    // Neumann axis) or in the window of n cells centred on the target's
    // cell (a periodic axis; c then stands for its wrapped cell, each cell
    // once).
    auto cell_in = [&](int a, int c, int* w) -> bool {
      const int na = A.g.n[a];
      if ((A.g.per >> a) & 1) {
        const int lo_w = ci[a] - na / 2;
        if (c < lo_w || c >= lo_w + na) return false;
        *w = c < 0 ? c + na : (c >= na ? c - na : c);
        return true;
      }
      *w = c;
      return c >= 0 && c < na;
    };
    for (int cz = lo[2]; cz <= hi[2]; ++cz) {
      int wz = 0;
      if (D == 3 && !cell_in(2, cz, &wz)) continue;
      for (int cy = lo[1]; cy <= hi[1]; ++cy) {
        int wy;
        if (!cell_in(1, cy, &wy)) continue;
        bool yz_edge = (cy == lo[1] || cy == hi[1]) || (D == 3 && (cz == lo[2] || cz == hi[2]));
        int step = (yz_edge || R == 0) ? 1 : 2 * R;
        for (int cx = lo[0]; cx <= hi[0]; cx += step) {
          int wx;
          if (!cell_in(0, cx, &wx)) continue;
          int64_t c = wx + (int64_t)A.g.n[0] * (wy + (int64_t)A.g.n[1] * wz);
          int s0 = A.start[c], s1 = A.start[c + 1];
          for (int s = s0; s < s1; ++s) {
            int nid = A.sorted[s];
            double dx = axis_diff(A.xyz[nid], xt[0], A.g, 0);
            double dy = axis_diff(A.xyz[A.M + nid], xt[1], A.g, 1);
            double d2 = D == 2 ? sq_sum2(dx, dy)
                               : sq_sum3(dx, dy, axis_diff(A.xyz[2 * A.M + nid], xt[2], A.g, 2));
            ++found;
            if (key_lt(d2, nid, ld[0], li[0])) {
              ld[0] = d2;
              li[0] = nid;
#pragma unroll
              for (int j = 0; j + 1 < KMAX; ++j) {
                if (j + 1 < k && key_lt(ld[j], li[j], ld[j + 1], li[j + 1])) {
                  double td = ld[j];
                  ld[j] = ld[j + 1];
                  ld[j + 1] = td;
                  int ti = li[j];
                  li[j] = li[j + 1];
                  li[j + 1] = ti;
                }
              }
            }
          }
        }
      }
    }
    // every unscanned node lies at least (R + off) hmin away (a cell centre
    // is 1/2 h inside its cell, a vertex sits on its corner)
    double bound = (R + A.g.off) * hmin;
    if (found >= k && ld[0] < bound * bound * (1.0 - 1e-12)) break;
  }
  if (found < k) {
    atomicOr(GA.bad, 2);
    return;
  }
  // ---- WLS (Eqs. 13-17) ----
  const double rk = sqrt(ld[0]);
  const double ht = fmax(GA.hsup, rk);
  const double iht = 1.0 / ht;
  double Cm[MU * (MU + 1) / 2];
#pragma unroll
  for (int j = 0; j < MU * (MU + 1) / 2; ++j) Cm[j] = 0.0;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < k) {
      int nid = li[j];
      double xi[3];
#pragma unroll
      for (int a = 0; a < D; ++a) xi[a] = axis_diff(A.xyz[a * A.M + nid], xt[a], A.g, a) / ht;
      double w = exp((-GA.eps * ld[j]) / (ht * ht));
      double q[MU];
      basis<D>(xi, q);
#pragma unroll
      for (int r = 0; r < MU; ++r) {
        double wq = w * q[r];
#pragma unroll
        for (int c = 0; c <= r; ++c) Cm[tri(r, c)] += wq * q[c];
      }
    }
  }
  double ratio = cholesky<MU>(Cm);
  if (!(ratio >= SINGULAR_RATIO)) {
    atomicOr(GA.bad, 1);
    return;
  }
  double y[D][MU];
#pragma unroll
  for (int a = 0; a < D; ++a) chol_unit_solve<MU>(Cm, 1 + a, y[a]);
  const int64_t G = A.g.G;
  // Storage order: by the node's offset from the target in whole grid
  // spacings (rounded per axis, each clamped to [-4, 4]), shortest offsets
  // first, ties by the offset's coordinates (z, y, x), then by node index.
  // The stencils of neighbouring grid points hold the same nearby offsets
  // (the 3^d nodes around a cell centre nearly always, farther ones by
  // turns), so entry i lies at the same offset from its target in most lanes
  // of a wavefront and the gathers of the transfer kernels are close to
  // contiguous.
  int okey[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    okey[j] = 0x7fffffff;
    if (j < k) {
      int o2 = 0, lex = 0;
#pragma unroll
      for (int a = D - 1; a >= 0; --a) {
        const double t = axis_diff(A.xyz[a * A.M + li[j]], xt[a], A.g, a) / A.g.h[a];
        const int o = (int)fmin(fmax(rint(t), -4.0), 4.0);
        o2 += o * o;
        lex = lex * 9 + (o + 4);
      }
      okey[j] = o2 * 729 + lex;
    }
  }
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < k) {
      int nid = li[j];
      int pos = 0;
#pragma unroll
      for (int jj = 0; jj < KMAX; ++jj)
        if (jj < k && (okey[jj] < okey[j] || (okey[jj] == okey[j] && li[jj] < nid))) ++pos;
      double xi[3];
#pragma unroll
      for (int a = 0; a < D; ++a) xi[a] = axis_diff(A.xyz[a * A.M + nid], xt[a], A.g, a) / ht;
      double w = exp((-GA.eps * ld[j]) / (ht * ht));
      double q[MU];
      basis<D>(xi, q);
      GA.gidx[(int64_t)pos * G + p] = nid;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double t = 0.0;
#pragma unroll
        for (int r = 0; r < MU; ++r) t += y[a][r] * q[r];
        double cval = w * t * iht;
        if (GA.gcoef) GA.gcoef[((int64_t)a * k + pos) * G + p] = cval;
        if (GA.gcoef32) GA.gcoef32[((int64_t)a * k + pos) * G + p] = (float)cval;
      }
    }
  }
}

// ---- node-target stencils ------------------------------------------------------
struct NodeStencilArgs {
  const double* xyz;
  int64_t M;
  GridDesc g;
  int m, bn, k;
  double eps, hsup;
  int32_t* nbase;   // [M]
  int64_t ms;       // coefficient stream stride (>= M)
  double* ncoef;    // [d][bn][ms]
  float* ncoef32;
  int32_t* bad;
};

template <int D>
__global__ void __launch_bounds__(64) k_node_stencils(NodeStencilArgs A) {
  constexpr int MU = D == 2 ? 6 : 10;
  const int64_t n = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (n >= A.M) return;
  const int m = A.m, bn = A.bn, k = A.k;
  double x[3];
  // base: the block's low line along each axis, unwrapped (a periodic axis
  // may start it at -1 or end it past n - 1: those lines are the periodic
  // images of the lines at the other face)
  int base[3] = {0, 0, 0};
  int64_t flat0 = 0, stride = 1;
  bool wraps = false;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    x[a] = A.xyz[a * A.M + n];
    double lo = floor(x[a] / A.g.h[a] - (0.5 * m - 1.0 + A.g.off));
    if (!((A.g.per >> a) & 1)) lo = fmin(fmax(lo, 0.0), (double)(A.g.n[a] - m));
    base[a] = (int)lo;
    const int na = A.g.n[a];
    const int bw = base[a] < 0 ? base[a] + na : base[a];
    wraps = wraps || base[a] < 0 || base[a] + m > na;
    flat0 += (int64_t)bw * stride;
    stride *= na;
  }
  // squared distances of the block points
  double d2[BNMAX];
  int64_t fl[BNMAX];
#pragma unroll
  for (int o = 0; o < BNMAX; ++o) {
    d2[o] = INFINITY;
    fl[o] = 0;
    if (o < bn) {
      int oc[3] = {o % m, (o / m) % m, o / (m * m)};
      double dd[3];
      int64_t f = 0, st = 1;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        int cc = base[a] + oc[a];
        dd[a] = ((double)cc + A.g.off) * A.g.h[a] - x[a];
        const int na = A.g.n[a];
        f += (int64_t)(cc < 0 ? cc + na : (cc >= na ? cc - na : cc)) * st;
        st *= na;
      }
      d2[o] = D == 2 ? sq_sum2(dd[0], dd[1]) : sq_sum3(dd[0], dd[1], dd[2]);
      fl[o] = f;
    }
  }
  // selection: the k smallest (d^2, flat index) keys of the block
  bool sel[BNMAX];
  double rk2 = 0.0;
#pragma unroll
  for (int o = 0; o < BNMAX; ++o) {
    sel[o] = false;
    if (o < bn) {
      int rank = 0;
      if (k < bn) {
#pragma unroll
        for (int q = 0; q < BNMAX; ++q)
          if (q < bn && key_lt(d2[q], (int)fl[q], d2[o], (int)fl[o])) ++rank;
      }
      sel[o] = rank < k;
      if (sel[o]) rk2 = fmax(rk2, d2[o]);
    }
  }
  const double ht = fmax(A.hsup, sqrt(rk2));
  const double iht = 1.0 / ht;
  double Cm[MU * (MU + 1) / 2];
#pragma unroll
  for (int j = 0; j < MU * (MU + 1) / 2; ++j) Cm[j] = 0.0;
#pragma unroll
  for (int o = 0; o < BNMAX; ++o) {
    if (o < bn && sel[o]) {
      int oc[3] = {o % m, (o / m) % m, o / (m * m)};
      double xi[3];
#pragma unroll
      for (int a = 0; a < D; ++a)
        xi[a] = ((((double)(base[a] + oc[a]) + A.g.off) * A.g.h[a]) - x[a]) / ht;
      double w = exp((-A.eps * d2[o]) / (ht * ht));
      double q[MU];
      basis<D>(xi, q);
#pragma unroll
      for (int r = 0; r < MU; ++r) {
        double wq = w * q[r];
#pragma unroll
        for (int c = 0; c <= r; ++c) Cm[tri(r, c)] += wq * q[c];
      }
    }
  }
  double ratio = cholesky<MU>(Cm);
  if (!(ratio >= SINGULAR_RATIO)) {
    atomicOr(A.bad, 1);
    return;
  }
  double y[D][MU];
#pragma unroll
  for (int a = 0; a < D; ++a) chol_unit_solve<MU>(Cm, 1 + a, y[a]);
  // a block that wraps around a periodic axis is marked by storing the
  // one's complement of its low corner (the gathers then wrap its entries)
  A.nbase[n] = wraps ? ~(int32_t)flat0 : (int32_t)flat0;
  const int64_t ms = A.ms;
#pragma unroll
  for (int o = 0; o < BNMAX; ++o) {
    if (o < bn) {
      double cv[3] = {0.0, 0.0, 0.0};
      if (sel[o]) {
        int oc[3] = {o % m, (o / m) % m, o / (m * m)};
        double xi[3];
#pragma unroll
        for (int a = 0; a < D; ++a)
          xi[a] = ((((double)(base[a] + oc[a]) + A.g.off) * A.g.h[a]) - x[a]) / ht;
        double w = exp((-A.eps * d2[o]) / (ht * ht));
        double q[MU];
        basis<D>(xi, q);
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double t = 0.0;
#pragma unroll
          for (int r = 0; r < MU; ++r) t += y[a][r] * q[r];
          cv[a] = w * t * iht;
        }
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        if (A.ncoef) A.ncoef[((int64_t)a * bn + o) * ms + n] = cv[a];
        if (A.ncoef32) A.ncoef32[((int64_t)a * bn + o) * ms + n] = (float)cv[a];
      }
    }
  }
}

// ---- node-to-node stencils (the first fractional step) ------------------------------
// Eq. 11 polynomial vector of the known-value form (2D: x, y, x^2/2, xy, y^2/2;
// 3D: x, y, z, x^2/2, xy, xz, y^2/2, yz, z^2/2) of scaled offsets.
template <int D>
__device__ __forceinline__ void basis_known(const double* xi, double* q) {
  if (D == 2) {
    q[0] = xi[0]; q[1] = xi[1];
    q[2] = 0.5 * xi[0] * xi[0]; q[3] = xi[0] * xi[1]; q[4] = 0.5 * xi[1] * xi[1];
  } else {
    q[0] = xi[0]; q[1] = xi[1]; q[2] = xi[2];
    q[3] = 0.5 * xi[0] * xi[0]; q[4] = xi[0] * xi[1]; q[5] = xi[0] * xi[2];
    q[6] = 0.5 * xi[1] * xi[1]; q[7] = xi[1] * xi[2]; q[8] = 0.5 * xi[2] * xi[2];
  }
}

struct SelfStencilArgs {
  RingArgs r;
  int k;
  double eps, hsup;
  int64_t ms;       // stream stride
  int32_t* sidx;    // [k][ms] neighbour node, ascending
  double* scoef;    // [d+1][k][ms]: d first-derivative rows, then the Laplacian row
  float* scoef32;
  int32_t* bad;
};

// Every node's k nearest other nodes and the known-value WLS rows of
// Eqs. 13-15 (data f(x_i) - f(x)): first derivatives and the Laplacian
// (the sum of the pure second-derivative rows), in float64.
template <int D>
__global__ void __launch_bounds__(64) k_self_stencils(SelfStencilArgs SA) {
  constexpr int MU = D == 2 ? 5 : 9;
  const RingArgs& A = SA.r;
  const int64_t n = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (n >= A.M) return;
  const int k = SA.k;
  double xt[3];
  int ci[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    xt[a] = A.xyz[a * A.M + n];
    const double t = floor(xt[a] / A.g.h[a]);
    ci[a] = (int)fmin(fmax(t, 0.0), (double)(A.g.n[a] - 1));
  }
  double ld[KMAX];
  int li[KMAX];
  const int found = knn_ring<D, true>(A, xt, ci, k, (int)n, 0.0, ld, li);
  if (found < k) {
    atomicOr(SA.bad, 2);
    return;
  }
  const double ht = fmax(SA.hsup, sqrt(ld[0]));
  const double iht = 1.0 / ht;
  double Cm[MU * (MU + 1) / 2];
#pragma unroll
  for (int j = 0; j < MU * (MU + 1) / 2; ++j) Cm[j] = 0.0;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < k) {
      const int nid = li[j];
      double xi[3];
#pragma unroll
      for (int a = 0; a < D; ++a) xi[a] = axis_diff(A.xyz[a * A.M + nid], xt[a], A.g, a) / ht;
      const double w = exp((-SA.eps * ld[j]) / (ht * ht));
      double q[MU];
      basis_known<D>(xi, q);
#pragma unroll
      for (int r = 0; r < MU; ++r) {
        const double wq = w * q[r];
#pragma unroll
        for (int c = 0; c <= r; ++c) Cm[tri(r, c)] += wq * q[c];
      }
    }
  }
  if (!(cholesky<MU>(Cm) >= SINGULAR_RATIO)) {
    atomicOr(SA.bad, 1);
    return;
  }
  // rows of C^-1: the first derivatives (unknowns 0..D-1) and the sum of the
  // pure second derivatives (2D: unknowns 2, 4; 3D: 3, 6, 8)
  double y[D + 1][MU];
#pragma unroll
  for (int a = 0; a < D; ++a) chol_unit_solve<MU>(Cm, a, y[a]);
  {
    double t0[MU], t1[MU], t2[MU];
    chol_unit_solve<MU>(Cm, D == 2 ? 2 : 3, t0);
    chol_unit_solve<MU>(Cm, D == 2 ? 4 : 6, t1);
    if (D == 3) chol_unit_solve<MU>(Cm, 8, t2);
#pragma unroll
    for (int r = 0; r < MU; ++r) y[D][r] = D == 2 ? t0[r] + t1[r] : (t0[r] + t1[r]) + t2[r];
  }
  const int64_t ms = SA.ms;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < k) {
      const int nid = li[j];
      int pos = 0;  // ascending node index (near-contiguous gathers)
#pragma unroll
      for (int jj = 0; jj < KMAX; ++jj)
        if (jj < k && li[jj] < nid) ++pos;
      double xi[3];
#pragma unroll
      for (int a = 0; a < D; ++a) xi[a] = axis_diff(A.xyz[a * A.M + nid], xt[a], A.g, a) / ht;
      const double w = exp((-SA.eps * ld[j]) / (ht * ht));
      double q[MU];
      basis_known<D>(xi, q);
      SA.sidx[(int64_t)pos * ms + n] = nid;
#pragma unroll
      for (int a = 0; a <= D; ++a) {
        double t = 0.0;
#pragma unroll
        for (int r = 0; r < MU; ++r) t += y[a][r] * q[r];
        // first derivatives scale by 1/h_t, the Laplacian by 1/h_t^2
        const double cval = a < D ? w * t * iht : w * t * (iht * iht);
        if (SA.scoef) SA.scoef[((int64_t)a * k + pos) * ms + n] = cval;
        if (SA.scoef32) SA.scoef32[((int64_t)a * k + pos) * ms + n] = (float)cval;
      }
    }
  }
}

// ---- IB lists ------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_near_flags(const int32_t* __restrict__ gidx, int64_t G,
                                                    int k, const uint8_t* __restrict__ kind,
                                                    uint8_t* __restrict__ flag) {
  int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= G) return;
  int cnt = 0;
  for (int i = 0; i < k; ++i) cnt += kind[gidx[(int64_t)i * G + p]] != PC_KIND_F;
  flag[p] = (uint8_t)(cnt > 255 ? 255 : cnt);
}

__global__ void __launch_bounds__(256) k_slot_map(const int32_t* __restrict__ ib, int64_t nib,
                                                  int32_t* __restrict__ slot) {
  int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s < nib) slot[ib[s]] = (int32_t)s;
}

template <typename T>
__global__ void __launch_bounds__(256) k_near_fill(const int32_t* __restrict__ near, int64_t nnear,
                                                   int64_t nns, int W,
                                                   const int32_t* __restrict__ gidx,
                                                   const T* __restrict__ gcoef, int64_t G, int k,
                                                   int d, const int32_t* __restrict__ slot,
                                                   int32_t* __restrict__ nslot,
                                                   T* __restrict__ ncoefib) {
  int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= nnear) return;
  int64_t p = near[q];
  int e = 0;
  for (int i = 0; i < k; ++i) {
    int nid = gidx[(int64_t)i * G + p];
    int s = slot[nid];
    if (s >= 0 && e < W) {
      nslot[(int64_t)e * nns + q] = s;
      for (int a = 0; a < d; ++a)
        ncoefib[((int64_t)a * W + e) * nns + q] = gcoef[((int64_t)a * k + i) * G + p];
      ++e;
    }
  }
  for (; e < W; ++e) {
    nslot[(int64_t)e * nns + q] = -1;
    for (int a = 0; a < d; ++a) ncoefib[((int64_t)a * W + e) * nns + q] = T(0);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_ib_gather(const int32_t* __restrict__ ib, int64_t nib,
                                                   const int32_t* __restrict__ nbase,
                                                   const T* __restrict__ ncoef, int64_t ms,
                                                   int rows, int64_t ibs,
                                                   int32_t* __restrict__ ibbase,
                                                   T* __restrict__ ibcoef) {
  int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= nib) return;
  int64_t nid = ib[s];
  if (ibbase) ibbase[s] = nbase[nid];
  for (int r = 0; r < rows; ++r) ibcoef[(int64_t)r * ibs + s] = ncoef[(int64_t)r * ms + nid];
}

// Node block bases for export: the low corner, with the wrap mark removed.
__global__ void __launch_bounds__(256) k_base_export(const int32_t* __restrict__ in, int64_t n,
                                                     int32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const int32_t v = in[i];
    out[i] = v < 0 ? ~v : v;
  }
}

// Stencils of selected targets, for inspection: grid stencils of the grid
// points pts[t] and node stencils of the nodes nds[t] (one thread per target
// and array); an index out of range sets *bad and is skipped.
__global__ void __launch_bounds__(256) k_export_at(const int32_t* __restrict__ gidx,
                                                   const double* __restrict__ gcoef, int64_t G,
                                                   int kg, int d, const int64_t* __restrict__ pts,
                                                   int64_t np_, int32_t* __restrict__ oidx,
                                                   double* __restrict__ ocoef,
                                                   const int32_t* __restrict__ nbase,
                                                   const double* __restrict__ ncoef, int64_t M,
                                                   int64_t ms, int bn,
                                                   const int64_t* __restrict__ nds, int64_t nn,
                                                   int32_t* __restrict__ obase,
                                                   double* __restrict__ oncoef,
                                                   int32_t* __restrict__ bad) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < np_) {
    const int64_t p = pts[t];
    if (p < 0 || p >= G) {
      *bad = 1;
    } else {
      for (int i = 0; i < kg; ++i) {
        if (oidx) oidx[(int64_t)i * np_ + t] = gidx[(int64_t)i * G + p];
        if (ocoef)
          for (int a = 0; a < d; ++a)
            ocoef[((int64_t)a * kg + i) * np_ + t] = gcoef[((int64_t)a * kg + i) * G + p];
      }
    }
  }
  if (t < nn) {
    const int64_t n = nds[t];
    if (n < 0 || n >= M) {
      *bad = 1;
    } else {
      if (obase) {
        const int32_t v = nbase[n];
        obase[t] = v < 0 ? ~v : v;
      }
      if (oncoef)
        for (int r = 0; r < d * bn; ++r) oncoef[(int64_t)r * nn + t] = ncoef[(int64_t)r * ms + n];
    }
  }
}

int scan_exclusive(const int32_t* in, int64_t n, int32_t* out, hipStream_t s) {
  int64_t nb = (n + SCAN_B - 1) / SCAN_B;
  int64_t* bsum = nullptr;
  PC_TRY(dev_alloc((void**)&bsum, (size_t)nb * sizeof(int64_t), "scan sums"));
  hipLaunchKernelGGL(k_scan_blocksum, dim3((unsigned)nb), dim3(SCAN_B), 0, s, in, n, bsum);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_B), 0, s, bsum, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_B), 0, s, in, n, bsum, out);
  hipError_t e = hipStreamSynchronize(s);
  dev_free(bsum);
  if (e != hipSuccess) return fail(PC_ERR_HIP, std::string("scan: ") + hipGetErrorString(e));
  return PC_OK;
}

unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void geom_free(pc_geom* g) {
  if (!g) return;
  void* ptrs[] = {g->gidx,   g->gcoef,  g->gcoef32, g->nbase,  g->ncoef,  g->ncoef32,
                  g->ib,     g->near,   g->nslot,   g->ncoefib, g->ncoefib32, g->ibbase,
                  g->ibcoef, g->ibcoef32, g->sidx,  g->scoef,   g->scoef32,  g->vlist,
                  g->perm};
  for (void* p : ptrs) dev_free(p);
}

struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) dev_free(p);
  }
  int alloc(void** p, size_t bytes, const char* what) {
    int rc = dev_alloc(p, bytes, what);
    if (rc == PC_OK) ptrs.push_back(*p);
    return rc;
  }
};

// Device bytes held by a geometry with these counts (the arrays of
// pc_wls_build; the node permutation of PC_ORDER_CELL not included).
int64_t geom_bytes_for(int d, int64_t G, int64_t M, int k_grid, int bn, int64_t n_ib,
                       int64_t n_near, int near_w, bool want64, bool want32, int k_self,
                       int64_t n_v) {
  const int64_t ms = (M + 63) / 64 * 64, ibs = (n_ib + 63) / 64 * 64;
  const int64_t ell = n_near ? (int64_t)near_w * ((n_near + 63) / 64 * 64) : 0;
  // indices, bases and lists (every geometry)
  int64_t bytes = (int64_t)k_grid * G * 4 + M * 4 + n_ib * 4 + n_near * 4 + ell * 4 +
                  n_ib * 4 + (int64_t)k_self * ms * 4 + n_v * 4;
  // coefficients, per kept precision (s bytes a value)
  for (int s : {8, 4}) {
    if (!(s == 8 ? want64 : want32)) continue;
    bytes += ((int64_t)d * k_grid * G + (int64_t)d * bn * ms + ell * d + ibs * (int64_t)d * bn +
              (int64_t)k_self * ms * (d + 1)) * s;
  }
  return bytes;
}

// The stencil copies a build keeps, from pc_wls_opts.dtype_mask: bit
// (1 << PC_F64) float64, bit (1 << PC_F32) float32; 0 means float64 only.
int dtype_keep(const pc_wls_opts* o, bool* want64, bool* want32) {
  const int mask = o ? o->dtype_mask : 0;
  if (mask & ~((1 << PC_F64) | (1 << PC_F32)))
    return fail(PC_ERR_INVALID_ARG, "dtype_mask takes the bits (1 << PC_F64) and (1 << PC_F32)");
  *want64 = mask == 0 || (mask & (1 << PC_F64));
  *want32 = (mask & (1 << PC_F32)) != 0;
  return PC_OK;
}

// Scratch a build holds at most at once besides the geometry's own arrays:
// the cell list (counts, starts, cursors, sorted nodes), flags, the scan
// sums, the near flags and the slot map; PC_ORDER_CELL adds its own cell
// list and the nodes in cell order.
int64_t build_scratch_bytes(int d, int64_t G, int64_t M, bool cell_order) {
  int64_t b = 4 * G + 4 * (G + 1) + 4 * G + 4 * M + 256 + G + 4 * M + 8 * ((G + 1023) / 1024);
  if (cell_order) b += 4 * G + 4 * (G + 1) + 4 * G + 256 + 8 * (int64_t)d * M + M;
  return b;
}

GridDesc grid_desc(const pc_plan* P) {
  GridDesc gd;
  gd.per = 0;
  for (int a = 0; a < 3; ++a) {
    gd.n[a] = P->n[a];
    gd.h[a] = P->h[a];
    gd.L[a] = (double)P->n[a] * P->h[a];
    if (a < P->d && P->bc[a] == PC_BC_PERIODIC) gd.per |= 1 << a;
  }
  gd.G = P->G;
  gd.off = P->vertex ? 0.0 : 0.5;
  return gd;
}

int build(const pc_plan* P, const double* xyz, const uint8_t* kind, int64_t M,
          const pc_wls_opts* o, hipStream_t s, pc_geom* g);

// PC_ORDER_CELL: the nodes sorted by grid cell (cells x fastest; within a
// cell by position, then caller index) into g->perm, and the stencils built
// on the cloud in that order.
int build_cell_order(const pc_plan* P, const double* xyz, const uint8_t* kind, int64_t M,
                     const pc_wls_opts* o, hipStream_t s, pc_geom* g) {
  const int d = P->d;
  const int64_t G = P->G;
  const GridDesc gd = grid_desc(P);
  Scratch tmp;
  int32_t *count, *start, *cursor, *bad;
  PC_TRY(tmp.alloc((void**)&count, (size_t)G * 4, "cell counts"));
  PC_TRY(tmp.alloc((void**)&start, (size_t)(G + 1) * 4, "cell starts"));
  PC_TRY(tmp.alloc((void**)&cursor, (size_t)G * 4, "cell cursors"));
  PC_TRY(tmp.alloc((void**)&bad, 256, "flags"));
  PC_TRY(dev_alloc((void**)&g->perm, (size_t)M * 4, "node permutation"));
  PC_TRY(fill_zero(count, (size_t)G * 4, s));
  PC_TRY(fill_zero(cursor, (size_t)G * 4, s));
  PC_TRY(fill_zero(bad, 256, s));
  if (d == 2)
    hipLaunchKernelGGL(k_cell_count<2>, dim3(nblocks(M, 256)), dim3(256), 0, s, xyz, M, gd, count,
                       bad);
  else
    hipLaunchKernelGGL(k_cell_count<3>, dim3(nblocks(M, 256)), dim3(256), 0, s, xyz, M, gd, count,
                       bad);
  PC_HIP_CHECK(hipGetLastError());
  PC_TRY(scan_exclusive(count, G, start, s));
  if (d == 2) {
    hipLaunchKernelGGL(k_cell_fill<2>, dim3(nblocks(M, 256)), dim3(256), 0, s, xyz, M, gd, start,
                       cursor, g->perm);
    hipLaunchKernelGGL(k_cell_order<2>, dim3(nblocks(G, 256)), dim3(256), 0, s, xyz, M, G, start,
                       g->perm);
  } else {
    hipLaunchKernelGGL(k_cell_fill<3>, dim3(nblocks(M, 256)), dim3(256), 0, s, xyz, M, gd, start,
                       cursor, g->perm);
    hipLaunchKernelGGL(k_cell_order<3>, dim3(nblocks(G, 256)), dim3(256), 0, s, xyz, M, G, start,
                       g->perm);
  }
  PC_HIP_CHECK(hipGetLastError());
  double* xi;
  uint8_t* ki;
  PC_TRY(tmp.alloc((void**)&xi, (size_t)d * M * 8, "node positions in cell order"));
  PC_TRY(tmp.alloc((void**)&ki, (size_t)M, "node kinds in cell order"));
  hipLaunchKernelGGL(k_gather_nodes, dim3(nblocks(M, 256)), dim3(256), 0, s, g->perm, M, d, xyz,
                     kind, xi, ki);
  PC_HIP_CHECK(hipGetLastError());
  PC_TRY(build(P, xi, ki, M, o, s, g));
  g->bytes += M * 4;
  return PC_OK;
}

int build(const pc_plan* P, const double* xyz, const uint8_t* kind, int64_t M,
          const pc_wls_opts* o, hipStream_t s, pc_geom* g) {
  const int d = P->d;
  const int MU = d == 2 ? 6 : 10;
  int k_grid = o && o->k_grid ? o->k_grid : 16;
  int k_node = o && o->k_node ? o->k_node : (d == 2 ? 16 : 27);
  double eps = o && o->eps != 0.0 ? o->eps : 6.3;
  double support = o && o->support != 0.0 ? o->support : 3.0;
  double delta = o ? o->delta : 0.0;
  bool want64 = true, want32 = false;
  PC_TRY(dtype_keep(o, &want64, &want32));
  const int k_self = o ? o->k_self : 0;
  if (k_self != 0 && (k_self < (d == 2 ? 5 : 9) || k_self > KMAX))
    return fail(PC_ERR_INVALID_ARG, "k_self must be 0 or in [5 (2D) / 9 (3D), PC_MAX_K_GRID]");
  if (k_self >= M) return fail(PC_ERR_INVALID_ARG, "k_self must be below the number of nodes");
  if (k_grid < MU || k_node < MU)
    return fail(PC_ERR_INVALID_ARG, "k_grid and k_node must be at least the number of unknowns");
  if (k_grid > KMAX) return fail(PC_ERR_UNSUPPORTED_SIZE, "k_grid above PC_MAX_K_GRID");
  if (M < k_grid) return fail(PC_ERR_INVALID_ARG, "fewer nodes than k_grid");
  if (M > INT32_MAX - 1) return fail(PC_ERR_UNSUPPORTED_SIZE, "more than 2^31-2 nodes");
  int m = 1;
  while ((int)std::pow(m, d) < k_node) ++m;
  if (m < 3) m = 3;  // a quadratic fit needs three lines per axis
  int bn = 1;
  for (int a = 0; a < d; ++a) bn *= m;
  if (bn > BNMAX) return fail(PC_ERR_UNSUPPORTED_SIZE, "k_node block above PC_MAX_K_NODE");
  for (int a = 0; a < d; ++a)
    if (P->n[a] < m) return fail(PC_ERR_UNSUPPORTED_SIZE, "grid smaller than the node block");
  if (!(eps > 0.0) || !(support > 0.0) || delta < 0.0)
    return fail(PC_ERR_INVALID_ARG, "eps and support must be positive, delta non-negative");
  if (delta == 0.0) {
    bool iso = true;
    for (int a = 1; a < d; ++a) iso = iso && P->h[a] == P->h[0];
    if (iso) {
      delta = P->h[0];
    } else {
      double prod = 1.0;
      for (int a = 0; a < d; ++a) prod *= P->h[a];
      delta = std::pow(prod, 1.0 / d);
    }
  }
  const int64_t G = P->G;
  g->d = d;
  g->M = M;
  g->G = G;
  for (int a = 0; a < 3; ++a) {
    g->n[a] = P->n[a];
    g->h[a] = P->h[a];
  }
  g->k_grid = k_grid;
  g->k_node = k_node;
  g->m_node = m;
  g->bn = bn;
  g->has32 = want32;
  g->has64 = want64;
  const GridDesc gd = grid_desc(P);
  g->per = gd.per;
  g->vertex = P->vertex;

  Scratch tmp;
  int32_t *count, *start, *cursor, *sorted, *bad;
  PC_TRY(tmp.alloc((void**)&count, (size_t)G * 4, "cell counts"));
  PC_TRY(tmp.alloc((void**)&start, (size_t)(G + 1) * 4, "cell starts"));
  PC_TRY(tmp.alloc((void**)&cursor, (size_t)G * 4, "cell cursors"));
  PC_TRY(tmp.alloc((void**)&sorted, (size_t)M * 4, "sorted nodes"));
  PC_TRY(tmp.alloc((void**)&bad, 256, "flags"));
  PC_TRY(fill_zero(count, (size_t)G * 4, s));
  PC_TRY(fill_zero(cursor, (size_t)G * 4, s));
  PC_TRY(fill_zero(bad, 256, s));
  if (d == 2)
    hipLaunchKernelGGL(k_cell_count<2>, dim3(nblocks(M, 256)), dim3(256), 0, s, xyz, M, gd, count,
                       bad);
  else
    hipLaunchKernelGGL(k_cell_count<3>, dim3(nblocks(M, 256)), dim3(256), 0, s, xyz, M, gd, count,
                       bad);
  PC_HIP_CHECK(hipGetLastError());
  PC_TRY(scan_exclusive(count, G, start, s));
  if (d == 2)
    hipLaunchKernelGGL(k_cell_fill<2>, dim3(nblocks(M, 256)), dim3(256), 0, s, xyz, M, gd, start,
                       cursor, sorted);
  else
    hipLaunchKernelGGL(k_cell_fill<3>, dim3(nblocks(M, 256)), dim3(256), 0, s, xyz, M, gd, start,
                       cursor, sorted);
  PC_HIP_CHECK(hipGetLastError());

  // grid-target stencils
  PC_TRY(dev_alloc((void**)&g->gidx, (size_t)k_grid * G * 4, "grid stencil indices"));
  if (want64)
    PC_TRY(dev_alloc((void**)&g->gcoef, (size_t)d * k_grid * G * 8, "grid stencil coefficients"));
  if (want32)
    PC_TRY(dev_alloc((void**)&g->gcoef32, (size_t)d * k_grid * G * 4, "grid stencil f32"));
  const RingArgs ring{xyz, M, gd, start, sorted};
  GridStencilArgs ga{ring, k_grid, eps, support * delta, g->gidx, g->gcoef, g->gcoef32, bad};
  if (d == 2)
    hipLaunchKernelGGL(k_grid_stencils<2>, dim3(nblocks(G, 64)), dim3(64), 0, s, ga);
  else
    hipLaunchKernelGGL(k_grid_stencils<3>, dim3(nblocks(G, 64)), dim3(64), 0, s, ga);
  PC_HIP_CHECK(hipGetLastError());

  // node-target stencils
  PC_TRY(dev_alloc((void**)&g->nbase, (size_t)M * 4, "node stencil bases"));
  g->ms = (M + 63) / 64 * 64;
  if (want64)
    PC_TRY(dev_alloc((void**)&g->ncoef, (size_t)d * bn * g->ms * 8, "node stencil coefficients"));
  if (want32)
    PC_TRY(dev_alloc((void**)&g->ncoef32, (size_t)d * bn * g->ms * 4, "node stencil f32"));
  NodeStencilArgs na{xyz, M, gd, m, bn, k_node, eps, support * delta, g->nbase, g->ms, g->ncoef,
                     g->ncoef32, bad};
  if (d == 2)
    hipLaunchKernelGGL(k_node_stencils<2>, dim3(nblocks(M, 64)), dim3(64), 0, s, na);
  else
    hipLaunchKernelGGL(k_node_stencils<3>, dim3(nblocks(M, 64)), dim3(64), 0, s, na);
  PC_HIP_CHECK(hipGetLastError());

  // node-to-node stencils (the first fractional step)
  g->k_self = k_self;
  if (k_self) {
    PC_TRY(dev_alloc((void**)&g->sidx, (size_t)k_self * g->ms * 4, "node-node indices"));
    if (want64)
      PC_TRY(dev_alloc((void**)&g->scoef, (size_t)(d + 1) * k_self * g->ms * 8,
                       "node-node coefs"));
    if (want32)
      PC_TRY(dev_alloc((void**)&g->scoef32, (size_t)(d + 1) * k_self * g->ms * 4,
                       "node-node coefs f32"));
    SelfStencilArgs sa{ring, k_self, eps, support * delta, g->ms, g->sidx, g->scoef, g->scoef32,
                       bad};
    if (d == 2)
      hipLaunchKernelGGL(k_self_stencils<2>, dim3(nblocks(M, 64)), dim3(64), 0, s, sa);
    else
      hipLaunchKernelGGL(k_self_stencils<3>, dim3(nblocks(M, 64)), dim3(64), 0, s, sa);
    PC_HIP_CHECK(hipGetLastError());
  }

  int32_t hbad = 0;
  PC_HIP_CHECK(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s));
  PC_HIP_CHECK(hipStreamSynchronize(s));
  if (hbad & 4)
    return fail(PC_ERR_INVALID_ARG, "positions along a periodic axis must lie in [0, n h)");
  if (hbad & 2) return fail(PC_ERR_INVALID_ARG, "a grid point found fewer than k_grid nodes");
  if (hbad & 1)
    return fail(PC_ERR_SINGULAR_STENCIL, "a WLS normal matrix is singular (squared pivot ratio "
                                         "below 1e-12)");

  // boundary + virtual node list (ascending)
  std::vector<uint8_t> hkind((size_t)M);
  PC_HIP_CHECK(hipMemcpy(hkind.data(), kind, (size_t)M, hipMemcpyDeviceToHost));
  std::vector<int32_t> hib, hv;
  for (int64_t n = 0; n < M; ++n) {
    if (hkind[n] > PC_KIND_V) return fail(PC_ERR_INVALID_ARG, "node kind must be 0, 1 or 2");
    if (hkind[n] != PC_KIND_F) hib.push_back((int32_t)n);
    if (hkind[n] == PC_KIND_V) hv.push_back((int32_t)n);
  }
  g->n_ib = (int64_t)hib.size();
  g->n_v = (int64_t)hv.size();
  if (g->n_v) {
    PC_TRY(dev_alloc((void**)&g->vlist, (size_t)g->n_v * 4, "virtual list"));
    PC_HIP_CHECK(hipMemcpy(g->vlist, hv.data(), (size_t)g->n_v * 4, hipMemcpyHostToDevice));
  }
  // near-IB grid points and their compact stencils
  uint8_t* nflag;
  PC_TRY(tmp.alloc((void**)&nflag, (size_t)G, "near flags"));
  hipLaunchKernelGGL(k_near_flags, dim3(nblocks(G, 256)), dim3(256), 0, s, g->gidx, G, k_grid,
                     kind, nflag);
  PC_HIP_CHECK(hipGetLastError());
  std::vector<uint8_t> hflag((size_t)G);
  PC_HIP_CHECK(hipMemcpyAsync(hflag.data(), nflag, (size_t)G, hipMemcpyDeviceToHost, s));
  PC_HIP_CHECK(hipStreamSynchronize(s));
  std::vector<int32_t> hnear;
  int near_w = 0;
  int64_t near_entries = 0;
  for (int64_t p = 0; p < G; ++p) {
    if (hflag[p]) {
      hnear.push_back((int32_t)p);
      near_w = std::max(near_w, (int)hflag[p]);
      near_entries += hflag[p];
    }
  }
  g->n_near = (int64_t)hnear.size();
  g->n_near_entries = near_entries;
  // the ELL width is one of three compile-time bounds of the update kernel
  near_w = near_w <= 8 ? 8 : (near_w <= 16 ? 16 : (near_w <= 27 && d == 3 ? 27 : 32));
  g->near_w = near_w;
  g->nns = (g->n_near + 63) / 64 * 64;
  g->ibs = (g->n_ib + 63) / 64 * 64;
  if (g->n_ib) {
    PC_TRY(dev_alloc((void**)&g->ib, (size_t)g->n_ib * 4, "IB list"));
    PC_HIP_CHECK(hipMemcpy(g->ib, hib.data(), (size_t)g->n_ib * 4, hipMemcpyHostToDevice));
  }
  if (g->n_near) {
    const int64_t ell = (int64_t)near_w * g->nns;
    PC_TRY(dev_alloc((void**)&g->near, (size_t)g->n_near * 4, "near list"));
    PC_TRY(dev_alloc((void**)&g->nslot, (size_t)ell * 4, "near slots"));
    if (want64) PC_TRY(dev_alloc((void**)&g->ncoefib, (size_t)d * ell * 8, "near coefs"));
    if (want32) PC_TRY(dev_alloc((void**)&g->ncoefib32, (size_t)d * ell * 4, "near coefs"));
    PC_HIP_CHECK(hipMemcpy(g->near, hnear.data(), (size_t)g->n_near * 4, hipMemcpyHostToDevice));
    int32_t* slot;
    PC_TRY(tmp.alloc((void**)&slot, (size_t)M * 4, "slot map"));
    PC_HIP_CHECK(hipMemsetAsync(slot, 0xff, (size_t)M * 4, s));
    hipLaunchKernelGGL(k_slot_map, dim3(nblocks(g->n_ib, 256)), dim3(256), 0, s, g->ib, g->n_ib,
                       slot);
    if (want64)
      hipLaunchKernelGGL(k_near_fill<double>, dim3(nblocks(g->n_near, 256)), dim3(256), 0, s,
                         g->near, g->n_near, g->nns, near_w, g->gidx, g->gcoef, G, k_grid, d,
                         slot, g->nslot, g->ncoefib);
    if (want32)
      hipLaunchKernelGGL(k_near_fill<float>, dim3(nblocks(g->n_near, 256)), dim3(256), 0, s,
                         g->near, g->n_near, g->nns, near_w, g->gidx, g->gcoef32, G, k_grid,
                         d, slot, g->nslot, g->ncoefib32);
    PC_HIP_CHECK(hipGetLastError());
  }
  if (g->n_ib) {
    PC_TRY(dev_alloc((void**)&g->ibbase, (size_t)g->n_ib * 4, "IB bases"));
    // the first gather also writes the bases
    if (want64) {
      PC_TRY(dev_alloc((void**)&g->ibcoef, (size_t)d * bn * g->ibs * 8, "IB coefs"));
      hipLaunchKernelGGL(k_ib_gather<double>, dim3(nblocks(g->n_ib, 256)), dim3(256), 0, s,
                         g->ib, g->n_ib, g->nbase, g->ncoef, g->ms, d * bn, g->ibs, g->ibbase,
                         g->ibcoef);
    }
    if (want32) {
      PC_TRY(dev_alloc((void**)&g->ibcoef32, (size_t)d * bn * g->ibs * 4, "IB coefs"));
      hipLaunchKernelGGL(k_ib_gather<float>, dim3(nblocks(g->n_ib, 256)), dim3(256), 0, s, g->ib,
                         g->n_ib, g->nbase, g->ncoef32, g->ms, d * bn, g->ibs,
                         want64 ? (int32_t*)nullptr : g->ibbase, g->ibcoef32);
    }
    PC_HIP_CHECK(hipGetLastError());
  }
  PC_HIP_CHECK(hipStreamSynchronize(s));
  g->bytes = geom_bytes_for(d, G, M, k_grid, bn, g->n_ib, g->n_near, g->near_w, want64, want32,
                            k_self, g->n_v);
  return PC_OK;
}

}  // namespace
}  // namespace pc

using namespace pc;

extern "C" {

int pc_wls_build(const pc_plan* P, const double* xyz, const uint8_t* kind, int64_t M,
                 const pc_wls_opts* opts, void* stream, pc_geom** out) {
  if (!P || !xyz || !kind || !out) return fail(PC_ERR_INVALID_ARG, "pc_wls_build: null argument");
  *out = nullptr;
  if (M <= 0) return fail(PC_ERR_INVALID_ARG, "M must be positive");
  if (!aligned16(xyz)) return fail(PC_ERR_ALIGN, "positions must be 16-byte aligned");
  const int order = opts ? opts->order : PC_ORDER_CALLER;
  if (order != PC_ORDER_CALLER && order != PC_ORDER_CELL)
    return fail(PC_ERR_INVALID_ARG, "order must be PC_ORDER_CALLER or PC_ORDER_CELL");
  if (M > INT32_MAX - 1) return fail(PC_ERR_UNSUPPORTED_SIZE, "more than 2^31-2 nodes");
  pc_geom* g = new pc_geom();
  std::memset(g, 0, sizeof(*g));
  (void)hipGetDevice(&g->device);
  g->order = order;
  int rc = order == PC_ORDER_CELL ? build_cell_order(P, xyz, kind, M, opts, as_stream(stream), g)
                                  : build(P, xyz, kind, M, opts, as_stream(stream), g);
  if (rc != PC_OK) {
    std::string keep;
    {
      char buf[1024];
      pc_last_error(buf, sizeof(buf));
      keep = buf;
    }
    (void)hipStreamSynchronize(as_stream(stream));
    geom_free(g);
    delete g;
    set_error(keep);
    return rc;
  }
  *out = g;
  return PC_OK;
}

int pc_geom_destroy(pc_geom* g) {
  if (!g) return PC_OK;
  if (g->own_ws) pc_workspace_destroy(g->own_ws);
  geom_free(g);
  delete g;
  return PC_OK;
}

int pc_geom_info(const pc_geom* g, int64_t* c) {
  if (!g || !c) return fail(PC_ERR_INVALID_ARG, "pc_geom_info: null argument");
  c[0] = g->M;
  c[1] = g->n_ib;
  c[2] = g->n_near;
  c[3] = g->k_grid;
  c[4] = g->bn;
  c[5] = g->bytes;
  c[6] = g->n_near_entries;
  c[7] = g->near_w;
  return PC_OK;
}

int pc_geom_export_self(const pc_geom* g, int32_t* idx, double* coef, void* stream) {
  if (!g) return fail(PC_ERR_INVALID_ARG, "pc_geom_export_self: null geometry");
  if (!g->k_self) return fail(PC_ERR_INVALID_ARG, "the geometry has no node-to-node stencils");
  if (coef && !g->has64)
    return fail(PC_ERR_INVALID_ARG, "the geometry holds float32 stencils only");
  hipStream_t s = as_stream(stream);
  if (idx)
    PC_HIP_CHECK(hipMemcpy2DAsync(idx, (size_t)g->M * 4, g->sidx, (size_t)g->ms * 4,
                                  (size_t)g->M * 4, (size_t)g->k_self, hipMemcpyDeviceToDevice,
                                  s));
  if (coef)
    PC_HIP_CHECK(hipMemcpy2DAsync(coef, (size_t)g->M * 8, g->scoef, (size_t)g->ms * 8,
                                  (size_t)g->M * 8, (size_t)(g->d + 1) * g->k_self,
                                  hipMemcpyDeviceToDevice, s));
  return PC_OK;
}

int pc_geom_export(const pc_geom* g, int32_t* gidx, double* gcoef, int32_t* nbase,
                   double* ncoef, int32_t* ib, int32_t* near, void* stream) {
  if (!g) return fail(PC_ERR_INVALID_ARG, "pc_geom_export: null geometry");
  if ((gcoef || ncoef) && !g->has64)
    return fail(PC_ERR_INVALID_ARG, "the geometry holds float32 stencils only");
  hipStream_t s = as_stream(stream);
  auto cp = [&](void* dst, const void* src, size_t bytes) -> int {
    if (dst && src && bytes)
      PC_HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
    return PC_OK;
  };
  PC_TRY(cp(gidx, g->gidx, (size_t)g->k_grid * g->G * 4));
  PC_TRY(cp(gcoef, g->gcoef, (size_t)g->d * g->k_grid * g->G * 8));
  if (nbase && g->M) {
    hipLaunchKernelGGL(k_base_export, dim3(nblocks(g->M, 256)), dim3(256), 0, s, g->nbase, g->M,
                       nbase);
    PC_HIP_CHECK(hipGetLastError());
  }
  if (ncoef && g->M)
    PC_HIP_CHECK(hipMemcpy2DAsync(ncoef, (size_t)g->M * 8, g->ncoef, (size_t)g->ms * 8,
                                  (size_t)g->M * 8, (size_t)g->d * g->bn,
                                  hipMemcpyDeviceToDevice, s));
  PC_TRY(cp(ib, g->ib, (size_t)g->n_ib * 4));
  PC_TRY(cp(near, g->near, (size_t)g->n_near * 4));
  return PC_OK;
}

int pc_geom_footprint(const pc_plan* P, int64_t M, int64_t n_ib, int64_t n_near,
                      const pc_wls_opts* o, int64_t* geom_bytes, int64_t* build_peak_bytes,
                      int64_t* ws_bytes) {
  if (!P) return fail(PC_ERR_INVALID_ARG, "pc_geom_footprint: null plan");
  if (M <= 0 || n_ib < 0 || n_ib > M || n_near < 0 || n_near > P->G)
    return fail(PC_ERR_INVALID_ARG, "pc_geom_footprint: counts out of range");
  const int d = P->d;
  const int k_grid = o && o->k_grid ? o->k_grid : 16;
  const int k_node = o && o->k_node ? o->k_node : (d == 2 ? 16 : 27);
  bool want64 = true, want32 = false;
  PC_TRY(dtype_keep(o, &want64, &want32));
  const int k_self = o ? o->k_self : 0;
  const bool cell = o && o->order == PC_ORDER_CELL;
  int m = 1;
  while ((int)std::pow(m, d) < k_node) ++m;
  if (m < 3) m = 3;
  int bn = 1;
  for (int a = 0; a < d; ++a) bn *= m;
  // the near table is as wide as the most B+V entries of a near point: at
  // most k_grid, rounded up to the kernel's widths
  const int near_w = k_grid <= 8 ? 8 : (k_grid <= 16 ? 16 : (k_grid <= 27 && d == 3 ? 27 : 32));
  const int64_t gb = geom_bytes_for(d, P->G, M, k_grid, bn, n_ib, n_near, near_w, want64, want32,
                                    k_self, n_ib) + (cell ? M * 4 : 0);
  if (geom_bytes) *geom_bytes = gb;
  if (build_peak_bytes) *build_peak_bytes = gb + build_scratch_bytes(d, P->G, M, cell);
  if (ws_bytes) {
    const int modes[3] = {PC_F64, PC_F32, PC_MIXED};
    for (int i = 0; i < 3; ++i) ws_bytes[i] = workspace_bytes_for(P, true, n_ib, n_near, modes[i]);
  }
  return PC_OK;
}

int pc_geom_permutation(const pc_geom* g, int32_t* perm, void* stream) {
  if (!g || !perm) return fail(PC_ERR_INVALID_ARG, "pc_geom_permutation: null argument");
  hipStream_t s = as_stream(stream);
  if (g->perm)
    PC_HIP_CHECK(hipMemcpyAsync(perm, g->perm, (size_t)g->M * 4, hipMemcpyDeviceToDevice, s));
  else
    hipLaunchKernelGGL(k_iota, dim3(nblocks(g->M, 256)), dim3(256), 0, s, perm, g->M);
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

int pc_geom_permute(const pc_geom* g, int dtype, int ncomp, int to_internal, const void* src,
                    void* dst, void* stream) {
  if (!g || !src || !dst) return fail(PC_ERR_INVALID_ARG, "pc_geom_permute: null argument");
  if (dtype != PC_F64 && dtype != PC_F32) return fail(PC_ERR_INVALID_ARG, "dtype");
  if (ncomp < 1 || ncomp > 64) return fail(PC_ERR_INVALID_ARG, "ncomp must be in [1, 64]");
  if (src == dst) return fail(PC_ERR_INVALID_ARG, "pc_geom_permute: src and dst must differ");
  hipStream_t s = as_stream(stream);
  const size_t es = dtype == PC_F64 ? 8 : 4;
  if (!g->perm) {
    PC_HIP_CHECK(hipMemcpyAsync(dst, src, (size_t)ncomp * g->M * es, hipMemcpyDeviceToDevice, s));
    return PC_OK;
  }
  const int ti = to_internal ? 1 : 0;
  if (dtype == PC_F64)
    hipLaunchKernelGGL(k_permute<double>, dim3(nblocks(g->M, 256)), dim3(256), 0, s, g->perm, g->M,
                       ncomp, ti, (const double*)src, (double*)dst);
  else
    hipLaunchKernelGGL(k_permute<float>, dim3(nblocks(g->M, 256)), dim3(256), 0, s, g->perm, g->M,
                       ncomp, ti, (const float*)src, (float*)dst);
  PC_HIP_CHECK(hipGetLastError());
  return PC_OK;
}

int pc_geom_export_at(const pc_geom* g, const int64_t* grid_pts, int64_t n_grid,
                      int32_t* grid_idx, double* grid_coef, const int64_t* nodes, int64_t n_nodes,
                      int32_t* node_base, double* node_coef, void* stream) {
  if (!g) return fail(PC_ERR_INVALID_ARG, "pc_geom_export_at: null geometry");
  if (n_grid < 0 || n_nodes < 0 || (n_grid && !grid_pts) || (n_nodes && !nodes))
    return fail(PC_ERR_INVALID_ARG, "pc_geom_export_at: bad target list");
  if ((grid_coef || node_coef) && !g->has64)
    return fail(PC_ERR_INVALID_ARG, "the geometry holds float32 stencils only");
  const int64_t n = std::max(n_grid, n_nodes);
  if (n == 0) return PC_OK;
  hipStream_t s = as_stream(stream);
  Scratch tmp;
  int32_t* bad;
  PC_TRY(tmp.alloc((void**)&bad, 256, "flags"));
  PC_TRY(fill_zero(bad, 256, s));
  hipLaunchKernelGGL(k_export_at, dim3(nblocks(n, 256)), dim3(256), 0, s, g->gidx, g->gcoef, g->G,
                     g->k_grid, g->d, grid_pts, n_grid, grid_idx, grid_coef, g->nbase, g->ncoef,
                     g->M, g->ms, g->bn, nodes, n_nodes, node_base, node_coef, bad);
  PC_HIP_CHECK(hipGetLastError());
  int32_t hbad = 0;
  PC_HIP_CHECK(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s));
  PC_HIP_CHECK(hipStreamSynchronize(s));
  if (hbad) return fail(PC_ERR_INVALID_ARG, "pc_geom_export_at: target index out of range");
  return PC_OK;
}

}  // extern "C"
