// Internal declarations shared by the HIP translation units of libpcorr.
// Not part of the ABI (see include/pcorr.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "pcorr.h"

namespace pc {

// ---- error handling --------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define PC_HIP_CHECK(expr)                                                       \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      return ::pc::fail(PC_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define PC_TRY(expr)          \
  do {                        \
    int rc_ = (expr);         \
    if (rc_ < 0) return rc_;  \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int dev_alloc(void** p, size_t bytes, const char* what);
void dev_free(void* p);

// ---- device-side small complex --------------------------------------------
template <typename T>
struct cplx {
  T re, im;
};

// ---- per-axis transform tables (device) ------------------------------------
// For an axis of N cells (H = N/2):
//   twH[j]  = exp(-2 pi i j / H),      j = 0..H-1   (half-length FFT)
//   tN[k]   = exp(-2 pi i k / N),      k = 0..H     (real-FFT split)
//   t4N[k]  = exp(-i pi k / (2N)),     k = 0..H     (cosine-transform shift)
//   lam[s]  = the 1D eigenvalue of slot s, s = 0..N-1:
//             -(4 / h^2) sin^2(pi s / (2N))  (Neumann axis, DCT-II index s)
//             -(4 / h^2) sin^2(pi s / N)     (periodic axis: slots s and N-s
//                                             both hold mode s)
//             or, with pseudo-spectral eigenvalues, -(pi s / L)^2 (Neumann)
//             and -(2 pi min(s, N-s) / L)^2 (periodic), L = N h
template <typename T>
struct AxisTables {
  const cplx<T>* twH;
  const cplx<T>* tN;
  const cplx<T>* t4N;
  const T* lam;
};

}  // namespace pc

// ---- opaque handle bodies ----------------------------------------------------
struct pc_plan {
  int d;
  int32_t n[3];
  double h[3];
  int32_t bc[3];  // PC_BC_NEUMANN or PC_BC_PERIODIC per axis
  int32_t eig;    // PC_EIG_FD2 or PC_EIG_SPECTRAL
  int32_t vertex; // 1: grid points at i h (regular grid, DCT-I); 0: cell centres
  int64_t G;
  int device;
  // one allocation per precision holding all axis tables
  void* tab64;
  void* tab32;
  pc::AxisTables<double> ax64[3];
  pc::AxisTables<float> ax32[3];
  pc_workspace* own_ws;  // lazily created default workspace (solve-only)
};

struct pc_geom {
  int d;
  int64_t M, G;
  int32_t n[3];
  double h[3];
  int per;      // bit a set: axis a of the plan was periodic
  int vertex;   // the plan's grid points sit at i h (1) or (i + 1/2) h (0)
  int k_grid;   // stencil size of grid targets
  int k_node;   // selected entries of node stencils
  int m_node;   // block lines per axis; block size bn = m^d
  int bn;
  int64_t n_ib, n_near, n_near_entries;
  int device;
  bool has32;   // float32 stencil copies (PC_F32)
  bool has64;   // float64 stencils (PC_F64, PC_MIXED); a float32-only
                // geometry keeps null float64 coefficient arrays
  // grid-target stencils
  int32_t* gidx;   // [k_grid][G]
  double* gcoef;   // [d][k_grid][G] or null (float32 only)
  float* gcoef32;  // [d][k_grid][G] or null
  // node stencils (block order)
  int32_t* nbase;   // [M] flat index of the block's low corner; ~corner
                    // (negative) for a block that wraps around a periodic axis
  int64_t ms;       // stride of the node coefficient streams: M rounded up
                    // to 64, so that every stream starts on a 512-byte line
  double* ncoef;    // [d][bn][ms]
  float* ncoef32;   // [d][bn][ms] or null
  // IB lists
  int32_t* ib;          // [n_ib] node index
  int32_t* near;        // [n_near] grid index
  // near-IB stencils restricted to their B+V entries, ELL layout of width
  // near_w (8, 16, 27 or 32, at least the most B+V entries of any near
  // point; 27, the 3D stencil of the workloads, only in 3D):
  // entry e of near point q at e*nns + q, slot -1 / coefficient 0 past the
  // point's last entry; nns = n_near rounded up to 64
  int near_w;
  int64_t nns;
  int32_t* nslot;       // [near_w][nns] ib slot
  double* ncoefib;      // [d][near_w][nns]
  float* ncoefib32;
  // compact node stencils of the B+V nodes; ibs = n_ib rounded up to 64
  int64_t ibs;
  int32_t* ibbase;      // [n_ib]
  double* ibcoef;       // [d][bn][ibs]
  float* ibcoef32;
  // node-to-node stencils of the first fractional step (k_self = 0: none):
  // neighbour node sidx [k_self][ms] (ascending), coefficients
  // scoef [d+1][k_self][ms] (d first-derivative rows, then the Laplacian row)
  int k_self;
  int32_t* sidx;
  double* scoef;
  float* scoef32;
  int64_t n_v;       // virtual nodes
  int32_t* vlist;    // [n_v] their indices
  int64_t bytes;
  pc_workspace* own_ws;
  // node order (PC_ORDER_CALLER, PC_ORDER_CELL): with PC_ORDER_CELL every
  // node index above is internal and internal node i is the caller's node
  // perm[i]; null for PC_ORDER_CALLER
  int order;
  int32_t* perm;
};

namespace pc {
// Whether a geometry was built on a plan of this grid (shape, spacing and
// boundary conditions).
inline bool same_grid(const pc_plan* P, const pc_geom* g) {
  if (P->d != g->d || P->G != g->G) return false;
  int per = 0;
  for (int a = 0; a < P->d; ++a) {
    if (P->n[a] != g->n[a] || P->h[a] != g->h[a]) return false;
    if (P->bc[a] == PC_BC_PERIODIC) per |= 1 << a;
  }
  return per == g->per && P->vertex == g->vertex;
}
}  // namespace pc

struct pc_workspace {
  const pc_plan* plan;
  const pc_geom* geom;
  int mode;
  int device;
  int64_t bytes;
  void* block;       // single allocation; the pointers below point into it
  void* b;           // [G] field dtype  (right-hand side)
  void* phi;         // [G] field dtype
  float* w32;        // [G] float32 transform buffer (MIXED)
  void* bnear;       // [n_near] field dtype: b_u at the near points
  void* uib;         // [d][n_ib] field dtype: u* at B+V nodes
  void* gib;         // [d][n_ib] field dtype: IB force (times dt)
  void* gradib;      // [d][n_ib] field dtype
  double* partial;   // reduction partials
  double* part2;     // PC_MIXED: block sums of the near-IB RHS update (mean of b)
  double* scal;      // small float64 scalars: [0] bmean, [1] num, [2] den, [3] mean phi
  int32_t* flag;     // [0] converged flag
  int32_t* hflag;    // pinned host mirror of the flag
  double* hscal;     // pinned host mirror of scal
  int nblk;          // partial-sum blocks
  hipEvent_t ev[2];  // convergence-flag copies of alternate iterations
  // Resident transforms of the IB iteration (F64/F32 with a geometry): the
  // forward transforms of the right-hand side stay in `phi` (first axis) and
  // `w1b` (3D: second axis) between iterations, so later iterations redo
  // only the lines that hold near-IB points, and the inverse transforms run
  // only on the lines the B+V gradient reads until the loop has ended.
  int resident;
  void* w1b;         // [G] field dtype (3D only)
  int32_t* tiles;    // device tile lists, list l at tl[l]
  int32_t* tl[6];
  int ntl[6];
  // PC_MIXED with a geometry: the first correction sweep of every IB
  // iteration after the first solves the change of the right-hand side,
  // which is nonzero only at the near-IB points, through the forward
  // transforms of the lines holding them (tile lists above, float32 tiles).
  int delta;
  double* dgrid;     // [G] b_it - b_(it-1) at the near points, 0 elsewhere
  float* dspec[2];   // [G] forward transforms of dgrid along axis 0 (and 1 in
                     // 3D) on those lines; 0 on every other line
};

namespace pc {
// tile lists of the resident transforms
enum { TL_FWD0 = 0, TL_FWD1, TL_INV1_IB, TL_INV1_REST, TL_INV0_IB, TL_INV0_REST };
}

namespace pc {
// ---- solve (pc_solve.hip) ---------------------------------------------------
// Solves sigma * lap_h x = b - mean(b), mean(x) = 0 (sigma = 1: phi;
// sigma = 3 dt / 2: the pressure itself).
// skip (nullable): device flag; every launch returns at once when it is set
// (used to enqueue IB iterations ahead of the convergence test).
int solve_f64(const pc_plan* P, const double* b, double* phi, double* bmean_dev,
              pc_workspace* ws, hipStream_t s, double sigma = 1.0,
              const int32_t* skip = nullptr);
int solve_f32(const pc_plan* P, const float* b, float* phi, double* bmean_dev,
              pc_workspace* ws, hipStream_t s, double sigma = 1.0,
              const int32_t* skip = nullptr);
// warm: start the sweeps from the phi passed in instead of S32(b);
// remove_mean = false leaves mean(phi) (of the order of the float32 rounding
// of the corrections) for the caller to remove.
int solve_mixed(const pc_plan* P, const double* b, double* phi, int sweeps, double* bmean_dev,
                pc_workspace* ws, hipStream_t s, double sigma = 1.0,
                const int32_t* skip = nullptr, bool warm = false, bool remove_mean = true,
                bool bmean_given = false, bool delta = false);
// Mean of a float64 grid field (trapezoid-weighted on a vertex grid).
int grid_mean_f64(const pc_plan* P, const double* x, double* partial, int nblk, double* out_dev,
                  hipStream_t s, const int32_t* skip = nullptr);
int remove_mean_f64(const pc_plan* P, double* phi, pc_workspace* ws, hipStream_t s,
                    const int32_t* skip = nullptr);
int ensure_plan_ws(const pc_plan* P, pc_workspace** ws);
// Complex values per thread of the register transform of an axis of N
// points: 8 (radix-8 plan, N a power of two from 32 to 4096), 10 (radix-10
// plan, N = 200, 400, 1000 or 2000), 0 (the generic kernel).
int rad_values(int N);
// Lines per workgroup tile of the register transform along `axis` for
// elements of `elem` bytes (0 when the axis uses the generic kernel).
int rad_tile_lines(const pc_plan* P, int axis, size_t elem);
// Tile geometry of a transform pass along an axis: lines per tile C, tiles
// along x tx (strided passes number tile o * tx + i / C), and the tile count.
struct PassTiles {
  int C;
  int64_t tx;
  int64_t ntile;
};
PassTiles pass_tiles(const pc_plan* P, int axis, size_t elem);
// Whether the resident IB-iteration transforms apply to this plan/geometry/mode.
bool resident_ok(const pc_plan* P, const pc_geom* g, int mode);
bool resident_possible(const pc_plan* P, int64_t n_ib, int mode);
// The MIXED counterpart: the change-of-RHS sweep (pc_workspace.delta).
bool delta_possible(const pc_plan* P, int64_t n_ib, int mode);
// Device bytes of a workspace (pc_workspace_bytes) from the geometry's counts.
int64_t workspace_bytes_for(const pc_plan* P, bool geometry, int64_t n_ib, int64_t n_near,
                            int mode);
// Upper bound of the total length of the six tile lists.
int64_t resident_tiles_max(const pc_plan* P, size_t elem);
// Tile lists (host) of the resident transforms: near_pts are the near-IB
// grid points, ib_base the block corners of the B+V node stencils (block
// of m grid lines per axis).
void resident_tiles(const pc_plan* P, size_t elem, const std::vector<int32_t>& near_pts,
                    const std::vector<int32_t>& ib_base, int m, std::vector<int32_t> out[6]);
// One resident solve.  phase 0: first iteration (every line); phase 1: a
// later iteration (forward passes on the near-IB lines only); both leave
// the inverse transforms done only on the lines read by the B+V gradient.
// phase 2: completes the inverse transforms on the remaining lines.
int solve_resident_f64(const pc_plan* P, const double* b, double* p, double* bmean_dev,
                       pc_workspace* ws, hipStream_t s, double sigma, const int32_t* skip,
                       int phase);
int solve_resident_f32(const pc_plan* P, const float* b, float* p, double* bmean_dev,
                       pc_workspace* ws, hipStream_t s, double sigma, const int32_t* skip,
                       int phase);
// deterministic mean of a float64 grid field into out_dev[0]
int mean_f64(const double* x, int64_t n, double* partial, int nblk, double* out_dev,
             hipStream_t s, const int32_t* skip = nullptr);
int fill_zero(void* p, size_t bytes, hipStream_t s);
}  // namespace pc
