/*
 * pcorr.h -- C ABI of the MI355X hybrid pressure-correction library.
 *
 * The library implements the pressure-correction sub-step of the hybrid
 * projection method of J. Fang, "A fast hybrid pressure-correction algorithm
 * for simulating incompressible flows by projection methods" (arXiv
 * 2304.14690), Sec. 2.2-2.3:
 *
 *   u^{n+1} = u* - (3/2) dt grad p + dt f~                  (Eq. 18)
 *   f~      = -u* / dt + (3/2) grad p  on boundary/virtual points, 0 elsewhere
 *                                                           (Eq. 19)
 *   lap p   = (2/(3 dt)) div u* + (2/3) div f~              (Eq. 20)
 *
 * solved on a uniform cell-centred pressure grid covering an extended box,
 * with the divergence and the gradient carried between the scattered
 * velocity points ("nodes") and the grid by second-order weighted least
 * squares (Sec. 2.2, Eqs. 9-17), the Poisson equation solved directly by
 * transforms (Sec. 2.3, the three-step transform algorithm: cosine
 * transforms for the homogeneous Neumann condition of Eq. 7, real Fourier
 * transforms along periodic axes), and the immersed-boundary force found by
 * the fixed-point iteration of Sec. 2.3.  Options cover the solver
 * variants Sec. 3 reports as interchangeable (pseudo-spectral eigenvalues,
 * the regular vertex grid with the DCT-I), grid sizes that are not powers
 * of two, and the first fractional step (Eq. 3) for whole time steps.
 *
 * Internally the library works with phi = (3 dt / 2) p and g = dt f~, for
 * which Eqs. 18-20 read u^{n+1} = u* - grad phi + g, lap phi = div(u* + g),
 * g = -u* + grad phi on boundary and virtual points.
 *
 * Conventions shared by every entry point
 *   - Every call returns an int status: PC_OK (0), a negative PC_ERR_* code,
 *     or a positive PC_WARN_* code.  pc_last_error() gives a thread-local
 *     message for the last failing call of the calling thread.  No C++
 *     exception crosses the ABI.
 *   - Pointers named *_dev are device pointers (HBM of the current HIP
 *     device), at least 16-byte aligned; the caller owns them and the library
 *     never frees them.  Host structs (opts, stats) are read or written
 *     during the call only.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls only
 *     enqueue work on it, except where a call says it synchronises.
 *   - Node fields are structure-of-arrays [d][M] (component a of node n at
 *     a*M + n).  Grid fields are [G] with G = n0*n1(*n2), x fastest: cell
 *     (i, j, k) at i + n0*(j + n1*k), centred at ((i+1/2) h0, (j+1/2) h1,
 *     (k+1/2) h2); the box is [0, n0 h0] x [0, n1 h1] (x [0, n2 h2]).
 *   - Node kinds: PC_KIND_F (velocity point), PC_KIND_B (boundary point on
 *     the obstacle surface), PC_KIND_V (virtual point inside the obstacle).
 *     The provisional velocity at virtual points must be zero (Sec. 2.3:
 *     the frozen fluid inside the immersed boundary).
 *   - The library-owned handles (pc_plan, pc_geom, pc_workspace) hold device
 *     memory on the device that was current at creation; use them with that
 *     device current.  Handles are not thread-safe; calls that share a
 *     workspace must not overlap.
 */
#ifndef PCORR_H
#define PCORR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PC_OK 0
#define PC_WARN_IB_NOT_CONVERGED 1   /* max_it reached before the criterion */
#define PC_ERR_INVALID_ARG (-1)      /* null pointer, bad enum, k too small  */
#define PC_ERR_UNSUPPORTED_SIZE (-2) /* n odd or outside [8, 4096], d not 2  */
                                     /* or 3, k above the maximum            */
#define PC_ERR_ALIGN (-3)            /* device pointer not 16-byte aligned   */
#define PC_ERR_OOM (-4)              /* device allocation failed             */
#define PC_ERR_SINGULAR_STENCIL (-5) /* a WLS normal matrix is singular      */
#define PC_ERR_HIP (-6)              /* a HIP runtime call failed            */
#define PC_ERR_NO_DEVICE (-7)        /* no HIP device is visible             */

/* ---- precision modes ---------------------------------------------------- */
#define PC_F64 1   /* all arithmetic and storage in float64                  */
#define PC_F32 2   /* fields, stencils and transforms in float32             */
#define PC_MIXED 3 /* float64 fields and transfers; transforms in float32    */
                   /* followed by float64 defect-correction sweeps          */

/* ---- subsets ------------------------------------------------------------ */
#define PC_ALL 0
#define PC_NEAR_IB 1 /* grid points whose stencil holds a B or V node        */
#define PC_IB 2      /* boundary and virtual nodes, in ascending node order  */

/* ---- boundary condition of a grid axis ------------------------------------ */
#define PC_BC_NEUMANN 0  /* homogeneous Neumann on both faces (Eq. 7)        */
#define PC_BC_PERIODIC 1 /* periodic (the lateral condition of the paper's   */
                         /* verification cases, Sec. 3)                     */

/* ---- eigenvalues of the Poisson solve --------------------------------------- */
#define PC_EIG_FD2 0      /* central differences (the variant of the paper's   */
                          /* timings, Sec. 3.2)                                */
#define PC_EIG_SPECTRAL 1 /* pseudo-spectral: minus the squared wavenumber of  */
                          /* each mode (a variant Sec. 3 reports as giving no  */
                          /* noticeable difference)                            */

/* ---- placement of the pressure grid points ---------------------------------- */
#define PC_GRID_CELL 0   /* cell centres (i + 1/2) h: the staggered grid of the */
                         /* paper's timings (Sec. 3.2)                         */
#define PC_GRID_VERTEX 1 /* vertices i h of n - 1 intervals: the regular grid, */
                         /* a variant Sec. 3 reports as interchangeable        */

#define PC_KIND_F 0
#define PC_KIND_B 1
#define PC_KIND_V 2

#define PC_MAX_K_GRID 32 /* largest grid-point stencil                      */
#define PC_MAX_K_NODE 64 /* largest node stencil block (m^d)                */

typedef struct pc_plan pc_plan;           /* grid + transform tables         */
typedef struct pc_geom pc_geom;           /* WLS stencils of one node cloud  */
typedef struct pc_workspace pc_workspace; /* scratch of one in-flight solve  */

/* Options of pc_wls_build (Sec. 2.2).  Zero fields take the default. */
typedef struct pc_wls_opts {
  int32_t k_grid;    /* nodes per grid-point stencil (default 16)           */
  int32_t k_node;    /* grid points per node stencil (default 16 in 2D,     */
                     /* 27 in 3D)                                           */
  double eps;        /* Gaussian shape parameter of Eq. 17 (default 6.3)    */
  double support;    /* support radius in mean spacings (default 3)         */
  double delta;      /* mean point spacing (default: the grid spacing, or   */
                     /* the geometric mean of the per-axis spacings)        */
  int32_t dtype_mask;/* stencil precisions to keep: bit (1 << PC_F64)       */
                     /* float64 (PC_F64 and PC_MIXED), bit (1 << PC_F32)    */
                     /* float32 (PC_F32); 0 = float64 only.  A float32-only */
                     /* geometry (1 << PC_F32) holds half the coefficient   */
                     /* bytes (the 512^3 case of Sec. 3 fits only so in     */
                     /* float32) and refuses float64 calls and coefficient  */
                     /* exports with PC_ERR_INVALID_ARG; other bits: the    */
                     /* same error                                          */
  int32_t k_self;    /* > 0: also build node-to-node stencils of k_self     */
                     /* other nodes for the first fractional step           */
                     /* (pc_momentum_predict); 0 = none                    */
  int32_t order;     /* PC_ORDER_CALLER (default) or PC_ORDER_CELL: the     */
                     /* order of the node fields of this geometry           */
} pc_wls_opts;

/* pc_wls_opts.order.  The nodes may be given in any order (Sec. 2.2: the
 * points can be distributed arbitrarily), but the transfers gather node
 * values per grid point and grid values per node, and they stay near
 * contiguous only if nodes close in space are close in index.
 *   PC_ORDER_CALLER  node fields are in the caller's order (right when the
 *                    caller's order is already spatially coherent, such as a
 *                    lattice order);
 *   PC_ORDER_CELL    the library sorts the nodes by pressure-grid cell (cells
 *                    x fastest; within a cell by x, then y, then z, then the
 *                    caller's index, so the order depends only on the point
 *                    set) and every node field of the geometry -- u, u_out,
 *                    the IB force and lists, the momentum fields, exported
 *                    node stencils -- is in that internal order.
 *                    pc_geom_permutation gives the order, pc_geom_permute
 *                    moves fields between the two orders.
 * The k nearest nodes are chosen by (d^2, node index) in the geometry's own
 * order: with PC_ORDER_CELL the stencils, and so the results bit for bit,
 * depend only on the point set, not on the caller's numbering.  Where two
 * candidates lie exactly equally far (points on an obstacle face that runs
 * along a grid line, for one), the two orders may choose different, equally
 * valid stencils. */
#define PC_ORDER_CALLER 0
#define PC_ORDER_CELL 1

/* Options of the IB-force iteration (Sec. 2.3). */
typedef struct pc_ib_opts {
  double tol;        /* criterion tolerance (default 1e-3)                  */
  int32_t max_it;    /* iteration cap (default 50)                          */
  int32_t fixed_it;  /* > 0: run exactly this many iterations               */
  int32_t sweeps;    /* PC_MIXED defect-correction sweeps per IB iteration  */
                     /* (default 2): the first iteration corrects a        */
                     /* float32 solve, later ones start from the previous  */
                     /* iteration's pressure (its right-hand side differs  */
                     /* only near the IB), the first of their sweeps on    */
                     /* that change; mean(p) is removed at the end         */
  int32_t gauge;     /* 0: zero-mean pressure; 1: zero at the first cell    */
  int32_t flags;     /* PC_IB_* bits below                                  */
} pc_ib_opts;

/* pc_ib_opts.flags: transform every grid line in every IB iteration.  By
 * default (PC_F64, PC_F32, cell-centred grids) iterations after the first
 * redo the forward transforms only on the grid lines that hold near-IB
 * points (the only ones whose right-hand side changes, Sec. 2.3) and run
 * the inverse transforms only on the lines the B+V gradient reads; the
 * remaining lines are completed after the last iteration.  The results are
 * identical bit for bit; this flag exists to show that.  PC_MIXED: by
 * default the first correction sweep of each iteration after the first
 * solves the change of the right-hand side (transformed forward on those
 * lines only) instead of the whole residual; with the flag every sweep
 * takes the whole residual (the results agree within the mode's
 * tolerance, not bit for bit). */
#define PC_IB_FULL_TRANSFORMS 1

typedef struct pc_stats {
  int32_t n_it;      /* IB iterations run                                   */
  int32_t converged; /* 1 if the criterion was met                          */
  double bmean;      /* mean of the last right-hand side (removed; the      */
                     /* compatibility defect of the Neumann problem)        */
  double ib_num;     /* last criterion numerator  sum (|g|-|g_old|)^2       */
  double ib_den;     /* last criterion denominator sum |g_old|^2            */
} pc_stats;

/* ---- library ------------------------------------------------------------ */

/* ABI version (major*100 + minor): 115. */
int pc_version(void);

/* Copies the calling thread's last error message into buf (NUL-terminated,
 * truncated to n bytes).  Returns the message length. */
int pc_last_error(char* buf, size_t n);

/* Device memory of the library.  By default plans, geometries, workspaces
 * and the scratch of a call take their device memory from hipMalloc and
 * return it with hipFree.  A caller that accounts device memory itself (a
 * serving loop's admission, a framework's caching allocator) installs its
 * own pair: alloc(user, bytes, &ptr) returns 0 and a device pointer aligned
 * to at least 256 bytes, or nonzero when it cannot (the library call then
 * fails with PC_ERR_OOM); free(user, ptr) takes back a pointer that alloc
 * returned.  Both are called on the calling thread, from inside library
 * calls, with the current device unchanged.  A call may free its scratch
 * while work it queued on its stream still uses it: the pair must order
 * reuse after that stream's work (as a caching allocator bound to the same
 * stream does) or wait for it.  (NULL, NULL) restores
 * hipMalloc/hipFree.  Every allocation is returned to whoever gave it out:
 * objects created before a pair was installed go back to hipFree, objects
 * created through a pair go back to that pair's free.  The pair can be
 * replaced only while no allocation made through it is outstanding (every
 * object created with it destroyed): otherwise PC_ERR_INVALID_ARG.  Pinned
 * host memory (the convergence flags of a workspace) still comes from
 * hipHostMalloc. */
typedef int (*pc_alloc_fn)(void* user, size_t bytes, void** ptr);
typedef void (*pc_free_fn)(void* user, void* ptr);
int pc_set_allocator(pc_alloc_fn alloc, pc_free_fn free_fn, void* user);

/* ---- plan: grid and transform tables ------------------------------------ */

/* Creates the plan of a d-dimensional cell-centred grid with n[a] cells of
 * spacing h[a] per axis (Sec. 2.3, Fig. 1: the uniform pressure grid over
 * the extended rectangle).  Builds, in float64 on the host, the twiddle
 * tables of the cosine transforms and the 1D eigenvalues
 * -(4/h_a^2) sin^2(pi k / (2 n_a)) of the mirror-ghost central-difference
 * Laplacian (homogeneous Neumann condition, Eq. 7), and uploads them (plus
 * float32 copies).  n[a] must be even and in [8, 4096], and the grid may
 * hold at most 2^31 - 2 points (flat grid indices are int32; larger grids
 * give PC_ERR_UNSUPPORTED_SIZE).  Powers of two of
 * at least 32 take the register-resident transform kernels; other lengths
 * (such as the 400 x 402 and 280 x 480 grids of Sec. 3) take a mixed-radix
 * kernel staged in LDS whose cost per line grows with the sum of the prime
 * factors of n/2, and the IB iteration then transforms every line.
 * Synchronises `stream`.  Release with pc_plan_destroy. */
int pc_plan_create(int d, const int32_t* n, const double* h, void* stream, pc_plan** out);

/* pc_plan_create with a boundary condition per axis, a choice of eigenvalues
 * and of grid-point placement.
 *   bc[a] = PC_BC_NEUMANN or PC_BC_PERIODIC (bc NULL: Neumann everywhere).
 *     A periodic axis of n cells (n even, in [8, 4096]) joins cell n-1 to
 *     cell 0 (the 400 x 400 doubly periodic grid of Sec. 3, or a periodic
 *     axis beside a Neumann one); its transform is the real DFT, packed into
 *     n reals (slot k: Re X_k, slot n-k: Im X_k, slot n/2: X_{n/2}), and
 *     its central-difference eigenvalues are -(4/h_a^2) sin^2(pi k / n_a),
 *     those of the wrap-around 3-point Laplacian.  Every entry point that
 *     takes the plan follows its axes' conditions: the solve, and the WLS
 *     stencils of pc_wls_build (a periodic axis wraps node positions and
 *     neighbourhoods around the box).
 *   eig = PC_EIG_FD2 (the eigenvalues above and in pc_plan_create) or
 *     PC_EIG_SPECTRAL: -(pi k / L_a)^2 for cosine mode k of a Neumann axis,
 *     -(2 pi m / L_a)^2 for Fourier mode m of a periodic axis (L_a = n_a h_a).
 *     PC_MIXED needs PC_EIG_FD2 (its defect correction evaluates the
 *     3-point Laplacian); with PC_EIG_SPECTRAL it returns
 *     PC_ERR_INVALID_ARG.
 *   grid = PC_GRID_CELL (points at (i + 1/2) h, box [0, n h]) or
 *     PC_GRID_VERTEX (points at i h, box [0, (n - 1) h], n in [9, 2049],
 *     Neumann axes only): the homogeneous Neumann condition mirrors about
 *     the end vertex (phi_{-1} = phi_1), the transform is the DCT-I (the real
 *     DFT of the even extension, on the mixed-radix kernel) and the
 *     eigenvalues are -(4/h^2) sin^2(pi k / (2(n - 1))) (pseudo-spectral:
 *     -(pi k / ((n - 1) h))^2).  The operator is symmetric in the trapezoid
 *     weights (1/2 at the end points of each axis): bmean is the weighted
 *     mean and phi has zero weighted mean; PC_MIXED evaluates its float64
 *     residual with the same mirror and removes weighted means.  The WLS
 *     stencils of pc_wls_build use the same placement. */
int pc_plan_create_ex(int d, const int32_t* n, const double* h, const int32_t* bc, int32_t eig,
                      int32_t grid, void* stream, pc_plan** out);
int pc_plan_destroy(pc_plan* plan);

/* ---- the Poisson solve ---------------------------------------------------- */

/* Solves lap_h phi = b - mean(b) with mean(phi) = 0 on the plan's grid
 * (Sec. 2.3: forward transforms along each axis, division by the sum of the
 * 1D eigenvalues, backward transforms; the zero mode is dropped and the
 * compatibility defect mean(b) removed; on a vertex grid both means are
 * weighted by the trapezoid rule).
 *   mode PC_F64:   b_dev, phi_dev float64 [G].
 *   mode PC_F32:   b_dev, phi_dev float32 [G].
 *   mode PC_MIXED: b_dev, phi_dev float64 [G]; transforms in float32 with
 *                  `sweeps` float64 defect-correction sweeps
 *                  r = b - mean(b) - lap_h phi, phi += solve32(r).
 * b_dev and phi_dev may alias (in place) in PC_F64 and PC_F32, not in
 * PC_MIXED (the residual re-reads b).  bmean_dev (nullable) receives
 * mean(b) as one float64.  ws: a workspace of this plan (nullable: the
 * plan's own, which makes concurrent calls on the plan race). */
int pc_poisson_fft_solve(const pc_plan* plan, int mode, const void* b_dev, void* phi_dev,
                         int sweeps, double* bmean_dev, pc_workspace* ws, void* stream);

/* ---- WLS stencils --------------------------------------------------------- */

/* Builds the WLS stencils of one node cloud (Sec. 2.2; computed once per
 * geometry, last paragraph of Sec. 2.2):
 *   - every grid point takes its k_grid nearest nodes (key (d^2, node
 *     index), d^2 = ((dx*dx) + dy*dy) + dz*dz rounded term by term);
 *   - every node takes the k_node nearest grid points (same key, flat grid
 *     index) inside the block of the m = ceil(k_node^(1/d)) grid lines
 *     nearest to it along each axis, clamped inside the box (along a
 *     periodic axis the block wraps around; grid lines sit at the cell
 *     centres or, on a vertex grid, at i h);
 *   - for each target, the Eq. 16 polynomial vector (10 terms in 3D) in
 *     coordinates scaled by the support radius h_t = max(support*delta,
 *     r_k), the Eq. 17 weights exp(-eps r^2/h_t^2), C = sum w q q^T
 *     (Eq. 14) and the first-derivative rows of C^-1 A (Eq. 13);
 *   - the lists of boundary/virtual nodes and of grid points near them.
 * xyz_dev: float64 [d][M] node positions; kind_dev: uint8 [M].
 * Synchronises `stream`.  Returns PC_ERR_SINGULAR_STENCIL if any normal
 * matrix has a squared pivot ratio below 1e-12 (e.g. collinear nodes).
 * Release with pc_geom_destroy. */
int pc_wls_build(const pc_plan* plan, const double* xyz_dev, const uint8_t* kind_dev, int64_t M,
                 const pc_wls_opts* opts, void* stream, pc_geom** out);
int pc_geom_destroy(pc_geom* geom);

/* Sizes of a geometry: counts[0] = M, [1] = number of B+V nodes, [2] =
 * number of near-IB grid points, [3] = k_grid, [4] = k_node block size
 * m^d, [5] = device bytes held by the geometry, [6] = number of B+V entries
 * over all near-IB stencils, [7] = width of the near-IB table (8, 16, 27
 * (3D only) or 32).  counts8 holds 8 values. */
int pc_geom_info(const pc_geom* geom, int64_t* counts8);

/* Copies the stencils out (for inspection and tests).
 *   grid_idx_dev  int32   [k_grid][G]      node index (the selection is by
 *                                          (d^2, idx)); entries ordered by
 *                                          the node's offset from the grid
 *                                          point in whole grid spacings
 *                                          (rounded per axis, clamped to
 *                                          [-4, 4]): shortest first, then by
 *                                          its (z, y, x) components, then by
 *                                          node index
 *   grid_coef_dev float64 [d][k_grid][G]   derivative coefficients
 *   node_base_dev int32   [M]              flat grid index of the block's
 *                                          low corner (entries past a
 *                                          periodic face wrap around)
 *   node_coef_dev float64 [d][m^d][M]      coefficients in block order
 *                                          (x fastest); 0 for block points
 *                                          outside the k_node selection
 *   ib_dev        int32   [n_ib]           boundary+virtual node indices
 *   near_dev      int32   [n_near]         near-IB grid points
 * Any pointer may be NULL. */
int pc_geom_export(const pc_geom* geom, int32_t* grid_idx_dev, double* grid_coef_dev,
                   int32_t* node_base_dev, double* node_coef_dev, int32_t* ib_dev,
                   int32_t* near_dev, void* stream);

/* Device memory a geometry would take, before it is built (for admission
 * by memory, as a serving loop needs it): for M nodes of which n_ib are
 * boundary/virtual points, with at most n_near near-IB grid points (the
 * grid points whose stencil holds a B/V node, known exactly only after the
 * build: pass a bound), and the options of pc_wls_build:
 *   geom_bytes       the arrays the geometry keeps (pc_geom_info counts[5]
 *                    after the build, when n_near is exact), an upper bound;
 *   build_peak_bytes geom_bytes plus the scratch pc_wls_build holds at most
 *                    at once (cell lists, flags);
 *   ws_bytes[3]      pc_workspace_bytes of a workspace for PC_F64, PC_F32,
 *                    PC_MIXED on that geometry.
 * Any output pointer may be NULL.  Host only. */
int pc_geom_footprint(const pc_plan* plan, int64_t M, int64_t n_ib, int64_t n_near,
                      const pc_wls_opts* opts, int64_t* geom_bytes, int64_t* build_peak_bytes,
                      int64_t* ws_bytes);

/* The internal node order: perm_dev int32 [M], internal node i is the
 * caller's node perm_dev[i] (the identity for PC_ORDER_CALLER). */
int pc_geom_permutation(const pc_geom* geom, int32_t* perm_dev, void* stream);

/* Moves ncomp node fields [ncomp][M] (dtype PC_F64 or PC_F32) between the
 * caller's order and the geometry's internal order: to_internal != 0 gives
 * dst[c][i] = src[c][perm[i]], to_internal == 0 the inverse.  src and dst
 * must not alias (a plain copy for PC_ORDER_CALLER). */
int pc_geom_permute(const pc_geom* geom, int dtype, int ncomp, int to_internal,
                    const void* src_dev, void* dst_dev, void* stream);

/* The stencils of selected targets (for inspection and tests where a whole
 * export does not fit in device memory, such as 512^3 grids):
 *   grid_pts_dev  int64   [n_grid]            flat grid indices
 *   grid_idx_dev  int32   [k_grid][n_grid]    as in pc_geom_export, per target
 *   grid_coef_dev float64 [d][k_grid][n_grid]
 *   nodes_dev     int64   [n_nodes]           node indices
 *   node_base_dev int32   [n_nodes]
 *   node_coef_dev float64 [d][m^d][n_nodes]
 * Output pointers may be NULL.  Synchronises `stream`; an index out of range
 * gives PC_ERR_INVALID_ARG (the other targets are still copied). */
int pc_geom_export_at(const pc_geom* geom, const int64_t* grid_pts_dev, int64_t n_grid,
                      int32_t* grid_idx_dev, double* grid_coef_dev, const int64_t* nodes_dev,
                      int64_t n_nodes, int32_t* node_base_dev, double* node_coef_dev,
                      void* stream);

/* Copies the node-to-node stencils out (geometry built with k_self > 0):
 *   idx_dev  int32   [k_self][M]       neighbour node indices, ascending (the
 *                                      selection is by (d^2, idx), the node
 *                                      itself excluded)
 *   coef_dev float64 [d+1][k_self][M]  rows d_x, d_y(, d_z) and the Laplacian,
 *                                      applied to f(x_i) - f(x)
 * Either pointer may be NULL. */
int pc_geom_export_self(const pc_geom* geom, int32_t* idx_dev, double* coef_dev, void* stream);

/* ---- right-hand side ------------------------------------------------------ */

/* b = WLS divergence of v at the grid points (Sec. 2.3, Eq. 20 right-hand
 * side, with v = u* + g):  b_p = sum_a sum_i c^a_{p,i} v_a[idx_{p,i}].
 *   subset PC_ALL:     v_dev [d][M], writes b_dev[G].
 *   subset PC_NEAR_IB: v_dev [d][n_ib] holds values at the B+V nodes only
 *                      (zero assumed elsewhere) and the result is ADDED to
 *                      b_dev at the near-IB grid points (Sec. 2.3: after the
 *                      first iteration only these points see the force).
 * dtype PC_F64 or PC_F32 selects float64 or float32 fields and stencils. */
int pc_div_to_grid(const pc_geom* geom, int dtype, const void* v_dev, void* b_dev, int subset,
                   void* stream);

/* ---- gradient transfer ---------------------------------------------------- */

/* grad = WLS gradient of phi at the nodes (Sec. 2.3):
 * grad_a(n) = sum_j c^a_{n,j} phi[src_{n,j}].
 *   subset PC_ALL: grad_dev [d][M];  subset PC_IB: grad_dev [d][n_ib] at the
 *   boundary and virtual nodes in ascending node order. */
int pc_grad_to_nodes(const pc_geom* geom, int dtype, const void* phi_dev, void* grad_dev,
                     int subset, void* stream);

/* ---- one IB-force update -------------------------------------------------- */

/* g_new = -u* + grad at the B+V nodes (Eq. 19 times dt); sums the criterion
 * of Sec. 2.3, num = sum (|g_new| - |g_old|)^2 and den = sum |g_old|^2, into
 * sums_dev[0..1] (float64, deterministic order), sets *conv_dev = 1 if
 * num < tol * den or num == 0 (else 0), and overwrites g_dev with g_new.
 * u_dev [d][M] (dtype); grad_ib_dev, g_dev [d][n_ib] (dtype).  Allocates
 * its own device scratch and synchronises `stream` before freeing it
 * (pc_pressure_correct runs the same step without either). */
int pc_ib_update(const pc_geom* geom, int dtype, const void* u_dev, const void* grad_ib_dev,
                 void* g_dev, double tol, double* sums_dev, int32_t* conv_dev, void* stream);

/* pc_ib_update without device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same update with its scratch (the partial sums and u* at
 * the B+V nodes) in a static device array of PC_NOALLOC_SCRATCH_BYTES that
 * each device holds until the process ends, and without synchronising
 * `stream`.  Geometries with more than PC_NOALLOC_MAX_IB boundary/virtual
 * nodes in float64 (twice as many in float32, in 2D 3/2 times as many) give
 * PC_ERR_UNSUPPORTED_SIZE.  Every call on a device shares that device's
 * array: calls that overlap on one device (other streams, other threads)
 * race and must be ordered by the caller.  Results equal pc_ib_update's bit
 * for bit. */
#define PC_NOALLOC_SCRATCH_BYTES (64ll << 20)
#define PC_NOALLOC_MAX_IB 2796000 /* 3D float64: (64 MiB - 4352 B) / 24 B */
int pc_ib_update_noalloc(const pc_geom* geom, int dtype, const void* u_dev,
                         const void* grad_ib_dev, void* g_dev, double tol, double* sums_dev,
                         int32_t* conv_dev, void* stream);

/* ---- projection ----------------------------------------------------------- */

/* u_out = u* - grad + g (Eq. 18 with phi, g): u* - grad on velocity points
 * and exactly 0 on boundary and virtual points, where Eq. 19 cancels it.
 * u_dev, grad_dev, u_out_dev [d][M] (dtype).  u_out may alias u. */
int pc_project(const pc_geom* geom, int dtype, const void* u_dev, const void* grad_dev,
               void* u_out_dev, void* stream);

/* ---- the first fractional step (Eq. 3) ------------------------------------- */

/* The intermediate velocity of the second-order Adams-Bashforth step with the
 * pressure gradient dropped from R^n (Eq. 3):
 *   R     = -u_j d_j u + nu lap u + F   at every node, from the node-to-node
 *           stencils of the geometry (pc_wls_opts.k_self > 0: the known-value
 *           WLS form of Sec. 2.2, Eqs. 10-15, over the k_self nearest other
 *           nodes);
 *   u*    = u + dt (3/2 R - 1/2 R_prev), or u + dt R when r_prev_dev is NULL
 *           (the first step); 0 at the virtual points (the frozen fluid of
 *           Sec. 2.3).
 * u_dev, r_prev_dev (nullable), r_dev (out: R) and ustar_dev (out) are
 * [d][M] in dtype (PC_F32 needs a geometry built with float32 stencils).
 * force (host, nullable) is the body force F, d values.  ustar_dev must not
 * alias u_dev; r_dev may alias r_prev_dev.  Pass u* to pc_pressure_correct,
 * then pc_momentum_pressure for the next step's R_prev. */
int pc_momentum_predict(const pc_geom* geom, int dtype, const void* u_dev, const void* r_prev_dev,
                        double dt, double nu, const double* force, void* r_dev, void* ustar_dev,
                        void* stream);

/* R_prev for the next step: R^n - grad p^n at every node (R^{n-1} of Eq. 3
 * includes the pressure gradient), where Eq. 18 gives grad p^n =
 * 2 (u* - u^{n+1} + g) / (3 dt) with g the IB force times dt at the B+V
 * nodes.  r_dev, ustar_dev, unew_dev, r_prev_dev [d][M]; g_ib_dev [d][n_ib]
 * as returned by pc_pressure_correct (nullable: zero); r_prev_dev may alias
 * r_dev. */
int pc_momentum_pressure(const pc_geom* geom, int dtype, const void* r_dev, const void* ustar_dev,
                         const void* unew_dev, const void* g_ib_dev, double dt, void* r_prev_dev,
                         void* stream);

/* ---- the whole sub-step ------------------------------------------------------ */

/* Workspace for pc_pressure_correct / pc_poisson_fft_solve in `mode` on this
 * plan and geometry (geom may be NULL for solve-only use). */
int pc_workspace_create(const pc_plan* plan, const pc_geom* geom, int mode, pc_workspace** out);
int pc_workspace_destroy(pc_workspace* ws);
/* Device bytes a workspace of this mode would hold. */
int64_t pc_workspace_bytes(const pc_plan* plan, const pc_geom* geom, int mode);

/* One pressure-correction sub-step (Sec. 2.3): b_u = div u*; loop { RHS
 * update near the IB; Poisson solve; grad phi at B+V; IB-force update;
 * criterion } ; final grad phi at all nodes and the projection of Eq. 18;
 * p = 2 phi / (3 dt).
 *   mode PC_F64 / PC_MIXED: u_dev, u_out_dev [d][M] and p_dev [G] float64.
 *   mode PC_F32:            the same arrays in float32.
 *   g_inout_dev (nullable) [d][n_ib] in the field dtype: the warm start of
 *   the IB force times dt (Sec. 2.3: taken from the previous time step) and
 *   its final value.  NULL starts from zero.
 *   stats (nullable) is filled after the call synchronises `stream`.
 *   ws: a workspace created for this plan, geometry and mode, or NULL for
 *   the geometry's own (created on first use, replaced when the mode
 *   changes); calls that share a workspace, including the geometry's own,
 *   must not overlap.
 * The host waits once per IB iteration for that iteration's convergence
 * flag (written by the device into pinned host memory) while the next
 * iteration is already queued; a queued iteration after convergence exits
 * at once on a device-side flag.  Not when fixed_it > 0.  u_out_dev must
 * not alias u_dev.  Returns PC_WARN_IB_NOT_CONVERGED when max_it is
 * reached first. */
int pc_pressure_correct(const pc_geom* geom, const pc_plan* plan, int mode, const void* u_dev,
                        double dt, void* u_out_dev, void* p_dev, void* g_inout_dev,
                        const pc_ib_opts* opts, pc_stats* stats, pc_workspace* ws,
                        void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PCORR_H */
