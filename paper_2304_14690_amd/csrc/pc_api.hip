// C ABI entry points of libpcorr: errors, plans, workspaces and the Poisson
// solve.  Geometry entry points live in pc_wls.hip, the transfers and the
// whole sub-step in pc_step.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>

#include "pc_internal.h"

namespace pc {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

namespace {
// The caller's allocator (pc_set_allocator), and the owner of every live
// allocation made through an installed pair: each pointer is returned to the
// pair that gave it out, whatever is installed when it is freed, and a
// pointer with no record came from hipMalloc.  A pair cannot be replaced
// while allocations of it are live (its `user` may not outlive the swap).
struct Owner {
  pc_free_fn free_fn;
  void* user;
};
std::mutex g_alloc_mu;
pc_alloc_fn g_alloc = nullptr;
pc_free_fn g_free = nullptr;
void* g_alloc_user = nullptr;
std::unordered_map<void*, Owner> g_owner;
}  // namespace

int dev_alloc(void** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (bytes == 0) return PC_OK;
  pc_alloc_fn fa;
  pc_free_fn ff;
  void* user;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    fa = g_alloc;
    ff = g_free;
    user = g_alloc_user;
  }
  if (fa) {
    if (fa(user, bytes, p) != 0 || !*p) {
      *p = nullptr;
      return fail(PC_ERR_OOM, std::string("the installed allocator failed for ") + what + " (" +
                                  std::to_string(bytes) + " bytes)");
    }
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_owner[*p] = Owner{ff, user};
    return PC_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(PC_ERR_OOM, std::string("hipMalloc failed for ") + what + " (" +
                                std::to_string(bytes) + " bytes): " + hipGetErrorString(e));
  }
  return PC_OK;
}

void dev_free(void* p) {
  if (!p) return;
  Owner o{nullptr, nullptr};
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_owner.find(p);
    if (it != g_owner.end()) {
      o = it->second;
      g_owner.erase(it);
    }
  }
  if (o.free_fn)
    o.free_fn(o.user, p);
  else
    (void)hipFree(p);
}

namespace {

// Host float64 tables of one axis of n grid points, in the order twH[H]
// (complex), tN[H+1] (complex), t4N[H+1] (complex), lam[n], where the real
// sequence transformed has length NS = n (cell-centred axis) or 2(n-1) (the
// even extension of a vertex axis, whose DCT-I is its real DFT) and H = NS/2.
int axis_real_length(int n, bool vertex) { return vertex ? 2 * (n - 1) : n; }

size_t axis_table_reals(int n, bool vertex) {
  const int H = axis_real_length(n, vertex) / 2;
  return 2 * (size_t)H + 2 * (size_t)(H + 1) * 2 + (size_t)n;
}

void fill_axis_tables(int n, double h, bool periodic, bool vertex, bool spectral,
                      std::vector<double>& out) {
  const long double PI = 3.141592653589793238462643383279502884L;
  const int NS = axis_real_length(n, vertex);
  const int H = NS / 2;
  out.clear();
  out.reserve(axis_table_reals(n, vertex));
  for (int j = 0; j < H; ++j) {
    long double a = 2.0L * PI * (long double)j / (long double)H;
    out.push_back((double)cosl(a));
    out.push_back((double)-sinl(a));
  }
  for (int k = 0; k <= H; ++k) {
    long double a = 2.0L * PI * (long double)k / (long double)NS;
    out.push_back((double)cosl(a));
    out.push_back((double)-sinl(a));
  }
  for (int k = 0; k <= H; ++k) {
    long double a = PI * (long double)k / (2.0L * (long double)NS);
    out.push_back((double)cosl(a));
    out.push_back((double)-sinl(a));
  }
  // eigenvalue of slot k: DCT-II index k (Neumann), mode min(k, n-k)
  // (periodic; sin^2 is the same for both) or DCT-I index k (vertex axis)
  const long double den = periodic ? (long double)n
                                   : (vertex ? 2.0L * (long double)(n - 1) : 2.0L * (long double)n);
  if (spectral) {
    const long double L = (long double)(vertex ? n - 1 : n) * (long double)h;
    for (int k = 0; k < n; ++k) {
      const long double w = periodic ? 2.0L * PI * (long double)std::min(k, n - k) / L
                                     : PI * (long double)k / L;
      out.push_back((double)(-(w * w)));
    }
    return;
  }
  for (int k = 0; k < n; ++k) {
    long double sn = sinl(PI * (long double)k / den);
    out.push_back((double)(-(4.0L / ((long double)h * (long double)h)) * sn * sn));
  }
}

template <typename T>
void set_axis_ptrs(AxisTables<T>& A, T* base, int n, bool vertex) {
  const int H = axis_real_length(n, vertex) / 2;
  A.twH = reinterpret_cast<const cplx<T>*>(base);
  A.tN = reinterpret_cast<const cplx<T>*>(base + 2 * (size_t)H);
  A.t4N = reinterpret_cast<const cplx<T>*>(base + 2 * (size_t)H + 2 * (size_t)(H + 1));
  A.lam = base + 2 * (size_t)H + 4 * (size_t)(H + 1);
}

// Reduction partials: 1024 blocks for grid means, two per 256-node block of
// the IB update.
int64_t partial_doubles(const pc_geom* g) {
  int64_t n = 1024;
  // two partial sums per block of the IB iteration kernel (64 threads)
  if (g) n = std::max<int64_t>(n, 2 * ((g->n_ib + 63) / 64));
  return n;
}

int check_mode(int mode) {
  if (mode != PC_F64 && mode != PC_F32 && mode != PC_MIXED)
    return fail(PC_ERR_INVALID_ARG, "mode must be PC_F64, PC_F32 or PC_MIXED");
  return PC_OK;
}

}  // namespace

int ensure_plan_ws(const pc_plan* P, pc_workspace** ws) {
  if (*ws) return PC_OK;
  pc_plan* mp = const_cast<pc_plan*>(P);
  if (!mp->own_ws) PC_TRY(pc_workspace_create(P, nullptr, PC_MIXED, &mp->own_ws));
  *ws = mp->own_ws;
  return PC_OK;
}

}  // namespace pc

using namespace pc;

extern "C" {

int pc_version(void) { return 115; }

int pc_set_allocator(pc_alloc_fn alloc, pc_free_fn free_fn, void* user) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(PC_ERR_INVALID_ARG, "pc_set_allocator: give both functions or neither");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  if (!g_owner.empty())
    return fail(PC_ERR_INVALID_ARG,
                "pc_set_allocator: allocations of the installed allocator are outstanding");
  g_alloc = alloc;
  g_free = free_fn;
  g_alloc_user = alloc ? user : nullptr;
  return PC_OK;
}

int pc_last_error(char* buf, size_t n) {
  const std::string& m = g_last_error;
  if (buf && n) {
    size_t c = m.size() < n - 1 ? m.size() : n - 1;
    std::memcpy(buf, m.data(), c);
    buf[c] = '\0';
  }
  return (int)m.size();
}

int pc_plan_create(int d, const int32_t* n, const double* h, void* stream, pc_plan** out) {
  return pc_plan_create_ex(d, n, h, nullptr, PC_EIG_FD2, PC_GRID_CELL, stream, out);
}

int pc_plan_create_ex(int d, const int32_t* n, const double* h, const int32_t* bc, int32_t eig,
                      int32_t grid, void* stream, pc_plan** out) {
  if (!out || !n || !h) return fail(PC_ERR_INVALID_ARG, "pc_plan_create: null argument");
  *out = nullptr;
  if (eig != PC_EIG_FD2 && eig != PC_EIG_SPECTRAL)
    return fail(PC_ERR_INVALID_ARG, "eig must be PC_EIG_FD2 or PC_EIG_SPECTRAL");
  if (grid != PC_GRID_CELL && grid != PC_GRID_VERTEX)
    return fail(PC_ERR_INVALID_ARG, "grid must be PC_GRID_CELL or PC_GRID_VERTEX");
  const bool vertex = grid == PC_GRID_VERTEX;
  if (d != 2 && d != 3) return fail(PC_ERR_UNSUPPORTED_SIZE, "d must be 2 or 3");
  for (int a = 0; a < d; ++a) {
    const int32_t b = bc ? bc[a] : PC_BC_NEUMANN;
    if (b != PC_BC_NEUMANN && b != PC_BC_PERIODIC)
      return fail(PC_ERR_INVALID_ARG, "bc[a] must be PC_BC_NEUMANN or PC_BC_PERIODIC");
    if (vertex) {
      if (b != PC_BC_NEUMANN)
        return fail(PC_ERR_INVALID_ARG, "a vertex grid has Neumann axes only");
      if (n[a] < 9 || n[a] > 2049)
        return fail(PC_ERR_UNSUPPORTED_SIZE, "a vertex axis needs n[a] in [9, 2049]");
    } else if (n[a] < 8 || n[a] > 4096 || (n[a] & 1)) {
      return fail(PC_ERR_UNSUPPORTED_SIZE, "n[a] must be even and in [8, 4096]");
    }
    if (!(h[a] > 0.0) || !std::isfinite(h[a]))
      return fail(PC_ERR_INVALID_ARG, "h[a] must be positive and finite");
  }
  {
    // flat grid indices are stored as int32 (stencil sources, block corners
    // and their one's-complement wrap mark)
    int64_t G = 1;
    for (int a = 0; a < d; ++a) G *= n[a];
    if (G > (int64_t)INT32_MAX - 1)
      return fail(PC_ERR_UNSUPPORTED_SIZE, "the grid has more than 2^31 - 2 points");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(PC_ERR_NO_DEVICE, "no HIP device visible");
  }
  pc_plan* P = new pc_plan();
  std::memset(P, 0, sizeof(*P));
  P->d = d;
  P->G = 1;
  for (int a = 0; a < 3; ++a) {
    P->n[a] = a < d ? n[a] : 1;
    P->h[a] = a < d ? h[a] : 1.0;
    P->bc[a] = (a < d && bc) ? bc[a] : PC_BC_NEUMANN;
    P->eig = eig;
    P->vertex = vertex ? 1 : 0;
    P->G *= P->n[a];
  }
  if (hipGetDevice(&P->device) != hipSuccess) {
    delete P;
    return fail(PC_ERR_HIP, "hipGetDevice failed");
  }
  std::vector<double> all, one;
  size_t offs[3];
  for (int a = 0; a < d; ++a) {
    offs[a] = all.size();
    fill_axis_tables(P->n[a], P->h[a], P->bc[a] == PC_BC_PERIODIC, vertex, eig == PC_EIG_SPECTRAL,
                     one);
    all.insert(all.end(), one.begin(), one.end());
  }
  std::vector<float> all32(all.size());
  for (size_t i = 0; i < all.size(); ++i) all32[i] = (float)all[i];
  int rc = dev_alloc(&P->tab64, all.size() * sizeof(double), "plan tables");
  if (rc == PC_OK) rc = dev_alloc(&P->tab32, all32.size() * sizeof(float), "plan tables");
  if (rc != PC_OK) {
    pc_plan_destroy(P);
    return rc;
  }
  hipStream_t s = as_stream(stream);
  hipError_t e = hipMemcpyAsync(P->tab64, all.data(), all.size() * sizeof(double),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(P->tab32, all32.data(), all32.size() * sizeof(float),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    pc_plan_destroy(P);
    return fail(PC_ERR_HIP, std::string("plan upload: ") + hipGetErrorString(e));
  }
  for (int a = 0; a < d; ++a) {
    set_axis_ptrs(P->ax64[a], reinterpret_cast<double*>(P->tab64) + offs[a], P->n[a], vertex);
    set_axis_ptrs(P->ax32[a], reinterpret_cast<float*>(P->tab32) + offs[a], P->n[a], vertex);
  }
  *out = P;
  return PC_OK;
}

int pc_plan_destroy(pc_plan* P) {
  if (!P) return PC_OK;
  if (P->own_ws) pc_workspace_destroy(P->own_ws);
  dev_free(P->tab64);
  dev_free(P->tab32);
  delete P;
  return PC_OK;
}

}  // extern "C"

namespace pc {
// Device bytes of a workspace of `mode` for a geometry with n_ib B+V nodes
// and n_near near-IB points (geometry false: solve-only).  Every region is
// rounded up to 256 bytes, as pc_workspace_create lays them out.
int64_t workspace_bytes_for(const pc_plan* P, bool geometry, int64_t n_ib, int64_t n_near,
                            int mode) {
  size_t s = mode == PC_F32 ? 4 : 8;
  int64_t bytes = 0;
  auto add = [&](int64_t b) { bytes += (b + 255) / 256 * 256; };
  if (geometry) {
    add(P->G * (int64_t)s);              // b
    add(P->G * (int64_t)s);              // phi
    add(n_near * (int64_t)s);            // bnear
    for (int i = 0; i < 3; ++i) add((int64_t)P->d * n_ib * (int64_t)s);  // uib, gib, gradib
  }
  if (mode == PC_MIXED) add(P->G * 4);   // w32
  if (mode == PC_MIXED && geometry) add(8 * ((n_near + 255) / 256));  // part2
  if (geometry && pc::resident_possible(P, n_ib, mode)) {
    if (P->d == 3) add(P->G * (int64_t)s);             // w1b
    add(4 * pc::resident_tiles_max(P, s));            // tile lists
  }
  if (geometry && pc::delta_possible(P, n_ib, mode)) {
    add(P->G * 8);                                    // dgrid
    for (int a = 0; a < P->d - 1; ++a) add(P->G * 4);  // dspec
    add(4 * pc::resident_tiles_max(P, 4));            // tile lists
  }
  // reduction partials: 1024 blocks for grid means, two per 64-node block of
  // the IB iteration kernel
  add(8 * std::max<int64_t>(1024, geometry ? 2 * ((n_ib + 63) / 64) : 0));
  add(16 * 8);                           // scalars
  add(16 * 4);                           // flags
  return bytes;
}
}  // namespace pc

extern "C" {

int64_t pc_workspace_bytes(const pc_plan* P, const pc_geom* g, int mode) {
  if (!P || check_mode(mode) != PC_OK) return -1;
  return pc::workspace_bytes_for(P, g != nullptr, g ? g->n_ib : 0, g ? g->n_near : 0, mode);
}

}  // extern "C"

namespace {

// Builds the tile lists of the resident transforms from the geometry's
// near-IB points and B+V stencil blocks and uploads them.
int resident_setup(const pc_plan* P, const pc_geom* g, size_t elem, pc_workspace* W) {
  std::vector<int32_t> near_pts(g->n_near), ib_base(g->n_ib);
  if (g->n_near)
    PC_HIP_CHECK(hipMemcpy(near_pts.data(), g->near, 4 * g->n_near, hipMemcpyDeviceToHost));
  if (g->n_ib)
    PC_HIP_CHECK(hipMemcpy(ib_base.data(), g->ibbase, 4 * g->n_ib, hipMemcpyDeviceToHost));
  std::vector<int32_t> lists[6];
  pc::resident_tiles(P, elem, near_pts, ib_base, g->m_node, lists);
  std::vector<int32_t> all;
  for (int l = 0; l < 6; ++l) {
    W->tl[l] = W->tiles + all.size();
    W->ntl[l] = (int)lists[l].size();
    all.insert(all.end(), lists[l].begin(), lists[l].end());
  }
  if ((int64_t)all.size() > pc::resident_tiles_max(P, elem))
    return fail(PC_ERR_INVALID_ARG, "resident tile lists exceed their bound");
  if (!all.empty())
    PC_HIP_CHECK(hipMemcpy(W->tiles, all.data(), 4 * all.size(), hipMemcpyHostToDevice));
  return PC_OK;
}

}  // namespace

extern "C" {

int pc_workspace_create(const pc_plan* P, const pc_geom* g, int mode, pc_workspace** out) {
  if (!P || !out) return fail(PC_ERR_INVALID_ARG, "pc_workspace_create: null argument");
  *out = nullptr;
  PC_TRY(check_mode(mode));
  if (g && !same_grid(P, g)) return fail(PC_ERR_INVALID_ARG, "geometry and plan grids differ");
  pc_workspace* W = new pc_workspace();
  std::memset(W, 0, sizeof(*W));
  W->plan = P;
  W->geom = g;
  W->mode = mode;
  W->nblk = 1024;
  (void)hipGetDevice(&W->device);
  W->bytes = pc_workspace_bytes(P, g, mode);
  int rc = dev_alloc(&W->block, (size_t)W->bytes, "workspace");
  if (rc != PC_OK) {
    delete W;
    return rc;
  }
  size_t s = mode == PC_F32 ? 4 : 8;
  char* cur = reinterpret_cast<char*>(W->block);
  auto take = [&](int64_t b) {
    char* p = cur;
    cur += (b + 255) / 256 * 256;
    return (void*)p;
  };
  if (g) {
    W->b = take(P->G * (int64_t)s);
    W->phi = take(P->G * (int64_t)s);
    W->bnear = take(g->n_near * (int64_t)s);
    W->uib = take((int64_t)g->d * g->n_ib * (int64_t)s);
    W->gib = take((int64_t)g->d * g->n_ib * (int64_t)s);
    W->gradib = take((int64_t)g->d * g->n_ib * (int64_t)s);
  }
  if (mode == PC_MIXED) W->w32 = reinterpret_cast<float*>(take(P->G * 4));
  if (mode == PC_MIXED && g) W->part2 = reinterpret_cast<double*>(take(8 * ((g->n_near + 255) / 256)));
  if (pc::resident_ok(P, g, mode)) {
    if (P->d == 3) W->w1b = take(P->G * (int64_t)s);
    W->tiles = reinterpret_cast<int32_t*>(take(4 * pc::resident_tiles_max(P, s)));
    W->resident = 1;
  }
  if (g && pc::delta_possible(P, g->n_ib, mode)) {
    W->dgrid = reinterpret_cast<double*>(take(P->G * 8));
    for (int a = 0; a < P->d - 1; ++a) W->dspec[a] = reinterpret_cast<float*>(take(P->G * 4));
    W->tiles = reinterpret_cast<int32_t*>(take(4 * pc::resident_tiles_max(P, 4)));
    W->delta = 1;
  }
  W->partial = reinterpret_cast<double*>(take(8 * partial_doubles(g)));
  W->scal = reinterpret_cast<double*>(take(16 * 8));
  W->flag = reinterpret_cast<int32_t*>(take(16 * 4));
  if (cur - reinterpret_cast<char*>(W->block) > W->bytes) {
    // the layout above and pc_workspace_bytes must agree region by region
    dev_free(W->block);
    delete W;
    return fail(PC_ERR_HIP, "workspace layout exceeds its allocation");
  }
  // coherent: the IB kernel's flag store (system-scope fence) is read by the
  // host while later kernels of the stream are still running
  if (hipHostMalloc((void**)&W->hscal, 16 * 8 + 16 * 4, hipHostMallocCoherent) != hipSuccess) {
    (void)hipGetLastError();
    dev_free(W->block);
    delete W;
    return fail(PC_ERR_OOM, "pinned host scalars");
  }
  W->hflag = reinterpret_cast<int32_t*>(W->hscal + 16);
  if (W->resident || W->delta) {
    int rc2 = resident_setup(P, g, W->delta ? 4 : s, W);
    if (rc2 != PC_OK) {
      pc_workspace_destroy(W);
      return rc2;
    }
  }
  if (W->delta) {
    // zero outside the near points and their lines, for good: every later
    // write lands on those (the same lists every iteration)
    hipError_t e = hipMemset(W->dgrid, 0, (size_t)P->G * 8);
    for (int a = 0; a < P->d - 1 && e == hipSuccess; ++a)
      e = hipMemset(W->dspec[a], 0, (size_t)P->G * 4);
    // complete before the caller's streams (which need not synchronise with
    // the null stream) use the workspace
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      (void)hipGetLastError();
      pc_workspace_destroy(W);
      return fail(PC_ERR_HIP, "workspace clear failed");
    }
  }
  for (int i = 0; i < 2; ++i) {
    if (hipEventCreateWithFlags(&W->ev[i], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      pc_workspace_destroy(W);
      return fail(PC_ERR_HIP, "hipEventCreate failed");
    }
  }
  *out = W;
  return PC_OK;
}

int pc_workspace_destroy(pc_workspace* W) {
  if (!W) return PC_OK;
  for (int i = 0; i < 2; ++i)
    if (W->ev[i]) (void)hipEventDestroy(W->ev[i]);
  dev_free(W->block);
  if (W->hscal) (void)hipHostFree(W->hscal);
  delete W;
  return PC_OK;
}

int pc_poisson_fft_solve(const pc_plan* P, int mode, const void* b, void* phi, int sweeps,
                         double* bmean_dev, pc_workspace* ws, void* stream) {
  if (!P || !b || !phi) return fail(PC_ERR_INVALID_ARG, "pc_poisson_fft_solve: null argument");
  PC_TRY(check_mode(mode));
  if (!aligned16(b) || !aligned16(phi)) return fail(PC_ERR_ALIGN, "fields must be 16-byte aligned");
  if (sweeps < 0 || sweeps > 16) return fail(PC_ERR_INVALID_ARG, "sweeps must be in [0, 16]");
  hipStream_t s = as_stream(stream);
  if (mode == PC_F64)
    return solve_f64(P, (const double*)b, (double*)phi, bmean_dev, ws, s);
  if (mode == PC_F32) return solve_f32(P, (const float*)b, (float*)phi, bmean_dev, ws, s);
  if (b == phi) return fail(PC_ERR_INVALID_ARG, "PC_MIXED needs b and phi to be distinct");
  if (P->eig != PC_EIG_FD2)
    return fail(PC_ERR_INVALID_ARG, "PC_MIXED needs the central-difference eigenvalues");
  if (ws && ws->mode != PC_MIXED)
    return fail(PC_ERR_INVALID_ARG, "PC_MIXED needs a workspace created for PC_MIXED");
  PC_TRY(ensure_plan_ws(P, &ws));
  return solve_mixed(P, (const double*)b, (double*)phi, sweeps, bmean_dev, ws, s);
}

}  // extern "C"
