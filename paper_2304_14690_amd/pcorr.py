"""Thin Python binding of libpcorr (include/pcorr.h).

Argument marshalling only: every step of the pressure-correction path runs
in the HIP kernels of libpcorr.so.  Tensors are torch CUDA tensors (device
memory of the current HIP device); the HIP stream defaults to torch's current
stream.  The functions keep the C names without the `pc_` prefix.  There is
no CPU fallback: if the library is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcorr.so")

PC_OK = 0
PC_WARN_IB_NOT_CONVERGED = 1
PC_ERR_INVALID_ARG = -1
PC_ERR_UNSUPPORTED_SIZE = -2
PC_ERR_ALIGN = -3
PC_ERR_OOM = -4
PC_ERR_SINGULAR_STENCIL = -5
PC_ERR_HIP = -6
PC_ERR_NO_DEVICE = -7

PC_F64, PC_F32, PC_MIXED = 1, 2, 3
PC_ALL, PC_NEAR_IB, PC_IB = 0, 1, 2
PC_KIND_F, PC_KIND_B, PC_KIND_V = 0, 1, 2
PC_BC_NEUMANN, PC_BC_PERIODIC = 0, 1
BCS = {"neumann": PC_BC_NEUMANN, "periodic": PC_BC_PERIODIC}
PC_EIG_FD2, PC_EIG_SPECTRAL = 0, 1
EIGS = {"fd2": PC_EIG_FD2, "spectral": PC_EIG_SPECTRAL}
PC_GRID_CELL, PC_GRID_VERTEX = 0, 1
GRIDS = {"cell": PC_GRID_CELL, "vertex": PC_GRID_VERTEX}

MODES = {"f64": PC_F64, "f32": PC_F32, "mixed": PC_MIXED}

# every symbol include/pcorr.h declares
EXPORTS = [
    "pc_version", "pc_last_error", "pc_plan_create", "pc_plan_create_ex", "pc_plan_destroy",
    "pc_poisson_fft_solve", "pc_wls_build", "pc_geom_destroy", "pc_geom_info",
    "pc_geom_export", "pc_div_to_grid", "pc_grad_to_nodes", "pc_ib_update", "pc_project",
    "pc_workspace_create", "pc_workspace_destroy", "pc_workspace_bytes",
    "pc_pressure_correct", "pc_geom_export_self", "pc_momentum_predict", "pc_momentum_pressure",
    "pc_set_allocator", "pc_geom_export_at", "pc_ib_update_noalloc", "pc_geom_permutation",
    "pc_geom_permute", "pc_geom_footprint",
]

# pc_alloc_fn / pc_free_fn
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                            ctypes.POINTER(ctypes.c_void_p))
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class PcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libpcorr error {code}: {msg}")
        self.code = code


class WlsOpts(ctypes.Structure):
    _fields_ = [("k_grid", ctypes.c_int32), ("k_node", ctypes.c_int32),
                ("eps", ctypes.c_double), ("support", ctypes.c_double),
                ("delta", ctypes.c_double), ("dtype_mask", ctypes.c_int32),
                ("k_self", ctypes.c_int32), ("order", ctypes.c_int32)]


PC_ORDER_CALLER, PC_ORDER_CELL = 0, 1
ORDERS = {"caller": PC_ORDER_CALLER, "cell": PC_ORDER_CELL}


def _dtype_mask(want_f32: bool, f32_only: bool) -> int:
    """pc_wls_opts.dtype_mask: float64 stencils unless f32_only, float32
    copies if want_f32 or f32_only."""
    if f32_only:
        return 1 << PC_F32
    return (1 << PC_F64) | ((1 << PC_F32) if want_f32 else 0)


PC_IB_FULL_TRANSFORMS = 1


class IbOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_it", ctypes.c_int32),
                ("fixed_it", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("gauge", ctypes.c_int32), ("flags", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("n_it", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("bmean", ctypes.c_double), ("ib_num", ctypes.c_double),
                ("ib_den", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2304_14690_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "pc_version": ([], ctypes.c_int),
        "pc_last_error": ([ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
        "pc_plan_create": ([ctypes.c_int, vp, vp, vp, ctypes.POINTER(vp)], ctypes.c_int),
        "pc_plan_create_ex": ([ctypes.c_int, vp, vp, vp, i32, i32, vp, ctypes.POINTER(vp)],
                              ctypes.c_int),
        "pc_plan_destroy": ([vp], ctypes.c_int),
        "pc_poisson_fft_solve": ([vp, ctypes.c_int, vp, vp, ctypes.c_int, vp, vp, vp],
                                 ctypes.c_int),
        "pc_wls_build": ([vp, vp, vp, i64, ctypes.POINTER(WlsOpts), vp, ctypes.POINTER(vp)],
                         ctypes.c_int),
        "pc_geom_destroy": ([vp], ctypes.c_int),
        "pc_geom_info": ([vp, ctypes.POINTER(i64)], ctypes.c_int),
        "pc_geom_export": ([vp, vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "pc_div_to_grid": ([vp, ctypes.c_int, vp, vp, ctypes.c_int, vp], ctypes.c_int),
        "pc_grad_to_nodes": ([vp, ctypes.c_int, vp, vp, ctypes.c_int, vp], ctypes.c_int),
        "pc_ib_update": ([vp, ctypes.c_int, vp, vp, vp, dbl, vp, vp, vp], ctypes.c_int),
        "pc_ib_update_noalloc": ([vp, ctypes.c_int, vp, vp, vp, dbl, vp, vp, vp], ctypes.c_int),
        "pc_project": ([vp, ctypes.c_int, vp, vp, vp, vp], ctypes.c_int),
        "pc_workspace_create": ([vp, vp, ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "pc_workspace_destroy": ([vp], ctypes.c_int),
        "pc_workspace_bytes": ([vp, vp, ctypes.c_int], i64),
        "pc_pressure_correct": ([vp, vp, ctypes.c_int, vp, dbl, vp, vp, vp,
                                 ctypes.POINTER(IbOpts), ctypes.POINTER(Stats), vp, vp],
                                ctypes.c_int),
        "pc_geom_export_self": ([vp, vp, vp, vp], ctypes.c_int),
        "pc_geom_export_at": ([vp, vp, i64, vp, vp, vp, i64, vp, vp, vp], ctypes.c_int),
        "pc_geom_permutation": ([vp, vp, vp], ctypes.c_int),
        "pc_geom_footprint": ([vp, i64, i64, i64, ctypes.POINTER(WlsOpts), vp, vp, vp],
                              ctypes.c_int),
        "pc_geom_permute": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp],
                            ctypes.c_int),
        "pc_momentum_predict": ([vp, ctypes.c_int, vp, vp, dbl, dbl, vp, vp, vp, vp],
                                ctypes.c_int),
        "pc_momentum_pressure": ([vp, ctypes.c_int, vp, vp, vp, vp, dbl, vp, vp], ctypes.c_int),
        "pc_set_allocator": ([ALLOC_FN, FREE_FN, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        if hasattr(lib, name):
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def last_error() -> str:
    buf = ctypes.create_string_buffer(1024)
    _lib.pc_last_error(buf, 1024)
    return buf.value.decode(errors="replace")


def _check(rc: int) -> int:
    if rc < 0:
        raise PcError(rc, last_error())
    return rc


def _stream(stream):
    if stream is None:
        if not torch.cuda.is_available():
            return None  # the library then reports that no device is visible
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return PC_F64
    if t.dtype == torch.float32:
        return PC_F32
    raise ValueError(f"unsupported dtype {t.dtype}")


class Plan:
    """Grid and transform tables (pc_plan).  bc: per-axis "neumann" or
    "periodic" (or the PC_BC_* codes); None is Neumann everywhere.  eig:
    "fd2" (central differences) or "spectral" (pseudo-spectral).  grid:
    "cell" (points at (i + 1/2) h) or "vertex" (points at i h)."""

    def __init__(self, d: int, n: Sequence[int], h: Sequence[float], stream=None,
                 bc: Optional[Sequence] = None, eig: str = "fd2", grid: str = "cell"):
        nn = (ctypes.c_int32 * 3)(*(list(n) + [1] * (3 - len(n))))
        hh = (ctypes.c_double * 3)(*(list(h) + [1.0] * (3 - len(h))))
        out = ctypes.c_void_p()
        if bc is None and eig == "fd2" and grid == "cell":
            _check(_lib.pc_plan_create(d, ctypes.addressof(nn), ctypes.addressof(hh),
                                       _stream(stream), ctypes.byref(out)))
            self.bc = ("neumann",) * d
        else:
            codes = [BCS[b] if isinstance(b, str) else int(b) for b in (bc or ("neumann",) * d)]
            bb = (ctypes.c_int32 * 3)(*(codes + [0] * (3 - len(codes))))
            e = EIGS[eig] if isinstance(eig, str) else int(eig)
            gt = GRIDS[grid] if isinstance(grid, str) else int(grid)
            _check(_lib.pc_plan_create_ex(d, ctypes.addressof(nn), ctypes.addressof(hh),
                                          ctypes.addressof(bb), e, gt, _stream(stream),
                                          ctypes.byref(out)))
            names = {v: k for k, v in BCS.items()}
            self.bc = tuple(names.get(c, str(c)) for c in codes)
        self.eig = eig
        self.grid = grid
        self.h_ = out
        self.d, self.n, self.h = d, tuple(n), tuple(h)
        self.G = 1
        for v in n:
            self.G *= v

    def __del__(self):
        if getattr(self, "h_", None) and _lib is not None:
            _lib.pc_plan_destroy(self.h_)
            self.h_ = None


class Geometry:
    """WLS stencils of one node cloud (pc_geom)."""

    def __init__(self, handle, plan: Plan):
        self.h_ = handle
        self.plan = plan
        info = (ctypes.c_int64 * 8)()
        _check(_lib.pc_geom_info(self.h_, info))
        (self.M, self.n_ib, self.n_near, self.k_grid, self.bn, self.bytes, self.near_entries,
         self.near_w) = (int(v) for v in info)

    def __del__(self):
        if getattr(self, "h_", None) and _lib is not None:
            _lib.pc_geom_destroy(self.h_)
            self.h_ = None


class Workspace:
    def __init__(self, plan: Plan, geom: Optional[Geometry], mode: int):
        out = ctypes.c_void_p()
        _check(_lib.pc_workspace_create(plan.h_, geom.h_ if geom else None, mode,
                                        ctypes.byref(out)))
        self.h_ = out
        self.plan, self.geom, self.mode = plan, geom, mode

    def __del__(self):
        if getattr(self, "h_", None) and _lib is not None:
            _lib.pc_workspace_destroy(self.h_)
            self.h_ = None


def version() -> int:
    return _lib.pc_version()


def plan_create(d, n, h, stream=None) -> Plan:
    return Plan(d, n, h, stream)


def workspace_create(plan: Plan, geom: Optional[Geometry], mode: int) -> Workspace:
    return Workspace(plan, geom, mode)


def workspace_bytes(plan: Plan, geom: Optional[Geometry], mode: int) -> int:
    return int(_lib.pc_workspace_bytes(plan.h_, geom.h_ if geom else None, mode))


def poisson_fft_solve(plan: Plan, b: torch.Tensor, phi: torch.Tensor, mode: int = PC_F64,
                      sweeps: int = 2, bmean: Optional[torch.Tensor] = None,
                      ws: Optional[Workspace] = None, stream=None) -> int:
    return _check(_lib.pc_poisson_fft_solve(plan.h_, mode, _ptr(b), _ptr(phi), sweeps,
                                            _ptr(bmean), ws.h_ if ws else None,
                                            _stream(stream)))


def wls_build(plan: Plan, xyz: torch.Tensor, kind: torch.Tensor, k_grid: int = 0,
              k_node: int = 0, eps: float = 0.0, support: float = 0.0, delta: float = 0.0,
              want_f32: bool = False, stream=None, k_self: int = 0,
              order: str = "caller", f32_only: bool = False) -> Geometry:
    assert xyz.dtype == torch.float64 and kind.dtype == torch.uint8
    opts = WlsOpts(k_grid, k_node, eps, support, delta, _dtype_mask(want_f32, f32_only), k_self,
                   ORDERS[order] if isinstance(order, str) else int(order))
    out = ctypes.c_void_p()
    _check(_lib.pc_wls_build(plan.h_, _ptr(xyz), _ptr(kind), kind.numel(), ctypes.byref(opts),
                             _stream(stream), ctypes.byref(out)))
    return Geometry(out, plan)


def geom_export(geom: Geometry, grid_idx=None, grid_coef=None, node_base=None,
                node_coef=None, ib=None, near=None, stream=None) -> int:
    return _check(_lib.pc_geom_export(geom.h_, _ptr(grid_idx), _ptr(grid_coef),
                                      _ptr(node_base), _ptr(node_coef), _ptr(ib), _ptr(near),
                                      _stream(stream)))


def geom_footprint(plan: Plan, M: int, n_ib: int, n_near: int, k_grid: int = 0,
                   k_node: int = 0, want_f32: bool = False, k_self: int = 0,
                   order: str = "caller", f32_only: bool = False):
    """(geometry bytes, build peak bytes, {mode: workspace bytes}) before a
    build (pc_geom_footprint); n_near is a bound on the near-IB points."""
    opts = WlsOpts(k_grid, k_node, 0.0, 0.0, 0.0, _dtype_mask(want_f32, f32_only), k_self,
                   ORDERS[order] if isinstance(order, str) else int(order))
    gb, pk = ctypes.c_int64(), ctypes.c_int64()
    ws = (ctypes.c_int64 * 3)()
    _check(_lib.pc_geom_footprint(plan.h_, M, n_ib, n_near, ctypes.byref(opts),
                                  ctypes.byref(gb), ctypes.byref(pk), ws))
    return int(gb.value), int(pk.value), {PC_F64: int(ws[0]), PC_F32: int(ws[1]),
                                          PC_MIXED: int(ws[2])}


def geom_permutation(geom: Geometry, perm: torch.Tensor, stream=None) -> int:
    """perm (int32 [M]): internal node i is the caller's node perm[i]."""
    assert perm.dtype == torch.int32 and perm.numel() == geom.M
    return _check(_lib.pc_geom_permutation(geom.h_, _ptr(perm), _stream(stream)))


def geom_permute(geom: Geometry, src: torch.Tensor, dst: torch.Tensor, to_internal: bool = True,
                 stream=None) -> int:
    """[ncomp][M] node fields between the caller's order and the internal one."""
    assert src.shape == dst.shape and src.dtype == dst.dtype and src.shape[-1] == geom.M
    ncomp = src.numel() // geom.M
    return _check(_lib.pc_geom_permute(geom.h_, _dtype_code(src), ncomp, 1 if to_internal else 0,
                                       _ptr(src), _ptr(dst), _stream(stream)))


def geom_export_at(geom: Geometry, grid_pts: Optional[torch.Tensor] = None, grid_idx=None,
                   grid_coef=None, nodes: Optional[torch.Tensor] = None, node_base=None,
                   node_coef=None, stream=None) -> int:
    """Stencils of the grid points grid_pts and the nodes `nodes` (int64
    device tensors) into [k][S], [d][k][S], [T] and [d][bn][T] tensors."""
    ng = 0 if grid_pts is None else grid_pts.numel()
    nn = 0 if nodes is None else nodes.numel()
    for t in (grid_pts, nodes):
        assert t is None or t.dtype == torch.int64
    return _check(_lib.pc_geom_export_at(geom.h_, _ptr(grid_pts), ng, _ptr(grid_idx),
                                         _ptr(grid_coef), _ptr(nodes), nn, _ptr(node_base),
                                         _ptr(node_coef), _stream(stream)))


def div_to_grid(geom: Geometry, v: torch.Tensor, b: torch.Tensor, subset: int = PC_ALL,
                stream=None) -> int:
    return _check(_lib.pc_div_to_grid(geom.h_, _dtype_code(v), _ptr(v), _ptr(b), subset,
                                      _stream(stream)))


def grad_to_nodes(geom: Geometry, phi: torch.Tensor, grad: torch.Tensor, subset: int = PC_ALL,
                  stream=None) -> int:
    return _check(_lib.pc_grad_to_nodes(geom.h_, _dtype_code(phi), _ptr(phi), _ptr(grad),
                                        subset, _stream(stream)))


def ib_update(geom: Geometry, u: torch.Tensor, grad_ib: torch.Tensor, g: torch.Tensor,
              tol: float, sums: torch.Tensor, conv: torch.Tensor, stream=None) -> int:
    return _check(_lib.pc_ib_update(geom.h_, _dtype_code(u), _ptr(u), _ptr(grad_ib), _ptr(g),
                                    tol, _ptr(sums), _ptr(conv), _stream(stream)))


def ib_update_noalloc(geom: Geometry, u: torch.Tensor, grad_ib: torch.Tensor, g: torch.Tensor,
                      tol: float, sums: torch.Tensor, conv: torch.Tensor, stream=None) -> int:
    return _check(_lib.pc_ib_update_noalloc(geom.h_, _dtype_code(u), _ptr(u), _ptr(grad_ib),
                                            _ptr(g), tol, _ptr(sums), _ptr(conv),
                                            _stream(stream)))


def project(geom: Geometry, u: torch.Tensor, grad: torch.Tensor, u_out: torch.Tensor,
            stream=None) -> int:
    return _check(_lib.pc_project(geom.h_, _dtype_code(u), _ptr(u), _ptr(grad), _ptr(u_out),
                                  _stream(stream)))


def pressure_correct(geom: Geometry, plan: Plan, mode: int, u: torch.Tensor, dt: float,
                     u_out: torch.Tensor, p: torch.Tensor, g: Optional[torch.Tensor] = None,
                     tol: float = 1e-3, max_it: int = 50, fixed_it: int = 0, sweeps: int = 2,
                     gauge: int = 0, ws: Optional[Workspace] = None, stream=None,
                     want_stats: bool = True, full_transforms: bool = False):
    opts = IbOpts(tol, max_it, fixed_it, sweeps, gauge,
                  PC_IB_FULL_TRANSFORMS if full_transforms else 0)
    st = Stats()
    rc = _check(_lib.pc_pressure_correct(geom.h_, plan.h_, mode, _ptr(u), dt, _ptr(u_out),
                                         _ptr(p), _ptr(g), ctypes.byref(opts),
                                         ctypes.byref(st) if want_stats else None,
                                         ws.h_ if ws else None, _stream(stream)))
    return rc, st.as_dict()


_allocator = None  # the installed callbacks, kept alive while installed


def set_allocator(alloc=None, free=None) -> int:
    """Routes the library's device allocations through alloc(nbytes) -> int
    device pointer and free(ptr) (both None: hipMalloc/hipFree again); see
    pc_set_allocator.  An exception in alloc reports PC_ERR_OOM."""
    global _allocator
    if alloc is None and free is None:
        _check(_lib.pc_set_allocator(ALLOC_FN(), FREE_FN(), None))
        _allocator = None
        return PC_OK

    def _a(user, nbytes, out):
        try:
            ptr = int(alloc(int(nbytes)))
        except Exception:
            return 1
        out[0] = ptr
        return 0 if ptr else 1

    def _f(user, ptr):
        free(int(ptr))

    cbs = (ALLOC_FN(_a), FREE_FN(_f))
    _check(_lib.pc_set_allocator(cbs[0], cbs[1], None))
    _allocator = cbs
    return PC_OK


def torch_allocator():
    """(alloc, free) through torch's caching allocator on the current device,
    so that torch's memory statistics and limits cover the library."""
    import torch

    def alloc(nbytes: int) -> int:
        return torch.cuda.caching_allocator_alloc(nbytes)

    def free(ptr: int) -> None:
        torch.cuda.caching_allocator_delete(ptr)
    return alloc, free


def geom_export_self(geom: Geometry, idx=None, coef=None, stream=None) -> int:
    return _check(_lib.pc_geom_export_self(geom.h_, _ptr(idx), _ptr(coef), _stream(stream)))


def momentum_predict(geom: Geometry, u: torch.Tensor, r_prev: Optional[torch.Tensor], dt: float,
                     nu: float, r: torch.Tensor, ustar: torch.Tensor, force=None,
                     stream=None) -> int:
    """The first fractional step (Eq. 3): r <- R^n, ustar <- u*."""
    f = None
    if force is not None:
        f = (ctypes.c_double * 3)(*(list(force) + [0.0] * (3 - len(force))))
    return _check(_lib.pc_momentum_predict(geom.h_, _dtype_code(u), _ptr(u), _ptr(r_prev), dt, nu,
                                           ctypes.addressof(f) if f is not None else None,
                                           _ptr(r), _ptr(ustar), _stream(stream)))


def momentum_pressure(geom: Geometry, r: torch.Tensor, ustar: torch.Tensor, unew: torch.Tensor,
                      g_ib: Optional[torch.Tensor], dt: float, r_prev: torch.Tensor,
                      stream=None) -> int:
    """r_prev <- R^n - grad p^n for the next step."""
    return _check(_lib.pc_momentum_pressure(geom.h_, _dtype_code(r), _ptr(r), _ptr(ustar),
                                            _ptr(unew), _ptr(g_ib), dt, _ptr(r_prev),
                                            _stream(stream)))
