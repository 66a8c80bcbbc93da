"""The hybrid pressure-correction step (Sec. 2.3), in float64.

Notation: phi = (3 dt / 2) p and g = dt * f~ (the IB force of Eq. 19 times
the time step).  With these, Eqs. (18)-(20) read
    u^{n+1} = u* - grad phi + g,
    lap phi = div(u* + g),
    g = -u* + grad phi   at boundary and virtual points, 0 elsewhere.

Steps, in the order of Sec. 2.3:
  1. WLS stencils, computed once per geometry (Sec. 2.2, last paragraph):
     every grid point takes its k_g nearest velocity/boundary/virtual points;
     every node takes its k_n nearest grid points within the block of grid
     lines nearest to it (oracle.knn.knn_grid_window).
  2. The right-hand side is the WLS divergence of u* + g at the grid points.
     Written in split form b = D u* + D g; D g vanishes away from the points
     whose stencil holds a boundary or virtual point, which is why only
     those need re-evaluating after the first iteration.
  3. Cosine-transform Poisson solve (oracle.poisson.solve).
  4. WLS gradient of phi at the boundary and virtual points; IB-force update.
  5. Repeat 2-4 until the IB force converges.  Criterion: the mean squared
     difference of the force magnitude between two iterations is below the
     tolerance times the mean squared magnitude of the previous iteration
     (read literally: (|g^it| - |g^{it-1}|)^2 per point).  A criterion whose
     numerator is exactly zero also counts as converged.
  6. At the last iteration the gradient is evaluated at all nodes and the
     velocity projected: u* - grad phi on fluid points and exactly 0 on
     boundary and virtual points (where Eqs. 18 and 19 cancel).  The
     pressure is p = 2 phi / (3 dt).

Test infrastructure only.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import knn as _knn
from . import poisson as _poisson
from . import wls as _wls
from .grid import Grid

KIND_F, KIND_B, KIND_V = 0, 1, 2


@dataclasses.dataclass
class Stencils:
    grid: Grid
    grid_idx: np.ndarray    # [G, k_g] node index, sorted by (d^2, index)
    grid_coef: np.ndarray   # [G, d, k_g]
    node_idx: np.ndarray    # [M, k_n] flat grid index, sorted by (d^2, index)
    node_base: np.ndarray   # [M, d] low corner of each node's grid block
    node_coef: np.ndarray   # [M, d, k_n]
    ib: np.ndarray          # ascending indices of boundary+virtual nodes
    near: np.ndarray        # ascending grid points whose stencil holds an ib node
    singular_grid: np.ndarray
    singular_node: np.ndarray


def build_stencils(grid: Grid, x: np.ndarray, kind: np.ndarray, k_grid: int, k_node: int,
                   eps: float = _wls.EPS_DEFAULT, support: float = _wls.SUPPORT_DEFAULT,
                   delta: Optional[float] = None, workers: int = -1) -> Stencils:
    """x: [M, d] node positions; kind: [M].  Along a periodic axis of the
    grid the positions must lie in [0, n h) and offsets are minimal images."""
    delta = _wls.default_delta(grid.h) if delta is None else float(delta)
    lengths = _lengths(grid, x)
    gc = grid.centres()
    gi, gd2 = _knn.knn(gc, x, k_grid, workers=workers, lengths=lengths)
    Xg = _knn.offsets(gc, x, gi, lengths) if lengths else None
    gcoef, _, gs = _wls.derivative_coefficients(gc, x, gi, gd2, delta, eps, support, X=Xg)
    ni, nd2, nbase, Xn = _knn.knn_grid_window(x, grid, k_node)
    ncoef, _, ns = _wls.derivative_coefficients(x, gc, ni, nd2, delta, eps, support, X=Xn)
    ib = np.flatnonzero(kind != KIND_F).astype(np.int64)
    is_ib = kind != KIND_F
    near = np.flatnonzero(is_ib[gi].any(axis=1)).astype(np.int64)
    return Stencils(grid, gi, gcoef, ni, nbase, ncoef, ib, near, gs, ns)


def _lengths(grid: Grid, x: np.ndarray):
    """Box lengths of the periodic axes (None elsewhere), or None when no
    axis is periodic; checks that the positions lie in the periodic box."""
    if not any(grid.periodic(a) for a in range(grid.d)):
        return None
    out = []
    for a in range(grid.d):
        if grid.periodic(a):
            L = grid.length[a]
            if not (np.all(x[:, a] >= 0.0) and np.all(x[:, a] < L)):
                raise ValueError("positions along a periodic axis must lie in [0, n h)")
            out.append(L)
        else:
            out.append(None)
    return tuple(out)


def window_candidates(targets: np.ndarray, x: np.ndarray, w: float,
                      chunk: int = 1 << 24) -> np.ndarray:
    """Ascending indices of the nodes x [M, d] that lie in the cubes of side
    w adjacent to (or holding) a target's cube, cubes taken at multiples of
    w.  Every node closer than w to a target is among them (its cube index
    differs by at most one per axis)."""
    d = x.shape[1]
    ct = np.floor(targets / w).astype(np.int64)
    lo = min(int(ct.min()), int(np.floor(x.min() / w))) - 1
    hi = max(int(ct.max()), int(np.floor(x.max() / w))) + 1
    nc = hi - lo + 1
    if nc ** d > 1 << 28:
        raise ValueError("candidate window too fine for the extent of the cloud")
    mark = np.zeros(nc ** d, dtype=bool)
    shifts = np.stack(np.meshgrid(*[np.arange(-1, 2)] * d, indexing="ij"), -1).reshape(-1, d)
    for sh in shifts:
        c = ct + sh - lo
        key = np.zeros(c.shape[0], dtype=np.int64)
        for a in reversed(range(d)):
            key = key * nc + c[:, a]
        mark[key] = True
    out = []
    for s in range(0, x.shape[0], chunk):
        c = np.floor(x[s:s + chunk] / w).astype(np.int64) - lo
        key = np.zeros(c.shape[0], dtype=np.int64)
        for a in reversed(range(d)):
            key = key * nc + c[:, a]
        out.append(s + np.flatnonzero(mark[key]))
    return np.concatenate(out)


def sample_stencils(grid: Grid, x: np.ndarray, k_grid: int, k_node: int,
                    grid_pts: np.ndarray, nodes: np.ndarray,
                    eps: float = _wls.EPS_DEFAULT, support: float = _wls.SUPPORT_DEFAULT,
                    delta: Optional[float] = None, workers: int = -1,
                    image_margin: Optional[float] = None, window: Optional[float] = None):
    """The stencils of build_stencils for a subset of targets only: the
    grid points `grid_pts` (flat indices) over all nodes x [M, d], and the
    nodes `nodes` over the grid.  For checks at sizes where building every
    stencil on the CPU is too slow.  image_margin: on a periodic box, keep
    only the periodic images within this distance of the box (the neighbour
    search raises if a stencil reaches further).  window (non-periodic
    grids): search the grid points' neighbours only among the nodes of
    window_candidates(..., window), and raise if a k-th neighbour is not
    closer than the window (then a nearer node could have been missed).
    Returns (grid_idx [S, k_g], grid_coef [S, d, k_g], node_idx [T, k_n],
    node_coef [T, d, k_n])."""
    delta = _wls.default_delta(grid.h) if delta is None else float(delta)
    lengths = _lengths(grid, x)
    centres = grid.centres()
    gc = centres[grid_pts]
    if window is not None:
        if lengths is not None:
            raise ValueError("the candidate window is for grids without periodic axes")
        cand = window_candidates(gc, x, window)
        li, gd2 = _knn.knn(gc, x[cand], k_grid, workers=workers)
        if not np.all(gd2[:, -1] < window * window * (1.0 - 1e-9)):
            raise ValueError("a k-th neighbour reaches the edge of the candidate window")
        gi = cand[li]
    else:
        gi, gd2 = _knn.knn(gc, x, k_grid, workers=workers, lengths=lengths, margin=image_margin)
    Xg = _knn.offsets(gc, x, gi, lengths) if lengths else None
    gcoef, _, _ = _wls.derivative_coefficients(gc, x, gi, gd2, delta, eps, support, X=Xg)
    xn = x[nodes]
    ni, nd2, _, Xn = _knn.knn_grid_window(xn, grid, k_node)
    ncoef, _, _ = _wls.derivative_coefficients(xn, centres, ni, nd2, delta, eps, support, X=Xn)
    return gi, gcoef, ni, ncoef


def div_to_grid(st: Stencils, v: np.ndarray, rows: Optional[np.ndarray] = None,
                chunk: int = 1 << 18) -> np.ndarray:
    """b_p = sum_a sum_i coef[p, a, i] v[idx[p, i], a] for the grid points
    `rows` (all if None).  v: [M, d] -> [len]."""
    sel = np.arange(st.grid_idx.shape[0]) if rows is None else rows
    out = np.empty(sel.size)
    for s in range(0, sel.size, chunk):
        e = min(sel.size, s + chunk)
        p = sel[s:e]
        vals = v[st.grid_idx[p]]                        # [t, k, d]
        out[s:e] = np.einsum("tak,tka->t", st.grid_coef[p], vals)
    return out


def grad_to_nodes(st: Stencils, phi: np.ndarray, nodes: Optional[np.ndarray] = None,
                  chunk: int = 1 << 18) -> np.ndarray:
    """G_n,a = sum_j coef[n, a, j] phi[idx[n, j]] for the given nodes (all if
    None).  Returns [len, d]."""
    sel = np.arange(st.node_idx.shape[0]) if nodes is None else nodes
    out = np.empty((sel.size, st.node_coef.shape[1]))
    for s in range(0, sel.size, chunk):
        e = min(sel.size, s + chunk)
        n = sel[s:e]
        vals = phi[st.node_idx[n]]                      # [t, k]
        out[s:e] = np.einsum("tak,tk->ta", st.node_coef[n], vals)
    return out


def ib_sums(g_new: np.ndarray, g_old: np.ndarray):
    """Numerator and denominator of the IB-force criterion (Sec. 2.3):
    sum (|g_new| - |g_old|)^2 and sum |g_old|^2 over the IB points."""
    mn = np.sqrt(np.sum(g_new * g_new, axis=1))
    mo = np.sqrt(np.sum(g_old * g_old, axis=1))
    return float(np.sum((mn - mo) ** 2)), float(np.sum(mo * mo))


def pressure_correct(st: Stencils, u: np.ndarray, dt: float = 1.0, tol: float = 1e-3,
                     max_it: int = 50, fixed_it: int = 0, g0: Optional[np.ndarray] = None,
                     solver=None):
    """One hybrid pressure-correction sub-step.  u: [M, d] provisional
    velocity (zero at virtual points, Sec. 2.3).  g0: optional [n_ib, d] warm
    start of the IB force (times dt).  fixed_it > 0 runs exactly that many
    iterations.  `solver(b) -> (phi, bmean)` defaults to the cosine-transform
    solve.  Returns a dict."""
    grid = st.grid
    solver = solver or (lambda b: _poisson.solve(grid, b))
    M, d = u.shape
    ib = st.ib
    g = np.zeros((M, d))
    if g0 is not None:
        g[ib] = g0
    b_u = div_to_grid(st, u)
    it = 0
    hist = []
    while True:
        it += 1
        b = b_u.copy()
        if it > 1 or g0 is not None:
            # only grid points near the IB see the force (Sec. 2.3)
            b[st.near] = b_u[st.near] + div_to_grid(st, g, st.near)
        phi, bmean = solver(b)
        if ib.size == 0:
            break
        G_ib = grad_to_nodes(st, phi, ib)
        g_new = -u[ib] + G_ib
        num, den = ib_sums(g_new, g[ib])
        hist.append((num, den))
        g[ib] = g_new
        if fixed_it > 0:
            if it >= fixed_it:
                break
            continue
        if num < tol * den or num == 0.0 or it >= max_it:
            break
    converged = bool(ib.size == 0 or (hist and (hist[-1][0] < tol * hist[-1][1]
                                                 or hist[-1][0] == 0.0)))
    G_all = grad_to_nodes(st, phi)
    u_new = u - G_all
    u_new[ib] = 0.0
    return dict(u_new=u_new, phi=phi, p=2.0 * phi / (3.0 * dt), g_ib=g[ib].copy(),
                n_it=it, bmean=bmean, b_u=b_u, b_last=b, history=hist, converged=converged)
