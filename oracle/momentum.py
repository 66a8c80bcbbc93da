"""The first fractional step (Eq. 3) on the node cloud, in float64: the
intermediate velocity by the second-order Adams-Bashforth scheme with the
pressure gradient dropped from R^n, its spatial derivatives from the
weighted-least-squares form whose value at the target is known (Sec. 2.2,
Eqs. 9-15: unknowns f_x, f_y, f_xx, f_xy, f_yy, data f(x_i) - f(x)).

Readings:
  * node stencils: the k nearest other nodes by the (d^2, index) key (the
    target itself excluded; minimal image along periodic axes);
  * support and weight as for the transfers: h_t = max(support * Delta, r_k),
    exp(-eps r^2 / h_t^2) (Eq. 17), the basis in coordinates scaled by h_t;
  * 3D unknowns: f_x, f_y, f_z, f_xx, f_xy, f_xz, f_yy, f_yz, f_zz (the
    extension Sec. 2.2 calls straightforward); the Laplacian row is the sum
    of the rows of the pure second derivatives;
  * R^n = -u^n_j d_j u^n_i + nu lap u^n_i + F_i and R^{n-1} is the same
    expression at n-1 plus -d_i p^{n-1} (Eq. 3); the first step, which has no
    R^{n-1}, takes u* = u^n + dt R^n;
  * virtual points carry u* = 0 (Sec. 2.3: the frozen fluid inside the
    body); boundary points are advanced like velocity points;
  * the pressure gradient at the nodes for R^{n-1} comes from the projection
    of the previous step: Eq. 18 gives grad phi = u* - u^{n+1} + g with
    phi = (3 dt / 2) p and g the IB force times dt (zero off the B+V points).

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import knn as _knn
from . import wls as _wls

KIND_F, KIND_B, KIND_V = 0, 1, 2


def basis_known(xi: np.ndarray) -> np.ndarray:
    """Eq. (11) polynomial vector (2D: x, y, x^2/2, xy, y^2/2) or its 3D
    extension (x, y, z, x^2/2, xy, xz, y^2/2, yz, z^2/2).  xi [..., d]."""
    d = xi.shape[-1]
    if d == 2:
        x, y = xi[..., 0], xi[..., 1]
        return np.stack([x, y, 0.5 * x * x, x * y, 0.5 * y * y], axis=-1)
    x, y, z = xi[..., 0], xi[..., 1], xi[..., 2]
    return np.stack([x, y, z, 0.5 * x * x, x * y, x * z, 0.5 * y * y, y * z, 0.5 * z * z],
                    axis=-1)


def wls_known_rows(targets, sources, idx, d2, delta, eps=_wls.EPS_DEFAULT,
                   support=_wls.SUPPORT_DEFAULT, X=None):
    """C^-1 A of Eqs. (13)-(15) for targets whose value is known: rows
    [T, m, k] acting on b_i = f(x_i) - f(x), with m = 5 (2D) or 9 (3D), in
    the order of basis_known.  Solved by QR of W^1/2 Q.  Returns (rows, h_t,
    singular)."""
    T, k = idx.shape
    d = targets.shape[1]
    m = 5 if d == 2 else 9
    if k < m:
        raise ValueError(f"k={k} < {m} unknowns")
    Xc = (sources[idx] - targets[:, None, :]) if X is None else X
    ht = np.maximum(support * delta, np.sqrt(d2[:, -1]))
    w = np.exp(-eps * d2 / (ht[:, None] * ht[:, None]))
    Q = basis_known(Xc / ht[:, None, None])
    sw = np.sqrt(w)
    Qr, R = np.linalg.qr(sw[:, :, None] * Q)
    dg = np.abs(np.diagonal(R, axis1=1, axis2=2))
    sing = ~((dg.min(axis=1) / dg.max(axis=1)) ** 2 >= _wls.SINGULAR_RATIO)
    Rs = R.copy()
    if sing.any():
        Rs[sing] = np.eye(m)
    Z = np.linalg.solve(Rs, np.swapaxes(Qr, 1, 2))
    order = np.array([1] * d + [2] * (m - d), dtype=np.float64)
    rows = Z * sw[:, None, :] / (ht[:, None, None] ** order[None, :, None])
    return rows, ht, sing


def self_stencils(x: np.ndarray, k: int, delta: float, lengths=None,
                  eps=_wls.EPS_DEFAULT, support=_wls.SUPPORT_DEFAULT):
    """Stencils of every node over the other nodes.  x [M, d].  Returns
    (idx [M, k], coef [M, d + 1, k]: the d first-derivative rows and the
    Laplacian row, singular [M])."""
    M, d = x.shape
    idx1, d21 = _knn.knn(x, x, k + 1, lengths=lengths)
    own = idx1 == np.arange(M)[:, None]
    if not np.all(own.sum(axis=1) == 1):
        raise ValueError("a node is not its own nearest neighbour")
    keep = ~own
    idx = idx1[keep].reshape(M, k)
    d2 = d21[keep].reshape(M, k)
    X = _knn.offsets(x, x, idx, lengths) if lengths is not None else None
    rows, _, sing = wls_known_rows(x, x, idx, d2, delta, eps, support, X)
    pure = [2, 4] if d == 2 else [3, 6, 8]  # f_xx, f_yy (, f_zz) in basis_known order
    lap = rows[:, pure, :].sum(axis=1)
    coef = np.concatenate([rows[:, :d, :], lap[:, None, :]], axis=1)
    return idx, coef, sing


def momentum_rhs(idx, coef, u: np.ndarray, nu: float, force=None) -> np.ndarray:
    """R_i = -u_j d_j u_i + nu lap u_i + F_i at every node.  u [M, d]."""
    M, d = u.shape
    du = u[idx] - u[:, None, :]                         # [M, k, d]
    grad = np.einsum("mak,mkc->mac", coef[:, :d, :], du)  # grad[m, a, c] = d_a u_c
    lap = np.einsum("mk,mkc->mc", coef[:, d, :], du)
    R = -np.einsum("ma,mac->mc", u, grad) + nu * lap
    if force is not None:
        R = R + np.asarray(force, dtype=np.float64)[None, :]
    return R


def predict(u, R, R_prev, dt: float, kind) -> np.ndarray:
    """Eq. 3: u* = u^n + (3/2) dt R^n - (1/2) dt R^{n-1}; u* = u^n + dt R^n
    when R_prev is None (the first step); 0 at virtual points."""
    if R_prev is None:
        us = u + dt * R
    else:
        us = u + dt * (1.5 * R - 0.5 * R_prev)
    us[kind == KIND_V] = 0.0
    return us


def r_prev_next(R, ustar, unew, g_full, dt: float) -> np.ndarray:
    """R^n with the pressure gradient of this step: R^n - grad p^n, where
    grad p = 2 (u* - u^{n+1} + g) / (3 dt) at the nodes (Eq. 18)."""
    return R - (2.0 / (3.0 * dt)) * (ustar - unew + g_full)


def advance(st, self_idx, self_coef, kind, u0: np.ndarray, dt: float, nu: float, steps: int,
            force=None, solver=None):
    """Time steps of the two fractional steps: Eq. 3 (this module), then the
    pressure-correction sub-step (oracle.projection.pressure_correct, Eqs.
    18-20) with the IB force warm-started from the previous step (Sec. 2.3).
    st: the transfer stencils; self_idx/self_coef: self_stencils.  Returns
    (u [M, d], the last sub-step's result dict)."""
    from . import projection as _proj
    u = u0.copy()
    R_prev = None
    g_ib = None
    res = None
    M, d = u.shape
    for _ in range(steps):
        R = momentum_rhs(self_idx, self_coef, u, nu, force)
        us = predict(u, R, R_prev, dt, kind)
        res = _proj.pressure_correct(st, us, dt=dt, g0=g_ib, solver=solver)
        g_ib = res["g_ib"]
        g_full = np.zeros((M, d))
        g_full[st.ib] = g_ib
        R_prev = r_prev_next(R, us, res["u_new"], g_full, dt)
        u = res["u_new"]
    return u, res
