"""Weighted-least-squares derivative coefficients (Sec. 2.2).

The transfers of the hybrid step evaluate a field at points where it is not
known (grid points are not velocity points and vice versa), so they use the
form of Sec. 2.2 in which the value at the target is an unknown too: the
unknown vector is [f, f_1, f_2, f_11, f_12, f_22] and the polynomial vector
is Eq. (16).  The 3D extension has the ten terms
[1, x, y, z, x^2/2, xy, xz, y^2/2, yz, z^2/2].  The weights are the Gaussian
of Eq. (17) with epsilon = 6.3.  Minimising J (Eq. 12) gives a = C^-1 A b
(Eqs. 13-15); rows 1..d of C^-1 A are the first-derivative coefficients
("like the coefficients of a finite difference scheme").

Readings:
  * support radius: h_t = max(support * Delta, r_k), where r_k is the
    distance to the k-th neighbour, so every selected neighbour has r <= h_t
    and a positive weight (Eq. 17 is inclusive); Delta is the average point
    spacing and support = 3 (Sec. 2.2).  The weight of a selected neighbour
    is exp(-eps r^2 / h_t^2) with no further cut-off test;
  * the polynomial vector is evaluated in coordinates scaled by h_t, which is
    a diagonal change of basis and leaves the derivative estimates unchanged
    once divided back by h_t;
  * the least-squares problem is solved by a QR factorisation of W^1/2 Q
    (not the normal equations), and a stencil whose smallest-to-largest
    squared diagonal of R falls below 1e-12 is rejected as singular.

The 5-unknown form (Eqs. 10-15, value known at the target) is provided for
self-checks only; the hybrid step does not use it.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

EPS_DEFAULT = 6.3
SUPPORT_DEFAULT = 3.0
SINGULAR_RATIO = 1e-12


def basis6(xi: np.ndarray) -> np.ndarray:
    """Eq. (16) polynomial vector (2D, 6 terms) or its 3D 10-term extension.
    xi [..., d] -> [..., m]."""
    d = xi.shape[-1]
    one = np.ones(xi.shape[:-1])
    if d == 2:
        x, y = xi[..., 0], xi[..., 1]
        return np.stack([one, x, y, 0.5 * x * x, x * y, 0.5 * y * y], axis=-1)
    if d == 3:
        x, y, z = xi[..., 0], xi[..., 1], xi[..., 2]
        return np.stack([one, x, y, z, 0.5 * x * x, x * y, x * z, 0.5 * y * y, y * z,
                         0.5 * z * z], axis=-1)
    raise ValueError("d must be 2 or 3")


def basis5(xi: np.ndarray) -> np.ndarray:
    """Eq. (11) polynomial vector (2D, value known at the target)."""
    x, y = xi[..., 0], xi[..., 1]
    return np.stack([x, y, 0.5 * x * x, x * y, 0.5 * y * y], axis=-1)


def gaussian_weight(r2: np.ndarray, h: np.ndarray, eps: float = EPS_DEFAULT) -> np.ndarray:
    """Eq. (17): exp(-eps r^2 / h^2) for r <= h, else 0."""
    w = np.exp(-eps * r2 / (h * h))
    return np.where(r2 <= h * h, w, 0.0)


def default_delta(h) -> float:
    """Average point spacing: the grid spacing when isotropic, else the
    geometric mean of the per-axis spacings."""
    h = [float(v) for v in h]
    if all(v == h[0] for v in h):
        return h[0]
    return float(np.prod(h)) ** (1.0 / len(h))


def wls_rows(targets: np.ndarray, sources: np.ndarray, idx: np.ndarray, d2: np.ndarray,
             delta: float, eps: float = EPS_DEFAULT, support: float = SUPPORT_DEFAULT,
             chunk: int = 1 << 16, X: np.ndarray | None = None):
    """Full C^-1 A (Eq. 13) for every target, in unscaled coordinates.

    targets [T, d], sources [S, d], idx/d2 [T, k] from knn.  X (optional)
    [T, k, d]: the source-minus-target offsets, when they are not the plain
    differences (periodic images).
    Returns (rows [T, m, k], h_t [T], singular [T] bool) where rows[t, j, i]
    is the weight of f(x_i) in the j-th unknown of target t."""
    T, k = idx.shape
    d = targets.shape[1]
    m = 6 if d == 2 else 10
    if k < m:
        raise ValueError(f"k={k} < {m} unknowns")
    rows = np.empty((T, m, k), dtype=np.float64)
    hts = np.empty(T, dtype=np.float64)
    sing = np.zeros(T, dtype=bool)
    # derivative order of each basis term, to undo the scaling
    order = np.array([0] + [1] * d + [2] * (m - 1 - d), dtype=np.float64)
    for s in range(0, T, chunk):
        e = min(T, s + chunk)
        Xc = (sources[idx[s:e]] - targets[s:e, None, :]) if X is None else X[s:e]
        r2 = d2[s:e]
        ht = np.maximum(support * delta, np.sqrt(r2[:, -1]))
        # the selected neighbours lie inside the support by construction
        # (r <= r_k <= h_t); re-testing r <= h_t after the square root could
        # drop the k-th neighbour on a rounding of sqrt(r_k^2)^2
        w = np.exp(-eps * r2 / (ht[:, None] * ht[:, None]))
        xi = Xc / ht[:, None, None]
        Q = basis6(xi)                                          # [t, k, m]
        sw = np.sqrt(w)
        Qr, R = np.linalg.qr(sw[:, :, None] * Q)                # [t,k,m], [t,m,m]
        dg = np.abs(np.diagonal(R, axis1=1, axis2=2))
        ratio = (dg.min(axis=1) / dg.max(axis=1)) ** 2
        bad = ~(ratio >= SINGULAR_RATIO)
        sing[s:e] = bad
        Rs = R.copy()
        if bad.any():
            Rs[bad] = np.eye(m)
        Z = np.linalg.solve(Rs, np.swapaxes(Qr, 1, 2))          # [t, m, k]
        rows[s:e] = Z * sw[:, None, :] / (ht[:, None, None] ** order[None, :, None])
        hts[s:e] = ht
    return rows, hts, sing


def derivative_coefficients(targets, sources, idx, d2, delta, eps=EPS_DEFAULT,
                            support=SUPPORT_DEFAULT, chunk: int = 1 << 16, X=None):
    """First-derivative rows of C^-1 A: coef [T, d, k] with
    df/dx_a (target t) ~= sum_i coef[t, a, i] f(x_idx[t, i])."""
    d = targets.shape[1]
    rows, ht, sing = wls_rows(targets, sources, idx, d2, delta, eps, support, chunk, X)
    return np.ascontiguousarray(rows[:, 1:1 + d, :]), ht, sing


def wls5_rows(target: np.ndarray, nbrs: np.ndarray, h: float, eps: float = EPS_DEFAULT):
    """Eqs. (10)-(15) for one target whose value is known (2D): returns the
    [5, n] matrix C^-1 A acting on b_i = f(x_i) - f(x)."""
    X = nbrs - target[None, :]
    r2 = np.einsum("nd,nd->n", X, X)
    w = gaussian_weight(r2, np.float64(h), eps)
    q = basis5(X)                                   # [n, 5]
    C = (q * w[:, None]).T @ q                      # Eq. (14)
    A = (q * w[:, None]).T                          # Eq. (15)
    return np.linalg.solve(C, A)
