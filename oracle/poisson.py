"""Pressure Poisson solve on the extended box (Sec. 2.3).

The three-step transform algorithm of Sec. 2.3: forward 1D transforms along
every axis, division by the eigenvalues (the sum of the 1D eigenvalues), and
backward 1D transforms.  Readings (the paper delegates the choice of
transform and eigenvalues to a table of Fuka 2015 that is not reproduced):

  * grid: staggered / cell-centred (the grid used with Neumann walls in
    Sec. 3.3);
  * boundary condition per axis: the homogeneous Neumann condition, Eq. (7),
    discretised with mirror ghosts phi_{-1} = phi_0, phi_n = phi_{n-1}; or
    periodic (phi_{-1} = phi_{n-1}, phi_n = phi_0), the lateral condition of
    the verification cases of Sec. 3;
  * method: central finite differences (the variant used for the reported
    timings of Sec. 3.2), or the pseudo-spectral eigenvalues (the squared
    wavenumbers of the transform's modes), one of the variants Sec. 3
    reports as interchangeable.  The mirror-ghost 3-point operator is diagonalised
    by the DCT-II, with eigenvalues -(4/h^2) sin^2(pi k / (2n)); the periodic
    one by the DFT, with eigenvalues -(4/h^2) sin^2(pi k / n);
  * zero mode: with Neumann walls everywhere the operator is singular; the
    mean of the right-hand side (the compatibility defect) is removed and
    reported, and the solution is taken with zero mean (the mode-0
    coefficient is set to zero).  Fixing the pressure at one point
    (Sec. 2.3, reference method; Sec. 3.1: zero at the left-bottom corner)
    is an output gauge applied afterwards.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .grid import Grid


def eigenvalues_1d(grid: Grid, a: int) -> np.ndarray:
    """1D eigenvalues of axis a.  Central differences: -(4/h^2) sin^2(pi k /
    (2n)) (Neumann, DCT-II index k) or -(4/h^2) sin^2(pi k / n) (periodic,
    DFT index k).  Pseudo-spectral: minus the squared wavenumber of the
    mode, -(pi k / L)^2 (Neumann: cos(pi k x / L)) or -(2 pi m / L)^2 with
    m = min(k, n - k) (periodic), L = n h."""
    n = grid.n[a]
    k = np.arange(n, dtype=np.float64)
    if grid.eig == "spectral":
        L = grid.length[a]
        if grid.periodic(a):
            return -(2.0 * np.pi * np.minimum(k, n - k) / L) ** 2
        return -(np.pi * k / L) ** 2
    if grid.eig != "fd2":
        raise ValueError(grid.eig)
    if grid.vertex:  # DCT-I index k of the mirror-about-the-vertex operator
        return -(4.0 / (grid.h[a] ** 2)) * np.sin(np.pi * k / (2.0 * (n - 1))) ** 2
    den = n if grid.periodic(a) else 2.0 * n
    return -(4.0 / (grid.h[a] ** 2)) * np.sin(np.pi * k / den) ** 2


def weights(grid: Grid) -> np.ndarray:
    """Quadrature weights of the grid points (flat [G]): 1, except 1/2 per
    vertex-grid axis at its two end points (the trapezoid rule; the vertex
    operator is symmetric in the inner product they define)."""
    w = np.ones(grid.shape_zyx)
    if grid.vertex:
        for a in range(grid.d):
            wa = np.ones(grid.n[a])
            wa[0] = wa[-1] = 0.5
            shape = [1] * grid.d
            shape[grid.d - 1 - a] = grid.n[a]
            w = w * wa.reshape(shape)
    return w.reshape(-1)


def eigenvalues(grid: Grid) -> np.ndarray:
    """Sum of the 1D eigenvalues, as an array of the grid's (z, y, x) shape."""
    lam = np.zeros(grid.shape_zyx)
    for a in range(grid.d):
        la = eigenvalues_1d(grid, a)
        shape = [1] * grid.d
        shape[grid.d - 1 - a] = grid.n[a]
        lam = lam + la.reshape(shape)
    return lam


def solve(grid: Grid, b: np.ndarray, workers: int = -1):
    """phi with L_h phi = b - mean(b) and mean(phi) = 0.  b: flat [G].
    Returns (phi flat [G], bmean).  On a vertex grid the transform is the
    DCT-I, bmean the weighted mean (weights()) and phi has zero weighted
    mean."""
    w = weights(grid)
    bm = float(np.sum(w * b) / np.sum(w)) if grid.vertex else float(np.mean(b))
    B = grid.to_array(b - bm)
    neu = tuple(grid.d - 1 - a for a in range(grid.d) if not grid.periodic(a))
    per = tuple(grid.d - 1 - a for a in range(grid.d) if grid.periodic(a))
    ttype = 1 if grid.vertex else 2
    Bh = sfft.dctn(B, type=ttype, axes=neu, workers=workers) if neu else B
    if per:
        Bh = sfft.fftn(Bh, axes=per, workers=workers)
    lam = eigenvalues(grid)
    lam.flat[0] = 1.0
    Ph = Bh / lam
    Ph.flat[0] = 0.0
    if per:
        Ph = sfft.ifftn(Ph, axes=per, workers=workers).real
    phi = sfft.idctn(Ph, type=ttype, axes=neu, workers=workers) if neu else Ph
    return np.ascontiguousarray(phi).reshape(-1), bm


def laplacian(grid: Grid, phi: np.ndarray) -> np.ndarray:
    """Central-difference Laplacian with mirror ghosts (Neumann axes) or
    wrap-around (periodic axes): the operator solve() inverts.  phi flat
    [G] -> flat [G]."""
    P = grid.to_array(phi)
    out = np.zeros_like(P)
    for a in range(grid.d):
        ax = grid.d - 1 - a
        if grid.periodic(a):
            up = np.roll(P, -1, axis=ax)
            dn = np.roll(P, 1, axis=ax)
        elif grid.vertex:  # mirror about the end vertex: phi_{-1} = phi_1
            n = grid.n[a]
            up = np.take(P, list(range(1, n)) + [n - 2], axis=ax)
            dn = np.take(P, [1] + list(range(0, n - 1)), axis=ax)
        else:
            lo = np.concatenate([np.take(P, [0], axis=ax), P], axis=ax)
            hi = np.concatenate([P, np.take(P, [grid.n[a] - 1], axis=ax)], axis=ax)
            up = np.take(hi, np.arange(1, grid.n[a] + 1), axis=ax)
            dn = np.take(lo, np.arange(0, grid.n[a]), axis=ax)
        out = out + (up - 2.0 * P + dn) / (grid.h[a] ** 2)
    return out.reshape(-1)


def laplacian_dense(grid: Grid) -> np.ndarray:
    """The same operator as a dense [G, G] matrix, assembled cell by cell
    with its ghost rule per axis (for tiny grids only)."""
    G = grid.G
    L = np.zeros((G, G))
    strides = [int(np.prod(grid.n[:a])) for a in range(grid.d)]
    for p in range(G):
        rem = p
        coords = []
        for a in range(grid.d):
            coords.append(rem % grid.n[a])
            rem //= grid.n[a]
        for a in range(grid.d):
            inv = 1.0 / grid.h[a] ** 2
            for step in (-1, 1):
                c = coords[a] + step
                if grid.periodic(a):
                    q = p + ((c % grid.n[a]) - coords[a]) * strides[a]
                elif grid.vertex and (c < 0 or c >= grid.n[a]):
                    q = p - step * strides[a]  # the mirror image of the neighbour
                else:
                    q = p if (c < 0 or c >= grid.n[a]) else p + step * strides[a]
                L[p, q] += inv
                L[p, p] -= inv
    return L


def solve_bordered(grid: Grid, b: np.ndarray):
    """Dense LU of [[L, 1], [w^T, 0]] [phi; mu] = [b; 0] (w = weights()).
    mu equals the (weighted) mean of b and phi has zero (weighted) mean.
    Tiny grids only."""
    G = grid.G
    K = np.zeros((G + 1, G + 1))
    K[:G, :G] = laplacian_dense(grid)
    K[:G, G] = 1.0
    K[G, :G] = weights(grid)
    rhs = np.concatenate([b, [0.0]])
    sol = np.linalg.solve(K, rhs)
    return sol[:G], float(sol[G])
