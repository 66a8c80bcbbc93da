"""k-nearest-neighbour selection for the WLS support domains.

Sec. 2.2 selects the neighbours of a point as the cloud points inside a
circular support domain found with a linked-list cell search.  The workloads
here fix the stencil size instead (k nearest sources), so the selection is
written as its plain definition: the k sources with the smallest key
(d^2, source index), where d^2 = ((dx*dx) + dy*dy) + dz*dz is evaluated in
float64 with every product and sum rounded separately (no fused multiply-add).
The index in the key makes the set unique when distances tie exactly, which
happens for points placed on grid symmetry lines.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def exact_d2(targets: np.ndarray, sources: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Squared distances with the fixed operation order.  targets [T, d],
    sources [S, d], idx [T, c] -> [T, c]."""
    d = targets.shape[1]
    acc = None
    for a in range(d):
        diff = sources[idx, a] - targets[:, a:a + 1]
        sq = diff * diff
        acc = sq if acc is None else acc + sq
    return acc


def _sort_by_key(d2: np.ndarray, idx: np.ndarray):
    order = np.lexsort((idx, d2), axis=-1)
    return (np.take_along_axis(d2, order, axis=-1),
            np.take_along_axis(idx, order, axis=-1))


def knn_brute(targets: np.ndarray, sources: np.ndarray, k: int):
    """Definition by exhaustion: every source is a candidate.  O(T*S); for
    tiny inputs and for pinning knn() below."""
    S = sources.shape[0]
    idx = np.broadcast_to(np.arange(S, dtype=np.int64), (targets.shape[0], S)).copy()
    d2 = exact_d2(targets, sources, idx)
    d2s, idxs = _sort_by_key(d2, idx)
    return idxs[:, :k], d2s[:, :k]


def knn(targets: np.ndarray, sources: np.ndarray, k: int, extra: int = 8,
        workers: int = -1, chunk: int = 1 << 18, tree: cKDTree | None = None):
    """Same result as knn_brute, found through a k-d tree: the tree proposes
    k+extra candidates, the exact key re-ranks them, and a target whose k-th
    key is not safely inside the candidate radius is re-queried with more
    candidates.  Returns (idx [T, k] int64, d2 [T, k] float64)."""
    S = sources.shape[0]
    if k > S:
        raise ValueError("k larger than the number of sources")
    T = targets.shape[0]
    tree = tree if tree is not None else cKDTree(sources)
    out_i = np.empty((T, k), dtype=np.int64)
    out_d = np.empty((T, k), dtype=np.float64)
    for s in range(0, T, chunk):
        e = min(T, s + chunk)
        todo = np.arange(s, e)
        kk = min(S, k + extra)
        while todo.size:
            dist, cand = tree.query(targets[todo], k=kk, workers=workers)
            cand = cand.astype(np.int64)
            d2 = exact_d2(targets[todo], sources, cand)
            d2s, cs = _sort_by_key(d2, cand)
            out_i[todo] = cs[:, :k]
            out_d[todo] = d2s[:, :k]
            if kk == S:
                break
            # A source outside the candidate set lies at tree distance
            # >= dist[:, -1]; require a relative margin far above rounding.
            rlim = dist[:, -1]
            safe = d2s[:, k - 1] < (rlim * rlim) * (1.0 - 1e-9)
            todo = todo[~safe]
            kk = min(S, 2 * kk)
    return out_i, out_d


def window_m(k: int, d: int) -> int:
    """Smallest m with m^d >= k: the number of grid lines per axis in the
    block a node's stencil is drawn from."""
    m = 1
    while m ** d < k:
        m += 1
    return m


def node_window_base(x: np.ndarray, n, h, m: int) -> np.ndarray:
    """Lowest grid line of the m lines nearest to each node along each axis,
    clamped so the block lies inside the box.  Grid line i sits at
    (i + 1/2) h, so the m nearest lines start at floor(x/h - m/2 + 1/2).
    x [T, d] -> [T, d] int64."""
    out = np.empty(x.shape, dtype=np.int64)
    for a in range(x.shape[1]):
        lo = np.floor(x[:, a] / h[a] - (0.5 * m - 0.5)).astype(np.int64)
        out[:, a] = np.clip(lo, 0, n[a] - m)
    return out


def knn_grid_window(x: np.ndarray, grid, k: int):
    """Stencils of nodes over the regular grid.  Reading of the k-neighbour
    rule for this transfer: the k nearest grid points, by the (d^2, flat
    index) key, among the m^d points of the block of the m grid lines
    nearest to the node along each axis (m = ceil(k^(1/d)), block clamped
    inside the box).  Unrestricted k-nearest selection can fall on only two
    grid planes next to a box face in 3D (k = 27), where the quadratic fit of
    Eq. (16) is singular; the block always spans at least three lines per
    axis.  Returns (idx [T, k] flat grid index, d2 [T, k], base [T, d])."""
    d = x.shape[1]
    m = window_m(k, d)
    if any(v < m for v in grid.n):
        raise ValueError("grid smaller than the stencil block")
    base = node_window_base(x, grid.n, grid.h, m)
    offs = np.indices((m,) * d).reshape(d, -1)[::-1].T      # [m^d, d], x fastest
    cell = base[:, None, :] + offs[None, :, :]              # [T, m^d, d]
    stride = np.cumprod([1] + list(grid.n[:-1]))
    flat = np.einsum("tcd,d->tc", cell, stride)
    centres = np.empty(cell.shape, dtype=np.float64)
    for a in range(d):
        centres[..., a] = (cell[..., a] + 0.5) * grid.h[a]
    acc = None
    for a in range(d):
        diff = centres[..., a] - x[:, a:a + 1]
        sq = diff * diff
        acc = sq if acc is None else acc + sq
    d2s, idxs = _sort_by_key(acc, flat)
    return idxs[:, :k], d2s[:, :k], base
