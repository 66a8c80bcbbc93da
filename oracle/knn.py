"""k-nearest-neighbour selection for the WLS support domains.

Sec. 2.2 selects the neighbours of a point as the cloud points inside a
circular support domain found with a linked-list cell search.  The workloads
here fix the stencil size instead (k nearest sources), so the selection is
written as its plain definition: the k sources with the smallest key
(d^2, source index), where d^2 = ((dx*dx) + dy*dy) + dz*dz is evaluated in
float64 with every product and sum rounded separately (no fused multiply-add).
The index in the key makes the set unique when distances tie exactly, which
happens for points placed on grid symmetry lines.

Periodic axes (the lateral condition of the verification cases of Sec. 3)
measure offsets by the minimal image: t = x_s - x_t, then t - L if t > L/2
or t + L if t < -L/2 (one rounding each), L the box length of the axis.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def wrap_offset(t: np.ndarray, L: float) -> np.ndarray:
    """Minimal-image offset along a periodic axis of length L."""
    return np.where(t > 0.5 * L, t - L, np.where(t < -0.5 * L, t + L, t))


def offsets(targets: np.ndarray, sources: np.ndarray, idx: np.ndarray,
            lengths=None) -> np.ndarray:
    """Source-minus-target offsets [T, c, d]; lengths[a] (None for a
    non-periodic axis) selects the minimal image along axis a."""
    d = targets.shape[1]
    out = np.empty(idx.shape + (d,))
    for a in range(d):
        t = sources[idx, a] - targets[:, a:a + 1]
        if lengths is not None and lengths[a] is not None:
            t = wrap_offset(t, lengths[a])
        out[..., a] = t
    return out


def exact_d2(targets: np.ndarray, sources: np.ndarray, idx: np.ndarray,
             lengths=None) -> np.ndarray:
    """Squared distances with the fixed operation order.  targets [T, d],
    sources [S, d], idx [T, c] -> [T, c]."""
    X = offsets(targets, sources, idx, lengths)
    acc = None
    for a in range(targets.shape[1]):
        sq = X[..., a] * X[..., a]
        acc = sq if acc is None else acc + sq
    return acc


def _sort_by_key(d2: np.ndarray, idx: np.ndarray):
    order = np.lexsort((idx, d2), axis=-1)
    return (np.take_along_axis(d2, order, axis=-1),
            np.take_along_axis(idx, order, axis=-1))


def knn_brute(targets: np.ndarray, sources: np.ndarray, k: int, lengths=None):
    """Definition by exhaustion: every source is a candidate.  O(T*S); for
    tiny inputs and for pinning knn() below."""
    S = sources.shape[0]
    idx = np.broadcast_to(np.arange(S, dtype=np.int64), (targets.shape[0], S)).copy()
    d2 = exact_d2(targets, sources, idx, lengths)
    d2s, idxs = _sort_by_key(d2, idx)
    return idxs[:, :k], d2s[:, :k]


def _images(sources: np.ndarray, lengths, margin=None):
    """The sources and their copies shifted by -L and +L along every
    periodic axis, as (points, source index of each point).  With a margin,
    only the copies that land within `margin` of the box are kept."""
    d = sources.shape[1]
    pts, src = sources, np.arange(sources.shape[0], dtype=np.int64)
    for a in range(d):
        if lengths is None or lengths[a] is None:
            continue
        L = lengths[a]
        parts, ids = [pts], [src]
        for sgn in (-1.0, 1.0):
            q = pts.copy()
            q[:, a] = pts[:, a] + sgn * L
            keep = slice(None) if margin is None else (q[:, a] > -margin) & (q[:, a] < L + margin)
            parts.append(q[keep])
            ids.append(src[keep])
        pts, src = np.concatenate(parts), np.concatenate(ids)
    return pts, src


def knn(targets: np.ndarray, sources: np.ndarray, k: int, extra: int = 8,
        workers: int = -1, chunk: int = 1 << 18, tree: cKDTree | None = None,
        lengths=None, margin=None):
    """Same result as knn_brute, found through a k-d tree: the tree proposes
    k+extra candidates, the exact key re-ranks them, and a target whose k-th
    key is not safely inside the candidate radius is re-queried with more
    candidates.  With periodic axes the tree holds the periodic images of
    the sources (all of them, or those within `margin` of the box, for
    targets inside the box; a k-th neighbour beyond the margin is an error);
    candidates map back to their source and are ranked by the minimal-image
    key.  Returns (idx [T, k] int64, d2 [T, k] float64)."""
    S = sources.shape[0]
    if k > S:
        raise ValueError("k larger than the number of sources")
    T = targets.shape[0]
    periodic = lengths is not None and any(v is not None for v in lengths)
    src_of = None
    if periodic:
        pts, src_of = _images(sources, lengths, margin)
        tree = cKDTree(pts)
    elif tree is None:
        tree = cKDTree(sources)
    SX = tree.n
    out_i = np.empty((T, k), dtype=np.int64)
    out_d = np.empty((T, k), dtype=np.float64)
    for s in range(0, T, chunk):
        e = min(T, s + chunk)
        todo = np.arange(s, e)
        kk = min(SX, k + extra)
        while todo.size:
            dist, cand = tree.query(targets[todo], k=kk, workers=workers)
            cand = cand.astype(np.int64)
            if periodic:
                cand = src_of[cand]
            d2 = exact_d2(targets[todo], sources, cand, lengths)
            if periodic:
                # two images of one source: keep one
                o = np.argsort(cand, axis=1, kind="stable")
                cs_ = np.take_along_axis(cand, o, 1)
                dup = np.zeros(cs_.shape, dtype=bool)
                dup[:, 1:] = cs_[:, 1:] == cs_[:, :-1]
                d2 = d2.copy()
                np.put_along_axis(d2, o, np.where(dup, np.inf, np.take_along_axis(d2, o, 1)), 1)
            d2s, cs = _sort_by_key(d2, cand)
            out_i[todo] = cs[:, :k]
            out_d[todo] = d2s[:, :k]
            if kk == SX:
                break
            # A source outside the candidate set lies at tree distance
            # >= dist[:, -1]; require a relative margin far above rounding.
            rlim = dist[:, -1]
            safe = d2s[:, k - 1] < (rlim * rlim) * (1.0 - 1e-9)
            todo = todo[~safe]
            kk = min(SX, 2 * kk)
    if periodic and margin is not None and not np.all(out_d[:, -1] < margin * margin):
        raise ValueError("a k-th neighbour lies beyond the image margin")
    return out_i, out_d


def window_m(k: int, d: int) -> int:
    """Smallest m with m^d >= k: the number of grid lines per axis in the
    block a node's stencil is drawn from."""
    m = 1
    while m ** d < k:
        m += 1
    return m


def node_window_base(x: np.ndarray, n, h, m: int, periodic=None,
                     offset: float = 0.5) -> np.ndarray:
    """Lowest grid line of the m lines nearest to each node along each axis,
    clamped so the block lies inside the box (not along a periodic axis,
    where the block may run past a face and wraps around).  Grid line i sits
    at (i + offset) h (offset 1/2 on the cell-centred grid, 0 on the vertex
    grid), so the m nearest lines start at floor(x/h - offset - m/2 + 1).
    x [T, d] -> [T, d] int64 (unwrapped: -1 or above n - m on a periodic
    axis)."""
    out = np.empty(x.shape, dtype=np.int64)
    for a in range(x.shape[1]):
        lo = np.floor(x[:, a] / h[a] - (0.5 * m - 1.0 + offset)).astype(np.int64)
        out[:, a] = lo if (periodic is not None and periodic[a]) else np.clip(lo, 0, n[a] - m)
    return out


def knn_grid_window(x: np.ndarray, grid, k: int):
    """Stencils of nodes over the regular grid.  Reading of the k-neighbour
    rule for this transfer: the k nearest grid points, by the (d^2, flat
    index) key, among the m^d points of the block of the m grid lines
    nearest to the node along each axis (m = ceil(k^(1/d)), block clamped
    inside the box).  Unrestricted k-nearest selection can fall on only two
    grid planes next to a box face in 3D (k = 27), where the quadratic fit of
    Eq. (16) is singular; the block always spans at least three lines per
    axis.  Along a periodic axis the block is not clamped: its lines past a
    face are the periodic images of the lines at the other side (flat index
    of the wrapped line, offset to the unwrapped centre).
    Returns (idx [T, k] flat grid index, d2 [T, k], base [T, d] wrapped low
    corner, X [T, k, d] offsets of the selected centres from the node)."""
    d = x.shape[1]
    m = window_m(k, d)
    if any(v < m for v in grid.n):
        raise ValueError("grid smaller than the stencil block")
    per = [grid.periodic(a) for a in range(d)]
    base = node_window_base(x, grid.n, grid.h, m, per, grid.offset)
    offs = np.indices((m,) * d).reshape(d, -1)[::-1].T      # [m^d, d], x fastest
    cell = base[:, None, :] + offs[None, :, :]              # [T, m^d, d], unwrapped
    wrapped = cell % np.array(grid.n)[None, None, :]
    stride = np.cumprod([1] + list(grid.n[:-1]))
    flat = np.einsum("tcd,d->tc", wrapped, stride)
    diffs = np.empty(cell.shape, dtype=np.float64)
    for a in range(d):
        diffs[..., a] = (cell[..., a] + grid.offset) * grid.h[a] - x[:, a:a + 1]
    acc = None
    for a in range(d):
        sq = diffs[..., a] * diffs[..., a]
        acc = sq if acc is None else acc + sq
    order = np.lexsort((flat, acc), axis=-1)[:, :k]
    X = np.take_along_axis(diffs, order[:, :, None], axis=1)
    return (np.take_along_axis(flat, order, 1), np.take_along_axis(acc, order, 1),
            base % np.array(grid.n)[None, :], X)
