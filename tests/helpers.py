"""Shared test helpers: error metrics and layout conversion between the
oracle's [T, ...] arrays and the library's structure-of-arrays layout."""
import numpy as np


def rel_l2(x, ref):
    """The paper's error metric (Sec. 3.1): root-mean-squared difference
    normalised by the root-mean-squared reference value."""
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / den) if den > 0 else float(np.linalg.norm(x))


def to_np(t):
    return t.detach().cpu().numpy()


def stored_order(grid, x, idx, targets=None):
    """Per row of idx [T, k] (the oracle's grid-point stencils, node indices
    into x [M, d]), the argsort that puts the row into the library's storage
    order (include/pcorr.h, pc_geom_export): by the node's offset from the
    grid point in whole grid spacings, rounded per axis and clamped to
    [-4, 4], shortest first, then by its (z, y, x) components, then by node
    index.  targets: flat indices of the rows' grid points (all if None)."""
    from oracle import knn
    centres = grid.centres()
    if targets is not None:
        centres = centres[targets]
    d = grid.d
    lengths = None
    if any(grid.periodic(a) for a in range(d)):
        lengths = tuple(grid.length[a] if grid.periodic(a) else None for a in range(d))
    X = knn.offsets(centres, x, idx, lengths)
    o = np.clip(np.rint(X / np.asarray(grid.h, dtype=np.float64)), -4, 4).astype(np.int64)
    key = (o * o).sum(-1) * 729
    lex = np.zeros_like(key)
    for a in reversed(range(d)):
        lex = lex * 9 + (o[..., a] + 4)
    return np.lexsort((idx, key + lex), axis=-1)
