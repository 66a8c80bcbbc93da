"""Pins for the periodic parts of the oracle's WLS transfers: the minimal-
image key against a pure-Python definition over the three images of every
source, the k-d-tree selection against exhaustion, and the periodic stencils
against the non-periodic oracle run on the cloud tiled three times along
every periodic axis (the periodic box seen as one cell of an infinite
lattice; the non-periodic stencils are pinned in test_oracle_knn and
test_oracle_wls)."""
import itertools

import numpy as np
import pytest

from oracle import Grid, knn, wls
from oracle import projection as P


def _py_key(t, s, L):
    acc = 0.0
    for a in range(len(t)):
        diff = float(s[a]) - float(t[a])
        if L[a] is not None:
            # the image nearest to the target
            diff = min((diff + sh * L[a] for sh in (-1, 0, 1)), key=abs)
        acc = acc + diff * diff
    return acc


@pytest.mark.parametrize("L", [(1.0, None), (None, 0.5), (1.0, 0.5)])
def test_minimal_image_key_by_definition(rng, L):
    box = [v if v is not None else 1.0 for v in L]
    t = rng.uniform(size=(7, 2)) * box
    s = rng.uniform(size=(30, 2)) * box
    idx, d2 = knn.knn_brute(t, s, 11, lengths=L)
    for i in range(7):
        keys = sorted((_py_key(t[i], s[j], L), j) for j in range(30))[:11]
        assert [j for _, j in keys] == list(idx[i])
        assert [k for k, _ in keys] == list(d2[i])


@pytest.mark.parametrize("d,k,L", [(2, 16, (1.0, None)), (2, 12, (1.0, 1.0)),
                                   (3, 27, (1.0, None, 1.0)), (3, 27, (1.0, 1.0, 1.0))])
def test_periodic_tree_equals_brute(rng, d, k, L):
    s = rng.uniform(size=(700, d))
    # targets everywhere, and packed against the faces
    t = np.concatenate([rng.uniform(size=(200, d)),
                        np.clip(rng.uniform(size=(200, d)) * 0.04, 0, 1),
                        1.0 - rng.uniform(size=(100, d)) * 0.04])
    i1, d1 = knn.knn(t, s, k, lengths=L)
    i2, d2 = knn.knn_brute(t, s, k, lengths=L)
    np.testing.assert_array_equal(i1, i2)
    np.testing.assert_array_equal(d1, d2)


def _tiled(grid, x):
    """The cloud and grid tiled three times along every periodic axis and
    shifted by one box length there, as a non-periodic problem.  Returns
    (tiled grid, tiled nodes, source map tiled node -> node, map of the
    tiled grid's flat index -> original flat index, offsets of the middle
    copy's grid points)."""
    d = grid.d
    per = [grid.periodic(a) for a in range(d)]
    L = grid.length
    nt = tuple(3 * grid.n[a] if per[a] else grid.n[a] for a in range(d))
    tg = Grid(d, nt, grid.h)
    M = x.shape[0]
    shifts = list(itertools.product(*[(-1, 0, 1) if per[a] else (0,) for a in range(d)]))
    xs, src = [], []
    for sh in shifts:
        y = x.copy()
        for a in range(d):
            if per[a]:
                y[:, a] = x[:, a] + (sh[a] + 1) * L[a]
        xs.append(y)
        src.append(np.arange(M))
    cells = np.indices(tuple(reversed(nt))).reshape(d, -1)[::-1].T   # [Gt, d], x fastest
    orig = cells % np.array(grid.n)[None, :]
    stride = np.cumprod([1] + list(grid.n[:-1]))
    tmap = orig @ stride
    mid = np.array([grid.n[a] if per[a] else 0 for a in range(d)])
    return tg, np.concatenate(xs), np.concatenate(src), tmap, mid


@pytest.mark.parametrize("n,bc,k_grid,k_node", [
    ((32, 32), ("periodic", "neumann"), 16, 16),
    ((32, 64), ("periodic", "periodic"), 12, 16),
    ((32, 16), ("neumann", "periodic"), 16, 9),
    ((16, 16, 16), ("periodic", "neumann", "periodic"), 27, 27),
    ((40, 24), ("periodic", "periodic"), 16, 16),
    ((12, 10, 14), ("periodic", "neumann", "periodic"), 27, 27),
])
def test_periodic_stencils_equal_tiled_cloud(rng, n, bc, k_grid, k_node):
    d = len(n)
    h = tuple(1.0 / v for v in n)
    grid = Grid(d, n, h, bc)
    # a jittered lattice in the box (inside [0, L) along every axis)
    cells = np.indices(tuple(reversed(n))).reshape(d, -1)[::-1].T
    x = (cells + 0.5 + rng.uniform(-0.45, 0.45, size=cells.shape)) * np.array(h)
    kind = np.zeros(x.shape[0], np.uint8)
    st = P.build_stencils(grid, x, kind, k_grid, k_node)

    tg, xt, src, tmap, mid = _tiled(grid, x)
    delta = wls.default_delta(h)
    # grid points: the middle copy of every original point
    stride_t = np.cumprod([1] + list(tg.n[:-1]))
    gcell = np.indices(tuple(reversed(n))).reshape(d, -1)[::-1].T + mid[None, :]
    gc = tg.centres()[gcell @ stride_t]
    gi, gd2 = knn.knn(gc, xt, k_grid)
    gcoef, _, _ = wls.derivative_coefficients(gc, xt, gi, gd2, delta)
    np.testing.assert_array_equal(src[gi], st.grid_idx)
    np.testing.assert_allclose(gcoef, st.grid_coef, rtol=0,
                               atol=1e-12 * np.abs(st.grid_coef).max())
    # nodes: the middle copy of every node
    xm = x + mid[None, :] * np.array(h)[None, :]
    ni, nd2, nbase, Xn = knn.knn_grid_window(xm, tg, k_node)
    ncoef, _, _ = wls.derivative_coefficients(xm, tg.centres(), ni, nd2, delta, X=Xn)
    np.testing.assert_array_equal(tmap[ni], st.node_idx)
    np.testing.assert_array_equal(nbase % np.array(n)[None, :], st.node_base)
    np.testing.assert_allclose(ncoef, st.node_coef, rtol=0,
                               atol=1e-12 * np.abs(st.node_coef).max())
    # some stencils really do reach across a periodic face
    per_axes = [a for a in range(d) if grid.periodic(a)]
    a0 = per_axes[0]
    s0 = int(np.prod(n[:a0]))
    ci = (st.node_idx // s0) % n[a0]
    assert np.any(ci.max(axis=1) - ci.min(axis=1) > n[a0] // 2)


def test_positions_outside_periodic_box_rejected(rng):
    grid = Grid(2, (32, 32), (1 / 32, 1 / 32), ("periodic", "neumann"))
    x = rng.uniform(size=(1024, 2))
    x[5, 0] = 1.0
    with pytest.raises(ValueError):
        P.build_stencils(grid, x, np.zeros(1024, np.uint8), 16, 16)


@pytest.mark.parametrize("d,L", [(2, (1.0, None)), (3, (1.0, None, 1.0))])
def test_image_margin_same_selection(rng, d, L):
    s = rng.uniform(size=(3000, d))
    t = np.concatenate([rng.uniform(size=(300, d)), rng.uniform(size=(300, d)) * 0.05])
    i1, d1 = knn.knn(t, s, 16, lengths=L)
    i2, d2 = knn.knn(t, s, 16, lengths=L, margin=0.2)
    np.testing.assert_array_equal(i1, i2)
    np.testing.assert_array_equal(d1, d2)
    with pytest.raises(ValueError):
        knn.knn(t, s, 16, lengths=L, margin=0.01)
