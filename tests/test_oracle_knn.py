"""Pins for oracle.knn: the k-d-tree selection equals the definition by
exhaustion, including exact distance ties, and the distance key is the
unfused float64 expression."""
import numpy as np
import pytest

from oracle import knn


def _py_d2(t, s):
    acc = 0.0
    for a in range(len(t)):
        diff = float(s[a]) - float(t[a])
        acc = acc + diff * diff
    return acc


@pytest.mark.parametrize("d", [2, 3])
def test_exact_d2_matches_scalar_loop(rng, d):
    t = rng.uniform(size=(5, d))
    s = rng.uniform(size=(7, d))
    idx = np.tile(np.arange(7), (5, 1))
    d2 = knn.exact_d2(t, s, idx)
    for i in range(5):
        for j in range(7):
            assert d2[i, j] == _py_d2(t[i], s[j])


def test_brute_is_pure_python_definition(rng):
    t = rng.uniform(size=(6, 2))
    s = rng.uniform(size=(40, 2))
    idx, d2 = knn.knn_brute(t, s, 9)
    for i in range(6):
        keys = sorted((_py_d2(t[i], s[j]), j) for j in range(40))[:9]
        assert [j for _, j in keys] == list(idx[i])
        assert [k for k, _ in keys] == list(d2[i])


@pytest.mark.parametrize("d,k", [(2, 12), (2, 16), (3, 27)])
def test_tree_equals_brute_random(rng, d, k):
    s = rng.uniform(size=(600, d))
    t = rng.uniform(size=(300, d))
    i1, d1 = knn.knn(t, s, k)
    i2, d2 = knn.knn_brute(t, s, k)
    np.testing.assert_array_equal(i1, i2)
    np.testing.assert_array_equal(d1, d2)


@pytest.mark.parametrize("d,k", [(2, 12), (3, 27)])
def test_tree_equals_brute_with_ties(d, k):
    # sources on an exact lattice, targets on cell centres and lattice
    # points: many neighbours tie exactly, the index decides
    n = 6 if d == 3 else 12
    g = np.indices((n,) * d).reshape(d, -1).T.astype(np.float64) * 0.125
    t = np.concatenate([g[::7] + 0.0625, g[::5]], axis=0)
    i1, d1 = knn.knn(t, g, k, extra=1)
    i2, d2 = knn.knn_brute(t, g, k)
    np.testing.assert_array_equal(i1, i2)
    np.testing.assert_array_equal(d1, d2)
    # ties really are present and resolved by index
    tied = (np.diff(d2, axis=1) == 0)
    assert tied.any()
    inc = np.diff(i2, axis=1) > 0
    assert np.all(inc[tied])


@pytest.mark.parametrize("d,k,n", [(2, 12, 9), (2, 16, 7), (3, 27, 5)])
def test_grid_window_is_knn_inside_block(rng, d, k, n):
    """Within the clamped block of the m nearest grid lines per axis the
    selection is plain k-nearest; the block itself is checked line by line."""
    from oracle import Grid
    grid = Grid(d, (n,) * d, (1.0 / n,) * d)
    x = rng.uniform(-0.02, 1.02, size=(200, d))
    idx, d2, base, _ = knn.knn_grid_window(x, grid, k)
    m = knn.window_m(k, d)
    centres = grid.centres()
    for t in range(0, 200, 7):
        lines = []
        for a in range(d):
            c = np.arange(n)
            dist = np.abs((c + 0.5) / n - x[t, a])
            near = np.sort(np.lexsort((c, dist))[:m])
            # clamp: if the m nearest lines are not contiguous (never) or run
            # past the box, the block is the clamped contiguous range
            lo = min(max(int(near[0]), 0), n - m)
            assert base[t, a] == lo or abs(dist[base[t, a]] - dist[lo]) < 1e-15 \
                or abs((base[t, a] + m - 1 + 0.5) / n - x[t, a]) == abs((lo + 0.5) / n - x[t, a])
            lines.append(np.arange(base[t, a], base[t, a] + m))
        cells = np.stack(np.meshgrid(*lines, indexing="ij"), -1).reshape(-1, d)
        flat = cells[:, 0] + n * cells[:, 1] + (n * n * cells[:, 2] if d == 3 else 0)
        bi, bd = knn.knn_brute(x[t:t + 1], centres[flat], k)
        np.testing.assert_array_equal(np.sort(flat[bi[0]]), np.sort(idx[t]))


def test_window_spans_three_lines_per_axis(rng):
    from oracle import Grid
    grid = Grid(3, (8, 8, 8), (0.125,) * 3)
    x = rng.uniform(0, 1, size=(500, 3))
    idx, _, _, _ = knn.knn_grid_window(x, grid, 27)
    cells = np.stack([idx % 8, (idx // 8) % 8, idx // 64], -1)
    for a in range(3):
        assert all(len(np.unique(cells[t, :, a])) >= 3 for t in range(500))


@pytest.mark.parametrize("d,k", [(2, 16), (3, 27)])
def test_vertex_node_window_by_exhaustion(rng, d, k):
    """On the vertex grid (points at i h) the block holds the m grid lines
    nearest to the node along each axis, clamped inside the box, and the
    stencil is the k smallest keys of the block."""
    from oracle import Grid
    n = (9, 12, 7)[:d]
    h = (0.1, 0.07, 0.13)[:d]
    grid = Grid(d, n, h, vertex=True)
    x = rng.uniform(size=(200, d)) * np.array([(v - 1) * hh for v, hh in zip(n, h)])
    idx, d2, base, X = knn.knn_grid_window(x, grid, k)
    m = knn.window_m(k, d)
    for t in range(x.shape[0]):
        for a in range(d):
            lines = np.arange(n[a])
            dist = np.abs(lines * h[a] - x[t, a])
            near = np.sort(np.argsort(dist, kind="stable")[:m])
            # the m nearest lines form a run; the block is that run
            assert base[t, a] == near[0] or abs(dist[near[0]] - dist[base[t, a] + m - 1]) < 1e-12
        cells = np.indices((m,) * d).reshape(d, -1)[::-1].T + base[t]
        stride = np.cumprod([1] + list(n[:-1]))
        flat = cells @ stride
        pos = cells * np.array(h)
        dd = ((pos - x[t]) ** 2).sum(1)
        order = np.lexsort((flat, dd))[:k]
        assert set(flat[order]) == set(idx[t])
    np.testing.assert_allclose(X, grid.centres()[idx] - x[:, None, :], atol=1e-15)
