"""Pins for oracle.wls against what Sec. 2.2 and the mathematics fix:
exact reproduction of quadratics (Eqs. 9, 13, 16), the weighted normal
equations (Eq. 13 is the minimiser of Eq. 12 with the weights of Eq. 17), a
closed form on a symmetric stencil, rotation equivariance, and the weight
function itself."""
import math

import numpy as np
import pytest

from oracle import Grid, knn, wls


def _quad(rng, d):
    """Random quadratic f(x) = c + g.x + x.H.x/2 with value, gradient."""
    c = rng.normal()
    g = rng.normal(size=d)
    A = rng.normal(size=(d, d))
    H = A + A.T

    def f(x):
        return c + x @ g + 0.5 * np.einsum("...i,ij,...j->...", x, H, x)

    def grad(x):
        return g + x @ H
    return f, grad, H


def _cloud(rng, d, n):
    h = 1.0 / n
    g = (np.indices((n,) * d).reshape(d, -1).T + 0.5) * h
    return g + rng.uniform(-0.3 * h, 0.3 * h, size=g.shape), g, h


@pytest.mark.parametrize("d,k", [(2, 12), (2, 16), (3, 27)])
def test_reproduces_quadratics_grid_targets(rng, d, k):
    n = 16 if d == 2 else 8
    nodes, centres, h = _cloud(rng, d, n)
    idx, d2 = knn.knn(centres, nodes, k)
    coef, ht, sing = wls.derivative_coefficients(centres, nodes, idx, d2, h)
    assert not sing.any()
    f, grad, _ = _quad(rng, d)
    fv = f(nodes)
    est = np.einsum("tak,tk->ta", coef, fv[idx])
    ref = grad(centres)
    assert np.max(np.abs(est - ref)) <= 1e-9 * np.max(np.abs(ref))
    # derivative rows annihilate constants: sum_i c_i = 0
    assert np.max(np.abs(coef.sum(axis=2))) <= 1e-10 / h


@pytest.mark.parametrize("d,k", [(2, 16), (3, 27)])
def test_reproduces_quadratics_node_targets_all_rows(rng, d, k):
    n = 16 if d == 2 else 8
    nodes, centres, h = _cloud(rng, d, n)
    grid = Grid(d, (n,) * d, (h,) * d)
    idx, d2, _, _ = knn.knn_grid_window(nodes, grid, k)
    rows, ht, sing = wls.wls_rows(nodes, centres, idx, d2, h)
    assert not sing.any()
    f, grad, H = _quad(rng, d)
    fv = f(centres)[idx]
    est = np.einsum("tmk,tk->tm", rows, fv)
    scale = np.max(np.abs(f(nodes)))
    np.testing.assert_allclose(est[:, 0], f(nodes), atol=1e-11 * scale)
    np.testing.assert_allclose(est[:, 1:1 + d], grad(nodes), atol=1e-9 * np.abs(grad(nodes)).max())
    # second derivatives in the Eq. (16) order
    if d == 2:
        want = [H[0, 0], H[0, 1], H[1, 1]]
    else:
        want = [H[0, 0], H[0, 1], H[0, 2], H[1, 1], H[1, 2], H[2, 2]]
    for j, w in enumerate(want):
        np.testing.assert_allclose(est[:, 1 + d + j], w, atol=1e-6 * np.abs(H).max())


def test_weighted_normal_equations(rng):
    """For arbitrary data b, a = C^-1 A b satisfies sum_i w_i q_i e_i = 0 with
    e = M a - b (the stationarity condition of J, Eq. 12), where the weights
    are evaluated here straight from Eq. (17)."""
    nodes, centres, h = _cloud(rng, 2, 12)
    idx, d2 = knn.knn(centres[:50], nodes, 16)
    rows, ht, _ = wls.wls_rows(centres[:50], nodes, idx, d2, h)
    for t in range(50):
        X = nodes[idx[t]] - centres[t]
        r = np.sqrt((X ** 2).sum(1))
        w = np.array([math.exp(-6.3 * ri * ri / (ht[t] * ht[t])) for ri in r])
        q = np.stack([np.ones(16), X[:, 0], X[:, 1], X[:, 0] ** 2 / 2, X[:, 0] * X[:, 1],
                      X[:, 1] ** 2 / 2], axis=1)
        b = rng.normal(size=16)
        a = rows[t] @ b
        e = q @ a - b
        stat = q.T @ (w * e)
        assert np.max(np.abs(stat)) <= 1e-11 * np.max(np.abs(q.T @ (w * b)))
        # and the optimum is unique: perturbing a raises J
        J0 = np.sum(w * e * e)
        for _ in range(3):
            da = rng.normal(size=6) * 1e-3
            e2 = q @ (a + da) - b
            assert np.sum(w * e2 * e2) > J0


def test_closed_form_symmetric_stencil():
    """3x3 lattice of spacing s centred on the target: by symmetry the
    x-derivative decouples, c_x(i) = w_i dx_i / sum_j w_j dx_j^2."""
    s = 0.01
    pts = np.array([(i * s, j * s) for j in (-1, 0, 1) for i in (-1, 0, 1)], dtype=float)
    tgt = np.zeros((1, 2))
    idx = np.arange(9)[None, :]
    d2 = knn.exact_d2(tgt, pts, idx)
    order = np.lexsort((idx, d2), axis=-1)
    idx = np.take_along_axis(idx, order, -1)
    d2 = np.take_along_axis(d2, order, -1)
    delta = s  # support h_t = 3 s
    coef, ht, _ = wls.derivative_coefficients(tgt, pts, idx, d2, delta)
    assert ht[0] == 3 * s
    X = pts[idx[0]]
    w = np.exp(-6.3 * (X ** 2).sum(1) / (3 * s) ** 2)
    cx = w * X[:, 0] / np.sum(w * X[:, 0] ** 2)
    cy = w * X[:, 1] / np.sum(w * X[:, 1] ** 2)
    np.testing.assert_allclose(coef[0, 0], cx, rtol=0, atol=1e-12 / s)
    np.testing.assert_allclose(coef[0, 1], cy, rtol=0, atol=1e-12 / s)


def test_rotation_equivariance(rng):
    """The Gaussian weight is radial and the quadratic space is rotation
    invariant, so the gradient stencil of a rotated cloud is the rotated
    stencil."""
    X = rng.uniform(-1, 1, size=(16, 2)) * 0.02
    tgt = np.array([[0.3, 0.7]])
    th = 0.7
    Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    pts1 = tgt + X
    pts2 = tgt + X @ Rm.T
    idx = np.arange(16)[None, :]
    r2 = (X ** 2).sum(1)[None, :]
    c1, _, _ = wls.derivative_coefficients(tgt, pts1, idx, r2, 0.01)
    c2, _, _ = wls.derivative_coefficients(tgt, pts2, idx, r2, 0.01)
    np.testing.assert_allclose(c2[0], Rm @ c1[0], atol=1e-10 * np.abs(c1).max())


def test_gaussian_weight_eq17():
    h = np.float64(0.3)
    assert wls.gaussian_weight(np.float64(0.0), h) == 1.0
    assert wls.gaussian_weight(h * h, h) == pytest.approx(math.exp(-6.3), rel=1e-15)
    assert wls.gaussian_weight(np.float64(0.0901), h) == 0.0   # r > h
    assert wls.EPS_DEFAULT == 6.3 and wls.SUPPORT_DEFAULT == 3.0


def test_singular_collinear_stencil_flagged():
    pts = np.stack([np.linspace(0, 1, 16), np.zeros(16)], axis=1) * 0.01
    tgt = np.array([[0.005, 0.001]])
    idx = np.arange(16)[None, :]
    d2 = knn.exact_d2(tgt, pts, idx)
    _, _, sing = wls.derivative_coefficients(tgt, pts, idx, d2, 0.001)
    assert sing[0]


def test_five_unknown_form_reproduces(rng):
    """Eqs. (10)-(15): with f known at the target, C^-1 A (f_i - f) gives the
    exact first and second derivatives of a quadratic."""
    f, grad, H = _quad(rng, 2)
    tgt = np.array([0.4, 0.6])
    nbrs = tgt + rng.uniform(-1, 1, size=(12, 2)) * 0.03
    R = wls.wls5_rows(tgt, nbrs, 0.1)
    a = R @ (f(nbrs) - f(tgt))
    np.testing.assert_allclose(a[:2], grad(tgt), rtol=1e-9)
    np.testing.assert_allclose(a[2:], [H[0, 0], H[0, 1], H[1, 1]], rtol=1e-6)
