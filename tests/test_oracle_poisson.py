"""Pins for oracle.poisson against the mathematics of the Neumann-box
problem (Sec. 2.3, Eq. 7): discrete eigenfunctions, the dense bordered
system on tiny grids (an independent LU solve of the same operator, also at
sizes that are not powers of two and with anisotropic spacing), the
residual of the solved problem, and an exact rational solve."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import Grid, poisson


def _eigvec(grid, ks):
    idx = np.indices(grid.shape_zyx)
    v = np.ones(grid.shape_zyx)
    lam = 0.0
    for a in range(grid.d):
        i = idx[grid.d - 1 - a]
        v = v * np.cos(np.pi * ks[a] * (i + 0.5) / grid.n[a])
        lam += -(4.0 / grid.h[a] ** 2) * np.sin(np.pi * ks[a] / (2 * grid.n[a])) ** 2
    return v.reshape(-1), lam


@pytest.mark.parametrize("n,h,ks", [
    ((64, 64), (1 / 64, 1 / 64), (3, 5)),
    ((32, 16), (0.1, 0.03), (31, 1)),
    ((16, 8, 32), (1 / 16, 0.2, 0.01), (2, 7, 9)),
])
def test_eigenfunctions(n, h, ks):
    grid = Grid(len(n), n, h)
    v, lam = _eigvec(grid, ks)
    phi, bm = poisson.solve(grid, v)
    assert abs(bm) < 1e-14
    np.testing.assert_allclose(phi, v / lam, rtol=0, atol=1e-13 * np.abs(v / lam).max())
    # the mirror-ghost operator has exactly these eigenpairs
    np.testing.assert_allclose(poisson.laplacian(grid, v), lam * v, atol=1e-12 * abs(lam))


def test_constant_rhs_gives_zero():
    grid = Grid(2, (8, 16), (0.1, 0.2))
    phi, bm = poisson.solve(grid, np.full(128, 3.5))
    assert bm == pytest.approx(3.5, rel=1e-15)
    assert np.max(np.abs(phi)) < 1e-13


@pytest.mark.parametrize("n,h", [((3, 5), (0.3, 0.2)), ((8, 8), (1 / 8, 1 / 8)),
                                 ((4, 4, 4), (0.25, 0.25, 0.25)),
                                 ((2, 3, 5), (0.5, 0.1, 0.7))])
def test_bordered_lu(rng, n, h):
    grid = Grid(len(n), n, h)
    b = rng.normal(size=grid.G)
    phi, bm = poisson.solve(grid, b)
    phi2, mu = poisson.solve_bordered(grid, b)
    assert mu == pytest.approx(np.mean(b), abs=1e-13)
    assert bm == pytest.approx(mu, abs=1e-13)
    np.testing.assert_allclose(phi, phi2, atol=1e-12 * np.abs(phi2).max())
    assert abs(phi.mean()) < 1e-13 * np.abs(phi).max()


def test_dense_operator_matches_stencil(rng):
    grid = Grid(3, (3, 4, 5), (0.2, 0.3, 0.5))
    v = rng.normal(size=grid.G)
    np.testing.assert_allclose(poisson.laplacian_dense(grid) @ v, poisson.laplacian(grid, v),
                               atol=1e-12 * np.abs(v).max() / 0.04)


@pytest.mark.parametrize("n", [(64, 64), (16, 16, 16), (48, 40)])
def test_residual_vanishes(rng, n):
    """The FD divergence of the FD gradient of phi equals the compatible RHS."""
    grid = Grid(len(n), n, tuple(1.0 / v for v in n))
    b = rng.normal(size=grid.G) + 0.7
    phi, bm = poisson.solve(grid, b)
    r = (b - bm) - poisson.laplacian(grid, phi)
    assert np.linalg.norm(r) / np.linalg.norm(b - bm) < 1e-13


def _exact_solve(grid, b):
    """Gaussian elimination in rationals on the bordered system."""
    L = poisson.laplacian_dense(grid)
    G = grid.G
    K = [[Fraction(0)] * (G + 2) for _ in range(G + 1)]
    for i in range(G):
        for j in range(G):
            K[i][j] = Fraction(L[i, j]).limit_denominator(10 ** 6)
        K[i][G] = Fraction(1)
        K[i][G + 1] = b[i]
    for j in range(G):
        K[G][j] = Fraction(1)
    n = G + 1
    for c in range(n):
        p = next(r for r in range(c, n) if K[r][c] != 0)
        K[c], K[p] = K[p], K[c]
        for r in range(n):
            if r != c and K[r][c] != 0:
                f = K[r][c] / K[c][c]
                K[r] = [a - f * bb for a, bb in zip(K[r], K[c])]
    return [K[i][G + 1] / K[i][i] for i in range(n)]


def test_exact_rational_tiny():
    grid = Grid(2, (3, 2), (1.0, 0.5))
    b = [Fraction(v) for v in (1, -2, 3, 5, 0, -4)]
    sol = _exact_solve(grid, b)
    phi, bm = poisson.solve(grid, np.array([float(v) for v in b]))
    assert bm == pytest.approx(float(sol[-1]), abs=1e-15)
    np.testing.assert_allclose(phi, [float(v) for v in sol[:-1]], atol=1e-14)


# ---- periodic and mixed periodic x Neumann boxes (the lateral condition of
# the verification cases of Sec. 3) ----------------------------------------------

def _eigvec_mixed(grid, ks, phases):
    """Products of cos(pi k (i + 1/2) / n) along Neumann axes and
    cos(2 pi k i / n + theta) along periodic axes, with their eigenvalues
    written out from the 3-point stencil (not from oracle.poisson)."""
    idx = np.indices(grid.shape_zyx)
    v = np.ones(grid.shape_zyx)
    lam = 0.0
    for a in range(grid.d):
        i = idx[grid.d - 1 - a]
        if grid.periodic(a):
            v = v * np.cos(2 * np.pi * ks[a] * i / grid.n[a] + phases[a])
            lam += (2 * np.cos(2 * np.pi * ks[a] / grid.n[a]) - 2) / grid.h[a] ** 2
        else:
            v = v * np.cos(np.pi * ks[a] * (i + 0.5) / grid.n[a])
            lam += (2 * np.cos(np.pi * ks[a] / grid.n[a]) - 2) / grid.h[a] ** 2
    return v.reshape(-1), lam


@pytest.mark.parametrize("n,h,bc,ks,ph", [
    ((64, 64), (1 / 64, 1 / 64), ("periodic", "periodic"), (3, 5), (0.3, 1.1)),
    ((64, 32), (1 / 64, 1 / 32), ("periodic", "neumann"), (7, 4), (2.0, 0.0)),
    ((16, 32), (0.1, 0.03), ("neumann", "periodic"), (15, 1), (0.0, 0.7)),
    ((16, 8, 32), (1 / 16, 0.2, 0.01), ("periodic", "neumann", "periodic"), (2, 7, 9),
     (0.5, 0.0, 2.5)),
    ((32, 32), (1 / 32, 1 / 32), ("periodic", "periodic"), (16, 16), (0.4, 0.9)),
])
def test_eigenfunctions_mixed(n, h, bc, ks, ph):
    grid = Grid(len(n), n, h, bc)
    v, lam = _eigvec_mixed(grid, ks, ph)
    np.testing.assert_allclose(poisson.laplacian(grid, v), lam * v,
                               atol=1e-12 * abs(lam) * np.abs(v).max())
    phi, bm = poisson.solve(grid, v)
    assert abs(bm) < 1e-14
    np.testing.assert_allclose(phi, v / lam, rtol=0, atol=1e-13 * np.abs(v / lam).max())


@pytest.mark.parametrize("n,h,bc", [
    ((3, 5), (0.3, 0.2), ("periodic", "neumann")),
    ((4, 6), (0.25, 0.1), ("periodic", "periodic")),
    ((5, 3), (0.2, 0.4), ("neumann", "periodic")),
    ((4, 4, 4), (0.25, 0.25, 0.25), ("periodic", "neumann", "periodic")),
    ((2, 3, 5), (0.5, 0.1, 0.7), ("neumann", "periodic", "neumann")),
])
def test_bordered_lu_mixed(rng, n, h, bc):
    grid = Grid(len(n), n, h, bc)
    b = rng.normal(size=grid.G)
    phi, bm = poisson.solve(grid, b)
    phi2, mu = poisson.solve_bordered(grid, b)
    assert mu == pytest.approx(np.mean(b), abs=1e-13)
    assert bm == pytest.approx(mu, abs=1e-13)
    np.testing.assert_allclose(phi, phi2, atol=1e-12 * np.abs(phi2).max())


def test_dense_periodic_operator_matches_stencil(rng):
    grid = Grid(3, (3, 4, 5), (0.2, 0.3, 0.5), ("periodic", "neumann", "periodic"))
    v = rng.normal(size=grid.G)
    L = poisson.laplacian_dense(grid)
    np.testing.assert_allclose(L @ v, poisson.laplacian(grid, v),
                               atol=1e-12 * np.abs(v).max() / 0.04)
    # the wrap-around couples the first and last cells of a periodic row
    assert L[0, 2] == pytest.approx(1 / 0.04) and L[0, 1] == pytest.approx(1 / 0.04)


@pytest.mark.parametrize("n,bc", [((64, 64), ("periodic", "neumann")),
                                  ((16, 16, 16), ("periodic", "periodic", "periodic"))])
def test_residual_vanishes_mixed(rng, n, bc):
    grid = Grid(len(n), n, tuple(1.0 / v for v in n), bc)
    b = rng.normal(size=grid.G) + 0.7
    phi, bm = poisson.solve(grid, b)
    r = (b - bm) - poisson.laplacian(grid, phi)
    assert np.linalg.norm(r) / np.linalg.norm(b - bm) < 1e-13


def test_exact_rational_periodic():
    grid = Grid(2, (3, 2), (1.0, 0.5), ("periodic", "neumann"))
    b = [Fraction(v) for v in (1, -2, 3, 5, 0, -4)]
    sol = _exact_solve(grid, b)
    phi, bm = poisson.solve(grid, np.array([float(v) for v in b]))
    assert bm == pytest.approx(float(sol[-1]), abs=1e-15)
    np.testing.assert_allclose(phi, [float(v) for v in sol[:-1]], atol=1e-14)


# ---- pseudo-spectral eigenvalues (a solver variant Sec. 3 reports as giving
# no noticeable difference) -------------------------------------------------------

def _trig_field(grid, terms):
    """f = sum_t c_t prod_a m_{t,a}(x_a) at the cell centres, with
    m = cos(pi k x / L) on a Neumann axis or cos(2 pi k x / L + theta) on a
    periodic one, and its Laplacian written out analytically."""
    X = grid.centres()
    f = np.zeros(grid.G)
    lap = np.zeros(grid.G)
    for c, modes in terms:
        prod = np.full(grid.G, float(c))
        w2 = 0.0
        for a, (k, th) in enumerate(modes):
            L = grid.length[a]
            w = (2.0 * np.pi * k / L) if grid.periodic(a) else (np.pi * k / L)
            prod = prod * np.cos(w * X[:, a] + th)
            w2 += w * w
        f += prod
        lap -= w2 * prod
    return f, lap


@pytest.mark.parametrize("n,bc,terms", [
    ((32, 64), ("neumann", "neumann"), [(1.0, ((3, 0.0), (5, 0.0))), (0.3, ((7, 0.0), (0, 0.0)))]),
    ((64, 32), ("periodic", "neumann"), [(1.0, ((3, 0.4), (2, 0.0))), (-0.7, ((32, 0.3), (1, 0.0)))]),
    ((16, 8, 32), ("periodic", "neumann", "periodic"),
     [(1.0, ((2, 1.1), (3, 0.0), (5, 0.2))), (0.5, ((8, 0.0), (0, 0.0), (16, 0.9)))]),
])
def test_spectral_solve_exact_on_trig_polynomials(n, bc, terms):
    """The pseudo-spectral solve inverts the Laplacian of a trigonometric
    polynomial exactly (the central-difference one only to O(h^2))."""
    d = len(n)
    h = tuple(1.0 / v for v in n)
    grid = Grid(d, n, h, bc, eig="spectral")
    f, lap = _trig_field(grid, terms)
    phi, bm = poisson.solve(grid, lap)
    assert abs(bm) < 1e-9 * np.abs(lap).max()
    np.testing.assert_allclose(phi, f - f.mean(), atol=1e-12 * np.abs(f).max())
    fd, _ = poisson.solve(Grid(d, n, h, bc), lap)
    assert np.abs(fd - (f - f.mean())).max() > 1e-4 * np.abs(f).max()


# ---- the regular (vertex) grid with the DCT-I (a solver variant Sec. 3 reports
# as giving no noticeable difference) ---------------------------------------------

def _vertex_eig(grid, ks):
    """cos(pi k i / (n - 1)) per axis, eigenvalue of the 3-point stencil with
    mirror ghosts about the end vertices written out."""
    idx = np.indices(grid.shape_zyx)
    v = np.ones(grid.shape_zyx)
    lam = 0.0
    for a in range(grid.d):
        i = idx[grid.d - 1 - a]
        n = grid.n[a]
        v = v * np.cos(np.pi * ks[a] * i / (n - 1))
        lam += (2 * np.cos(np.pi * ks[a] / (n - 1)) - 2) / grid.h[a] ** 2
    return v.reshape(-1), lam


@pytest.mark.parametrize("n,h,ks", [((33, 17), (1 / 32, 1 / 16), (5, 16)),
                                    ((9, 12, 7), (0.1, 0.2, 0.05), (8, 3, 1))])
def test_vertex_eigenfunctions(n, h, ks):
    grid = Grid(len(n), n, h, vertex=True)
    v, lam = _vertex_eig(grid, ks)
    np.testing.assert_allclose(poisson.laplacian(grid, v), lam * v,
                               atol=1e-12 * abs(lam) * np.abs(v).max())
    phi, bm = poisson.solve(grid, v)
    assert abs(bm) < 1e-13
    np.testing.assert_allclose(phi, v / lam, atol=1e-13 * np.abs(v / lam).max())


@pytest.mark.parametrize("n,h", [((3, 5), (0.3, 0.2)), ((4, 4, 4), (0.25,) * 3),
                                 ((2, 3, 5), (0.5, 0.1, 0.7))])
def test_vertex_bordered_lu(rng, n, h):
    grid = Grid(len(n), n, h, vertex=True)
    b = rng.normal(size=grid.G)
    phi, bm = poisson.solve(grid, b)
    phi2, mu = poisson.solve_bordered(grid, b)
    w = poisson.weights(grid)
    assert mu == pytest.approx(float(np.sum(w * b) / np.sum(w)), abs=1e-13)
    assert bm == pytest.approx(mu, abs=1e-13)
    np.testing.assert_allclose(phi, phi2, atol=1e-12 * np.abs(phi2).max())


def test_vertex_dense_operator_and_exact_solve():
    grid = Grid(2, (3, 4), (1.0, 0.5), vertex=True)
    rng = np.random.Generator(np.random.PCG64(4))
    v = rng.normal(size=grid.G)
    np.testing.assert_allclose(poisson.laplacian_dense(grid) @ v, poisson.laplacian(grid, v),
                               atol=1e-12)
    # the end vertex's mirror neighbour counts twice: row 0 has 2/h^2 on its
    # x neighbour
    assert poisson.laplacian_dense(grid)[0, 1] == pytest.approx(2.0)
    b = [Fraction(v) for v in (1, -2, 3, 5, 0, -4, 2, 2, -1, 0, 1, 3)]
    # the bordered system with trapezoid weights, in rationals
    L = poisson.laplacian_dense(grid)
    w = poisson.weights(grid)
    G = grid.G
    K = [[Fraction(L[i, j]).limit_denominator(10 ** 6) for j in range(G)] + [Fraction(1), b[i]]
         for i in range(G)]
    K.append([Fraction(wj).limit_denominator(10) for wj in w] + [Fraction(0), Fraction(0)])
    n_ = G + 1
    for c in range(n_):
        p = next(r for r in range(c, n_) if K[r][c] != 0)
        K[c], K[p] = K[p], K[c]
        for r in range(n_):
            if r != c and K[r][c] != 0:
                f = K[r][c] / K[c][c]
                K[r] = [a - f * bb for a, bb in zip(K[r], K[c])]
    sol = [K[i][G + 1] / K[i][i] for i in range(n_)]
    phi, bm = poisson.solve(grid, np.array([float(v) for v in b]))
    assert bm == pytest.approx(float(sol[-1]), abs=1e-14)
    np.testing.assert_allclose(phi, [float(v) for v in sol[:-1]], atol=1e-13)


def test_vertex_spectral_exact_on_trig():
    n, h = (33, 17), (1 / 32, 1 / 16)
    grid = Grid(2, n, h, eig="spectral", vertex=True)
    f, lap = _trig_field(grid, [(1.0, ((3, 0.0), (5, 0.0))), (0.4, ((32, 0.0), (0, 0.0)))])
    phi, _ = poisson.solve(grid, lap)
    w = poisson.weights(grid)
    np.testing.assert_allclose(phi, f - np.sum(w * f) / np.sum(w), atol=1e-12 * np.abs(f).max())
