"""Pins for oracle.momentum (the first fractional step, Eq. 3): the
known-value WLS rows against the literal matrices of Eqs. (10)-(15) and
against exact derivatives of quadratics (2D and 3D), the self-excluding
neighbour search against exhaustion, and R^n against the analytic convection
and diffusion of a quadratic field."""
import numpy as np
import pytest

from oracle import knn, momentum, wls


def _quad(rng, d):
    A = rng.normal(size=(d, d))
    H = A + A.T
    g0 = rng.normal(size=d)
    c0 = rng.normal()

    def f(x):
        return c0 + x @ g0 + 0.5 * np.einsum("ti,ij,tj->t", x, H, x)

    def grad(x):
        return g0[None, :] + x @ H
    return f, grad, H


def test_known_rows_match_literal_equations(rng):
    """2D: the scaled QR rows equal C^-1 A of Eqs. (14)-(15) written out
    (oracle.wls.wls5_rows) for the same neighbours and support."""
    tgt = np.array([[0.4, 0.6]])
    nbrs = tgt + rng.uniform(-1, 1, size=(14, 2)) * 0.03
    idx = np.arange(14)[None, :]
    d2 = knn.exact_d2(tgt, nbrs, idx)
    o = np.lexsort((idx, d2), axis=-1)
    idx, d2 = np.take_along_axis(idx, o, -1), np.take_along_axis(d2, o, -1)
    rows, ht, sing = momentum.wls_known_rows(tgt, nbrs, idx, d2, 0.01)
    lit = wls.wls5_rows(tgt[0], nbrs[idx[0]], float(ht[0]))
    np.testing.assert_allclose(rows[0], lit, rtol=1e-9, atol=1e-9 * np.abs(lit).max())
    assert not sing[0]


@pytest.mark.parametrize("d,k", [(2, 12), (3, 20)])
def test_known_rows_reproduce_quadratics(rng, d, k):
    x = rng.uniform(size=(400, d))
    f, grad, H = _quad(rng, d)
    idx, coef, sing = momentum.self_stencils(x, k, delta=x.shape[0] ** (-1.0 / d))
    assert not sing.any()
    df = f(x)[idx] - f(x)[:, None]
    g = np.einsum("mak,mk->ma", coef[:, :d, :], df)
    lap = np.einsum("mk,mk->m", coef[:, d, :], df)
    np.testing.assert_allclose(g, grad(x), atol=1e-9 * np.abs(grad(x)).max())
    np.testing.assert_allclose(lap, np.trace(H), atol=1e-7 * np.abs(H).max())


@pytest.mark.parametrize("L", [None, (1.0, None), (1.0, 1.0, 1.0)])
def test_self_neighbours_by_exhaustion(rng, L):
    d = 2 if L is None or len(L) == 2 else 3
    x = rng.uniform(size=(300, d))
    idx, _, _ = momentum.self_stencils(x, 12, 0.05, lengths=L)
    ib, _ = knn.knn_brute(x, x, 13, lengths=L)
    for m in range(x.shape[0]):
        want = [j for j in ib[m] if j != m][:12]
        assert list(idx[m]) == want


def test_rhs_of_quadratic_field(rng):
    """u quadratic: grad u and lap u are exact, so R = -u.grad u + nu lap u
    + F holds to rounding."""
    d = 2
    x = rng.uniform(size=(500, d))
    f1, g1, H1 = _quad(rng, d)
    f2, g2, H2 = _quad(rng, d)
    u = np.stack([f1(x), f2(x)], axis=1)
    idx, coef, _ = momentum.self_stencils(x, 14, 0.045)
    nu, F = 0.3, np.array([0.1, -2.0])
    R = momentum.momentum_rhs(idx, coef, u, nu, F)
    G = np.stack([g1(x), g2(x)], axis=2)            # G[m, a, c] = d_a u_c
    want = -np.einsum("ma,mac->mc", u, G) + nu * np.array([np.trace(H1), np.trace(H2)]) + F
    np.testing.assert_allclose(R, want, atol=1e-6 * np.abs(want).max())


def test_predict_and_pressure_term():
    u = np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]])
    R = np.array([[0.5, 0.0], [1.0, 1.0], [2.0, 2.0]])
    Rp = np.array([[1.0, 1.0], [0.0, 0.0], [1.0, 1.0]])
    kind = np.array([0, 1, 2], dtype=np.uint8)
    us = momentum.predict(u, R, Rp, 0.1, kind)
    np.testing.assert_allclose(us[0], [1.0 + 0.1 * (0.75 - 0.5), 2.0 - 0.05])
    np.testing.assert_allclose(us[1], [3.0 + 0.15, 4.0 + 0.15])
    assert np.all(us[2] == 0.0)
    us1 = momentum.predict(u, R, None, 0.1, kind)
    np.testing.assert_allclose(us1[1], [3.1, 4.1])
    g = np.zeros_like(u)
    g[2] = [0.3, 0.3]
    rn = momentum.r_prev_next(R, us, u, g, 0.1)
    np.testing.assert_allclose(rn, R - (2.0 / 0.3) * (us - u + g), rtol=0, atol=1e-12)


def test_taylor_green_decay():
    """The Taylor-Green vortex u = (sin 2 pi x cos 2 pi y, -cos 2 pi x sin 2 pi y)
    exp(-8 pi^2 nu t) is an exact solution on the periodic unit box (its
    convection is a pressure gradient).  Both fractional steps together keep
    its shape and decay rate: after 20 steps the velocity matches the exact
    field to second order in h and dt (1% here), while the first step alone
    without the projection does not."""
    import oracle
    from oracle import projection as P
    from paper_2304_14690_amd import inputs
    n = (48, 48)
    h = (1 / 48, 1 / 48)
    bc = ("periodic", "periodic")
    grid = oracle.Grid(2, n, h, bc)
    x = inputs.jittered_lattice(n, h, 61).T.copy()
    kind = np.zeros(x.shape[0], np.uint8)
    st = P.build_stencils(grid, x, kind, 16, 16)
    L = (1.0, 1.0)
    sidx, scoef, sing = momentum.self_stencils(x, 16, 1 / 48, lengths=L)
    assert not sing.any()

    def tg(t, nu):
        a = np.exp(-8 * np.pi ** 2 * nu * t)
        return a * np.stack([np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1]),
                             -np.cos(2 * np.pi * x[:, 0]) * np.sin(2 * np.pi * x[:, 1])], 1)
    nu, dt, steps = 0.01, 0.004, 20
    u, _ = momentum.advance(st, sidx, scoef, kind, tg(0.0, nu), dt, nu, steps)
    exact = tg(dt * steps, nu)
    err = np.linalg.norm(u - exact) / np.linalg.norm(exact)
    decay = np.linalg.norm(u) / np.linalg.norm(tg(0.0, nu))
    want = np.exp(-8 * np.pi ** 2 * nu * dt * steps)
    print(f"TG: rel err {err:.2e}, decay {decay:.5f} (exact {want:.5f})")
    assert err < 1e-2 and abs(decay - want) < 1e-2 * want
    # without the projection the convection is not balanced
    u2 = tg(0.0, nu)
    for _ in range(steps):
        u2 = momentum.predict(u2, momentum.momentum_rhs(sidx, scoef, u2, nu), None, dt, kind)
    assert np.linalg.norm(u2 - exact) / np.linalg.norm(exact) > 5 * err
