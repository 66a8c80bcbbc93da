"""Pins for oracle.projection: the whole pressure-correction step against
independent formulations.

  * no obstacle + divergence-free quadratic velocity: WLS reproduces the
    (zero) divergence exactly, so phi = 0 and u^{n+1} = u* (Sec. 2.3);
  * dense-matrix pipeline: the transfers assembled as dense matrices and the
    Poisson solve replaced by the pseudo-inverse of the dense operator,
    iterated the same number of times (Eqs. 18-20, Sec. 2.3 iteration);
  * the IB iteration's limit equals the dense solution of its linear fixed
    point;
  * exact zeros at boundary and virtual points (Eqs. 18-19 cancel);
  * linearity at a fixed iteration count;
  * the convergence sums on hand-made data.
"""
import numpy as np
import pytest

from oracle import Grid, poisson, projection as P
from paper_2304_14690_amd import inputs


def _tiny_case(seed=7, N=8, R=0.2):
    return inputs.make_case("tiny", 2, N, [inputs.Obstacle("circle", (0.5, 0.5), (R,))],
                            12, 12, 4, seed, seed + 1)


def _stencils(c):
    grid = Grid(c.d, c.n, c.h)
    return P.build_stencils(grid, c.x.T.copy(), c.kind, c.k_grid, c.k_node)


def _dense(st, M, d):
    G = st.grid.G
    D = np.zeros((G, d * M))
    for p in range(G):
        for a in range(d):
            for i, node in enumerate(st.grid_idx[p]):
                D[p, a * M + node] += st.grid_coef[p, a, i]
    Gn = np.zeros((d * M, G))
    for n in range(M):
        for a in range(d):
            for j, q in enumerate(st.node_idx[n]):
                Gn[a * M + n, q] += st.node_coef[n, a, j]
    return D, Gn


def test_divergence_free_quadratic_no_obstacle(rng):
    for d, N, k in ((2, 32, 16), (3, 10, 27)):
        c = inputs.make_case("free", d, N, [], k, k, 1, 3, 4)
        x = c.x.T
        # u = curl of a cubic potential: divergence-free and quadratic
        A = rng.normal(size=(d, d, d))
        if d == 2:
            # psi = sum A_ijk x_i x_j x_k ; u = (psi_y, -psi_x)
            def grad_psi(x):
                g = np.zeros_like(x)
                for i in range(2):
                    for j in range(2):
                        for kk in range(2):
                            t = A[i, j, kk]
                            g[:, i] += t * x[:, j] * x[:, kk]
                            g[:, j] += t * x[:, i] * x[:, kk]
                            g[:, kk] += t * x[:, i] * x[:, j]
                return g
            gp = grad_psi(x)
            u = np.stack([gp[:, 1], -gp[:, 0]], axis=1)
        else:
            # u = curl(a) with a_m quadratic -> u linear, divergence-free
            B = rng.normal(size=(3, 3, 3))
            a_grad = np.einsum("mij,tj->tmi", B + B.transpose(0, 2, 1), x)
            u = np.stack([a_grad[:, 2, 1] - a_grad[:, 1, 2],
                          a_grad[:, 0, 2] - a_grad[:, 2, 0],
                          a_grad[:, 1, 0] - a_grad[:, 0, 1]], axis=1)
        st = _stencils(c)
        r = P.pressure_correct(st, u)
        scale = np.abs(u).max() / c.h[0]
        assert np.abs(r["b_u"]).max() < 1e-9 * scale
        assert np.abs(u - r["u_new"]).max() < 1e-9 * np.abs(u).max()
        assert r["n_it"] == 1


def test_dense_pipeline_agrees():
    c = _tiny_case()
    st = _stencils(c)
    M, d = c.M, c.d
    u = c.u.T.copy()
    r = P.pressure_correct(st, u)
    n_it = r["n_it"]
    assert n_it >= 2
    D, Gn = _dense(st, M, d)
    Lp = np.linalg.pinv(poisson.laplacian_dense(st.grid), rcond=1e-12)
    uf = u.T.reshape(-1)                       # [a*M + n]
    ibmask = np.zeros(M, bool)
    ibmask[st.ib] = True
    ibrows = np.concatenate([a * M + np.flatnonzero(ibmask) for a in range(d)])
    g = np.zeros(d * M)
    for it in range(n_it):
        phi = Lp @ (D @ (uf + g))
        grad = Gn @ phi
        g[ibrows] = -uf[ibrows] + grad[ibrows]
    unew = uf - grad
    unew[ibrows] = 0.0
    np.testing.assert_allclose(r["phi"], phi, atol=1e-12 * np.abs(phi).max())
    np.testing.assert_allclose(r["u_new"].T.reshape(-1), unew, atol=1e-12 * np.abs(unew).max())
    np.testing.assert_allclose(r["p"], 2 * phi / 3, atol=1e-12 * np.abs(phi).max())


def test_ib_limit_is_linear_fixed_point():
    c = _tiny_case(seed=11)
    st = _stencils(c)
    M, d = c.M, c.d
    u = c.u.T.copy()
    D, Gn = _dense(st, M, d)
    Lp = np.linalg.pinv(poisson.laplacian_dense(st.grid), rcond=1e-12)
    uf = u.T.reshape(-1)
    ibmask = np.zeros(M, bool)
    ibmask[st.ib] = True
    rows = np.concatenate([a * M + np.flatnonzero(ibmask) for a in range(d)])
    T = Gn[rows] @ Lp @ D[:, rows]
    rhs = -uf[rows] + Gn[rows] @ Lp @ D @ uf
    g_star = np.linalg.solve(np.eye(rows.size) - T, rhs)
    assert np.max(np.abs(np.linalg.eigvals(T))) < 1.0
    r = P.pressure_correct(st, u, fixed_it=300)
    g_it = r["g_ib"].T.reshape(-1)
    np.testing.assert_allclose(g_it, g_star, atol=1e-9 * np.abs(g_star).max())


def test_exact_zero_on_ib_and_linearity(rng):
    c = _tiny_case(seed=5, N=16)
    st = _stencils(c)
    u = c.u.T.copy()
    v = rng.normal(size=u.shape)
    v[c.kind == inputs.KIND_V] = 0.0
    r1 = P.pressure_correct(st, u, fixed_it=4)
    assert np.all(r1["u_new"][st.ib] == 0.0)
    r2 = P.pressure_correct(st, v, fixed_it=4)
    r3 = P.pressure_correct(st, 2.0 * u - 0.5 * v, fixed_it=4)
    want = 2.0 * r1["u_new"] - 0.5 * r2["u_new"]
    np.testing.assert_allclose(r3["u_new"], want, atol=1e-12 * np.abs(want).max())


def test_ib_sums_by_hand():
    g_new = np.array([[3.0, 4.0], [0.0, 1.0]])
    g_old = np.array([[0.0, 2.0], [1.0, 0.0]])
    num, den = P.ib_sums(g_new, g_old)
    assert num == (5.0 - 2.0) ** 2 + (1.0 - 1.0) ** 2
    assert den == 4.0 + 1.0


def test_near_list_and_split_rhs():
    """Grid points outside the near list never see the force: a full
    evaluation of D(u*+g) equals the split form."""
    c = _tiny_case(seed=3, N=16)
    st = _stencils(c)
    u = c.u.T.copy()
    r = P.pressure_correct(st, u, fixed_it=3)
    g = np.zeros_like(u)
    g[st.ib] = r["history"] and P.pressure_correct(st, u, fixed_it=2)["g_ib"]
    full = P.div_to_grid(st, u + g)
    np.testing.assert_allclose(r["b_last"], full, atol=1e-12 * np.abs(full).max())
    far = np.setdiff1d(np.arange(st.grid.G), st.near)
    assert np.all(P.div_to_grid(st, g)[far] == 0.0)


def test_sample_stencils_equal_full_build():
    """The subset builder gives exactly the rows of the full build."""
    from paper_2304_14690_amd import inputs
    c = inputs.config1()
    grid = Grid(c.d, c.n, c.h)
    x = c.x.T.copy()
    st = P.build_stencils(grid, x, c.kind, c.k_grid, c.k_node)
    rng = np.random.Generator(np.random.PCG64(3))
    gp = rng.choice(grid.G, 50, replace=False)
    nd = np.concatenate([rng.choice(c.M, 40, replace=False), st.ib[:10]])
    gi, gcf, ni, ncf = P.sample_stencils(grid, x, c.k_grid, c.k_node, gp, nd)
    np.testing.assert_array_equal(gi, st.grid_idx[gp])
    np.testing.assert_array_equal(gcf, st.grid_coef[gp])
    np.testing.assert_array_equal(ni, st.node_idx[nd])
    np.testing.assert_array_equal(ncf, st.node_coef[nd])


def _dense_history(st, u, K):
    """The IB iteration of Sec. 2.3 written out with dense matrices (the
    transfers assembled entry by entry, the Poisson solve as the
    pseudo-inverse of the dense Laplacian), and the criterion sums of every
    iteration added up point by point: [(num_1, den_1), ..., (num_K, den_K)]."""
    M, d = u.shape
    D, Gn = _dense(st, M, d)
    Lp = np.linalg.pinv(poisson.laplacian_dense(st.grid), rcond=1e-12)
    uf = u.T.reshape(-1)
    g = np.zeros(d * M)
    out = []
    for _ in range(K):
        grad = Gn @ (Lp @ (D @ (uf + g)))
        num = den = 0.0
        for n in st.ib:
            new = [-uf[a * M + n] + grad[a * M + n] for a in range(d)]
            old = [g[a * M + n] for a in range(d)]
            mag_new = np.sqrt(sum(v * v for v in new))
            mag_old = np.sqrt(sum(v * v for v in old))
            num += (mag_new - mag_old) ** 2
            den += mag_old ** 2
            for a in range(d):
                g[a * M + n] = new[a]
        out.append((num, den))
    return out


def test_ib_stops_at_first_qualifying_iteration():
    """The loop of Sec. 2.3 stops at the FIRST iteration whose criterion
    holds (iteration 1 from a zero force has a zero denominator and never
    does), reports convergence only then, and stops unconverged at the cap."""
    c = _tiny_case(seed=13)
    st = _stencils(c)
    u = c.u.T.copy()
    K = 12
    hist = _dense_history(st, u, K)
    assert hist[0][1] == 0.0
    ratios = [num / den if den > 0 else np.inf for num, den in hist]

    def first_stop(tol):
        for it, (num, den) in enumerate(hist, start=1):
            if num < tol * den or num == 0.0:
                return it
        return None

    # the default tolerance, and tolerances placed between consecutive
    # ratios so that a stop one iteration early or late changes n_it
    tols = [1e-3]
    for j in range(1, K - 1):
        lo, hi = sorted((ratios[j], ratios[j + 1]))
        if lo > 0 and hi / lo > 1.01:
            tols.append(float(np.sqrt(lo * hi)))
    assert len(tols) >= 4
    for tol in tols:
        want = first_stop(tol)
        assert want is not None and want >= 2
        r = P.pressure_correct(st, u, tol=tol)
        assert r["n_it"] == want, (tol, r["n_it"], want)
        assert r["converged"]
        num, den = r["history"][-1]
        np.testing.assert_allclose([num, den], hist[want - 1], rtol=1e-9)
        if want > 2:
            # capped one short of the stop: unconverged, at the cap
            rc = P.pressure_correct(st, u, tol=tol, max_it=want - 1)
            assert rc["n_it"] == want - 1 and not rc["converged"]
        # capped exactly at the stop: converged
        rc = P.pressure_correct(st, u, tol=tol, max_it=want)
        assert rc["n_it"] == want and rc["converged"]


def test_sample_stencils_window_equals_full_search():
    """The windowed candidate search gives the rows of the unrestricted one,
    and refuses a window the k-th neighbour reaches."""
    from paper_2304_14690_amd import inputs
    for c in (inputs.config1(),
              inputs.make_case("w3", 3, 12, [inputs.Obstacle("sphere", (0.4, 0.5, 0.5), (0.2,))],
                               27, 27, 4, 21, 22)):
        grid = Grid(c.d, c.n, c.h)
        x = c.x.T.copy()
        rng = np.random.Generator(np.random.PCG64(5))
        gp = rng.choice(grid.G, 60, replace=False)
        corners = np.array([0, grid.G - 1])
        gp = np.unique(np.concatenate([gp, corners]))
        nd = rng.choice(c.M, 30, replace=False)
        full = P.sample_stencils(grid, x, c.k_grid, c.k_node, gp, nd)
        win = P.sample_stencils(grid, x, c.k_grid, c.k_node, gp, nd, window=4 * c.h[0])
        for a, b in zip(full, win):
            np.testing.assert_array_equal(a, b)
        cand = P.window_candidates(grid.centres()[gp[:3]], x, 4 * c.h[0])
        assert cand.size < c.M and np.all(np.diff(cand) > 0)
        # every node closer than the window to a target is a candidate
        t = grid.centres()[gp[:3]]
        dist = np.sqrt(((x[None, :, :] - t[:, None, :]) ** 2).sum(-1)).min(0)
        assert np.all(np.isin(np.flatnonzero(dist < 4 * c.h[0]), cand))
        with pytest.raises(ValueError):
            P.sample_stencils(grid, x, c.k_grid, c.k_node, gp, nd, window=1.0 * c.h[0])
