"""Edge cases of the sub-step against the float64 oracle: no obstacle (no IB
iteration), anisotropic and non-square grids, axes shorter than the
register transform (generic path), the largest grid stencil, a warm start
of the IB force, the corner gauge, and the iteration cap."""
import math

import numpy as np
import pytest

import oracle
from oracle import projection as P
from paper_2304_14690_amd import inputs
from tests.helpers import rel_l2, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    from paper_2304_14690_amd import pcorr
    return pcorr


def custom_case(n, obstacles, k_grid, k_node, seed_nodes=21, seed_vel=22, modes=8):
    """A jittered lattice on [0, 1]^d with n[a] cells along axis a (spacing
    1/n[a]), like inputs.make_case but for any grid shape."""
    d = len(n)
    h = tuple(1.0 / v for v in n)
    lat = inputs.jittered_lattice(n, h, seed_nodes)
    inside = np.zeros(lat.shape[1], dtype=bool)
    for ob in obstacles:
        inside |= ob.inside(lat.T)
    kind = np.where(inside, inputs.KIND_V, inputs.KIND_F).astype(np.uint8)
    delta = math.exp(sum(math.log(v) for v in h) / d)
    surf = [ob.surface_points(delta) for ob in obstacles]
    x = lat
    if surf:
        bp = np.concatenate(surf)
        x = np.concatenate([lat, bp.T], axis=1)
        kind = np.concatenate([kind, np.full(bp.shape[0], inputs.KIND_B, np.uint8)])
    x = np.ascontiguousarray(x)
    u = inputs.fourier_velocity(x, modes, seed_vel)
    u[:, kind == inputs.KIND_V] = 0.0
    return inputs.Case("custom", d, tuple(n), h, x, kind, np.ascontiguousarray(u), 1.0,
                       k_grid, k_node, list(obstacles))


CIRCLE = [inputs.Obstacle("circle", (0.45, 0.55), (0.17,))]
SPHERE = [inputs.Obstacle("sphere", (0.5, 0.45, 0.5), (0.22,))]
CASES = {
    "2d_no_obstacle": lambda: custom_case((64, 64), [], 12, 12),
    "3d_no_obstacle": lambda: custom_case((32, 32, 32), [], 27, 27),
    "2d_aniso_64x128": lambda: custom_case((64, 128), CIRCLE, 16, 16),
    "2d_small_16": lambda: custom_case((16, 16), [inputs.Obstacle("circle", (0.5, 0.5),
                                                                   (0.25,))], 12, 12),
    "2d_rect_16x32": lambda: custom_case((16, 32), CIRCLE, 12, 12),
    "3d_mixed_16x32x32": lambda: custom_case((16, 32, 32), SPHERE, 27, 27),
    "2d_k32": lambda: custom_case((64, 64), CIRCLE, 32, 16),
}
_CACHE = {}


def case_and_stencils(name):
    if name not in _CACHE:
        c = CASES[name]()
        grid = oracle.Grid(c.d, c.n, c.h)
        st = P.build_stencils(grid, c.x.T.copy(), c.kind, c.k_grid, c.k_node)
        _CACHE[name] = (c, grid, st)
    return _CACHE[name]


def run(pc, c, mode, **kw):
    import torch
    plan = pc.Plan(c.d, c.n, c.h)
    geom = pc.wls_build(plan, torch.from_numpy(c.x).cuda(), torch.from_numpy(c.kind).cuda(),
                        c.k_grid, c.k_node, want_f32=(mode == pc.PC_F32))
    dtype = torch.float32 if mode == pc.PC_F32 else torch.float64
    u = torch.from_numpy(c.u).to(dtype).cuda()
    uo = torch.empty_like(u)
    p = torch.empty(c.G, dtype=dtype, device="cuda")
    g = kw.pop("g", None)
    rc, st = pc.pressure_correct(geom, plan, mode, u, 1.0, uo, p, g=g, **kw)
    torch.cuda.synchronize()
    return rc, st, to_np(uo), to_np(p)


@pytest.mark.parametrize("name", list(CASES))
def test_edge_case_all_modes(pc, name):
    c, grid, st = case_and_stencils(name)
    ref = P.pressure_correct(st, c.u.T.copy())
    rc, stats, uo, p = run(pc, c, pc.PC_F64)
    eu, ep = rel_l2(uo, ref["u_new"].T), rel_l2(p, ref["p"])
    print(f"{name}: n_it {stats['n_it']} (oracle {ref['n_it']}), u {eu:.2e} p {ep:.2e}")
    assert rc == 0 and stats["n_it"] == ref["n_it"]
    if st.ib.size == 0:
        assert stats["n_it"] == 1
    assert eu <= 1e-11 and ep <= 1e-11
    assert np.all(uo[:, st.ib] == 0.0)
    for mode, tol in ((pc.PC_MIXED, 1e-10), (pc.PC_F32, 5e-5)):
        u_in = c.u if mode != pc.PC_F32 else c.u.astype(np.float32).astype(np.float64)
        r2 = P.pressure_correct(st, u_in.T.copy(), fixed_it=ref["n_it"])
        rc, stats, uo, p = run(pc, c, mode, fixed_it=ref["n_it"])
        assert rel_l2(uo, r2["u_new"].T) <= tol and rel_l2(p, r2["p"]) <= tol


def test_warm_start_gauge_and_cap(pc):
    import torch
    c, grid, st = case_and_stencils("2d_aniso_64x128")
    rng = np.random.Generator(np.random.PCG64(8))
    g0 = 0.1 * rng.standard_normal((st.ib.size, c.d))
    ref = P.pressure_correct(st, c.u.T.copy(), g0=g0)
    g = torch.from_numpy(g0.T.copy()).cuda()
    rc, stats, uo, p = run(pc, c, pc.PC_F64, g=g, gauge=1)
    assert stats["n_it"] == ref["n_it"] and rc == 0
    assert rel_l2(uo, ref["u_new"].T) <= 1e-11
    # gauge 1: the pressure is zero in the first cell, otherwise the same field
    assert p[0] == 0.0
    assert rel_l2(p, ref["p"] - ref["p"][0]) <= 1e-11
    assert rel_l2(to_np(g).T, ref["g_ib"]) <= 1e-11
    # a cap below the needed iterations: warning, not converged, the capped result
    capped = P.pressure_correct(st, c.u.T.copy(), fixed_it=2)
    rc, stats, uo, p = run(pc, c, pc.PC_F64, max_it=2, tol=1e-14)
    assert rc == pc.PC_WARN_IB_NOT_CONVERGED and stats["converged"] == 0
    assert stats["n_it"] == 2
    assert rel_l2(uo, capped["u_new"].T) <= 1e-11
