"""GPU parity of the pseudo-spectral variant of the Poisson solve (one of the
solver variants Sec. 3 reports as giving no noticeable difference): the
eigenvalue of each transform mode is minus its squared wavenumber.  Solves
against the oracle (float64 1e-11, float32 5e-5) on Neumann, periodic and
mixed boxes, both register plans and the generic kernels (periodic and
Neumann axes that are short or not powers of two); exact inversion of
a trigonometric polynomial's analytic Laplacian at full size; the sub-step
with a pseudo-spectral plan against the oracle; PC_MIXED is refused (its
defect correction evaluates the 3-point Laplacian)."""
import numpy as np
import pytest

import oracle
from oracle import Grid, poisson, projection as P
from paper_2304_14690_amd import inputs
from tests.helpers import rel_l2, to_np

pytestmark = pytest.mark.gpu

PE, NE = "periodic", "neumann"
CASES = [
    ((64, 64), (NE, NE)), ((2048, 2048), (NE, NE)), ((64, 32), (PE, NE)), ((16, 64), (NE, PE)),
    ((32, 16, 64), (PE, NE, PE)), ((256, 256, 256), (NE, NE, NE)), ((64, 64, 64), (PE, PE, PE)),
    # generic kernels: periodic and Neumann axes that are short or not powers of two
    ((400, 400), (PE, PE)), ((400, 402), (PE, NE)), ((280, 480), (NE, NE)), ((16, 64), (PE, NE)),
    ((48, 40, 36), (PE, PE, NE)),
]


@pytest.fixture(scope="module")
def pc():
    from paper_2304_14690_amd import pcorr
    return pcorr


@pytest.mark.parametrize("n,bc", CASES, ids=["x".join(map(str, n)) + "-" + "".join(b[0] for b in bc)
                                             for n, bc in CASES])
def test_spectral_solve_matches_oracle(pc, n, bc):
    import torch
    d = len(n)
    h = tuple(1.0 / v for v in n)
    grid = Grid(d, n, h, bc, eig="spectral")
    plan = pc.Plan(d, n, h, bc=bc, eig="spectral")
    rng = np.random.Generator(np.random.PCG64(12))
    b = rng.normal(size=grid.G) + 0.2
    ref, bm_ref = poisson.solve(grid, b)
    bt = torch.from_numpy(b).cuda()
    phi = torch.empty_like(bt)
    bm = torch.zeros(1, dtype=torch.float64, device="cuda")
    pc.poisson_fft_solve(plan, bt, phi, pc.PC_F64, bmean=bm)
    b32 = torch.from_numpy(b.astype(np.float32)).cuda()
    phi32 = torch.empty_like(b32)
    pc.poisson_fft_solve(plan, b32, phi32, pc.PC_F32)
    torch.cuda.synchronize()
    ref32, _ = poisson.solve(grid, b.astype(np.float32).astype(np.float64))
    e64, e32 = rel_l2(to_np(phi), ref), rel_l2(to_np(phi32), ref32)
    print(f"spectral {n} {bc}: f64 {e64:.2e} f32 {e32:.2e}")
    assert e64 <= 1e-11 and e32 <= 5e-5
    assert abs(bm.item() - bm_ref) <= 1e-12 * max(1.0, abs(bm_ref))
    if d == 2 and n[0] == 64:
        ws = pc.Workspace(plan, None, pc.PC_MIXED)
        with pytest.raises(pc.PcError) as e:
            pc.poisson_fft_solve(plan, bt, phi, pc.PC_MIXED, ws=ws)
        assert e.value.code == pc.PC_ERR_INVALID_ARG


@pytest.mark.parametrize("n,bc,modes", [
    ((2048, 2048), (NE, NE), ((1021, 0.0), (6, 0.0))),
    ((2048, 2048), (PE, NE), ((1024, 0.7), (2047, 0.0))),
    ((256, 256, 256), (PE, NE, PE), ((3, 0.4), (200, 0.0), (128, 1.3))),
])
def test_spectral_inverts_trig_laplacian(pc, n, bc, modes):
    """f = prod_a cos(w_a x_a + theta_a) with the axis's wavenumber w (pi k / L
    on a Neumann axis, 2 pi k / L on a periodic one): the solve of its
    analytic Laplacian -(sum w^2) f returns f."""
    import torch
    d = len(n)
    h = tuple(1.0 / v for v in n)
    idx = np.indices(tuple(reversed(n)))
    f = np.ones(tuple(reversed(n)))
    w2 = 0.0
    for a in range(d):
        x = (idx[d - 1 - a] + 0.5) * h[a]
        k, th = modes[a]
        w = (2 * np.pi * k if bc[a] == PE else np.pi * k) / (n[a] * h[a])
        f = f * np.cos(w * x + th)
        w2 += w * w
    f = f.reshape(-1)
    plan = pc.Plan(d, n, h, bc=bc, eig="spectral")
    bt = torch.from_numpy(-w2 * f).cuda()
    pc.poisson_fft_solve(plan, bt, bt, pc.PC_F64)
    torch.cuda.synchronize()
    err = rel_l2(to_np(bt), f - f.mean())
    # rounding spread into other modes is amplified by |lambda| / |lambda_min|
    lam_min = min(((2 if bc[a] == PE else 1) * np.pi / (n[a] * h[a])) ** 2 for a in range(d))
    bound = 4e-16 * np.log2(f.size) * w2 / lam_min
    print(f"trig {n} {bc} {modes}: rel L2 {err:.2e} (bound {bound:.2e})")
    assert err <= max(1e-13, bound)


@pytest.mark.parametrize("name", ["cfg1", "2d_periodic"])
def test_spectral_sub_step(pc, name):
    import torch
    if name == "cfg1":
        c, bc = inputs.config1(), None
    else:
        bc = (PE, NE)
        c = inputs.make_case("sp", 2, 64, [inputs.Obstacle("circle", (0.05, 0.5), (0.15,))],
                             16, 16, 8, 51, 52, bc=bc)
    grid = Grid(c.d, c.n, c.h, bc, eig="spectral")
    st = P.build_stencils(grid, c.x.T.copy(), c.kind, c.k_grid, c.k_node)
    ref = P.pressure_correct(st, c.u.T.copy(), solver=lambda b: poisson.solve(grid, b))
    plan = pc.Plan(c.d, c.n, c.h, bc=bc, eig="spectral")
    geom = pc.wls_build(plan, torch.from_numpy(c.x).cuda(), torch.from_numpy(c.kind).cuda(),
                        c.k_grid, c.k_node)
    u = torch.from_numpy(c.u).cuda()
    uo = torch.empty_like(u)
    p = torch.empty(grid.G, dtype=torch.float64, device="cuda")
    rc, stats = pc.pressure_correct(geom, plan, pc.PC_F64, u, 1.0, uo, p)
    torch.cuda.synchronize()
    eu, ep = rel_l2(to_np(uo), ref["u_new"].T), rel_l2(to_np(p), ref["p"])
    print(f"{name}: n_it {stats['n_it']} (oracle {ref['n_it']}), u {eu:.2e} p {ep:.2e}")
    assert rc == 0 and stats["n_it"] == ref["n_it"] and eu <= 1e-11 and ep <= 1e-11
    with pytest.raises(pc.PcError):
        pc.pressure_correct(geom, plan, pc.PC_MIXED, u, 1.0, uo, p)
