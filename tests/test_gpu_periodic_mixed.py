"""Periodic axes of any even length: the 400 x 400 doubly periodic grid of
the flow over a square and the horizontally periodic channels of Sec. 3
(400 x 402, 280 x 480), short periodic axes (8, 10, 16 cells) and 3D boxes
that mix them with Neumann axes.  The packed real DFT of such an axis runs
on the mixed-radix kernel; the WLS gathers wrap node blocks with division
instead of masks.  Against the float64 oracle: the solve in every precision
(float64 1e-11, float32 5e-5, float32 transforms + float64 correction
1e-10, relative L2), a discrete eigenfunction at 400 x 400 including the
Nyquist mode, and the whole sub-step with obstacles that cross a periodic
face (index sets bit-exact, coefficients 1e-12)."""
import numpy as np
import pytest

from oracle import Grid, poisson, projection as P
from paper_2304_14690_amd import inputs
from tests.helpers import rel_l2, to_np
from tests.test_gpu_periodic import _case, check_stencils, check_transfers

pytestmark = pytest.mark.gpu

PE, NE = "periodic", "neumann"
SOLVES = [
    ((400, 400), (PE, PE)),
    ((400, 402), (PE, NE)),
    ((280, 480), (NE, PE)),
    ((10, 12), (PE, PE)),
    ((8, 16), (PE, PE)),
    ((16, 64), (PE, NE)),
    ((2048, 402), (PE, PE)),
    ((48, 40, 36), (PE, PE, NE)),
    ((26, 18, 14), (PE, NE, PE)),
    ((64, 134, 32), (NE, PE, PE)),
    ((8, 8, 8), (PE, PE, PE)),
    ((10, 8, 12), (PE, NE, PE)),
    ((4094, 8), (PE, NE)),
]
SIDS = ["x".join(map(str, n)) + "-" + "".join(b[0] for b in bc) for n, bc in SOLVES]


@pytest.fixture(scope="module")
def pc():
    from paper_2304_14690_amd import pcorr
    return pcorr


@pytest.mark.parametrize("n,bc", SOLVES, ids=SIDS)
def test_periodic_any_even_solve(pc, n, bc):
    import torch
    d = len(n)
    h = tuple(1.0 / v for v in n)
    grid = Grid(d, n, h, bc)
    plan = pc.Plan(d, n, h, bc=bc)
    rng = np.random.Generator(np.random.PCG64(23))
    b = rng.normal(size=grid.G) + 0.4
    ref, bm_ref = poisson.solve(grid, b)
    bt = torch.from_numpy(b).cuda()
    phi = torch.empty_like(bt)
    bm = torch.zeros(1, dtype=torch.float64, device="cuda")
    pc.poisson_fft_solve(plan, bt, phi, pc.PC_F64, bmean=bm)
    b32 = torch.from_numpy(b.astype(np.float32)).cuda()
    phi32 = torch.empty_like(b32)
    pc.poisson_fft_solve(plan, b32, phi32, pc.PC_F32)
    ws = pc.Workspace(plan, None, pc.PC_MIXED)
    phim = torch.empty_like(bt)
    pc.poisson_fft_solve(plan, bt, phim, pc.PC_MIXED, sweeps=2, ws=ws)
    torch.cuda.synchronize()
    ref32, _ = poisson.solve(grid, b.astype(np.float32).astype(np.float64))
    e64, e32, em = rel_l2(to_np(phi), ref), rel_l2(to_np(phi32), ref32), rel_l2(to_np(phim), ref)
    print(f"{n} {bc}: f64 {e64:.2e} f32 {e32:.2e} mixed {em:.2e}")
    assert e64 <= 1e-11 and e32 <= 5e-5 and em <= 1e-10
    assert abs(bm.item() - bm_ref) <= 1e-12 * max(1.0, abs(bm_ref))


@pytest.mark.parametrize("ks,ph", [((200, 7), (0.3, 1.1)), ((1, 199), (2.0, 0.0))])
def test_periodic_400_eigenfunction(pc, ks, ph):
    """cos(2 pi k i / n + theta) on both axes of the 400 x 400 periodic
    grid: the solve returns v / lambda, lambda from the wrap-around 3-point
    stencil (k = 200 is the Nyquist mode, whose sine part vanishes)."""
    import torch
    n, h = (400, 400), (1 / 400, 1 / 400)
    j, i = np.indices((n[1], n[0]))
    v = (np.cos(2 * np.pi * ks[0] * i / n[0] + ph[0]) *
         np.cos(2 * np.pi * ks[1] * j / n[1] + ph[1])).reshape(-1)
    lam = sum((2 * np.cos(2 * np.pi * ks[a] / n[a]) - 2) / h[a] ** 2 for a in range(2))
    plan = pc.Plan(2, n, h, bc=(PE, PE))
    bt = torch.from_numpy(v).cuda()
    pc.poisson_fft_solve(plan, bt, bt, pc.PC_F64)
    torch.cuda.synchronize()
    err = rel_l2(to_np(bt), v / lam)
    lam_min = 4 / h[0] ** 2 * np.sin(np.pi / n[0]) ** 2
    bound = 4e-16 * np.log2(v.size) * abs(lam) / lam_min
    print(f"eigenfunction 400^2 {ks}: rel L2 {err:.2e} (bound {bound:.2e})")
    assert err <= max(1e-13, bound)


CASES = {
    # flow over a square, periodic both ways (Sec. 3)
    "2d_pp_400_square": lambda: _case("2d_pp_400_square", (400, 400), (PE, PE),
                                      [inputs.Obstacle("box", (0.45, 0.45), (0.55, 0.55))], 16,
                                      16, 8, (41, 42)),
    # channel periodic horizontally, cylinder across the periodic face
    "2d_pn_280x480": lambda: _case("2d_pn_280x480", (280, 480), (PE, NE),
                                   [inputs.Obstacle("circle", (0.02, 0.5), (0.12,))], 12, 16, 8,
                                   (43, 44)),
    "3d_ppn_48x40x36": lambda: _case("3d_ppn_48x40x36", (48, 40, 36), (PE, PE, NE),
                                     [inputs.Obstacle("sphere", (0.97, 0.03, 0.5), (0.2,))], 27,
                                     27, 16, (45, 46)),
}
_CACHE = {}


def case(name):
    if name not in _CACHE:
        c, bc = CASES[name]()
        grid = Grid(c.d, c.n, c.h, bc)
        st = P.build_stencils(grid, c.x.T.copy(), c.kind, c.k_grid, c.k_node)
        _CACHE[name] = (c, bc, grid, st)
    return _CACHE[name]


@pytest.mark.parametrize("name", list(CASES))
def test_periodic_any_even_stencils(pc, name):
    check_stencils(pc, *case(name), name)


@pytest.mark.parametrize("name", list(CASES))
def test_periodic_any_even_transfers(pc, name):
    check_transfers(pc, *case(name))


@pytest.mark.parametrize("name", list(CASES))
def test_periodic_any_even_sub_step(pc, name):
    import torch
    c, bc, grid, st = case(name)
    ref = P.pressure_correct(st, c.u.T.copy())
    plan = pc.Plan(c.d, c.n, c.h, bc=bc)
    geom = pc.wls_build(plan, torch.from_numpy(c.x).cuda(), torch.from_numpy(c.kind).cuda(),
                        c.k_grid, c.k_node, want_f32=True)
    res = {}
    for mode, dtype in ((pc.PC_F64, torch.float64), (pc.PC_MIXED, torch.float64),
                        (pc.PC_F32, torch.float32)):
        u_in = c.u if mode != pc.PC_F32 else c.u.astype(np.float32).astype(np.float64)
        r = ref if mode != pc.PC_F32 else P.pressure_correct(st, u_in.T.copy(),
                                                             fixed_it=ref["n_it"])
        ut = torch.from_numpy(u_in).to(dtype).cuda()
        uo = torch.empty_like(ut)
        p = torch.empty(grid.G, dtype=dtype, device="cuda")
        rc, stats = pc.pressure_correct(geom, plan, mode, ut, 1.0, uo, p,
                                        fixed_it=0 if mode == pc.PC_F64 else ref["n_it"])
        torch.cuda.synchronize()
        res[mode] = (stats["n_it"], rel_l2(to_np(uo), r["u_new"].T), rel_l2(to_np(p), r["p"]))
    print(f"{name}: oracle n_it {ref['n_it']}, gpu {res}")
    assert res[pc.PC_F64][0] == ref["n_it"]
    assert res[pc.PC_F64][1] <= 1e-11 and res[pc.PC_F64][2] <= 1e-11
    assert res[pc.PC_MIXED][1] <= 1e-10 and res[pc.PC_MIXED][2] <= 1e-10
    assert res[pc.PC_F32][1] <= 5e-5 and res[pc.PC_F32][2] <= 5e-5


@pytest.mark.parametrize("name", list(CASES))
def test_periodic_any_even_resident_transforms_bitwise(pc, name):
    from tests.test_gpu_mixed_radix import resident_bitwise
    c, bc, grid, st = case(name)
    resident_bitwise(pc, c, bc)
