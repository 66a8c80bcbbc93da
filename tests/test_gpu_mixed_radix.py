"""Grids whose sizes are not powers of two (Sec. 3 runs 400 x 402 and
280 x 480 pressure grids): the mixed-radix line transform (any even n; the
prime factors of n/2 include 3, 5, 7, 13 and 67 here) against the oracle's
library DCT in every precision, alone and next to power-of-two axes, and the
whole sub-step on a 400 x 402 grid and a 3D grid.  Bars: float64 1e-11,
float32 5e-5, float32 transforms + float64 correction 1e-10 (relative L2)."""
import numpy as np
import pytest

import oracle
from oracle import Grid, poisson, projection as P
from paper_2304_14690_amd import inputs
from tests.helpers import rel_l2, to_np
from tests.test_gpu_edge import custom_case

pytestmark = pytest.mark.gpu

SHAPES = [(400, 402), (280, 480), (10, 12), (2048, 402), (400, 256), (3000, 10),
          (48, 40, 36), (26, 18, 14), (64, 134, 32)]


@pytest.fixture(scope="module")
def pc():
    from paper_2304_14690_amd import pcorr
    return pcorr


@pytest.mark.parametrize("n", SHAPES, ids=["x".join(map(str, n)) for n in SHAPES])
def test_mixed_radix_solve(pc, n):
    import torch
    d = len(n)
    h = tuple(1.0 / v for v in n)
    grid = Grid(d, n, h)
    plan = pc.Plan(d, n, h)
    rng = np.random.Generator(np.random.PCG64(21))
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
    print(f"{n}: f64 {e64:.2e} f32 {e32:.2e} mixed {em:.2e}")
    assert e64 <= 1e-11 and e32 <= 5e-5 and em <= 1e-10
    assert abs(bm.item() - bm_ref) <= 1e-12 * max(1.0, abs(bm_ref))


CASES = {
    "2d_400x402": lambda: custom_case((400, 402), [inputs.Obstacle("circle", (0.3, 0.5),
                                                                   (0.06,))], 16, 16),
    "2d_280x480": lambda: custom_case((280, 480), [inputs.Obstacle("circle", (0.5, 0.4),
                                                                   (0.1,))], 12, 16),
    "3d_48x40x36": lambda: custom_case((48, 40, 36), [inputs.Obstacle("sphere", (0.5, 0.5, 0.5),
                                                                      (0.2,))], 27, 27),
}


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_radix_sub_step(pc, name):
    import torch
    c = CASES[name]()
    grid = Grid(c.d, c.n, c.h)
    st = P.build_stencils(grid, c.x.T.copy(), c.kind, c.k_grid, c.k_node)
    ref = P.pressure_correct(st, c.u.T.copy())
    plan = pc.Plan(c.d, c.n, c.h)
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


def test_mixed_radix_plan_rules(pc):
    with pytest.raises(pc.PcError) as e:
        pc.Plan(2, (401, 402), (1.0, 1.0))
    assert e.value.code == pc.PC_ERR_UNSUPPORTED_SIZE
    with pytest.raises(pc.PcError) as e:
        pc.Plan(2, (400, 66), (1.0, 1.0), bc=("neumann", "periodic"), grid="vertex")
    assert e.value.code == pc.PC_ERR_INVALID_ARG
    # a periodic axis of any even length beside a mixed-radix one
    pc.Plan(2, (400, 64), (1.0, 1.0), bc=("neumann", "periodic"))


def resident_bitwise(pc, c, bc=None):
    """The sub-step with resident transforms (later IB iterations transform
    only the lines whose right-hand side changed and invert only the lines
    the B+V gradient reads) against every line transformed in every
    iteration: equal bit for bit, float64 and float32, cold and warm; and
    the correction mode with its change-of-RHS sweeps and with full
    residual sweeps, both within 1e-10 of float64."""
    import torch
    plan = pc.Plan(c.d, c.n, c.h, bc=bc)
    geom = pc.wls_build(plan, torch.from_numpy(c.x).cuda(), torch.from_numpy(c.kind).cuda(),
                        c.k_grid, c.k_node, want_f32=True)
    G = int(np.prod(c.n))
    for mode, dtype in ((pc.PC_F64, torch.float64), (pc.PC_F32, torch.float32)):
        ut = torch.from_numpy(c.u).to(dtype).cuda()
        outs = []
        for full in (False, True):
            res = []
            g = torch.zeros((c.d, geom.n_ib), dtype=dtype, device="cuda")
            for rep in range(2):  # cold, then warm from the first result
                uo = torch.empty_like(ut)
                p = torch.empty(G, dtype=dtype, device="cuda")
                rc, st = pc.pressure_correct(geom, plan, mode, ut, 1.0, uo, p, g=g,
                                             full_transforms=full)
                torch.cuda.synchronize()
                res.append((rc, st["n_it"], to_np(uo), to_np(p), to_np(g).copy()))
            outs.append(res)
        # the cold run iterates, so later iterations take the resident path
        assert outs[0][0][1] >= 2
        for ra, rb in zip(*outs):
            assert ra[0] == rb[0] and ra[1] == rb[1]
            for xa, xb in zip(ra[2:], rb[2:]):
                assert np.array_equal(xa, xb)
    # PC_MIXED: the change-of-RHS first sweep of later iterations (default)
    # against full residual sweeps (the flag), within the mode's tolerance,
    # both against float64
    ut = torch.from_numpy(c.u).cuda()
    res = []
    for mode, full in ((pc.PC_F64, False), (pc.PC_MIXED, False), (pc.PC_MIXED, True)):
        uo = torch.empty_like(ut)
        p = torch.empty(G, dtype=torch.float64, device="cuda")
        rc, st = pc.pressure_correct(geom, plan, mode, ut, 1.0, uo, p, full_transforms=full)
        torch.cuda.synchronize()
        res.append((st["n_it"], to_np(uo), to_np(p)))
    for n_it, uo, p in res[1:]:
        assert n_it == res[0][0]
        assert rel_l2(uo, res[0][1]) <= 1e-10 and rel_l2(p, res[0][2]) <= 1e-10


@pytest.mark.parametrize("name", list(CASES) + ["3d_16x32x24", "2d_200x1000", "2d_2000x400",
                                                 "3d_40x200x32"])
def test_mixed_radix_resident_transforms_bitwise(pc, name):
    if name == "3d_16x32x24":
        # a short axis (generic kernel) between two others, one not a power of two
        c = custom_case((16, 32, 24), [inputs.Obstacle("sphere", (0.5, 0.5, 0.5), (0.25,))],
                        27, 27)
    elif name == "2d_200x1000":
        # radix-10 plans on both axes: 10^2 and 10^2 * 5
        c = custom_case((200, 1000), [inputs.Obstacle("circle", (0.4, 0.5), (0.08,))], 16, 16)
    elif name == "3d_40x200x32":
        # the radix-10 plan on the middle (strided) axis of a 3D box
        c = custom_case((40, 200, 32), [inputs.Obstacle("sphere", (0.5, 0.5, 0.5), (0.25,))],
                        27, 27)
    elif name == "2d_2000x400":
        # three radix-10 stages on the rows, two and a radix-2 stage on the columns
        c = custom_case((2000, 400), [inputs.Obstacle("circle", (0.5, 0.5), (0.2,))], 16, 16)
    else:
        c = CASES[name]()
    resident_bitwise(pc, c)
