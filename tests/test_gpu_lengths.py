"""Every length of the register line transform (N = 32 ... 4096, half
lengths 16 ... 2048: one to three radix-8 stages and a final stage of radix
1, 2 or 4; and the radix-10 plan's N = 200, 400, 1000, 2000: two or three
radix-10 stages and a final stage of radix 1, 2 or 5) on each axis of a 2D
box, as a cosine transform (homogeneous
Neumann axis, Eq. 7) and as a packed real DFT (periodic axis), in float64,
float32 and float32 transforms with float64 defect correction, against the
oracle's solve (float64 to 1e-11, float32 to 5e-5, the correction to 1e-10,
relative L2).  In 2D the other axis is 16 points long (the generic kernel,
whose pass the register kernel's output feeds or reads) or 32 (register
kernel on both axes); in 3D the long axis is the middle one (the strided
pass between two generic axes) or the last one (the fused pass)."""
import numpy as np
import pytest

from oracle import Grid, poisson
from tests.helpers import rel_l2, to_np

pytestmark = pytest.mark.gpu

P, NE = "periodic", "neumann"
LENGTHS = [32, 64, 128, 256, 512, 1024, 2048, 4096, 200, 400, 1000, 2000]
CASES = []
for N in LENGTHS:
    for bc in (NE, P):
        CASES.append(((N, 16), (bc, NE)))   # long x rows, generic last axis
        CASES.append(((32, N), (NE, bc)))   # long last axis (fused pass)
for N in LENGTHS:
    for bc in (NE, P):
        CASES.append(((16, N, 8), (NE, bc, NE)))   # 3D middle axis (strided pass)
        CASES.append(((8, 16, N), (P, NE, bc)))    # 3D last axis (fused pass)
IDS = ["x".join(map(str, n)) + "-" + "".join(b[0] for b in bc) for n, bc in CASES]


@pytest.fixture(scope="module")
def pc():
    import torch  # noqa: F401
    from paper_2304_14690_amd import pcorr
    return pcorr


@pytest.mark.parametrize("n,bc", CASES, ids=IDS)
def test_register_lengths_all_modes(pc, n, bc):
    import torch
    d = len(n)
    h = tuple(1.0 / v for v in n)
    grid = Grid(d, n, h, bc)
    plan = pc.Plan(d, n, h, bc=bc)
    rng = np.random.Generator(np.random.PCG64(4000 + n[0] + 7 * n[1] + 13 * n[-1]))
    b = rng.normal(size=grid.G) + 0.3
    phi_ref, bm_ref = poisson.solve(grid, b)
    bt = torch.from_numpy(b).cuda()
    phi = torch.empty_like(bt)
    bm = torch.zeros(1, dtype=torch.float64, device="cuda")
    pc.poisson_fft_solve(plan, bt, phi, pc.PC_F64, bmean=bm)
    torch.cuda.synchronize()
    e64 = rel_l2(to_np(phi), phi_ref)
    assert abs(bm.item() - bm_ref) <= 1e-12 * max(1.0, abs(bm_ref))

    b32 = b.astype(np.float32)
    ref32, _ = poisson.solve(grid, b32.astype(np.float64))
    bt32 = torch.from_numpy(b32).cuda()
    phi32 = torch.empty_like(bt32)
    pc.poisson_fft_solve(plan, bt32, phi32, pc.PC_F32)
    torch.cuda.synchronize()
    e32 = rel_l2(to_np(phi32), ref32)

    ws = pc.Workspace(plan, None, pc.PC_MIXED)
    phim = torch.empty_like(bt)
    pc.poisson_fft_solve(plan, bt, phim, pc.PC_MIXED, sweeps=2, ws=ws)
    torch.cuda.synchronize()
    em = rel_l2(to_np(phim), phi_ref)
    print(f"{n} {bc}: f64 {e64:.2e} f32 {e32:.2e} mixed {em:.2e}")
    assert e64 <= 1e-11 and e32 <= 5e-5 and em <= 1e-10
