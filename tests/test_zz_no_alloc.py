"""The allocation-free IB update (pc_ib_update_noalloc, scratch in a static
device array) against pc_ib_update through the C ABI: equal bit for bit on
two calls in a row, the second on a smaller geometry (fewer B+V nodes), in
float64 and float32 and in 2D and 3D."""
import numpy as np
import pytest

from paper_2304_14690_amd import inputs

pytestmark = pytest.mark.gpu


def _case(d, N, R, seed):
    obs = [inputs.Obstacle("circle" if d == 2 else "sphere", (0.5,) * d, (R,))]
    return inputs.make_case(f"na{d}{N}", d, N, obs, 16 if d == 2 else 27,
                            16 if d == 2 else 27, 8, seed, seed + 1)


def _update_both(pc, c, dtype, rng):
    import torch
    plan = pc.Plan(c.d, c.n, c.h)
    geom = pc.wls_build(plan, torch.from_numpy(c.x).cuda(), torch.from_numpy(c.kind).cuda(),
                        c.k_grid, c.k_node, want_f32=True)
    nib = geom.n_ib
    assert nib > 0
    u = torch.from_numpy(c.u).to(dtype).cuda()
    grad = torch.from_numpy(rng.normal(size=(c.d, nib))).to(dtype).cuda()
    g0 = torch.from_numpy(rng.normal(size=(c.d, nib))).to(dtype).cuda()
    out = []
    for fn in (pc.ib_update, pc.ib_update_noalloc):
        g = g0.clone()
        sums = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
        conv = torch.full((2,), -7, dtype=torch.int32, device="cuda")
        fn(geom, u, grad, g, 1e-3, sums, conv)
        torch.cuda.synchronize()
        out.append((g.cpu().numpy(), sums.cpu().numpy(), int(conv[0].item())))
    (ga, sa, ca), (gb, sb, cb) = out
    assert np.array_equal(ga, gb) and np.array_equal(sa, sb) and ca == cb
    # against the definition (Eq. 19 and the criterion sums of Sec. 2.3)
    gn = -c.u[:, c.kind != inputs.KIND_F] + grad.double().cpu().numpy()
    go = g0.double().cpu().numpy()
    if dtype == torch.float64:
        np.testing.assert_allclose(gb, gn, rtol=0, atol=1e-15 * np.abs(gn).max())
        mn, mo = np.sqrt((gn * gn).sum(0)), np.sqrt((go * go).sum(0))
        np.testing.assert_allclose(sb, [((mn - mo) ** 2).sum(), (mo * mo).sum()], rtol=1e-12)
    return nib


@pytest.mark.parametrize("d", [2, 3])
def test_noalloc_ib_update_matches(d):
    import torch
    from paper_2304_14690_amd import pcorr as pc
    rng = np.random.Generator(np.random.PCG64(91))
    big, small = ((_case(2, 128, 0.2, 31), _case(2, 64, 0.1, 33)) if d == 2 else
                  (_case(3, 32, 0.25, 35), _case(3, 16, 0.2, 37)))
    for dtype in (torch.float64, torch.float32):
        n1 = _update_both(pc, big, dtype, rng)
        n2 = _update_both(pc, small, dtype, rng)
        assert n2 < n1
