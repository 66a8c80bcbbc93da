"""Float32-only geometries (pc_wls_opts.dtype_mask = 1 << PC_F32): the
float32 stencils are the same values as the float32 copies of a geometry
that keeps both precisions, so every float32 call gives the same bits; the
float64 calls and coefficient exports are refused; the byte counts follow
the kept precisions."""
import ctypes

import numpy as np
import pytest

from paper_2304_14690_amd import inputs
from tests.helpers import to_np

pytestmark = pytest.mark.gpu

CASES = {
    "2d_256": lambda: inputs.config2(256),
    "3d_32_box": lambda: inputs.make_case("box3", 3, 32,
                                          [inputs.Obstacle("sphere", (0.3, 0.5, 0.5), (0.12,)),
                                           inputs.Obstacle("box", (0.6, 0.4, 0.4),
                                                           (0.8, 0.6, 0.6))], 27, 27, 16, 7, 8),
}


@pytest.fixture(scope="module")
def pc():
    from paper_2304_14690_amd import pcorr
    return pcorr


def _build(pc, c, **kw):
    import torch
    plan = pc.Plan(c.d, c.n, c.h)
    x = torch.from_numpy(c.x).cuda()
    kind = torch.from_numpy(c.kind).cuda()
    return plan, x, kind, pc.wls_build(plan, x, kind, c.k_grid, c.k_node, **kw)


@pytest.mark.parametrize("name", list(CASES))
def test_f32_only_same_bits_as_both(pc, name):
    import torch
    c = CASES[name]()
    plan, x, kind, both = _build(pc, c, want_f32=True)
    g32 = pc.wls_build(plan, x, kind, c.k_grid, c.k_node, f32_only=True)
    g64 = pc.wls_build(plan, x, kind, c.k_grid, c.k_node)
    assert (g32.n_ib, g32.n_near, g32.near_w) == (both.n_ib, both.n_near, both.near_w)
    # bytes: both = I + C8 + C4, float64 only = I + C8, float32 only = I + C4, C8 = 2 C4
    assert both.bytes - g32.bytes == 2 * (both.bytes - g64.bytes) > 0
    gb, _, _ = pc.geom_footprint(plan, c.kind.size, g32.n_ib, g32.n_near, c.k_grid, c.k_node,
                                 f32_only=True)
    # the footprint bounds the virtual-node list by n_ib (4 bytes per B node more)
    assert gb - g32.bytes == 4 * int((c.kind == inputs.KIND_B).sum())
    G = int(np.prod(c.n))
    u = torch.from_numpy(c.u).to(torch.float32).cuda()
    outs = []
    for geom in (both, g32):
        b = torch.empty(G, dtype=torch.float32, device="cuda")
        pc.div_to_grid(geom, u, b)
        gr = torch.empty_like(u)
        pc.grad_to_nodes(geom, b, gr)
        uo = torch.empty_like(u)
        p = torch.empty(G, dtype=torch.float32, device="cuda")
        g = torch.zeros((c.d, geom.n_ib), dtype=torch.float32, device="cuda")
        rc, st = pc.pressure_correct(geom, plan, pc.PC_F32, u, 1.0, uo, p, g=g)
        torch.cuda.synchronize()
        outs.append((st["n_it"], to_np(b), to_np(gr), to_np(uo), to_np(p), to_np(g)))
    assert outs[0][0] == outs[1][0]
    for xa, xb in zip(outs[0][1:], outs[1][1:]):
        assert np.array_equal(xa, xb)
    print(f"{name}: n_it {outs[0][0]}, bytes both {both.bytes} f32 only {g32.bytes}")


def test_f32_only_refuses_float64(pc):
    import torch
    c = CASES["2d_256"]()
    plan, x, kind, g32 = _build(pc, c, f32_only=True)
    G = int(np.prod(c.n))
    u = torch.from_numpy(c.u).cuda()
    b = torch.empty(G, dtype=torch.float64, device="cuda")
    uo = torch.empty_like(u)
    with pytest.raises(pc.PcError) as e:
        pc.div_to_grid(g32, u, b)
    assert e.value.code == pc.PC_ERR_INVALID_ARG and "float32" in pc.last_error()
    for mode in (pc.PC_F64, pc.PC_MIXED):
        with pytest.raises(pc.PcError):
            pc.pressure_correct(g32, plan, mode, u, 1.0, uo, b)
    gc = torch.empty((c.d, c.k_grid, G), dtype=torch.float64, device="cuda")
    with pytest.raises(pc.PcError):
        pc.geom_export(g32, grid_coef=gc)
    gi = torch.empty((c.k_grid, G), dtype=torch.int32, device="cuda")
    pc.geom_export(g32, grid_idx=gi)  # indices are kept
    # unknown bits of the mask
    opts = pc.WlsOpts(c.k_grid, c.k_node, 0.0, 0.0, 0.0, 1, 0, 0)
    out = ctypes.c_void_p()
    rc = pc.lib().pc_wls_build(plan.h_, ctypes.c_void_p(x.data_ptr()),
                               ctypes.c_void_p(kind.data_ptr()), kind.numel(),
                               ctypes.byref(opts), None, ctypes.byref(out))
    assert rc == pc.PC_ERR_INVALID_ARG and "dtype_mask" in pc.last_error()
