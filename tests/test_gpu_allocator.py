"""Device memory through a caller's allocator (pc_set_allocator): a
sub-step with plan, geometry and workspace taken from torch's caching
allocator equals the same sub-step on hipMalloc memory bit for bit; torch's
statistics see the library's memory; every allocation is returned (the
scratch of the stencil build included); the pair cannot be replaced while
its allocations are outstanding."""
import gc

import numpy as np
import pytest

from paper_2304_14690_amd import inputs
from tests.helpers import to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    from paper_2304_14690_amd import pcorr
    return pcorr


def _run(pc, c):
    import torch
    plan = pc.Plan(c.d, c.n, c.h)
    geom = pc.wls_build(plan, torch.from_numpy(c.x).cuda(), torch.from_numpy(c.kind).cuda(),
                        c.k_grid, c.k_node)
    ws = pc.Workspace(plan, geom, pc.PC_F64)
    u = torch.from_numpy(c.u).cuda()
    uo = torch.empty_like(u)
    p = torch.empty(c.G, dtype=torch.float64, device="cuda")
    rc, st = pc.pressure_correct(geom, plan, pc.PC_F64, u, 1.0, uo, p, ws=ws)
    torch.cuda.synchronize()
    return (plan, geom, ws), (rc, st["n_it"], to_np(uo), to_np(p))


def test_caller_allocator(pc):
    import torch
    c = inputs.make_case("alloc", 2, 128, [inputs.Obstacle("circle", (0.4, 0.5), (0.1,))],
                         16, 16, 8, 61, 62)
    objs, ref = _run(pc, c)
    del objs
    gc.collect()

    alloc, free = pc.torch_allocator()
    count = {"alloc": 0, "free": 0, "bytes": 0}

    def a(nbytes):
        count["alloc"] += 1
        count["bytes"] += nbytes
        return alloc(nbytes)

    def f(ptr):
        count["free"] += 1
        free(ptr)

    pc.set_allocator(a, f)
    try:
        before = torch.cuda.memory_allocated()
        objs, got = _run(pc, c)
        held = torch.cuda.memory_allocated() - before
        plan, geom, ws = objs
        assert held >= geom.bytes > 0
        assert got[:2] == ref[:2]
        assert np.array_equal(got[2], ref[2]) and np.array_equal(got[3], ref[3])
        with pytest.raises(pc.PcError) as e:
            pc.set_allocator(None, None)
        assert e.value.code == pc.PC_ERR_INVALID_ARG
        del objs, plan, geom, ws
        gc.collect()
        print(f"allocator: {count['alloc']} allocations, {count['bytes']} bytes, "
              f"{count['free']} returned; torch saw {held} bytes held")
        assert count["alloc"] == count["free"] and count["alloc"] > 0
    finally:
        gc.collect()
        pc.set_allocator(None, None)


def test_objects_return_to_their_own_allocator(pc):
    """A plan and geometry made on hipMalloc memory and destroyed while a
    caller's pair is installed go back to hipFree: the pair's free is never
    called for them, and the pair can be removed afterwards."""
    import torch
    c = inputs.make_case("alloc2", 2, 64, [inputs.Obstacle("circle", (0.5, 0.5), (0.1,))],
                         12, 12, 8, 63, 64)
    plan = pc.Plan(c.d, c.n, c.h)
    geom = pc.wls_build(plan, torch.from_numpy(c.x).cuda(), torch.from_numpy(c.kind).cuda(),
                        c.k_grid, c.k_node)
    torch.cuda.synchronize()
    alloc, free = pc.torch_allocator()
    seen = {"alloc": set(), "freed": []}

    def a(nbytes):
        ptr = alloc(nbytes)
        seen["alloc"].add(ptr)
        return ptr

    def f(ptr):
        seen["freed"].append(ptr)
        free(ptr)

    pc.set_allocator(a, f)
    try:
        del geom, plan
        gc.collect()
        assert seen["freed"] == []
        # objects made through the pair go back to it, hipMalloc ones do not
        plan2 = pc.Plan(c.d, c.n, c.h)
        del plan2
        gc.collect()
        assert seen["freed"] and set(seen["freed"]) <= seen["alloc"]
        assert len(seen["freed"]) == len(seen["alloc"])
    finally:
        gc.collect()
        pc.set_allocator(None, None)
