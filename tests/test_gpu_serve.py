"""The serving loop on the GPU: requests of mixed 2D/3D sizes and both
precisions run concurrently on four streams; each result must equal the
same request run alone (one slot, one request in flight), bit for bit, and
agree with the float64 oracle (1e-11 for PC_F64, 1e-10 for PC_MIXED)."""
import numpy as np
import pytest

import oracle
from oracle import projection as P
from paper_2304_14690_amd import serve
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

F64, MIXED = 1, 3
SIZES = [(2, 64), (2, 128), (3, 32)]


@pytest.fixture(scope="module")
def data():
    import torch
    ds = serve.Dataset(SIZES, {k: 2 for k in SIZES}, 2, seed=11)
    torch.cuda.synchronize()
    return ds


def _intervals_overlap(reqs):
    ev = sorted([(r.admitted, 1) for r in reqs] + [(r.done, -1) for r in reqs])
    cur = best = 0
    for _, e in ev:
        cur += e
        best = max(best, cur)
    return best


def test_mix_equals_alone_and_oracle(data):
    reqs = serve.poisson_trace(24, 3000.0, 5, SIZES, {k: 2 for k in SIZES}, 2, [F64, MIXED])
    ex = serve.GpuExecutor(data, slots=4, keep_results=True)
    sch = serve.Scheduler(ex, budget=8 << 30, slots=4)
    mix = sch.run(reqs)
    assert all(r.rc == 0 for r in mix)
    print("max in flight", _intervals_overlap(mix), serve.summarize(mix))
    assert _intervals_overlap(mix) > 1

    # each request alone, in arrival order, one in flight, same resident state
    alone_reqs = [serve.Request(r.rid, 0.0, r.d, r.N, r.geom, r.vel, r.mode) for r in mix]
    ex1 = serve.GpuExecutor(data, slots=1, keep_results=True)
    sch1 = serve.Scheduler(ex1, budget=8 << 30, slots=1)
    alone = {r.rid: r for r in sch1.run(alone_reqs)}
    for r in mix:
        a = alone[r.rid]
        assert a.n_it == r.n_it
        assert np.array_equal(a.result["u"], r.result["u"])
        assert np.array_equal(a.result["p"], r.result["p"])

    # oracle parity on one request of each precision per size
    checked = set()
    for r in mix:
        if (r.d, r.N, r.mode) in checked:
            continue
        checked.add((r.d, r.N, r.mode))
        it = data[r.key]
        x = it["x"].cpu().numpy()
        kind = it["kind"].cpu().numpy()
        u = it["u"][r.vel].cpu().numpy()
        grid = oracle.Grid(r.d, it["n"], it["h"])
        st = P.build_stencils(grid, x.T.copy(), kind, it["k"], it["k"])
        ref = P.pressure_correct(st, u.T.copy(), fixed_it=r.n_it)
        tol = 1e-11 if r.mode == F64 else 1e-10
        eu = rel_l2(r.result["u"], ref["u_new"].T)
        ep = rel_l2(r.result["p"], ref["p"])
        print(f"{r.key} mode {r.mode}: u {eu:.2e} p {ep:.2e}")
        assert eu <= tol and ep <= tol
    sch.release()
    sch1.release()


def test_footprint_matches_the_built_geometry(data):
    """pc_geom_footprint before a build against what the geometry and its
    workspaces take afterwards: the same workspace bytes, geometry bytes
    equal for the exact near-point count up to the near table's width, and
    an upper bound for a larger near-point bound."""
    import torch
    from paper_2304_14690_amd import pcorr as pc
    for key in [(2, 128, 0), (3, 32, 1)]:
        it = data[key]
        plan = pc.Plan(key[0], it["n"], it["h"])
        for want_f32, order in ((False, "caller"), (True, "cell")):
            g = pc.wls_build(plan, it["x"], it["kind"], it["k"], it["k"], want_f32=want_f32,
                             order=order)
            n_ib = int((it["kind"] != 0).sum().item())
            assert g.n_ib == n_ib
            gb, peak, ws = pc.geom_footprint(plan, it["M"], n_ib, g.n_near, it["k"], it["k"],
                                             want_f32=want_f32, order=order)
            bound_w = 8 if it["k"] <= 8 else (16 if it["k"] <= 16 else
                                              (27 if it["k"] <= 27 and key[0] == 3 else 32))
            wide = g.near_w != bound_w
            # the footprint counts every B+V node in the virtual-node list
            n_b = int((it["kind"] == 1).sum().item())
            assert gb >= g.bytes and (wide or gb - g.bytes == 4 * n_b)
            assert peak > gb
            for mode in (pc.PC_F64, pc.PC_F32, pc.PC_MIXED):
                assert ws[mode] == pc.workspace_bytes(plan, g, mode)
            gb2, _, _ = pc.geom_footprint(plan, it["M"], n_ib, 4 * g.n_near, it["k"], it["k"],
                                          want_f32=want_f32, order=order)
            assert gb2 > gb
            del g
