"""Host-side checks of bench.py that need no GPU: the one-GPU contract and the
algorithmic byte counts its roofline fractions divide by, against counts
worked out by hand from what each kernel reads and writes."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_divergence_bytes_per_point(bench):
    # per grid point: k stencil entries of a 4-byte node index and d float64
    # coefficients, b written once; per node: u read once (d float64)
    G = M = 1000
    assert bench.bytes_div_all(G, M, 16, 2, 8) == G * 344      # 16 * 20 + 8 + 16
    assert bench.bytes_div_all(G, M, 27, 3, 8) == G * 788      # 27 * 28 + 8 + 24
    assert bench.bytes_div_all(G, M, 27, 3, 4) == G * 448      # 27 * 16 + 4 + 12


def test_gradient_bytes_per_node(bench):
    # per node: the block of bn grid points times d coefficients, the block
    # corner (4 B), the gradient written (d values); phi read once per point.
    # The projection also reads u* (d values) and writes u^{n+1} instead.
    G, M = 64, 100
    assert bench.bytes_grad(G, M, 16, 2, 8) == M * (256 + 4 + 16) + G * 8
    assert bench.bytes_grad_project(G, M, 27, 3, 8) == M * (648 + 4 + 48) + G * 8


def test_solve_bytes_per_point(bench):
    G = 10
    # every pass reads and writes the grid once: 3 passes in 2D, 5 in 3D
    assert bench.bytes_solve_mode(G, 2, "f64", 0) == G * 3 * 16
    assert bench.bytes_solve_mode(G, 3, "f32", 0) == G * 5 * 8
    # MIXED, cold, 2D, two sweeps: the float32 solve of b (f64 in, f32 out;
    # f32 in and out; f32 in, f64 out) = 12 + 8 + 12, then per sweep the
    # residual pass (b and phi in, f32 out) 20, the middle pass 8, the
    # accumulating pass (f32 and phi in, phi out) 20
    assert bench.bytes_solve_mode(G, 2, "mixed", 2) == G * (32 + 2 * 48)
    # 3D has three middle passes of 8 bytes (forward y, the fused last axis,
    # inverse y)
    assert bench.bytes_solve_mode(G, 3, "mixed", 3) == G * ((12 + 24 + 12) + 3 * (20 + 24 + 20))
    # warm, 2D, two sweeps, a quarter of the x rows holding near points: the
    # change of b transformed forward on those rows (f64 in, f32 out), the
    # last-axis pass (8), the accumulating inverse (20), then one full sweep
    G = 400
    assert bench.bytes_solve_mode(G, 2, "mixed", 2, True, (0.25, 0.0)) == \
        G * 12 // 4 + G * (8 + 20 + 48)


def test_step_bytes_compose(bench):
    # FP64, 2D, k = 16, bn = 16, three iterations: the divergence, the final
    # gradient with the projection, three solves, three IB steps and two
    # near-IB updates
    G, M, n_near, ent, n_ib = 4096, 4200, 50, 400, 104
    div = G * 344 + (M - G) * 16
    grad = M * (256 + 4 + 32) + G * 8
    solves = 3 * G * 48
    ib = 3 * n_ib * (256 + 4 + 48)
    near = 2 * (ent * 20 + n_near * 16)
    assert bench.bytes_step(G, M, 16, 16, 2, "f64", 2, 3, n_near, ent, n_ib) == \
        div + grad + solves + ib + near
