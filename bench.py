#!/usr/bin/env python3
"""Benchmark of the hybrid pressure-correction sub-step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 3d512]
                    [--extra 2d2048]

Workloads (all inputs seeded and synthetic, resident in HBM before timing):
  3d512   512^3 grid, 134M jittered-lattice nodes (jitter +-0.3h), a sphere of
          radius 0.1 at (0.3, 0.5, 0.5) plus the box [0.6, 0.8] x [0.4, 0.6]^2
          whose interior nodes are virtual points and whose surfaces carry the
          boundary points, 27-neighbour WLS stencils, 64 random Fourier modes,
          Neumann box; float64, and float32 transforms with 2 and 3 float64
          defect-correction sweeps against all-float64.  The largest
          single-GPU workload: the headline is quoted on it.
  2d2048  2048^2 grid, 4.2M nodes, a cylinder of radius 0.05 at (0.3, 0.5),
          16-neighbour stencils, 32 modes; float64, float32 and float32 +
          float64 correction.  Run after the headline (--extra).
  3d256   256^3 grid, 16.8M nodes, sphere of radius 0.1 at the centre,
          27-neighbour stencils, 64 modes.
  2d2048p 2d2048 with a periodic x axis (a channel: periodic lateral faces,
          as in the paper's verification cases, Sec. 3) and Neumann walls in y.
  3d256p  3d256 with periodic x and z axes and Neumann walls in y.
  2d2048pp, 3d256pp  the same, periodic along every axis; these also time
          whole time steps (the first fractional step of Eq. 3 + the sub-step):
          the first step needs velocity conditions on non-periodic faces,
          which are the caller's, so whole steps are timed without faces.
  2d400sq the grid of the flow over a square (Sec. 3): 400^2, periodic in x
          and y, the square [0.45, 0.55]^2, 16-neighbour stencils, 32 modes;
          also times whole time steps.
  2d1024c the 2d2048 node cloud (the same 4.2M nodes and cylinder) under a
          1024^2 pressure grid: a pressure grid coarser than the velocity
          cloud, the saving Sec. 3 reports (WLS mean spacing = node spacing).
The stencils are built once (timed separately, not part of a step).  A step
is one complete pressure-correction sub-step (RHS transfer, IB-force
iterations of Poisson solve + gradient at the IB + force update, final
gradient and projection) from a zero IB force.

One JSON line is printed: grid-points/s of the float64 sub-step, p50/p99 step
latency, the other precisions with their error against float64, per-kernel
HIP-event timings with the roofline of the dominant kernel and of the whole
sub-step, the extra workloads, the serving loop (unless --serve-seconds 0),
and the CPU oracle timed on this host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

WORKLOADS = {
    "2d2048": {"d": 2, "N": 2048, "modes": "f64,f32,mixed", "cpu_N": 1024,
               "desc": "2D 2048^2 grid, {M} jittered nodes, cylinder r=0.05 at (0.3,0.5), "
                       "16-NN WLS, 32-mode velocity, Neumann box, cold IB start"},
    "3d256": {"d": 3, "N": 256, "modes": "f64,f32,mixed", "cpu_N": 64,
              "desc": "3D 256^3 grid, {M} jittered nodes, sphere r=0.1 at the centre, 27-NN "
                      "WLS, 64-mode velocity, Neumann box, cold IB start"},
    "2d2000": {"d": 2, "N": 2000, "modes": "f64,f32,mixed", "cpu_N": 1000,
               "desc": "2D 2000^2 grid (n/2 = 2^3 5^3: the mixed-radix transforms), {M} "
                       "jittered nodes, cylinder r=0.05 at (0.3,0.5), 16-NN WLS, 32-mode "
                       "velocity, Neumann box, cold IB start"},
    "2d2048p": {"d": 2, "N": 2048, "modes": "f64,f32,mixed", "cpu_N": 1024,
                "bc": ("periodic", "neumann"),
                "desc": "2D 2048^2 grid, {M} jittered nodes, cylinder r=0.05 at (0.3,0.5), "
                        "16-NN WLS, 32-mode velocity, periodic in x, Neumann walls in y, "
                        "cold IB start"},
    "3d256p": {"d": 3, "N": 256, "modes": "f64,f32,mixed", "cpu_N": 64,
               "bc": ("periodic", "neumann", "periodic"),
               "desc": "3D 256^3 grid, {M} jittered nodes, sphere r=0.1 at the centre, 27-NN "
                       "WLS, 64-mode velocity, periodic in x and z, Neumann walls in y, "
                       "cold IB start"},
    "2d2048pp": {"d": 2, "N": 2048, "modes": "f64,f32,mixed", "cpu_N": 1024,
                 "bc": ("periodic", "periodic"),
                 "desc": "2D 2048^2 grid, {M} jittered nodes, cylinder r=0.05 at (0.3,0.5), "
                         "16-NN WLS, 32-mode velocity, periodic box, cold IB start"},
    "3d256pp": {"d": 3, "N": 256, "modes": "f64,f32,mixed", "cpu_N": 64,
                "bc": ("periodic", "periodic", "periodic"),
                "desc": "3D 256^3 grid, {M} jittered nodes, sphere r=0.1 at the centre, 27-NN "
                        "WLS, 64-mode velocity, periodic box, cold IB start"},
    "2d400sq": {"d": 2, "N": 400, "modes": "f64,f32,mixed", "cpu_N": 400,
                "bc": ("periodic", "periodic"),
                "desc": "2D 400^2 grid, {M} jittered nodes, square [0.45,0.55]^2 (the "
                        "flow-over-a-square grid), 16-NN WLS, 32-mode velocity, periodic box, "
                        "cold IB start"},
    "2d1024c": {"d": 2, "N": 1024, "modes": "f64,f32,mixed", "cpu_N": 512, "nodes_per_axis": 2,
                "desc": "2D 1024^2 pressure grid under the 2048^2 workload's {M} jittered "
                        "nodes (node spacing 1/2048), cylinder r=0.05 at (0.3,0.5), 16-NN WLS, "
                        "32-mode velocity, Neumann box, cold IB start"},
    "3d512": {"d": 3, "N": 512, "modes": "f64,mixed,mixed3,f32", "cpu_N": 64, "f32_own_geom": True,
              "cpu_note": "the oracle's stencils of the 512^3 workload need ~230 GB of host "
                          "memory and hours of build; 64^3 (same obstacles, k, modes) runs "
                          "in seconds",
              "desc": "3D 512^3 grid, {M} jittered nodes, sphere r=0.1 at (0.3,0.5,0.5) plus "
                      "box [0.6,0.8]x[0.4,0.6]^2, 27-NN WLS, 64-mode velocity, Neumann box, "
                      "cold IB start"},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="3d512", choices=list(WORKLOADS))
    ap.add_argument("--extra", default="2d2048",
                    help="comma list of workloads run after the headline one (reported "
                         "under 'extra'); empty: none")
    ap.add_argument("--size", type=int, default=0, help="override N of the headline workload")
    ap.add_argument("--modes", default="", help="comma list of f64, f32, mixed, mixed3")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-size", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (counter scaling)")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="length of the serving trace (0: no serving run)")
    ap.add_argument("--serve-rate", type=str, default="200,800",
                    help="comma list of arrival rates (requests/s) of the serving runs")
    ap.add_argument("--serve-geoms", type=int, default=2,
                    help="geometries per grid size in the serving pool")
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--no-shuffle", action="store_true",
                    help="skip the shuffled-node-order runs of the 2D extra workloads")
    ap.add_argument("--time-steps", type=int, default=20,
                    help="on a periodic-box workload, also time whole time steps (first "
                         "fractional step + sub-step); 0: off")
    return ap.parse_args()


# ---- algorithmic bytes ---------------------------------------------------------
def bytes_div_all(G, M, k, d, s):
    """idx (4 B) + d coefficients per stencil entry, b written once, u read once."""
    return G * (k * (4 + d * s) + s) + M * d * s


def bytes_solve_pass(G, s_in, s_out):
    return G * (s_in + s_out)


def bytes_solve(G, d, s):
    return (2 * d - 1) * bytes_solve_pass(G, s, s)


def bytes_grad(G, M, bn, d, s):
    """coefficients + block corner per node, phi read once, gradient written."""
    return M * (bn * d * s + 4 + d * s) + G * s


def bytes_grad_project(G, M, bn, d, s):
    """coefficients + block corner per node, u* read, u^{n+1} written, phi read once."""
    return M * (bn * d * s + 4 + 2 * d * s) + G * s


def bytes_momentum(M, k, d, s):
    """node-to-node stencil streams (index + d derivative rows + Laplacian
    row per entry), u read once, R_prev read, R and u* written."""
    return M * (k * (4 + (d + 1) * s) + 4 * d * s)


def make_workload(name, N):
    """Seeded inputs of a workload: (Case-like dict) with x, kind on the host
    and u on the device (2D: numpy velocity; 3D: the same modes evaluated
    with torch on the device, much faster at 16.8M-134M nodes)."""
    import torch
    from paper_2304_14690_amd import inputs
    bc = WORKLOADS[name].get("bc")
    if name == "2d1024c":
        c = inputs.coarse_grid_case(name, 2, N, 2 * N,
                                    [inputs.Obstacle("circle", (0.3, 0.5), (0.05,))],
                                    16, 16, 32, 3, 4)
        return {"d": 2, "n": c.n, "h": c.h, "x": c.x, "kind": c.kind, "k": c.k_grid,
                "u": torch.from_numpy(c.u).cuda(), "bc": None, "delta": 1.0 / (2 * N)}
    if name == "2d400sq":
        c = inputs.make_case(name, 2, N, [inputs.Obstacle("box", (0.45, 0.45), (0.55, 0.55))],
                             16, 16, 32, 3, 4, bc=bc)
        return {"d": 2, "n": c.n, "h": c.h, "x": c.x, "kind": c.kind, "k": c.k_grid,
                "u": torch.from_numpy(c.u).cuda(), "bc": bc}
    if name in ("2d2048", "2d2000", "2d2048p", "2d2048pp"):
        c = inputs.make_case(name, 2, N, [inputs.Obstacle("circle", (0.3, 0.5), (0.05,))],
                             16, 16, 32, 3, 4, bc=bc)
        return {"d": 2, "n": c.n, "h": c.h, "x": c.x, "kind": c.kind, "k": c.k_grid,
                "u": torch.from_numpy(c.u).cuda(), "bc": bc}
    if name in ("3d256", "3d256p", "3d256pp"):
        obs, sn, sv = [inputs.Obstacle("sphere", (0.5, 0.5, 0.5), (0.1,))], 5, 6
    else:
        obs, sn, sv = [inputs.Obstacle("sphere", (0.3, 0.5, 0.5), (0.1,)),
                       inputs.Obstacle("box", (0.6, 0.4, 0.4), (0.8, 0.6, 0.6))], 7, 8
    n, h, x, kind = inputs.make_geometry(3, N, obs, sn, bc=bc)
    xt = torch.from_numpy(x).cuda()
    u = inputs.fourier_velocity_torch(xt, 64, sv)
    u[:, torch.from_numpy(kind).cuda() == inputs.KIND_V] = 0.0
    del xt
    return {"d": 3, "n": n, "h": h, "x": x, "kind": kind, "k": 27, "u": u, "bc": bc}


def rel_l2(a, b):
    import torch
    a = a.double()
    b = b.double()
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def bytes_solve_mode(G, d, mode, sweeps, warm=False, near_lines=(0.0, 0.0)):
    """Algorithmic bytes of one Poisson solve: 2d - 1 passes, each reading and
    writing the grid once.  In the correction mode a cold solve's first pass
    reads the float64 right-hand side and writes float32, its last reads
    float32 and writes float64; each sweep's first pass reads b and phi
    (float64) and writes float32, its last pass reads float32 and phi and
    writes phi.  A warm solve (IB iterations after the first) starts from
    the previous phi, and its first sweep transforms the change of the
    right-hand side forward only on the lines holding near-IB points (the
    fractions near_lines of the x rows and, in 3D, of the y lines: float64
    in, float32 out, then float32 in and out), then runs the last-axis pass,
    the middle inverse (3D) and the accumulating inverse over the grid."""
    if mode == "f64":
        return bytes_solve(G, d, 8)
    if mode == "f32":
        return bytes_solve(G, d, 4)
    mid = 8 * (2 * d - 3)
    if warm:
        fwd = near_lines[0] * 12 + (near_lines[1] * 8 if d == 3 else 0.0)
        return int(G * (fwd + 8 * (d - 1) + 20 + (sweeps - 1) * (20 + mid + 20)))
    return G * ((12 + mid + 12) + sweeps * (20 + mid + 20))


def bytes_step(G, M, k, bn, d, mode, sweeps, n_it, n_near, near_entries, n_ib,
               near_lines=(0.0, 0.0)):
    """Algorithmic bytes of one sub-step: the RHS transfer at every grid
    point, n_it solves, the near-IB RHS update in every iteration after the
    first (the B+V entries of the near stencils, b_u read and b written at
    each near point; in the correction mode also the old b read and the
    change written), the IB step (gradient at the B+V nodes, force update)
    in every iteration, and the final gradient fused with the projection.
    The correction mode also takes mean(b_u) once and removes mean(phi) at
    the end (8 + 24 bytes per grid point)."""
    s = 4 if mode == "f32" else 8
    near = near_entries * (4 + d * s) + n_near * (2 + (2 if mode == "mixed" else 0)) * s
    ibstep = n_ib * (bn * d * s + 4 + 3 * d * s)
    solves = bytes_solve_mode(G, d, mode, sweeps)
    if mode == "mixed":
        solves += (n_it - 1) * bytes_solve_mode(G, d, mode, sweeps, True, near_lines)
        solves += 32 * G
    else:
        solves *= n_it
    return (bytes_div_all(G, M, k, d, s) + bytes_grad_project(G, M, bn, d, s)
            + solves + n_it * ibstep + (n_it - 1) * near)


def near_line_fractions(geom, n, d):
    """Fractions of the x rows and (3D) of the y lines that hold a near-IB
    grid point: the lines the correction mode's first warm sweep transforms."""
    import torch
    from paper_2304_14690_amd import pcorr as pc
    if geom.n_near == 0:
        return (0.0, 0.0)
    near = torch.empty(geom.n_near, dtype=torch.int32, device="cuda")
    pc.geom_export(geom, near=near)
    q = near.cpu().numpy().astype(np.int64)
    rows = np.unique(q // n[0]).size / (int(np.prod(n)) // n[0])
    if d == 2:
        return (rows, 0.0)
    planes = np.unique(q // (n[0] * n[1])).size / n[2]
    return (rows, planes)


def run_shuffled(args, name, N):
    """The float64 sub-step with the nodes handed over in a seeded random
    order: the library sorting them into cells (pc_wls_opts.order =
    PC_ORDER_CELL; fields permuted once, untimed) and, for contrast, kept in
    the shuffled order (PC_ORDER_CALLER)."""
    import torch
    from paper_2304_14690_amd import pcorr as pc
    case = make_workload(name, N)
    d = case["d"]
    G = int(np.prod(case["n"]))
    M = int(case["kind"].size)
    rng = np.random.Generator(np.random.PCG64(11))
    sh = rng.permutation(M)
    x = torch.from_numpy(np.ascontiguousarray(case["x"][:, sh])).cuda()
    kind = torch.from_numpy(np.ascontiguousarray(case["kind"][sh])).cuda()
    shd = torch.from_numpy(sh).cuda()
    u_sh = case["u"][:, shd].contiguous()
    plan = pc.Plan(d, case["n"], case["h"], bc=case["bc"])
    out = {}
    ref_u = None
    for order in ("cell", "caller"):
        geom = pc.wls_build(plan, x, kind, case["k"], case["k"], order=order)
        u = torch.empty_like(u_sh)
        pc.geom_permute(geom, u_sh, u, to_internal=True)
        uo = torch.empty_like(u)
        p = torch.empty(G, dtype=torch.float64, device="cuda")
        ws = pc.Workspace(plan, geom, pc.PC_F64)
        for _ in range(args.warmup):
            _, st = pc.pressure_correct(geom, plan, pc.PC_F64, u, 1.0, uo, p, ws=ws)
        torch.cuda.synchronize()
        lat = []
        t_start = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            _, st = pc.pressure_correct(geom, plan, pc.PC_F64, u, 1.0, uo, p, ws=ws)
            torch.cuda.synchronize()
            lat.append(1e3 * (time.perf_counter() - ts))
        sec = (time.perf_counter() - t_start) / args.steps
        # back to the lattice order of the unshuffled workload
        uc = torch.empty_like(uo)
        pc.geom_permute(geom, uo, uc, to_internal=False)
        ul = torch.empty_like(uc)
        ul[:, shd] = uc
        if ref_u is None:
            ref_u = ul
        out[order] = {"ms_per_step": 1e3 * sec, "p50_ms": float(np.percentile(lat, 50)),
                      "p99_ms": float(np.percentile(lat, 99)), "n_it": st["n_it"],
                      "value": G / sec, "u_vs_cell_order": rel_l2(ul, ref_u)}
        print(f"bench: {name} shuffled, order {order}: {1e3 * sec:.3f} ms/step",
              file=sys.stderr, flush=True)
        del geom, ws, u, uo, p, uc
    del x, kind, u_sh, plan, case
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return {"nodes": "the workload's nodes in a seeded random order (PCG64 seed 11)",
            "cell_order": out["cell"], "caller_order": out["caller"]}


def run_workload(args, name, N, modes_arg):
    """Times the sub-step of one workload in each mode and its kernels;
    returns a dict (the device memory is released on return)."""
    import torch
    from paper_2304_14690_amd import pcorr as pc
    wl = WORKLOADS[name]
    stream = torch.cuda.current_stream()
    print(f"bench: workload {name} N={N}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    case = make_workload(name, N)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    d = case["d"]
    G = int(np.prod(case["n"]))
    M = int(case["kind"].size)
    plan = pc.Plan(d, case["n"], case["h"], bc=case["bc"])
    x = torch.from_numpy(case["x"]).cuda()
    kind = torch.from_numpy(case["kind"]).cuda()
    modes = [m for m in (modes_arg or wl["modes"]).split(",") if m]
    # float32 on a float32-only geometry of its own, after the float64 modes
    # (at 512^3 the two stencil precisions do not fit beside each other)
    f32_own = wl.get("f32_own_geom", False) and "f32" in modes
    x_host = case["x"] if f32_own else None
    case["x"] = None
    want_f32 = "f32" in modes and not f32_own
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # whole time steps only on a box without faces (the first fractional step
    # has no velocity condition of its own on them)
    time_steps = args.time_steps
    if not (case["bc"] and all(b == "periodic" for b in case["bc"])):
        time_steps = 0
    k_self = (16 if d == 2 else 20) if time_steps > 0 else 0
    geom = pc.wls_build(plan, x, kind, case["k"], case["k"], want_f32=want_f32,
                        delta=case.get("delta", 0.0), k_self=k_self)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    del x, kind
    print(f"bench: {name} generated in {t_gen:.1f} s, stencils built in {t_build:.2f} s",
          file=sys.stderr, flush=True)

    results = {}
    ref = None
    near_lines = near_line_fractions(geom, case["n"], d)

    def run_mode(geom, mname):
        nonlocal ref
        mode = pc.MODES["mixed" if mname == "mixed3" else mname]
        sweeps = 3 if mname == "mixed3" else 2
        dtype = torch.float32 if mode == pc.PC_F32 else torch.float64
        u = case["u"].to(dtype)
        uo = torch.empty_like(u)
        p = torch.empty(G, dtype=dtype, device="cuda")
        ws = pc.Workspace(plan, geom, mode)
        stats = None
        for _ in range(args.warmup):
            _, stats = pc.pressure_correct(geom, plan, mode, u, 1.0, uo, p, ws=ws, sweeps=sweeps)
        torch.cuda.synchronize()
        lat = []
        t_start = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            _, stats = pc.pressure_correct(geom, plan, mode, u, 1.0, uo, p, ws=ws, sweeps=sweeps)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        total = time.perf_counter() - t_start
        lat_ms = sorted(1e3 * v for v in lat)
        sec = total / args.steps
        nb = bytes_step(G, M, geom.k_grid, geom.bn, d, "mixed" if mname == "mixed3" else mname,
                        sweeps, stats["n_it"], geom.n_near, geom.near_entries, geom.n_ib,
                        near_lines)
        results[mname] = {
            "value": G / sec,
            "ms_per_step": 1e3 * sec,
            "p50_ms": float(np.percentile(lat_ms, 50)),
            "p99_ms": float(np.percentile(lat_ms, 99)),
            "n_it": stats["n_it"],
            "converged": stats["converged"],
            "sweeps": sweeps if mode == pc.PC_MIXED else None,
            "step_bytes": nb,
            "step_GBs": round(nb / sec / 1e9, 1),
            "step_frac": round(nb / sec / 1e9 / HBM_PEAK_GBS, 4),
        }
        print(f"bench: {name} {mname}: {1e3 * sec:.3f} ms/step, n_it {stats['n_it']}",
              file=sys.stderr, flush=True)
        if mname == "f64":
            ref = (uo.clone(), p.clone(), stats["n_it"])
        elif ref is not None:
            # error against the float64 sub-step at the same iteration count
            _, st2 = pc.pressure_correct(geom, plan, mode, u, 1.0, uo, p, ws=ws, sweeps=sweeps,
                                         fixed_it=ref[2])
            results[mname]["vs_f64"] = {"u": rel_l2(uo, ref[0]), "p": rel_l2(p, ref[1]),
                                        "fixed_it": ref[2]}
        del ws, u, uo, p

    for mname in modes:
        if not (f32_own and mname == "f32"):
            run_mode(geom, mname)

    # ---- per-kernel HIP-event timings (same kernels, same launch shapes) ----------
    def time_launches(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3  # seconds per launch

    u64 = case["u"]
    # the outputs of these launches in one allocation, 256-byte aligned
    # regions, as the sub-step's workspace holds b and phi: the large
    # gathers' speed depends on where their output lands (k_div_all writing
    # into a separate 1 GiB allocation at 512^3 takes 22.8 ms, into a region
    # of a larger block 20.8 ms, inside the sub-step 20.9 ms)
    def aligned(n):
        return (n + 31) // 32 * 32
    blk = torch.empty(2 * aligned(G) + aligned(d * M), dtype=torch.float64, device="cuda")
    b64 = blk[:G]
    phi64 = blk[aligned(G):aligned(G) + G]
    gr64 = blk[2 * aligned(G):2 * aligned(G) + d * M].view(d, M)
    pc.div_to_grid(geom, u64, b64)
    pc.poisson_fft_solve(plan, b64, phi64, pc.PC_F64)
    reps = args.kernel_reps
    t_div = time_launches(lambda: pc.div_to_grid(geom, u64, b64), reps)
    t_solve = time_launches(lambda: pc.poisson_fft_solve(plan, b64, phi64, pc.PC_F64), reps)
    t_grad = time_launches(lambda: pc.grad_to_nodes(geom, phi64, gr64), reps)
    k, bn = geom.k_grid, geom.bn
    n_it = results.get("f64", {}).get("n_it", 1)
    # kernel: (device kernel, bytes per launch, seconds per launch, launches per step);
    # the solve call is 2d-1 kernels (forward passes, fused last-axis pass, inverse passes)
    kern = {
        "div_to_grid": {"kernel": f"k_div_all<double,{d},{k}>",
                        "bytes": bytes_div_all(G, M, k, d, 8), "s": t_div,
                        "launches_per_step": 1, "kernels_per_call": 1},
        "poisson_fft_solve": {"kernel": f"dct_rad x{2 * d - 1}", "bytes": bytes_solve(G, d, 8),
                              "s": t_solve, "launches_per_step": n_it,
                              "kernels_per_call": 2 * d - 1},
        "grad_to_nodes": {"kernel": f"k_grad_all<double,{d},{bn}>",
                          "bytes": bytes_grad(G, M, bn, d, 8),
                          "s": t_grad, "launches_per_step": 1, "kernels_per_call": 1},
    }
    for v in kern.values():
        v["GBs"] = v["bytes"] / v["s"] / 1e9
        v["frac"] = v["GBs"] / HBM_PEAK_GBS
        v["us"] = v["s"] * 1e6
    # the dominant single kernel: largest time per step among one-kernel calls
    single = [n for n in kern if kern[n]["kernels_per_call"] == 1]
    dom = max(single, key=lambda n: kern[n]["s"] * kern[n]["launches_per_step"])
    roof = {"bound": "hbm", "achieved": round(kern[dom]["GBs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(kern[dom]["frac"], 4),
            "traffic": measured_traffic(kern[dom]["kernel"], name, G),
            "kernel": kern[dom]["kernel"], "call": dom, "bytes_per_launch": kern[dom]["bytes"],
            "avg_launch_us": round(kern[dom]["us"], 2)}

    # ---- whole time steps: the first fractional step (Eq. 3) + the sub-step --------
    timestep = None
    if time_steps > 0:
        from paper_2304_14690_amd.timeloop import TimeStepper
        # dt at a convective CFL number of 0.1 for the largest speed of the
        # random-mode field
        dt_ts = 0.1 * min(case["h"]) / float(case["u"].abs().max())
        nu_ts = 1e-3
        u = case["u"].clone()
        u2 = torch.empty_like(u)
        ts = TimeStepper(plan, geom, pc.PC_F64, dt_ts, nu_ts)
        for _ in range(3):
            ts.step(u, u2)
            u, u2 = u2, u
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_its = []
        for _ in range(time_steps):
            st = ts.step(u, u2)
            n_its.append(st["n_it"])
            u, u2 = u2, u
        torch.cuda.synchronize()
        t_step = (time.perf_counter() - t0) / time_steps
        r = torch.empty_like(u)
        us = torch.empty_like(u)
        t_mom = time_launches(lambda: pc.momentum_predict(geom, u, ts.r_prev, dt_ts, nu_ts, r, us),
                              reps)
        bm = bytes_momentum(M, k_self, d, 8)
        timestep = {"ms_per_time_step": round(1e3 * t_step, 4), "steps": time_steps,
                    "dt": dt_ts, "nu": nu_ts, "k_self": k_self,
                    "n_it_per_step": [min(n_its), max(n_its)],
                    "momentum_predict": {"kernel": f"k_momentum<double,{d},{k_self}>",
                                         "us": round(t_mom * 1e6, 2), "bytes": bm,
                                         "GBs": round(bm / t_mom / 1e9, 1),
                                         "frac": round(bm / t_mom / 1e9 / HBM_PEAK_GBS, 4)}}
        del ts, u, u2, r, us
        torch.cuda.synchronize()

    info = {"G": G, "M": M, "k": k, "n_ib": geom.n_ib, "n_near": geom.n_near,
            "build_s": round(t_build, 3), "gen_s": round(t_gen, 3)}
    if f32_own:
        del geom
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        x = torch.from_numpy(x_host).cuda()
        kind = torch.from_numpy(case["kind"]).cuda()
        t0 = time.perf_counter()
        geom = pc.wls_build(plan, x, kind, case["k"], case["k"], f32_only=True,
                            delta=case.get("delta", 0.0))
        torch.cuda.synchronize()
        info["build_f32_only_s"] = round(time.perf_counter() - t0, 3)
        del x, kind, x_host
        run_mode(geom, "f32")
    del ref

    if args.copy_probe:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    del geom, plan, u64, b64, phi64, gr64, blk, case
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    f64 = results.get("f64") or next(iter(results.values()))
    step_roof = {"bound": "hbm", "achieved": f64["step_GBs"], "peak": HBM_PEAK_GBS,
                 "unit": "GB/s", "frac": f64["step_frac"], "bytes_per_step": f64["step_bytes"],
                 "what": "whole float64 sub-step: algorithmic bytes (RHS transfer, n_it "
                         "solves of 2d-1 passes, near-IB updates, IB steps, gradient + "
                         "projection) over the measured time per step"}
    return {"name": name, "N": N, "d": d, "desc": wl["desc"].format(M=M), "info": info,
            "modes": results, "kernels": {n: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                                              for kk, vv in v.items()} for n, v in kern.items()},
            "roofline": roof, "roofline_step": step_roof, "time_step": timestep}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs the sub-step on one GPU; "
                                   "--gpus above 1 is not supported (see the sharding "
                                   "design notes)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    torch.cuda.init()
    dev = torch.cuda.current_device()
    rates = [float(v) for v in args.serve_rate.split(",") if v]
    if args.serve_only:
        print(json.dumps({"serving": serving(args, rates)}))
        return
    wl = WORKLOADS[args.workload]
    N = args.size or wl["N"]
    head = run_workload(args, args.workload, N, args.modes)
    extras = {}
    for name in [w for w in args.extra.split(",") if w and w != args.workload]:
        extras[name] = run_workload(args, name, WORKLOADS[name]["N"], "")
        if WORKLOADS[name]["d"] == 2 and not args.no_shuffle:
            extras[name]["shuffled"] = run_shuffled(args, name, WORKLOADS[name]["N"])
    serving_out = None
    if args.serve_seconds > 0:
        serving_out = serving(args, rates)

    # ---- CPU oracle on a bounded sample ----------------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.workload, args.cpu_size or wl["cpu_N"])
        for name, e in extras.items():
            # 2D workloads at full size: the oracle's stencils fit in host memory
            if WORKLOADS[name]["d"] == 2:
                e["cpu_baseline"] = cpu_baseline(name, e["N"])

    f64 = head["modes"].get("f64") or next(iter(head["modes"].values()))
    out = {
        "metric": f"pressure-correction grid-pts/s (float64 sub-step, {N}^{head['d']})",
        "value": f64["value"],
        "unit": "grid-pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "p50_ms": f64["p50_ms"],
        "p99_ms": f64["p99_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": dict({"workload": head["desc"], "n_it": f64["n_it"]}, **head["info"]),
        "modes": head["modes"],
        "kernels": head["kernels"],
        "roofline": head["roofline"],
        "roofline_step": head["roofline_step"],
        "cpu_baseline": cpu,
        "time_step": head["time_step"],
        "extra": extras,
        "serving": serving_out,
        "device": torch.cuda.get_device_name(dev),
    }
    print(json.dumps(out))


def kernel_source_digest(name):
    """sha256 (16 hex digits) of a kernel's source text, its launch helper,
    and the stencil builder whose layout decides its gather pattern: a
    change to any of them invalidates old counters."""
    import hashlib
    import re
    root = os.path.dirname(os.path.abspath(__file__))
    csrc = os.path.join(root, "paper_2304_14690_amd", "csrc")
    step = open(os.path.join(csrc, "pc_step.hip")).read()
    wls = open(os.path.join(csrc, "pc_wls.hip")).read()
    parts = re.findall(r"template <[^\n]*>\n__global__[^\n]*\b" + name + r"\(.*?\n}\n", step, re.S)
    parts += re.findall(r"\nint launch_" + name[2:] + r"\(.*?\n}\n", step, re.S)
    parts += re.findall(r"template <[^\n]*>\n__global__[^\n]*\bk_grid_stencils\(.*?\n}\n",
                        wls, re.S)
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:16]


def serving(args, rates):
    """The continuous-batching loop on Poisson streams of mixed 2D/3D
    requests (float64 and float32+float64-correction) at each arrival rate,
    against float64 alone on the same slots and float64 one at a time, on the
    same arrivals and the same resident stencils."""
    import torch
    from paper_2304_14690_amd import pcorr as pc, serve
    sizes = [(2, 128), (2, 512), (2, 2048), (3, 64), (3, 128), (3, 256)]
    n_geom = {k: args.serve_geoms for k in sizes}
    n_geom[(3, 256)] = min(args.serve_geoms, 4)
    print("bench: serving", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ds = serve.Dataset(sizes, n_geom, 2, seed=9)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    free, total = torch.cuda.mem_get_info()
    budget = int(free - (16 << 30))
    slots = 4
    ex = serve.GpuExecutor(ds, slots=slots)
    sch = serve.Scheduler(ex, budget=budget, slots=slots)
    # warm-up (untimed): build every geometry's stencils and a workspace per mode
    warm = [serve.Request(i, 0.0, d, N, g, 0, m)
            for i, ((d, N, g), m) in enumerate((k, m) for k in ds.items
                                               for m in (pc.PC_F64, pc.PC_MIXED))]
    t0 = time.perf_counter()
    sch.run(warm)
    t_warm = time.perf_counter() - t0

    def by_size(reqs):
        out = {}
        for (d, N) in sizes:
            lat = [1e3 * r.latency for r in reqs if (r.d, r.N) == (d, N)]
            if lat:
                out[f"{N}^{d}"] = {"n": len(lat), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                                   "p99_ms": round(float(np.percentile(lat, 99)), 3)}
        return out

    runs = []
    for rate in rates:
        n_req = int(round(rate * args.serve_seconds))
        trace = serve.poisson_trace(n_req, rate, 9, sizes, n_geom, 2, [pc.PC_F64, pc.PC_MIXED])
        sch.slots = slots
        mix = sch.run(trace)
        s_mix = serve.summarize(mix)
        s_mix["evictions"] = sch.evictions
        s_mix["peak_gb"] = round(sch.peak_bytes / 2**30, 2)
        s_mix["not_converged"] = sum(1 for r in mix if r.rc != 0)
        base = [serve.Request(r.rid, r.arrival, r.d, r.N, r.geom, r.vel, pc.PC_F64)
                for r in trace]
        out_f64 = sch.run(base)
        s_f64 = serve.summarize(out_f64)
        base = [serve.Request(r.rid, r.arrival, r.d, r.N, r.geom, r.vel, pc.PC_F64)
                for r in trace]
        sch.slots = 1
        out_base = sch.run(base)
        s_base = serve.summarize(out_base)
        print(f"bench: serving at {rate:g}/s done", file=sys.stderr, flush=True)
        runs.append({
            "workload": f"Poisson arrivals {rate:g}/s for {args.serve_seconds:g} s, sizes uniform "
                        "over 128^2, 512^2, 2048^2, 64^3, 128^3, 256^3, precision uniform over "
                        "f64 and f32+f64 correction (2 sweeps), "
                        f"{slots} slots, stencils resident per geometry (LRU under the HBM "
                        "budget)",
            "rate": rate, "geometries": sum(n_geom.values()),
            "budget_gb": round(budget / 2**30, 1),
            "setup_s": {"data": round(t_data, 2), "warm_build": round(t_warm, 2)},
            "mix": s_mix, "fp64_batched": s_f64, "fp64_one_at_a_time": s_base,
            "per_size": {"mix": by_size(mix), "fp64_batched": by_size(out_f64),
                         "fp64_one_at_a_time": by_size(out_base)}})
    sch.release()
    del ex, sch, ds
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return runs


def measured_traffic(kernel, workload, G):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy
    of known size), or None when the summary is absent, was taken at another
    size, or the kernel source has changed since it was taken."""
    root = os.path.dirname(os.path.abspath(__file__))
    name = kernel.split("<")[0]
    path = os.path.join(root, "profiles", f"{name}_{workload}.traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            key, val = line.split(":", 1)
            vals[key.strip()] = val.strip()
    if vals.get("kernel") != name or vals.get("source_sha256_16") != kernel_source_digest(name) \
            or int(vals.get("G", -1)) != G:
        return None
    return float(vals["hbm_bytes_per_launch"])


def cpu_baseline(workload, N):
    """The float64 oracle's sub-step on this host: the same workload at N^d
    (same obstacles, stencil size and modes), stencils built first and not
    timed, median of three timed sub-steps."""
    import oracle
    from oracle import projection as P
    from paper_2304_14690_amd import inputs
    cores = len(os.sched_getaffinity(0))
    bc = WORKLOADS[workload].get("bc")
    delta = None
    if workload == "2d1024c":
        c = inputs.coarse_grid_case(workload, 2, N, 2 * N,
                                    [inputs.Obstacle("circle", (0.3, 0.5), (0.05,))],
                                    16, 16, 32, 3, 4)
        delta = 1.0 / (2 * N)
    elif workload == "2d400sq":
        c = inputs.make_case(workload, 2, N, [inputs.Obstacle("box", (0.45, 0.45), (0.55, 0.55))],
                             16, 16, 32, 3, 4, bc=bc)
    elif workload in ("2d2048", "2d2000", "2d2048p", "2d2048pp"):
        c = inputs.make_case(workload, 2, N, [inputs.Obstacle("circle", (0.3, 0.5), (0.05,))],
                             16, 16, 32, 3, 4, bc=bc)
    elif workload in ("3d256", "3d256p", "3d256pp"):
        c = inputs.make_case(workload, 3, N, [inputs.Obstacle("sphere", (0.5, 0.5, 0.5), (0.1,))],
                             27, 27, 64, 5, 6, bc=bc)
    else:
        c = inputs.config4(N)
    grid = oracle.Grid(c.d, c.n, c.h, bc)
    t0 = time.perf_counter()
    st = P.build_stencils(grid, c.x.T.copy(), c.kind, c.k_grid, c.k_node, workers=cores,
                          delta=delta)
    t_build = time.perf_counter() - t0
    u = c.u.T.copy()
    times = []
    n_it = None
    for _ in range(3):
        t0 = time.perf_counter()
        r = P.pressure_correct(st, u)
        times.append(time.perf_counter() - t0)
        n_it = r["n_it"]
    t = statistics.median(times)
    note = WORKLOADS[workload].get("cpu_note") if N != WORKLOADS[workload]["N"] else None
    return {"value": c.G / t, "unit": "grid-pts/s", "cores": cores, "kind": "oracle",
            "sample": f"the same workload at {N}^{c.d} ({c.M} nodes), float64 oracle sub-step, "
                      f"median of 3, n_it={n_it}; stencil build {t_build:.1f}s not timed"
                      + (f" ({note})" if note else ""),
            "s_per_step": t}


if __name__ == "__main__":
    main()
