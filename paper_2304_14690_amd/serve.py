"""Continuous-batching request loop for pressure-correction sub-steps.

Requests of mixed 2D/3D grid sizes arrive over time.  Each one names a
grid size, one geometry of a per-size pool (node cloud + obstacle), a
velocity field and a precision (PC_F64 or PC_MIXED).  The loop

  * keeps the per-size transform tables (plans) resident for the whole run;
  * keeps WLS stencils resident per geometry in an LRU cache under an HBM
    budget (stencils are built once per geometry, Sec. 2.2, and evicted only
    when an admission needs the room and nothing running uses them);
  * admits a waiting request when a slot (a HIP stream with its own host
    thread) is free and its memory fits: FIFO, with smaller requests allowed
    to go ahead of a head that does not fit, at most `max_skip` times per
    head, so the head cannot starve;
  * runs admitted requests concurrently on their slots' streams, so that
    their kernels overlap on the device;
  * records arrival, admission, start and completion times per request.

All device work goes through an executor.  GpuExecutor drives the C ABI
(libpcorr) through the Python binding; the scheduler itself is plain Python
and is tested on the CPU with a fake executor.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import queue
import threading
import time
from typing import Dict, List, Optional, Tuple

import numpy as np

GeomKey = Tuple[int, int, int]  # (d, N, geometry index in the pool)


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    d: int
    N: int
    geom: int               # index into the size's geometry pool
    vel: int                # index into the geometry's velocity pool
    mode: int               # PC_F64 or PC_MIXED
    # filled in by the loop
    admitted: float = math.nan
    done: float = math.nan
    slot: int = -1
    n_it: int = 0
    rc: int = 0
    built: bool = False     # the stencils were built for this request
    skipped: int = 0        # times another request was admitted ahead of it
    result: Optional[dict] = None

    @property
    def key(self) -> GeomKey:
        return (self.d, self.N, self.geom)

    @property
    def G(self) -> int:
        return self.N ** self.d

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def poisson_trace(n_req: int, rate: float, seed: int, sizes, n_geom: Dict, n_vel: int,
                  modes) -> List[Request]:
    """Requests with exponential inter-arrival times (Poisson arrivals at
    `rate` per second); size, geometry, velocity and precision drawn
    uniformly from the given pools."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=n_req)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_req):
        d, N = sizes[int(rng.integers(0, len(sizes)))]
        g = int(rng.integers(0, n_geom[(d, N)]))
        v = int(rng.integers(0, n_vel))
        m = modes[int(rng.integers(0, len(modes)))]
        out.append(Request(i, float(t[i]), d, N, g, v, m))
    return out


# ---- the scheduler -------------------------------------------------------------------

class _Resident:
    __slots__ = ("handle", "bytes", "users", "last", "building", "ready")

    def __init__(self, handle, nbytes):
        self.handle = handle
        self.bytes = nbytes
        self.users = 0
        self.last = 0.0
        self.building = False          # a worker is building it
        self.ready = threading.Event()  # set once built (or failed)
        if handle is not None:
            self.ready.set()


class Scheduler:
    """Admission, residency and dispatch.  `executor` does the device work;
    `budget` bounds the bytes of everything the loop holds: resident
    stencils, pooled workspaces and the fields of running requests."""

    def __init__(self, executor, budget: int, slots: int = 4, max_skip: int = 8):
        if slots < 1:
            raise ValueError("at least one slot")
        self.ex = executor
        self.budget = int(budget)
        self.slots = slots
        self.max_skip = max_skip
        self.geoms: "collections.OrderedDict[GeomKey, _Resident]" = collections.OrderedDict()
        self.ws_pool: Dict[Tuple[GeomKey, int], List[_Resident]] = {}
        self.inflight_bytes = 0
        self.peak_bytes = 0
        self.evictions = 0
        self.builds = 0
        self._lock = threading.Lock()

    # -- accounting (called with the lock held) --
    def _held(self) -> int:
        b = sum(r.bytes for r in self.geoms.values())
        b += sum(w.bytes for ws in self.ws_pool.values() for w in ws)
        return b + self.inflight_bytes

    def _need(self, r: Request) -> int:
        """Bytes admission must find for r: its stencils unless resident, a
        workspace unless one is pooled, and its output fields."""
        need = self.ex.field_bytes(r.key, r.mode)
        g = self.geoms.get(r.key)
        if g is None:
            need += self.ex.geometry_bytes(r.key)
        if not self.ws_pool.get((r.key, r.mode)):
            need += self.ex.workspace_bytes(r.key, r.mode, g.handle if g is not None else None)
        return need

    def _evict_for(self, need: int, keep: GeomKey, keep_mode: int) -> bool:
        """Frees idle residents, least recently used first, until `need`
        bytes fit.  The geometry `keep` and its pooled workspaces of
        `keep_mode` stay: `need` was computed counting on them.  Returns
        whether they fit."""
        while self._held() + need > self.budget:
            victim = None
            for k, g in self.geoms.items():  # oldest first
                if g.users == 0 and k != keep:
                    victim = k
                    break
            if victim is None:
                # pooled workspaces of idle geometries go with them; a pooled
                # workspace of `keep` in another mode can go alone
                for (k, m), ws in self.ws_pool.items():
                    if ws and (k, m) != (keep, keep_mode):  # pooled ones are idle
                        w = ws.pop()
                        self.ex.free_workspace(w.handle)
                        self.evictions += 1
                        break
                else:
                    return False
                continue
            g = self.geoms.pop(victim)
            for m in list(self.ws_pool):
                if m[0] == victim:
                    for w in self.ws_pool.pop(m):
                        self.ex.free_workspace(w.handle)
            if g.handle is not None:
                self.ex.free_geometry(g.handle)
            self.evictions += 1
        return True

    # -- the loop --
    def run(self, requests: List[Request], clock=time.perf_counter) -> List[Request]:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        done_q: "queue.Queue[Tuple[Request, int, BaseException]]" = queue.Queue()
        work_q = [queue.Queue() for _ in range(self.slots)]
        free_slots = list(range(self.slots))
        t0 = clock()

        def worker(slot):
            while True:
                item = work_q[slot].get()
                if item is None:
                    return
                r, g_res, ws_res, field_bytes = item
                err = None
                try:
                    # the first request of a geometry builds its stencils;
                    # others admitted meanwhile wait for them
                    with self._lock:
                        mine = g_res.handle is None and not g_res.building
                        if mine:
                            g_res.building = True
                    if mine:
                        try:
                            g_res.handle = self.ex.build_geometry(r.key, slot)
                            r.built = True
                        finally:
                            g_res.ready.set()
                    g_res.ready.wait()
                    if g_res.handle is None:
                        raise RuntimeError(f"stencils of {r.key} were not built")
                    if ws_res.handle is None:
                        ws_res.handle = self.ex.make_workspace(r.key, g_res.handle, r.mode)
                    r.result = self.ex.run(r, g_res.handle, ws_res.handle, slot)
                    r.n_it = int(r.result.get("n_it", 0)) if r.result else 0
                    r.rc = int(r.result.get("rc", 0)) if r.result else 0
                except BaseException as e:  # reported by the dispatcher
                    err = e
                r.done = clock() - t0
                done_q.put((r, slot, err, g_res, ws_res, field_bytes))

        threads = [threading.Thread(target=worker, args=(i,), daemon=True)
                   for i in range(self.slots)]
        for th in threads:
            th.start()

        pending: List[Request] = []
        nxt = 0
        n_done = 0
        error = None
        try:
            while n_done < len(reqs):
                now = clock() - t0
                while nxt < len(reqs) and reqs[nxt].arrival <= now:
                    pending.append(reqs[nxt])
                    nxt += 1
                # admissions
                with self._lock:
                    i = 0
                    while free_slots and i < len(pending):
                        r = pending[i]
                        head_blocked = i > 0 and pending[0].skipped >= self.max_skip
                        if head_blocked:
                            break
                        need = self._need(r)
                        if need > self.budget:
                            raise MemoryError(f"request {r.rid} needs {need} bytes, "
                                              f"more than the budget {self.budget}")
                        if not self._evict_for(need, r.key, r.mode):
                            i += 1
                            continue
                        # admit r
                        for q in pending[:i]:
                            q.skipped += 1
                        pending.pop(i)
                        slot = free_slots.pop(0)
                        g = self.geoms.get(r.key)
                        if g is None:
                            g = _Resident(None, self.ex.geometry_bytes(r.key))
                            self.geoms[r.key] = g
                            self.builds += 1
                        self.geoms.move_to_end(r.key)
                        g.users += 1
                        g.last = now
                        pool = self.ws_pool.setdefault((r.key, r.mode), [])
                        if pool:
                            ws = pool.pop()
                        else:
                            ws = _Resident(None, self.ex.workspace_bytes(r.key, r.mode, g.handle))
                        fb = self.ex.field_bytes(r.key, r.mode)
                        self.inflight_bytes += ws.bytes + fb
                        self.peak_bytes = max(self.peak_bytes, self._held())
                        r.admitted = now
                        r.slot = slot
                        work_q[slot].put((r, g, ws, fb))
                # wait for a completion or the next arrival
                timeout = None
                if nxt < len(reqs):
                    timeout = max(0.0, reqs[nxt].arrival - (clock() - t0))
                try:
                    item = done_q.get(timeout=timeout)
                except queue.Empty:
                    continue
                while True:
                    r, slot, err, g, ws, fb = item
                    n_done += 1
                    with self._lock:
                        g.users -= 1
                        self.inflight_bytes -= ws.bytes + fb
                        if ws.handle is not None:
                            self.ws_pool.setdefault((r.key, r.mode), []).append(ws)
                        if g.handle is not None:
                            g.bytes = self.ex.actual_geometry_bytes(g.handle, g.bytes)
                        elif g.users == 0 and self.geoms.get(r.key) is g:
                            del self.geoms[r.key]  # its build failed
                        free_slots.append(slot)
                        free_slots.sort()
                    if err is not None and error is None:
                        error = err
                    try:
                        item = done_q.get_nowait()
                    except queue.Empty:
                        break
                if error is not None:
                    raise error
        finally:
            for q in work_q:
                q.put(None)
            for th in threads:
                th.join(timeout=60)
        return reqs

    def release(self):
        """Frees everything the loop holds."""
        with self._lock:
            for ws in self.ws_pool.values():
                for w in ws:
                    self.ex.free_workspace(w.handle)
            self.ws_pool.clear()
            for g in self.geoms.values():
                if g.handle is not None:
                    self.ex.free_geometry(g.handle)
            self.geoms.clear()


def summarize(reqs: List[Request]) -> dict:
    """p50/p99/mean latency, throughput in grid points per second over the
    span of the run, and device utilisation (fraction of the span with at
    least one request running)."""
    lat = np.array([r.latency for r in reqs]) * 1e3
    start = min(r.arrival for r in reqs)
    end = max(r.done for r in reqs)
    span = end - start
    iv = sorted((r.admitted, r.done) for r in reqs)
    busy, cur_s, cur_e = 0.0, None, None
    for s, e in iv:
        if cur_e is None or s > cur_e:
            if cur_e is not None:
                busy += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    if cur_e is not None:
        busy += cur_e - cur_s
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()), "grid_pts_per_s": sum(r.G for r in reqs) / span,
            "span_s": span, "utilisation": busy / span if span > 0 else 0.0,
            "builds": sum(1 for r in reqs if r.built)}


# ---- the device executor -------------------------------------------------------------

class Dataset:
    """The per-size pools the requests draw from: node clouds, kinds and
    velocity fields, already in HBM (client data, not held by the loop)."""

    def __init__(self, sizes, n_geom: Dict, n_vel: int, seed: int, device="cuda"):
        import torch
        from . import inputs
        self.items = {}
        rng = np.random.Generator(np.random.PCG64(seed))
        for (d, N) in sizes:
            for gi in range(n_geom[(d, N)]):
                gseed = int(rng.integers(0, 2**31 - 1))
                obs, s_nodes, s_vel, k, modes = inputs.serving_geometry(d, N, gseed)
                n, h, x, kind = inputs.make_geometry(d, N, obs, s_nodes)
                xt = torch.from_numpy(x).to(device)
                kt = torch.from_numpy(kind).to(device)
                vmask = (kt == inputs.KIND_V)
                us = []
                for vi in range(n_vel):
                    u = inputs.fourier_velocity_torch(xt, modes, s_vel + vi)
                    u[:, vmask] = 0.0
                    us.append(u)
                self.items[(d, N, gi)] = {"n": n, "h": h, "x": xt, "kind": kt, "u": us,
                                          "k": k, "M": int(kind.size), "seed": gseed}

    def __getitem__(self, key):
        return self.items[key]


class GpuExecutor:
    """Device work of the loop through libpcorr: plans per size (resident),
    stencils per geometry, workspaces, and the sub-step on a slot's stream."""

    def __init__(self, dataset: Dataset, slots: int, sweeps: int = 2, keep_results=False):
        import torch
        from . import pcorr
        self.pc = pcorr
        self.torch = torch
        self.data = dataset
        self.streams = [torch.cuda.Stream() for _ in range(slots)]  # default priority
        self.plans = {}
        self.sweeps = sweeps
        self.keep_results = keep_results
        self._plan_lock = threading.Lock()

    def plan(self, d, N):
        with self._plan_lock:
            if (d, N) not in self.plans:
                it = next(v for k, v in self.data.items.items() if k[:2] == (d, N))
                self.plans[(d, N)] = self.pc.Plan(d, it["n"], it["h"])
            return self.plans[(d, N)]

    # Sizes used for admission, from the library's own accounting
    # (pc_geom_footprint before a geometry exists, pc_workspace_bytes and
    # pc_geom_info after).  The near-IB point count is known only after the
    # build; admission bounds it by four times the B+V nodes (about one near
    # point per B+V node for these obstacles: the grid points inside the body
    # and a thin shell around it).
    def _footprint(self, key):
        it = self.data[key]
        if "footprint" not in it:
            d, N, _ = key
            n_ib = int((it["kind"] != 0).sum().item())
            it["n_ib"] = n_ib
            it["footprint"] = self.pc.geom_footprint(self.plan(d, N), it["M"], n_ib,
                                                     min(N ** d, 4 * n_ib + 64), it["k"],
                                                     it["k"])
        return it["footprint"]

    def geometry_bytes(self, key) -> int:
        """Device bytes a build of key's stencils needs at its peak."""
        return self._footprint(key)[1]

    def actual_geometry_bytes(self, handle, estimate) -> int:
        return int(handle.bytes)

    def workspace_bytes(self, key, mode, geom=None) -> int:
        if geom is not None:
            d, N, _ = key
            return self.pc.workspace_bytes(self.plan(d, N), geom, mode)
        return self._footprint(key)[2][mode]

    def field_bytes(self, key, mode) -> int:
        d, N, _ = key
        return int(d * self.data[key]["M"] * 8 + N ** d * 8)

    def build_geometry(self, key, slot):
        it = self.data[key]
        plan = self.plan(key[0], key[1])
        with self.torch.cuda.stream(self.streams[slot]):
            return self.pc.wls_build(plan, it["x"], it["kind"], it["k"], it["k"],
                                     stream=self.streams[slot])

    def free_geometry(self, handle):
        del handle

    def make_workspace(self, key, geom, mode):
        return self.pc.Workspace(self.plan(key[0], key[1]), geom, mode)

    def free_workspace(self, handle):
        del handle

    def run(self, r: Request, geom, ws, slot):
        torch = self.torch
        it = self.data[r.key]
        s = self.streams[slot]
        plan = self.plan(r.d, r.N)
        u = it["u"][r.vel]
        with torch.cuda.stream(s):
            uo = torch.empty_like(u)
            p = torch.empty(r.G, dtype=torch.float64, device=u.device)
            rc, st = self.pc.pressure_correct(geom, plan, r.mode, u, 1.0, uo, p, ws=ws,
                                              stream=s, sweeps=self.sweeps)
        out = {"rc": rc, "n_it": st["n_it"], "converged": st["converged"]}
        if self.keep_results:
            s.synchronize()
            out["u"] = uo.cpu().numpy()
            out["p"] = p.cpu().numpy()
        return out
