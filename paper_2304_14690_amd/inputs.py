"""Seeded synthetic inputs for the hybrid pressure-correction step.

This module only *describes* a workload: where the meshless nodes sit, which
of them are fluid (F), boundary (B) or virtual (V) points, and the provisional
velocity u* carried by them.  It holds none of the method's arithmetic (no
stencils, no transforms, no projection), so the CPU oracle and the HIP library
can both be fed from it without sharing any of the computation they are
compared on.

Geometry follows the double discretisation of Sec. 2.3 (Fig. 1): a uniform
cell-centred pressure grid over the box [0, L]^d, plus an irregular cloud of
velocity points.  The cloud is a jittered lattice (one node per grid cell,
each coordinate displaced by U(-0.3 h, 0.3 h)); lattice nodes that fall
inside an obstacle become virtual points (the frozen fluid of Sec. 2.3), and
boundary points are laid on the obstacle surface at the lattice spacing.
The provisional velocity is a sum of random Fourier modes evaluated at F and
B points and set to zero at V points (Sec. 2.3: the virtual points carry a
zero intermediate velocity).  On a box with periodic axes (the lateral
condition of the verification cases of Sec. 3) obstacles wrap around the
periodic faces, every position lies in [0, L) along those axes, and the
modes (integer wavenumbers on the unit box) are periodic.

Random streams: numpy.random.Generator(PCG64(seed)).  The node seed drives the
jitter only; the velocity seed drives the mode draw in the order wavenumber
magnitudes, wavenumber signs, phases, amplitudes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

KIND_F = 0
KIND_B = 1
KIND_V = 2


@dataclasses.dataclass
class Obstacle:
    """A solid body immersed in the box.  shape: 'circle' (2D), 'sphere'
    (3D) or 'box' (2D/3D axis-aligned).  For circle/sphere `a` is the centre
    and `b` holds the radius; for a box `a` and `b` are the low/high corners."""
    shape: str
    a: Tuple[float, ...]
    b: Tuple[float, ...]

    def inside(self, x: np.ndarray, lengths=None) -> np.ndarray:
        """x: [T, d].  Strictly-inside test (points on the surface are fluid).
        lengths[a] (not None): axis a is periodic with that box length, and a
        circle/sphere wraps around it."""
        if self.shape in ("circle", "sphere"):
            c = np.asarray(self.a, dtype=np.float64)
            r = float(self.b[0])
            dx = x - c[None, :]
            if lengths is not None:
                for a, L in enumerate(lengths):
                    if L is not None:
                        dx[:, a] -= L * np.round(dx[:, a] / L)
            return np.einsum("td,td->t", dx, dx) < r * r
        if self.shape == "box":
            lo = np.asarray(self.a, dtype=np.float64)
            hi = np.asarray(self.b, dtype=np.float64)
            return np.all((x > lo[None, :]) & (x < hi[None, :]), axis=1)
        raise ValueError(self.shape)

    def surface_points(self, delta: float) -> np.ndarray:
        """Boundary points at spacing ~delta.  Returns [Nb, d]."""
        if self.shape == "circle":
            cx, cy = self.a
            r = float(self.b[0])
            nb = max(3, int(round(2.0 * math.pi * r / delta)))
            th = 2.0 * math.pi * np.arange(nb, dtype=np.float64) / nb
            return np.stack([cx + r * np.cos(th), cy + r * np.sin(th)], axis=1)
        if self.shape == "sphere":
            c = np.asarray(self.a, dtype=np.float64)
            r = float(self.b[0])
            nb = max(4, int(round(4.0 * math.pi * r * r / (delta * delta))))
            j = np.arange(nb, dtype=np.float64)
            z = 1.0 - (2.0 * j + 1.0) / nb
            rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
            ang = j * (math.pi * (3.0 - math.sqrt(5.0)))  # golden angle
            p = np.stack([rho * np.cos(ang), rho * np.sin(ang), z], axis=1)
            return c[None, :] + r * p
        if self.shape == "box":
            lo = np.asarray(self.a, dtype=np.float64)
            hi = np.asarray(self.b, dtype=np.float64)
            d = lo.size
            pts = []
            for ax in range(d):
                others = [o for o in range(d) if o != ax]
                cnt = [max(1, int(round((hi[o] - lo[o]) / delta))) for o in others]
                axes = [lo[o] + (np.arange(c, dtype=np.float64) + 0.5) * (hi[o] - lo[o]) / c
                        for o, c in zip(others, cnt)]
                mesh = np.meshgrid(*axes, indexing="ij")
                flat = [m.reshape(-1) for m in mesh]
                for face in (lo[ax], hi[ax]):
                    q = np.empty((flat[0].size, d), dtype=np.float64)
                    q[:, ax] = face
                    for o, f in zip(others, flat):
                        q[:, o] = f
                    pts.append(q)
            return np.concatenate(pts, axis=0)
        raise ValueError(self.shape)


@dataclasses.dataclass
class Case:
    """One synthetic pressure-correction problem.

    x    : [d, M] float64 node positions (structure of arrays)
    kind : [M] uint8, KIND_F / KIND_B / KIND_V
    u    : [d, M] float64 provisional velocity u* (zero on V)
    n, h : cells per axis and spacing per axis of the pressure grid
    """
    name: str
    d: int
    n: Tuple[int, ...]
    h: Tuple[float, ...]
    x: np.ndarray
    kind: np.ndarray
    u: np.ndarray
    dt: float
    k_grid: int
    k_node: int
    obstacles: List[Obstacle]

    @property
    def M(self) -> int:
        return int(self.kind.size)

    @property
    def G(self) -> int:
        return int(np.prod(self.n))

    def counts(self):
        return {k: int(np.count_nonzero(self.kind == v))
                for k, v in (("F", KIND_F), ("B", KIND_B), ("V", KIND_V))}


def jittered_lattice(n: Sequence[int], h: Sequence[float], seed: int,
                     jitter: float = 0.3) -> np.ndarray:
    """One node per grid cell at the cell centre plus U(-jitter*h, jitter*h)
    per coordinate.  Lattice order is x-fastest.  Returns [d, prod(n)]."""
    d = len(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    G = int(np.prod(n))
    off = rng.uniform(-jitter, jitter, size=(G, d))
    idx = np.indices(tuple(reversed(n)), dtype=np.float64)  # [d, n_last, ..., n_x]
    x = np.empty((d, G), dtype=np.float64)
    for ax in range(d):
        centre = (idx[d - 1 - ax].reshape(-1) + 0.5) * h[ax]
        x[ax] = centre + off[:, ax] * h[ax]
    return x


def fourier_modes(d: int, n_modes: int, seed: int, kmax: int = 4):
    """The random modes of the provisional velocity: wavenumbers k_m in
    {+-1..+-kmax}^d (magnitudes, then signs), phases theta_m ~ U[0, 2pi),
    amplitudes a_m ~ N(0, I_d), drawn in that order.  Returns (k [K, d],
    theta [K], a [K, d])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kmag = rng.integers(1, kmax + 1, size=(n_modes, d))
    sgn = rng.choice(np.array([-1, 1]), size=(n_modes, d))
    kvec = (kmag * sgn).astype(np.float64)
    theta = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    amp = rng.standard_normal(size=(n_modes, d))
    return kvec, theta, amp


def fourier_velocity(x: np.ndarray, n_modes: int, seed: int, kmax: int = 4,
                     chunk: int = 1 << 20) -> np.ndarray:
    """u*(x) = sum_m a_m cos(2 pi k_m . x + theta_m), k_m in {+-1..+-kmax}^d,
    theta_m ~ U[0, 2pi), a_m ~ N(0, I_d).  x: [d, M].  Returns [d, M].
    a_m is not orthogonal to k_m, so the field is divergent."""
    d, M = x.shape
    kvec, theta, amp = fourier_modes(d, n_modes, seed, kmax)
    u = np.zeros((d, M), dtype=np.float64)
    for s in range(0, M, chunk):
        e = min(M, s + chunk)
        ph = 2.0 * math.pi * (kvec @ x[:, s:e]) + theta[:, None]  # [K, T]
        u[:, s:e] = amp.T @ np.cos(ph)
    return u


def fourier_velocity_torch(x, n_modes: int, seed: int, kmax: int = 4):
    """The same field as fourier_velocity, evaluated with torch on x's device
    (x: [d, M] float64 tensor): the same modes, summed mode by mode (the
    rounding differs from fourier_velocity's matrix products)."""
    import torch
    d = x.shape[0]
    kvec, theta, amp = fourier_modes(d, n_modes, seed, kmax)
    u = torch.zeros_like(x)
    for m in range(n_modes):
        ph = x[0] * float(kvec[m, 0])
        for a in range(1, d):
            ph = ph + x[a] * float(kvec[m, a])
        c = torch.cos(ph * (2.0 * math.pi) + float(theta[m]))
        for a in range(d):
            u[a].add_(c, alpha=float(amp[m, a]))
    return u


def wrap_into_box(p: np.ndarray, lengths) -> np.ndarray:
    """Positions [T, d] moved into [0, L) along the periodic axes (lengths[a]
    not None)."""
    p = p.copy()
    for a, L in enumerate(lengths):
        if L is not None:
            v = np.mod(p[:, a], L)
            v[v >= L] = 0.0  # a tiny negative coordinate rounds up to L
            p[:, a] = v
    return p


def make_geometry(d: int, N: int, obstacles: Sequence[Obstacle], seed_nodes: int,
                  jitter: float = 0.3, L: float = 1.0, bc=None):
    """Node positions [d, M] and kinds [M] of a jittered lattice with the
    obstacles' interior nodes turned virtual and their surface points
    appended as boundary points.  bc: per-axis "neumann"/"periodic" (None:
    Neumann everywhere)."""
    n = tuple([N] * d)
    h = tuple([L / N] * d)
    return make_geometry_n(n, h, obstacles, seed_nodes, jitter, bc)


def make_geometry_n(n: Sequence[int], h: Sequence[float], obstacles: Sequence[Obstacle],
                    seed_nodes: int, jitter: float = 0.3, bc=None):
    """make_geometry for any grid shape n and spacing h."""
    n, h = tuple(n), tuple(h)
    d = len(n)
    lengths = None
    if bc is not None and any(b == "periodic" for b in bc):
        lengths = tuple(n[a] * h[a] if bc[a] == "periodic" else None for a in range(d))
    lat = jittered_lattice(n, h, seed_nodes, jitter)
    pts = lat.T
    inside = np.zeros(pts.shape[0], dtype=bool)
    for ob in obstacles:
        inside |= ob.inside(pts, lengths)
    kind = np.where(inside, KIND_V, KIND_F).astype(np.uint8)
    delta = h[0] if all(v == h[0] for v in h) else math.exp(sum(math.log(v) for v in h) / d)
    surf = [ob.surface_points(delta) for ob in obstacles]
    if lengths is not None:
        surf = [wrap_into_box(sp, lengths) for sp in surf]
    if surf:
        bpts = np.concatenate(surf, axis=0)
        x = np.concatenate([lat, bpts.T], axis=1)
        kind = np.concatenate([kind, np.full(bpts.shape[0], KIND_B, np.uint8)])
    else:
        x = lat
    return n, h, np.ascontiguousarray(x), kind


def make_case(name: str, d: int, N: int, obstacles: Sequence[Obstacle], k_grid: int,
              k_node: int, n_modes: int, seed_nodes: int, seed_vel: int,
              jitter: float = 0.3, kmax: int = 4, dt: float = 1.0,
              L: float = 1.0, bc=None) -> Case:
    n, h, x, kind = make_geometry(d, N, obstacles, seed_nodes, jitter, L, bc)
    u = fourier_velocity(x, n_modes, seed_vel, kmax)
    u[:, kind == KIND_V] = 0.0
    return Case(name, d, n, h, x, kind, np.ascontiguousarray(u), dt, k_grid, k_node,
                list(obstacles))


# ---- the five workloads ------------------------------------------------------

def config1() -> Case:
    """64^2 grid, 4096 jittered nodes, circle R=0.1 at the centre, 12-NN,
    8 Fourier modes (seeds 1/2): the single-projection parity case."""
    return make_case("cfg1_64sq", 2, 64, [Obstacle("circle", (0.5, 0.5), (0.1,))],
                     12, 12, 8, 1, 2)


def config2(N: int = 2048) -> Case:
    """2048^2 grid, 4.2M jittered nodes, cylinder R=0.05 at (0.3, 0.5),
    16-NN, 32 modes (seeds 3/4)."""
    return make_case(f"cfg2_{N}sq", 2, N, [Obstacle("circle", (0.3, 0.5), (0.05,))],
                     16, 16, 32, 3, 4)


def config3(N: int = 256) -> Case:
    """256^3 grid, 16.8M jittered nodes, sphere R=0.1 at the centre, 27-NN,
    64 modes (seeds 5/6)."""
    return make_case(f"cfg3_{N}cube", 3, N,
                     [Obstacle("sphere", (0.5, 0.5, 0.5), (0.1,))], 27, 27, 64, 5, 6)


def config4(N: int = 512) -> Case:
    """512^3 grid, 134M nodes, sphere R=0.1 at (0.3,0.5,0.5) plus the box
    [0.6,0.8]x[0.4,0.6]^2, 27-NN, 64 modes (seeds 7/8)."""
    return make_case(f"cfg4_{N}cube", 3, N,
                     [Obstacle("sphere", (0.3, 0.5, 0.5), (0.1,)),
                      Obstacle("box", (0.6, 0.4, 0.4), (0.8, 0.6, 0.6))], 27, 27, 64, 7, 8)


def coarse_grid_case(name: str, d: int, N_grid: int, N_nodes: int,
                     obstacles: Sequence[Obstacle], k_grid: int, k_node: int, n_modes: int,
                     seed_nodes: int, seed_vel: int) -> Case:
    """A pressure grid coarser than the velocity cloud (the 256^2 grid under
    a 400^2-density cloud of Sec. 3): an N_nodes^d jittered lattice of
    spacing 1/N_nodes on the unit box, with the pressure grid of N_grid
    cells per axis.  The case's n, h are the grid's; the node spacing is
    1/N_nodes (pass it as the WLS mean spacing)."""
    n_nodes = tuple([N_nodes] * d)
    h_nodes = tuple([1.0 / N_nodes] * d)
    _, _, x, kind = make_geometry_n(n_nodes, h_nodes, obstacles, seed_nodes)
    u = fourier_velocity(x, n_modes, seed_vel)
    u[:, kind == KIND_V] = 0.0
    n = tuple([N_grid] * d)
    h = tuple([1.0 / N_grid] * d)
    return Case(name, d, n, h, x, kind, np.ascontiguousarray(u), 1.0, k_grid, k_node,
                list(obstacles))


def serving_geometry(d: int, N: int, seed: int):
    """Geometry of one serving request family: a circle/sphere of radius
    U(0.05, 0.15) centred in U(0.3, 0.7)^d over its own jittered cloud.
    Returns (obstacles, node seed, velocity seed, k, modes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = float(rng.uniform(0.05, 0.15))
    c = tuple(float(v) for v in rng.uniform(0.3, 0.7, size=d))
    s_nodes, s_vel = (int(v) for v in rng.integers(0, 2**31 - 1, size=2))
    k = 16 if d == 2 else 27
    shape = "circle" if d == 2 else "sphere"
    return [Obstacle(shape, c, (R,))], s_nodes, s_vel, k, (32 if d == 2 else 64)


def serving_case(d: int, N: int, seed: int, k: Optional[int] = None) -> Case:
    """One request of the serving stream: its own node cloud, circle/sphere of
    radius U(0.05, 0.15) centred in U(0.3, 0.7)^d, and a random-mode field."""
    obs, s_nodes, s_vel, k0, modes = serving_geometry(d, N, seed)
    k = k if k is not None else k0
    return make_case(f"serve_{d}d_{N}_{seed}", d, N, obs, k, k, modes, s_nodes, s_vel)
