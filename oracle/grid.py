"""Uniform cell-centred pressure grid over an extended rectangular box
(Sec. 2.3, double discretisation, Fig. 1; staggered placement as used with
Neumann walls in Sec. 3.3).  Test infrastructure only."""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Grid:
    d: int
    n: Tuple[int, ...]      # cells per axis
    h: Tuple[float, ...]    # spacing per axis; box is [0, n_a h_a]
    # boundary condition per axis: "neumann" (homogeneous, Eq. 7, mirror
    # ghosts) or "periodic" (the lateral condition of the paper's cases in
    # Sec. 3); None means Neumann everywhere
    bc: Optional[Tuple[str, ...]] = None
    # eigenvalues of the solve: "fd2" (central differences, the variant of
    # the reported timings, Sec. 3.2) or "spectral" (pseudo-spectral, one of
    # the variants Sec. 3 reports as giving no noticeable difference)
    eig: str = "fd2"
    # grid points at the cell centres (i + 1/2) h (the staggered grid of the
    # paper's timings) or at the vertices i h of n - 1 intervals (the regular
    # grid, a variant Sec. 3 reports as interchangeable; Neumann axes only)
    vertex: bool = False

    def __post_init__(self):
        if self.vertex and any(self.periodic(a) for a in range(self.d)):
            raise ValueError("a vertex grid has Neumann axes only")

    def periodic(self, a: int) -> bool:
        return self.bc is not None and self.bc[a] == "periodic"

    @property
    def offset(self) -> float:
        """Position of grid point 0 in units of h."""
        return 0.0 if self.vertex else 0.5

    @property
    def length(self) -> Tuple[float, ...]:
        """Box length per axis: n h (cells), (n - 1) h (vertices)."""
        m = 1 if self.vertex else 0
        return tuple((self.n[a] - m) * self.h[a] for a in range(self.d))

    @property
    def G(self) -> int:
        return int(np.prod(self.n))

    @property
    def shape_zyx(self):
        """numpy array shape with x fastest (C order)."""
        return tuple(reversed(self.n))

    def centres(self) -> np.ndarray:
        """[G, d] cell centres (i_a + 1/2) h_a, flat index x-fastest."""
        idx = np.indices(self.shape_zyx)
        out = np.empty((self.G, self.d), dtype=np.float64)
        for a in range(self.d):
            out[:, a] = (idx[self.d - 1 - a].reshape(-1) + self.offset) * self.h[a]
        return out

    def to_array(self, flat: np.ndarray) -> np.ndarray:
        return flat.reshape(self.shape_zyx)
