"""CPU oracle for the hybrid pressure-correction step of Fang's hybrid
projection method (arXiv 2304.14690, Sec. 2.2-2.3).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, float64
statement of what the GPU library computes.  Only the test-suite, the smoke
entry point and the CPU-baseline leg of the benchmark may import it; the
product path never does, and it shares no code with the HIP library.

Modules
  grid        uniform cell-centred pressure grid (Sec. 2.3, Fig. 1)
  knn         k-nearest-neighbour selection with an exact (d^2, index) key
  wls         weighted-least-squares derivative coefficients (Eqs. 9-17)
  poisson     Neumann-box Poisson solve by cosine transforms (Sec. 2.3,
              the three-step transform algorithm) plus the mirror-ghost
              finite-difference Laplacian it diagonalises
  projection  RHS transfer, gradient transfer, IB-force iteration and the
              velocity projection (Eqs. 4, 18-20)

Every function cites the passage it follows.  Readings of passages where the
paper is silent or ambiguous are stated at the point of use.
"""
from .grid import Grid  # noqa: F401
from . import knn, wls, poisson, projection  # noqa: F401
