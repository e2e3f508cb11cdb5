"""Plain CPU FP64 oracle for the matrix-free DG acoustic solver -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU baseline leg of the benchmark may
import this package.  The product path (the HIP library and its binding)
never imports it and shares no code with it.

The oracle evaluates the same weak form as the GPU path, but in the plainest
possible way: d-dimensional Lagrange polynomials evaluated directly at points
(no sum factorization, no basis change, no collocation), full Gauss quadrature
and a dense per-cell mass matrix inverted by Cholesky factorization.  Every
function cites the part of the paper (Schoeder, Kormann, Wall, Kronbichler,
"Efficient explicit time stepping of high order discontinuous Galerkin schemes
for waves", arXiv:1805.03981) it follows.

Parity status: every function is pinned by a CPU test (tests/test_oracle_*.py);
the point-source injection through its convergence to the retarded solution
in a homogeneous periodic box (no closed form exists on curved meshes with
variable coefficients, which take the same code path).
"""
from . import basis, mesh, operator, timestep, ader, norms, sources  # noqa: F401
from .mesh import Mesh, BC_WALL, BC_ABSORBING, BC_PRESCRIBED  # noqa: F401
from .operator import apply_operator  # noqa: F401
