"""CPU FP64 oracle for the differentiable linear-static FEA path -- TEST INFRASTRUCTURE ONLY.

This package is the slow, plain, obviously-correct reference that the HIP path is checked
against.  Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product path never routes through it and shares no code with it (the only shared
module is ``meshgen``, which lays out seeded inputs and holds none of the method's arithmetic).

What it computes (paper: Sec. 2.2, Eqs. (1)-(3) "K u = f", the augmented Lagrange system and the
constraint V u = b; Sec. 2.3.1, Eqs. (5)-(6), the adjoint equation and the adjoint sensitivity):

* element stiffness for the 12-DOF space-frame member and the 4-node flat shell
  (:mod:`oracle.elements`),
* the global sparse pattern, the element-to-slot scatter map, the sort permutation and segment
  offsets, and the assembled K (:mod:`oracle.assembly`),
* the constrained solve by elimination with LAPACK banded Cholesky plus extended-precision
  iterative refinement, and the paper's Lagrange-multiplier form for tiny cross-checks
  (:mod:`oracle.solve`),
* objectives, the adjoint solve, complex-step element derivatives and the gathered gradient
  dg/dp, plus central finite differences of the whole pipeline (:mod:`oracle.sensitivity`),
* the penalised-volume objective of the size optimisation example and the sensitivity hat
  filter (:mod:`oracle.extras`).

Every function names the passage of the paper (or the published method the paper cites) that it
follows.  Parity unpinned: the drilling penalty factor, the frame choice of warped quads and the
input-definition choices (self-weight density, bump recipe) are fixed by specification and have
no closed form to pin them; every other part is pinned by the not-gpu tests.
"""
from . import elements, assembly, solve, sensitivity, extras  # noqa: F401
from .sensitivity import analyze, objective_and_grad_fd  # noqa: F401
