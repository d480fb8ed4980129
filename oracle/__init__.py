"""Plain FP64 CPU oracle for hybridized implicit-explicit flux reconstruction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP path: the only
common dependency is the seeded input package ``fr_inputs``.

Each function cites the passage of Pereira & Vermeire, "Hybridized
Implicit-Explicit Flux Reconstruction Methods" (arXiv 2401.16632) that it
follows.  Where the paper is silent or garbled the reading taken is stated in
the function's docstring.

Parity status: every function here is pinned by a test in tests/test_oracle_*
(closed forms, invariants, brute force on tiny inputs, or an independently
written special case).  No function is "parity unpinned".
"""
from .operators import RefOps
from .mesh import QuadMesh, FACE_EXPLICIT, FACE_UPSILON, FACE_TRACE, FACE_BOUNDARY
from .physics import Euler, EDAC, Advection
from . import residual, newton, imex, efr, modal_filter, boundary_trace

__all__ = ["RefOps", "QuadMesh", "Euler", "EDAC", "Advection", "residual", "newton",
           "imex", "efr", "modal_filter", "boundary_trace", "FACE_EXPLICIT", "FACE_UPSILON", "FACE_TRACE",
           "FACE_BOUNDARY"]
