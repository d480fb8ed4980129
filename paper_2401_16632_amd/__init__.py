"""MI355X (gfx950) hot path of hybridized implicit-explicit flux
reconstruction.  Thin Python binding over the C ABI in include/hfr_imex.h:
argument checking and marshalling only; every step of the method runs in
the HIP library.  PyTorch provides device memory and streams."""
from .api import (HfrError, Mesh, Solver, ImexStepper, load_library,
                  soa_from_elements, elements_from_soa, tableau)

__all__ = ["HfrError", "Mesh", "Solver", "ImexStepper", "load_library",
           "soa_from_elements", "elements_from_soa", "tableau"]
