"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This package holds only input generation: mesh vertex coordinates and
connectivity, boundary tags, and point-wise initial states as functions of
physical coordinates.  It contains none of the method's arithmetic (no basis,
no mapping to solution points, no flux, no residual), so that the oracle and
the product path can both import it without sharing any of the method.
"""
from .meshes import (periodic_quad_mesh, box_quad_mesh, cylinder_ogrid,
                     ogrid_ratio_for_outer, concat_meshes)
from .states import (isentropic_vortex, freestream_state, perturb_state,
                     edac_vortex, edac_freestream, EULER_GAMMA)

__all__ = ["periodic_quad_mesh", "box_quad_mesh", "concat_meshes", "cylinder_ogrid", "ogrid_ratio_for_outer",
           "isentropic_vortex", "freestream_state", "perturb_state",
           "edac_vortex", "edac_freestream",
           "EULER_GAMMA"]
