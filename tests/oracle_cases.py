"""Shared builders of oracle test cases (mesh + partition + state)."""
import numpy as np

import fr_inputs as fi
import oracle


def c1_mesh(p=2, n=8, perturb=0.0, seed=None, lo=-5.0, hi=5.0):
    d = fi.periodic_quad_mesh(n, n, lo, hi, lo, hi, perturb=perturb, seed=seed)
    cx = d["node_xy"][d["elem_nodes"], 0].mean(axis=1)
    return oracle.QuadMesh(d, p, implicit_mask=cx < 0.5 * (lo + hi))


def vortex_state(mesh):
    return fi.isentropic_vortex(mesh.x, mesh.y)
