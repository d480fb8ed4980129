"""Seeded workloads used by the parity tests: the same input arrays feed the
oracle and the HIP path (each builds its own mesh, operators and geometry)."""
import numpy as np

import fr_inputs as fi


def c1_desc(n=8, perturb=0.0, seed=None):
    """Doubly periodic square [-5,5]^2, elements with centroid x < 0 implicit."""
    d = fi.periodic_quad_mesh(n, n, -5, 5, -5, 5, perturb=perturb, seed=seed)
    cx = d["node_xy"][d["elem_nodes"], 0].mean(axis=1)
    return d, cx < 0.0


def cylinder_desc(n_theta=32, n_r=16, first=1e-3, ratio=1.2, n_implicit_rings=3):
    """O-grid around a unit-diameter cylinder; the innermost rings implicit."""
    d = fi.cylinder_ogrid(n_theta, n_r, first=first, ratio=ratio)
    ring = np.arange(n_theta * n_r) // n_theta
    return d, ring < n_implicit_rings


def vortex_state_at(x, y):
    return fi.isentropic_vortex(x, y)


def cylinder_state_at(x, y, seed=2, amp=1e-3, mach=0.2):
    u = np.broadcast_to(fi.freestream_state(mach), x.shape + (4,)).copy()
    return fi.perturb_state(u, amp, seed)
