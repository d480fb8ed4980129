"""Implicit stage with the boundary traces kept as unknowns (test
infrastructure: a brute-force check of the closed-form boundary trace).

The transmission condition of the hybridized region (eq:hfr2, eq:hfrimex)
sums the jump of the hybridized flux over interior trace faces and a normal
boundary flux F^BC over boundary faces.  Reading of F^BC: the jump of the
hybridized flux (eq:hfrriemann) across the boundary with the ghost state of
the boundary condition outside,
    g_b = w_q [ F_hat(u, uhat_b) . S + F_hat(u_g(u), uhat_b) . (-S) ],
collocated at the flux points like the interior condition.  The element
sees the hybridized flux against uhat_b on its boundary faces.

Here uhat_b is one more block of unknowns beside u and the interior trace,
and the whole stage system (h, g, g_b) is solved by Newton with a dense
Jacobian taken by the complex step: no condensation, no closed form.  It is
meant for meshes of a few elements; ``oracle.newton.solve_stage`` (which
eliminates uhat_b in closed form, ``oracle.physics.boundary_trace``) must
reach the same stage.
"""
import numpy as np

from .mesh import FACE_BOUNDARY
from .physics import hfr_flux, _unit
from .residual import (ROLE_HFR, ROLE_BCT, element_residual, implicit_roles,
                       implicit_outer, assemble_trace, trace_average,
                       face_values)

CSTEP = 1e-30


def _layout(mesh, nv):
    im = mesh.imp_elems
    bmask = mesh.elem_face_kind[im] == FACE_BOUNDARY          # (Nim, 4)
    nb = int(bmask.sum()) * mesh.P
    sizes = [len(im) * mesh.P * mesh.P * nv, mesh.Ntp * nv, nb * nv]
    return bmask, nb, sizes


def stage_residual(mesh, phys, u_all, ustar_im, aii_dt, uhat, uhat_b):
    """(h, g, g_b) of one implicit stage with explicit boundary traces.

    u_all: full state (explicit part used on Upsilon); uhat: (Ntp, nv);
    uhat_b: (number of boundary faces of implicit elements, P, nv), in the
    order of the boolean mask elem_face_kind[imp_elems] == FACE_BOUNDARY."""
    im = mesh.imp_elems
    bmask = mesh.elem_face_kind[im] == FACE_BOUNDARY
    u_im = u_all[im]
    roles = implicit_roles(mesh)
    roles = np.where(roles == ROLE_BCT, ROLE_HFR, roles)
    outer = implicit_outer(mesh, u_all, uhat).astype(np.result_type(
        u_all, uhat, uhat_b))
    outer[bmask] = uhat_b
    R, common = element_residual(mesh, phys, im, u_im, outer, roles)
    wq = mesh.ops.w[None, None, :, None]
    trace_faces = mesh.elem_face_kind[im] != FACE_BOUNDARY
    gk = np.where((roles == ROLE_HFR)[..., None, None] &
                  trace_faces[..., None, None], wq * common, 0.0)
    g = assemble_trace(mesh, gk)
    # boundary transmission: element side plus the ghost side
    uf = face_values(mesh.ops, u_im)[bmask]                    # (nbf, P, nv)
    S = mesh.S_face[im][bmask]
    tags = np.broadcast_to(mesh.elem_face_bc[im][bmask][:, None],
                           uf.shape[:-1])
    nx, ny, _ = _unit(S)
    ug = phys.ghost(uf, nx, ny, tags, mesh.uinf)
    gb = mesh.ops.w[None, :, None] * (hfr_flux(phys, uf, uhat_b, S) +
                                      hfr_flux(phys, ug, uhat_b, -S))
    h = u_im - ustar_im - aii_dt * R
    return h, g, gb


def solve_stage(mesh, phys, u_all, ustar_im, aii_dt, tol=1e-13, maxit=25):
    """Dense Newton for (u_im, uhat, uhat_b).  Initial guesses: u_all's
    implicit part, the two-sided average on the interior trace, the element's
    own face state on the boundary trace.  Returns (u_im, uhat, uhat_b,
    iterations)."""
    nv = phys.nv
    im = mesh.imp_elems
    P = mesh.P
    bmask, nb, sizes = _layout(mesh, nv)
    u0 = u_all.copy()
    uhat = trace_average(mesh, u_all)
    uhat_b = face_values(mesh.ops, u_all[im])[bmask].copy()
    x = np.concatenate([u0[im].ravel(), uhat.ravel(), uhat_b.ravel()])
    o1, o2 = sizes[0], sizes[0] + sizes[1]
    shp_u = u0[im].shape
    scale = max(1.0, float(np.max(np.abs(ustar_im))) if ustar_im.size else 1.0)

    def F(xv):
        ua = u0.astype(xv.dtype)
        ua[im] = xv[:o1].reshape(shp_u)
        h, g, gb = stage_residual(mesh, phys, ua, ustar_im, aii_dt,
                                  xv[o1:o2].reshape(-1, nv),
                                  xv[o2:].reshape(-1, P, nv))
        return np.concatenate([h.ravel(), g.ravel(), gb.ravel()])

    for it in range(maxit + 1):
        r = F(x)
        if np.max(np.abs(r)) <= tol * scale:
            u_im = x[:o1].reshape(shp_u)
            return (u_im, x[o1:o2].reshape(-1, nv),
                    x[o2:].reshape(-1, P, nv), it)
        K = np.zeros((r.size, x.size))
        for c in range(x.size):
            xc = x.astype(np.complex128)
            xc[c] += 1j * CSTEP
            K[:, c] = F(xc).imag / CSTEP
        x = x + np.linalg.solve(K, -r)
    raise RuntimeError("dense Newton with boundary traces did not converge")
