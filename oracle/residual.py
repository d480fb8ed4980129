"""Spatial residuals: standard FR (eq:freq1) and hybridized FR (eq:hfr1,
eq:hfr2, and the IMEX transmission condition eq:hfrimex).

Layout: an element state is (P, P, nv) indexed [j, i, v] with i the xi index
(fastest), j the eta index.  Face values are (4, P, nv) in the canonical
counter-clockwise flux-point order of ``oracle.mesh``.

Sign reading: the paper writes both du/dt + f = 0 and u - u* - a dt f = 0;
here R = du/dt = -(1/J) [div F^D + corrections], and every other quantity is
derived from R.
"""
import numpy as np

from .mesh import FACE_TRACE, FACE_UPSILON, FACE_BOUNDARY, FACE_EXPLICIT
from .physics import rusanov, hfr_flux, boundary_flux, hfr_boundary_flux

# element-face flux roles
ROLE_RUSANOV = 0    # standard FR flux against the outer state
ROLE_HFR = 1        # hybridized flux against the trace (outer = trace)
ROLE_BC = 2         # standard FR flux against the boundary ghost state
ROLE_BCT = 3        # hybridized flux against the boundary trace (implicit)


def face_values(ops, a):
    """Interpolate nodal values (..., P, P, k) to the four faces,
    counter-clockwise point order -> (..., 4, P, k)."""
    f0 = np.einsum("j,...jik->...ik", ops.lm, a)
    f1 = np.einsum("i,...jik->...jk", ops.lp, a)
    f2 = np.einsum("j,...jik->...ik", ops.lp, a)[..., ::-1, :]
    f3 = np.einsum("i,...jik->...jk", ops.lm, a)[..., ::-1, :]
    return np.stack([f0, f1, f2, f3], axis=-3)


def transformed_flux(mesh, phys, u):
    """Transformed flux at the solution points (eq:d9sfxda):
    f~ = y_eta F - x_eta G,  g~ = -y_xi F + x_xi G."""
    F, G = phys.flux(u)
    ft = mesh.y_eta[..., None] * F - mesh.x_eta[..., None] * G
    gt = -mesh.y_xi[..., None] * F + mesh.x_xi[..., None] * G
    return ft, gt


def transformed_flux_sel(mesh, phys, u, elems):
    F, G = phys.flux(u)
    ye, xe = mesh.y_eta[elems, ..., None], mesh.x_eta[elems, ..., None]
    yx, xx = mesh.y_xi[elems, ..., None], mesh.x_xi[elems, ..., None]
    return ye * F - xe * G, -yx * F + xx * G


def discontinuous_normal_flux(ops, ft, gt):
    """F~^D . n~ at the flux points: the transformed discontinuous flux
    polynomial evaluated on each face, dotted with the reference normal."""
    fv = face_values(ops, ft)
    gv = face_values(ops, gt)
    return np.stack([-gv[..., 0, :, :], fv[..., 1, :, :],
                     gv[..., 2, :, :], -fv[..., 3, :, :]], axis=-3)


def divergence(ops, ft, gt, H):
    """Reference divergence of the corrected flux (eq:freq1): derivative of
    the discontinuous flux plus sum over flux points of div(g) * H."""
    D = ops.D
    div = np.einsum("il,...jlk->...jik", D, ft) + \
        np.einsum("jl,...lik->...jik", D, gt)
    cl, cr = ops.corr_left, ops.corr_right
    div = div + H[..., 1, :, None, :] * cr[None, :, None]          # xi = +1
    div = div + H[..., 3, ::-1, None, :] * cl[None, :, None]       # xi = -1
    div = div + H[..., 0, None, :, :] * cl[:, None, None]          # eta = -1
    div = div + H[..., 2, None, ::-1, :] * cr[:, None, None]       # eta = +1
    return div


def element_residual(mesh, phys, elems, u, outer, roles):
    """R = -(1/J)(div F~^D + corrections) for the elements ``elems``.

    u: (E, P, P, nv) states of those elements; outer: (E, 4, P, nv) the other
    argument of each face's common flux (neighbour state or trace, in this
    element's point order); roles: (E, 4) ROLE_*.  Returns R (E, P, P, nv)
    and the transformed common normal flux (E, 4, P, nv)."""
    ops = mesh.ops
    uf = face_values(ops, u)
    ft, gt = transformed_flux_sel(mesh, phys, u, elems)
    fdn = discontinuous_normal_flux(ops, ft, gt)
    S = mesh.S_face[elems]
    tags = mesh.elem_face_bc[elems]
    common = np.zeros_like(uf)
    r = np.broadcast_to(roles[..., None], uf.shape[:-1])
    for role in (ROLE_RUSANOV, ROLE_HFR, ROLE_BC, ROLE_BCT):
        m = r == role
        if not m.any():
            continue
        if role == ROLE_RUSANOV:
            common[m] = rusanov(phys, uf[m], outer[m], S[m])
        elif role == ROLE_HFR:
            common[m] = hfr_flux(phys, uf[m], outer[m], S[m])
        else:
            tg = np.broadcast_to(tags[..., None], uf.shape[:-1])[m]
            bflux = boundary_flux if role == ROLE_BC else hfr_boundary_flux
            common[m] = bflux(phys, uf[m], S[m], tg, mesh.uinf)
    H = common - fdn
    div = divergence(ops, ft, gt, H)
    R = -div / mesh.J[elems][..., None]
    return R, common


def neighbour_face_values(mesh, uf_all, elems):
    """For each face of ``elems``, the neighbour's face values in this
    element's point order (zeros on boundary faces)."""
    nb_e = mesh.nb_e[elems]
    nb_l = mesh.nb_l[elems]
    out = uf_all[np.maximum(nb_e, 0), np.maximum(nb_l, 0)][..., ::-1, :]
    return np.where((nb_e >= 0)[..., None, None], out, 0.0)


def fr_residual(mesh, phys, u):
    """Standard FR residual (eq:freq1) of every element of the mesh: Rusanov
    on interior faces, the ghost-state flux on boundary faces.  Used for the
    explicit region; at Upsilon faces the implicit neighbour's current state
    is the outer state (eq:explicitimex)."""
    ops = mesh.ops
    elems = np.arange(mesh.Ne)
    uf = face_values(ops, u)
    outer = neighbour_face_values(mesh, uf, elems)
    roles = np.where(mesh.elem_face_kind == FACE_BOUNDARY, ROLE_BC,
                     ROLE_RUSANOV)
    R, _ = element_residual(mesh, phys, elems, u, outer, roles)
    return R


def implicit_roles(mesh):
    """Hybridized flux against the trace on trace faces and against the
    (locally solved) boundary trace on boundary faces; the standard FR flux
    on Upsilon, where there is no trace (last paragraph of Section 4)."""
    kinds = mesh.elem_face_kind[mesh.imp_elems]
    return np.where(kinds == FACE_TRACE, ROLE_HFR,
                    np.where(kinds == FACE_BOUNDARY, ROLE_BCT, ROLE_RUSANOV))


def implicit_outer(mesh, u_all, uhat):
    """Outer states for the implicit elements: the trace values (gathered
    through the trace map) on trace faces, the explicit neighbour's face
    values on Upsilon faces, zeros on boundary faces."""
    ops = mesh.ops
    im = mesh.imp_elems
    uf = face_values(ops, u_all)
    outer = neighbour_face_values(mesh, uf, im)
    tm = mesh.trace_map
    if uhat is not None and mesh.Ntp:
        gathered = uhat[np.maximum(tm, 0)]
        outer = np.where((tm >= 0)[..., None], gathered, outer)
    return outer


def hfr_local(mesh, phys, u_im, outer):
    """Element-local hybridized residual of the implicit elements (eq:hfr1
    with the IMEX interface flux of eq:hfrimex on Upsilon faces).

    Returns R_im (Nim, P, P, nv) and the element's share of the transmission
    residual at its own flux points, g^(k) = w_q F~_hat . n~ on trace faces
    (zero elsewhere), shape (Nim, 4, P, nv).

    The face integral of eq:hfr2 is read as collocated at the Gauss flux
    points (face mass matrix diag(w_q J_f)); J_f is already inside the
    transformed flux, so it is applied once."""
    roles = implicit_roles(mesh)
    R, common = element_residual(mesh, phys, mesh.imp_elems, u_im, outer,
                                 roles)
    wq = mesh.ops.w[None, None, :, None]
    gk = np.where((roles == ROLE_HFR)[..., None, None], wq * common, 0.0)
    return R, gk


def assemble_trace(mesh, gk):
    """Sum element shares into the global trace residual (eq:assembly2)."""
    nv = gk.shape[-1]
    g = np.zeros((mesh.Ntp, nv), dtype=gk.dtype)
    tm = mesh.trace_map
    m = tm >= 0
    np.add.at(g, tm[m], gk[m])
    return g


def hfr_residual(mesh, phys, u_all, uhat):
    """R^im of the implicit elements and the assembled transmission residual
    g (eq:galdkjad / eq:hfrimex) for a full state u_all and trace uhat."""
    u_im = u_all[mesh.imp_elems]
    outer = implicit_outer(mesh, u_all, uhat)
    R, gk = hfr_local(mesh, phys, u_im, outer)
    return R, assemble_trace(mesh, gk)


def trace_average(mesh, u_all):
    """Average of the two sides' interpolated states at every trace point
    (the initial trace guess, and the converged inviscid trace)."""
    ops = mesh.ops
    P = mesh.P
    uf = face_values(ops, u_all)
    tf = mesh.trace_faces
    e0, l0 = mesh.face_e[tf, 0], mesh.face_l[tf, 0]
    e1, l1 = mesh.face_e[tf, 1], mesh.face_l[tf, 1]
    a = uf[e0, l0]
    b = uf[e1, l1][:, ::-1]
    return (0.5 * (a + b)).reshape(mesh.Ntp, -1)
