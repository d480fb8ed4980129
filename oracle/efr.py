"""Interior-embedded flux reconstruction (EFR): the hybridized method with a
trace that is continuous on the interior faces of the hybridized region
(Section 2.3: the trace spaces eq:hfrspaces and the EFR choice in the
paragraph after them, Figure tracepoints; Section 4 for the IMEX coupling).

The trace is nodal at the Gauss-Lobatto-Legendre (GLL) points of every
trace face, and a node at a vertex is shared by all trace faces that meet
there.  Element residuals still evaluate fluxes at the Gauss flux points;
the trace is carried there by the GLL-to-Gauss interpolation on each face
(the additional interpolation operator the paper mentions for EFR).  The
transmission residual eq:hfr2 is tested with the nodal trace basis: with
the same collocated face quadrature as HFR (reading 5),
    g_i = sum over faces containing node i of sum_q phi_i(x_q) w_q [F.n]_q.
Faces of the IMEX interface and domain boundaries carry no trace (Section
4), exactly as in the HFR path.

Reading (the paper defers details to an earlier work): vertex nodes are
shared across every trace face incident to the vertex, including across
periodic identifications (topological vertex ids).

Node numbering (needed for bit-exact maps): trace faces in increasing trace
face order; on each, walking the owner's counter-clockwise direction, the
start vertex (if not yet numbered), the P - 2 interior GLL nodes, then the
end vertex (if not yet numbered).
"""
import numpy as np
from numpy.polynomial import legendre as npleg

from .operators import lagrange_matrix
from .residual import face_values, hfr_local, implicit_outer
from .newton import CSTEP, NewtonError, trace_solve

__all__ = ["gll_points", "EfrTrace", "efr_residual", "node_average",
           "condense", "solve_stage", "recover", "dense_full_system"]


def gll_points(P):
    """Gauss-Lobatto-Legendre points on [-1, 1]: the end points and the roots
    of the derivative of the degree P-1 Legendre polynomial."""
    if P < 2:
        raise ValueError("GLL needs at least two points")
    inner = npleg.Legendre.basis(P - 1).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


class EfrTrace:
    """Trace nodes of the EFR space on a QuadMesh with its implicit set."""

    def __init__(self, mesh):
        P = mesh.P
        self.P = P
        self.xg = gll_points(P)
        # I[q, i] = phi_i(x_q): GLL basis at the Gauss flux points
        self.I = lagrange_matrix(self.xg, mesh.ops.x)
        # Jg[i, q] = l_q(x_i): Gauss (flux point) basis at the GLL nodes
        self.Jg = lagrange_matrix(mesh.ops.x, self.xg)
        vid = {}
        fn = np.full((mesh.Ntf, P), -1, np.int64)
        nn = 0
        for t, f in enumerate(mesh.trace_faces):
            e0, l0 = mesh.face_e[f, 0], mesh.face_l[f, 0]
            a = mesh.elem_vtopo[e0, l0]
            b = mesh.elem_vtopo[e0, (l0 + 1) % 4]
            if a not in vid:
                vid[a] = nn
                nn += 1
            fn[t, 0] = vid[a]
            for i in range(1, P - 1):
                fn[t, i] = nn
                nn += 1
            if b not in vid:
                vid[b] = nn
                nn += 1
            fn[t, P - 1] = vid[b]
        self.face_nodes = fn
        self.Nn = nn
        # per implicit element and face, the nodes in the element's
        # counter-clockwise order (-1 off the trace)
        em = np.full((mesh.Nim, 4, P), -1, np.int64)
        for k, e in enumerate(mesh.imp_elems):
            for lf in range(4):
                t = mesh.face_to_trace[mesh.elem_face[e, lf]]
                if t < 0:
                    continue
                em[k, lf] = fn[t] if mesh.elem_side[e, lf] == 0 else fn[t, ::-1]
        self.elem_nodes = em

    def local_nodes(self, k):
        """Distinct trace nodes of implicit element k, in first-occurrence
        order over (face, i)."""
        seen = []
        for lf in range(4):
            for i in range(self.P):
                nd = self.elem_nodes[k, lf, i]
                if nd >= 0 and nd not in seen:
                    seen.append(int(nd))
        return np.array(seen, np.int64)


def outer_states(mesh, tr, u_all, U):
    """Outer states of the implicit elements: explicit neighbours' face
    values on Upsilon faces and the interpolated trace on trace faces."""
    outer = implicit_outer(mesh, u_all, None)
    em = tr.elem_nodes
    on = em >= 0
    interp = np.einsum("qi,kfiv->kfqv", tr.I, U[np.maximum(em, 0)] *
                       on[..., None])
    face_on = on.any(axis=2)
    return np.where(face_on[..., None, None], interp, outer)


def assemble_g(tr, gk):
    """g_i = sum over the (element, face) incidences of node i of
    sum_q phi_i(x_q) g^(k)_q  (gk already holds w_q F.n on trace faces)."""
    nv = gk.shape[-1]
    g = np.zeros((tr.Nn, nv), dtype=gk.dtype)
    gi = np.einsum("qi,kfqv->kfiv", tr.I, gk)
    em = tr.elem_nodes
    m = em >= 0
    np.add.at(g, em[m], gi[m])
    return g


def efr_residual(mesh, tr, phys, u_all, U):
    """R^im of the implicit elements (eq:hfr1) and the EFR transmission
    residual at the trace nodes (eq:hfr2 tested with the GLL basis)."""
    outer = outer_states(mesh, tr, u_all, U)
    R, gk = hfr_local(mesh, phys, u_all[mesh.imp_elems], outer)
    return R, assemble_g(tr, gk)


def node_average(mesh, tr, u_all):
    """Initial trace: at every node, the mean over its (element, face)
    incidences of the element's state interpolated to the node."""
    uf = face_values(mesh.ops, u_all[mesh.imp_elems])      # (Nim, 4, P, nv)
    at_nodes = np.einsum("iq,kfqv->kfiv", tr.Jg, uf)
    nv = uf.shape[-1]
    s = np.zeros((tr.Nn, nv))
    c = np.zeros(tr.Nn)
    em = tr.elem_nodes
    m = em >= 0
    np.add.at(s, em[m], at_nodes[m])
    np.add.at(c, em[m], 1.0)
    return s / c[:, None]


def element_blocks(mesh, tr, phys, u_im, outer, aii_dt):
    """A_k = dh_k/du_k, C = dg^(k)/du_k, and per face-node slot (face, i)
    B = dh_k/dU_slot, D = dg^(k)_slot/dU_slot, all by the complex step, with
    g^(k)_slot = sum_q phi_i(x_q) g^(k)_(face, q).  ``outer`` holds the
    element's outer states (interpolated trace on trace faces).  Slots of
    one node are summed by ``_slots_to_nodes``."""
    E, P, _, nv = u_im.shape
    n = P * P * nv
    M = 4 * P * nv
    face_on = (tr.elem_nodes >= 0).any(axis=2)               # (E, 4)
    oc = outer.astype(np.complex128)
    uc = u_im.astype(np.complex128)
    A = np.zeros((E, n, n))
    B = np.zeros((E, n, M))
    C = np.zeros((E, M, n))
    D = np.zeros((E, M, M))

    def gslot(gk):
        return np.einsum("qi,kfqv->kfiv", tr.I, gk)

    for col in range(n):
        j, i, v = np.unravel_index(col, (P, P, nv))
        up = uc.copy()
        up[:, j, i, v] += 1j * CSTEP
        R, gk = hfr_local(mesh, phys, up, oc)
        A[:, :, col] = -aii_dt * (R.imag / CSTEP).reshape(E, n)
        A[:, col, col] += 1.0
        C[:, :, col] = (gslot(gk).imag / CSTEP).reshape(E, M)
    for col in range(M):
        f, i, v = np.unravel_index(col, (4, P, nv))
        op = oc.copy()
        # a trace value at slot (f, i) reaches the face's flux points
        # through phi_i; faces off the trace have no slots
        op[:, f, :, v] += np.where(face_on[:, f, None],
                                   1j * CSTEP * tr.I[None, :, i], 0.0)
        R, gk = hfr_local(mesh, phys, uc, op)
        B[:, :, col] = -aii_dt * (R.imag / CSTEP).reshape(E, n)
        D[:, :, col] = (gslot(gk).imag / CSTEP).reshape(E, M)
    return A, B, C, D


def _slots_to_nodes(tr, k, nv):
    """Slot-to-local-node aggregation matrix S (M x m) of element k and the
    global unknowns of its local nodes: B_nodes = B S, C_nodes = S^T C,
    D_nodes = S^T D S."""
    P = tr.P
    nodes = tr.local_nodes(k)
    pos = {int(nd): a for a, nd in enumerate(nodes)}
    M = 4 * P * nv
    m = len(nodes) * nv
    S = np.zeros((M, m))
    for lf in range(4):
        for i in range(P):
            nd = tr.elem_nodes[k, lf, i]
            if nd < 0:
                continue
            for v in range(nv):
                S[(lf * P + i) * nv + v, pos[int(nd)] * nv + v] = 1.0
    glob = (nodes[:, None] * nv + np.arange(nv)[None, :]).ravel()
    return S, glob


def condense(mesh, tr, phys, u_all, U, ustar_im, aii_dt):
    """Residuals, element blocks and the condensed EFR trace system
    L dU = t with L = sum_k D_k - C_k A_k^-1 B_k (Section 3.2 with the EFR
    trace)."""
    import scipy.sparse as sp
    nv = phys.nv
    im = mesh.imp_elems
    u_im = u_all[im]
    E, P = len(im), mesh.P
    n = P * P * nv
    outer = outer_states(mesh, tr, u_all, U)
    R, gk = hfr_local(mesh, phys, u_im, outer)
    h = (u_im - ustar_im - aii_dt * R).reshape(E, n)
    g = assemble_g(tr, gk).reshape(-1)
    A, Bs, Cs, Ds = element_blocks(mesh, tr, phys, u_im, outer, aii_dt)
    gs = np.einsum("qi,kfqv->kfiv", tr.I, gk).reshape(E, -1)
    Nt = tr.Nn * nv
    rows, cols, vals = [], [], []
    t = np.zeros(Nt)
    XB, Xr, idx = [], [], []
    B, C, D = [], [], []
    for k in range(E):
        S, glob = _slots_to_nodes(tr, k, nv)
        Bk = Bs[k] @ S
        Ck = S.T @ Cs[k]
        Dk = S.T @ Ds[k] @ S
        sk = -(S.T @ gs[k])
        xb = np.linalg.solve(A[k], Bk)
        xr = np.linalg.solve(A[k], -h[k])
        Lk = Dk - Ck @ xb
        tk = sk - Ck @ xr
        rr, cc = np.meshgrid(glob, glob, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(Lk.ravel())
        np.add.at(t, glob, tk)
        XB.append(xb)
        Xr.append(xr)
        idx.append(glob)
        B.append(Bk)
        C.append(Ck)
        D.append(Dk)
    if Nt and E:
        L = sp.coo_matrix((np.concatenate(vals),
                           (np.concatenate(rows), np.concatenate(cols))),
                          shape=(Nt, Nt)).tocsr()
    else:
        L = sp.csr_matrix((Nt, Nt))
    return dict(h=h, g=g, A=A, B=B, C=C, D=D, XB=XB, Xr=Xr, idx=idx, L=L,
                t=t, R=R)


def recover(sysd, dU):
    """Local back-substitution (eq:localproblems) with the EFR trace."""
    return np.stack([xr - xb @ dU[gi] for xr, xb, gi in
                     zip(sysd["Xr"], sysd["XB"], sysd["idx"])])


def solve_stage(mesh, tr, phys, u_all, ustar_im, aii_dt, U0=None, tol=1e-13,
                maxit=25, history=None):
    """Newton iteration for (u_im, U) of one implicit stage with the EFR
    trace; the initial trace is the nodal average (``node_average``)."""
    nv = phys.nv
    u_all = u_all.copy()
    im = mesh.imp_elems
    P = mesh.P
    U = node_average(mesh, tr, u_all) if U0 is None else U0.copy()
    scale = max(1.0, float(np.max(np.abs(ustar_im))) if ustar_im.size else 1.0)
    for it in range(maxit + 1):
        sysd = condense(mesh, tr, phys, u_all, U, ustar_im, aii_dt)
        res = max(np.max(np.abs(sysd["h"]), initial=0.0),
                  np.max(np.abs(sysd["g"]), initial=0.0))
        if history is not None:
            history.append(res)
        if not np.isfinite(res):
            raise NewtonError("non-finite residual")
        if res <= tol * scale:
            return u_all[im], U, it
        if it == maxit:
            break
        dU = trace_solve(sysd["L"], sysd["t"])
        du = recover(sysd, dU)
        u_all[im] += du.reshape(len(im), P, P, nv)
        U = U + dU.reshape(-1, nv)
    raise NewtonError(f"Newton did not converge (residual {res:.3e})")


def dense_full_system(mesh, tr, phys, u_all, U, ustar_im, aii_dt):
    """Brute-force check object: the unhybridized Newton system in (u, U)
    over all implicit elements and trace nodes (small meshes only)."""
    nv = phys.nv
    sysd = condense(mesh, tr, phys, u_all, U, ustar_im, aii_dt)
    E = len(mesh.imp_elems)
    n = mesh.P * mesh.P * nv
    Nt = tr.Nn * nv
    K = np.zeros((E * n + Nt, E * n + Nt))
    rhs = np.zeros(E * n + Nt)
    for k in range(E):
        glob = sysd["idx"][k]
        K[k * n:(k + 1) * n, k * n:(k + 1) * n] = sysd["A"][k]
        K[k * n:(k + 1) * n, E * n + glob] += sysd["B"][k]
        K[E * n + glob, k * n:(k + 1) * n] += sysd["C"][k]
        K[np.ix_(E * n + glob, E * n + glob)] += sysd["D"][k]
        rhs[k * n:(k + 1) * n] = -sysd["h"][k]
    rhs[E * n:] = -sysd["g"]
    return K, rhs, sysd
