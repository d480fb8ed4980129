"""Quadrilateral mesh, skeleton, IMEX partition and trace map.

Follows Section 2 (elements, faces and skeleton; element mapping), the
surjective flux-point-to-trace-point map used in the element-by-element
assembly (eq:assembly, Section 3.2) and the domain partition of Section 4
(implicit region, explicit region, interface Upsilon, trace only on implicit
faces that are not on Upsilon), with the stiffness indicator E_s of Section 5.

Canonical numbering (the paper does not fix one; this is the reading both
implementations follow so their maps can be compared bit for bit):
  * local face f of a quad joins local vertices f and f+1 (counter-clockwise);
    f = 0: eta = -1, 1: xi = +1, 2: eta = +1, 3: xi = -1;
  * faces are numbered on first encounter in (element, local face) order and
    the first element met is the owner;
  * flux points on a face are listed counter-clockwise along the element, so
    point q of the owner is point P-1-q of the neighbour;
  * trace faces (both sides implicit) are numbered densely in face order and
    trace point id = trace_face * P + (owner's point index).
"""
import numpy as np

from .operators import RefOps

FACE_EXPLICIT = 0
FACE_UPSILON = 1
FACE_TRACE = 2
FACE_BOUNDARY = 3

BC_INTERIOR = 0
BC_WALL = 1
BC_FARFIELD = 2


class MeshError(ValueError):
    pass


def _bilinear_metrics(xc, yc, xi, eta):
    """Derivatives of the bilinear map (Section 2, element mapping with the
    four vertices as mapping points).  xc, yc: (..., 4) vertex coordinates;
    xi, eta broadcastable arrays.  Returns x, y, x_xi, x_eta, y_xi, y_eta."""
    x0, x1, x2, x3 = (xc[..., c, None, None] for c in range(4))
    y0, y1, y2, y3 = (yc[..., c, None, None] for c in range(4))
    N0 = 0.25 * (1 - xi) * (1 - eta)
    N1 = 0.25 * (1 + xi) * (1 - eta)
    N2 = 0.25 * (1 + xi) * (1 + eta)
    N3 = 0.25 * (1 - xi) * (1 + eta)
    x = N0 * x0 + N1 * x1 + N2 * x2 + N3 * x3
    y = N0 * y0 + N1 * y1 + N2 * y2 + N3 * y3
    x_xi = 0.25 * ((x1 - x0) * (1 - eta) + (x2 - x3) * (1 + eta))
    y_xi = 0.25 * ((y1 - y0) * (1 - eta) + (y2 - y3) * (1 + eta))
    x_eta = 0.25 * ((x3 - x0) * (1 - xi) + (x2 - x1) * (1 + xi))
    y_eta = 0.25 * ((y3 - y0) * (1 - xi) + (y2 - y1) * (1 + xi))
    return x, y, x_xi, x_eta, y_xi, y_eta


class QuadMesh:
    """Mesh of bilinear quads of uniform degree p with an IMEX partition.

    ``desc`` is a dict with node_xy, elem_nodes, node_topo, elem_face_bc
    (see fr_inputs.meshes).  Exactly one of ``implicit_mask`` (bool per
    element) or ``es_cutoff`` (implicit iff E_s <= cutoff) may be given; with
    neither, every element is explicit.
    """

    def __init__(self, desc, p, implicit_mask=None, es_cutoff=None,
                 uinf=None):
        self.ops = ops = RefOps(p)
        self.p, self.P = p, ops.P
        P = self.P
        xy = np.asarray(desc["node_xy"], np.float64)
        en = np.asarray(desc["elem_nodes"], np.int64)
        topo = np.asarray(desc.get("node_topo", np.arange(len(xy))), np.int64)
        bc = np.asarray(desc.get("elem_face_bc", np.zeros((len(en), 4))),
                        np.int64)
        self.Ne = Ne = len(en)
        self.uinf = None if uinf is None else np.asarray(uinf, np.float64)
        self.elem_vtopo = topo[en]              # topological vertex ids (Ne, 4)

        # ---- skeleton: faces on first encounter -------------------------
        directed = set()
        open_faces = {}
        f_e = [[], []]
        f_l = [[], []]
        for e in range(Ne):
            for lf in range(4):
                a = topo[en[e, lf]]
                b = topo[en[e, (lf + 1) % 4]]
                if a == b:
                    raise MeshError(f"degenerate edge in element {e}")
                if (a, b) in directed:
                    raise MeshError(f"edge {a}->{b} traversed twice "
                                    "(clockwise or non-conforming element)")
                directed.add((a, b))
                if (b, a) in open_faces:
                    f = open_faces.pop((b, a))
                    if f_e[0][f] == e:
                        raise MeshError(f"element {e} is its own neighbour")
                    f_e[1][f] = e
                    f_l[1][f] = lf
                else:
                    f = len(f_e[0])
                    f_e[0].append(e)
                    f_l[0].append(lf)
                    f_e[1].append(-1)
                    f_l[1].append(-1)
                    open_faces[(a, b)] = f
        self.Nf = Nf = len(f_e[0])
        self.face_e = np.array(f_e, np.int64).T          # (Nf, 2)
        self.face_l = np.array(f_l, np.int64).T
        self.face_bc = np.zeros(Nf, np.int64)
        for f in range(Nf):
            e0, l0 = self.face_e[f, 0], self.face_l[f, 0]
            if self.face_e[f, 1] < 0:
                if bc[e0, l0] == BC_INTERIOR:
                    raise MeshError(f"unmatched edge without boundary tag "
                                    f"(element {e0}, face {l0})")
                self.face_bc[f] = bc[e0, l0]
            elif bc[e0, l0] != BC_INTERIOR or \
                    bc[self.face_e[f, 1], self.face_l[f, 1]] != BC_INTERIOR:
                raise MeshError(f"boundary tag on an interior edge (face {f})")
        self.elem_face = np.zeros((Ne, 4), np.int64)
        self.elem_side = np.zeros((Ne, 4), np.int64)
        for s in range(2):
            m = self.face_e[:, s] >= 0
            self.elem_face[self.face_e[m, s], self.face_l[m, s]] = \
                np.nonzero(m)[0]
            self.elem_side[self.face_e[m, s], self.face_l[m, s]] = s

        # ---- geometry --------------------------------------------------
        xc, yc = xy[en, 0], xy[en, 1]                      # (Ne, 4)
        self.vert_x, self.vert_y = xc, yc
        xi = ops.x[None, :]          # varies along i (last axis)
        eta = ops.x[:, None]         # varies along j
        (self.x, self.y, self.x_xi, self.x_eta, self.y_xi,
         self.y_eta) = _bilinear_metrics(xc, yc, xi, eta)   # (Ne, P, P)
        self.J = self.x_xi * self.y_eta - self.x_eta * self.y_xi
        if np.any(self.J <= 0):
            bad = np.nonzero((self.J <= 0).any(axis=(1, 2)))[0]
            raise MeshError(f"non-positive Jacobian (clockwise or folded) "
                            f"in elements {bad[:8].tolist()}")
        # scaled outward normals S = J_f n at the flux points, own geometry,
        # counter-clockwise point order per face
        g = ops.x
        r = g[::-1]
        one = np.ones(P)
        pts = [(g, -one), (one, g), (r, one), (-one, r)]
        S = np.zeros((Ne, 4, P, 2))
        for f, (fx, fe) in enumerate(pts):
            _, _, x_xi, x_eta, y_xi, y_eta = _bilinear_metrics(
                xc, yc, fx[None, :], fe[None, :])
            x_xi, x_eta, y_xi, y_eta = (a[:, 0, :] for a in
                                        (x_xi, x_eta, y_xi, y_eta))
            if f == 0:
                S[:, f, :, 0], S[:, f, :, 1] = y_xi, -x_xi
            elif f == 1:
                S[:, f, :, 0], S[:, f, :, 1] = y_eta, -x_eta
            elif f == 2:
                S[:, f, :, 0], S[:, f, :, 1] = -y_xi, x_xi
            else:
                S[:, f, :, 0], S[:, f, :, 1] = -y_eta, x_eta
        self.S_own = S
        # face-owned normal as seen by each side (owner's value, negated and
        # reversed on the neighbour) so both sides use one geometry
        S_face = S.copy()
        for f in range(Nf):
            e1 = self.face_e[f, 1]
            if e1 >= 0:
                S_face[e1, self.face_l[f, 1]] = \
                    -S[self.face_e[f, 0], self.face_l[f, 0]][::-1]
        self.S_face = S_face

        # ---- stiffness indicator (Section 5): area / perimeter ---------
        area = 0.5 * np.sum(xc * np.roll(yc, -1, axis=1)
                            - np.roll(xc, -1, axis=1) * yc, axis=1)
        perim = np.sum(np.hypot(np.roll(xc, -1, axis=1) - xc,
                                np.roll(yc, -1, axis=1) - yc), axis=1)
        self.Es = area / perim

        # ---- partition (Section 4) -------------------------------------
        if implicit_mask is not None and es_cutoff is not None:
            raise ValueError("give implicit_mask or es_cutoff, not both")
        if implicit_mask is not None:
            mask = np.asarray(implicit_mask, bool)
        elif es_cutoff is not None:
            mask = self.Es <= es_cutoff
        else:
            mask = np.zeros(Ne, bool)
        self.implicit = mask
        self.imp_elems = np.nonzero(mask)[0]
        self.exp_elems = np.nonzero(~mask)[0]
        self.elem_to_imp = np.full(Ne, -1, np.int64)
        self.elem_to_imp[self.imp_elems] = np.arange(len(self.imp_elems))
        self.Nim = len(self.imp_elems)
        kind = np.empty(Nf, np.int64)
        for f in range(Nf):
            e0, e1 = self.face_e[f]
            if e1 < 0:
                kind[f] = FACE_BOUNDARY
            elif mask[e0] and mask[e1]:
                kind[f] = FACE_TRACE
            elif mask[e0] or mask[e1]:
                kind[f] = FACE_UPSILON
            else:
                kind[f] = FACE_EXPLICIT
        self.face_kind = kind
        self.trace_faces = np.nonzero(kind == FACE_TRACE)[0]
        self.Ntf = len(self.trace_faces)
        self.face_to_trace = np.full(Nf, -1, np.int64)
        self.face_to_trace[self.trace_faces] = np.arange(self.Ntf)
        self.Ntp = self.Ntf * P
        # trace map (eq:assembly's surjective index map), per implicit element
        tmap = np.full((self.Nim, 4, P), -1, np.int64)
        for k, e in enumerate(self.imp_elems):
            for lf in range(4):
                f = self.elem_face[e, lf]
                tf = self.face_to_trace[f]
                if tf < 0:
                    continue
                q = np.arange(P)
                if self.elem_side[e, lf] == 0:
                    tmap[k, lf] = tf * P + q
                else:
                    tmap[k, lf] = tf * P + (P - 1 - q)
        self.trace_map = tmap
        # element-face roles for the local residual
        self.elem_face_kind = kind[self.elem_face]            # (Ne, 4)
        self.elem_face_bc = self.face_bc[self.elem_face]      # (Ne, 4)
        # neighbour (element, local face) across each element face
        nb_e = np.full((Ne, 4), -1, np.int64)
        nb_l = np.full((Ne, 4), -1, np.int64)
        for f in range(Nf):
            (e0, e1), (l0, l1) = self.face_e[f], self.face_l[f]
            if e1 >= 0:
                nb_e[e0, l0], nb_l[e0, l0] = e1, l1
                nb_e[e1, l1], nb_l[e1, l1] = e0, l0
        self.nb_e, self.nb_l = nb_e, nb_l

    def counts(self):
        return dict(n_elems=self.Ne, n_faces=self.Nf,
                    n_implicit=self.Nim,
                    n_trace_faces=self.Ntf, n_trace_points=self.Ntp,
                    n_upsilon=int(np.sum(self.face_kind == FACE_UPSILON)),
                    n_boundary=int(np.sum(self.face_kind == FACE_BOUNDARY)))
