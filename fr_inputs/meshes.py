"""Synthetic quadrilateral meshes (vertex coordinates + connectivity only).

Conventions shared by both consumers of these inputs:
  * ``node_xy``   float64 (n_nodes, 2) vertex coordinates.
  * ``elem_nodes`` int32 (n_elems, 4) vertex ids, counter-clockwise.
  * ``node_topo`` int32 (n_nodes,) topological vertex id.  Two vertices with
    the same topological id are the same mesh vertex for connectivity
    purposes (periodic identification); geometry always uses ``node_xy``.
  * ``elem_face_bc`` int8 (n_elems, 4) boundary tag for the local edge
    (vertex f -> vertex f+1): 0 interior, 1 slip wall, 2 far field.
"""
import numpy as np

BC_INTERIOR = 0
BC_WALL = 1
BC_FARFIELD = 2


def periodic_quad_mesh(nx, ny, x0=-5.0, x1=5.0, y0=-5.0, y1=5.0,
                       perturb=0.0, seed=None):
    """Doubly periodic nx-by-ny grid of quads on [x0,x1]x[y0,y1].

    ``perturb`` moves every topological vertex by a seeded uniform random
    offset of at most ``perturb`` times the cell size in each direction; the
    periodic twins of a vertex move by the same offset, so opposite boundary
    edges stay translates of each other.
    """
    if nx < 3 or ny < 3:
        raise ValueError("periodic meshes need at least 3 cells per direction")
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    X, Y = np.meshgrid(xs, ys)                 # [j][i]
    node_xy = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1))
    topo = ((jj % ny) * nx + (ii % nx)).ravel().astype(np.int32)
    if perturb:
        rng = np.random.default_rng(seed)
        dx = (x1 - x0) / nx
        dy = (y1 - y0) / ny
        off = rng.uniform(-perturb, perturb, size=(nx * ny, 2))
        node_xy = node_xy + off[topo] * np.array([dx, dy])
    nid = lambda i, j: j * (nx + 1) + i
    elems = []
    for j in range(ny):
        for i in range(nx):
            elems.append([nid(i, j), nid(i + 1, j), nid(i + 1, j + 1),
                          nid(i, j + 1)])
    return dict(node_xy=node_xy, elem_nodes=np.asarray(elems, np.int32),
                node_topo=topo,
                elem_face_bc=np.zeros((nx * ny, 4), np.int8))


def box_quad_mesh(nx, ny, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0,
                  tags=(BC_FARFIELD,) * 4, perturb=0.0, seed=None):
    """Non-periodic nx-by-ny grid of quads on [x0,x1]x[y0,y1] whose boundary
    edges carry the tags (bottom, right, top, left).  ``perturb`` moves every
    interior vertex by a seeded uniform offset of at most ``perturb`` times
    the cell size; boundary vertices stay on the box."""
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    X, Y = np.meshgrid(xs, ys)
    node_xy = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    if perturb:
        rng = np.random.default_rng(seed)
        off = rng.uniform(-perturb, perturb, size=node_xy.shape)
        off *= np.array([(x1 - x0) / nx, (y1 - y0) / ny])
        ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1))
        inner = ((ii > 0) & (ii < nx) & (jj > 0) & (jj < ny)).ravel()
        node_xy[inner] += off[inner]
    nid = lambda i, j: j * (nx + 1) + i
    elems, bc = [], []
    for j in range(ny):
        for i in range(nx):
            elems.append([nid(i, j), nid(i + 1, j), nid(i + 1, j + 1),
                          nid(i, j + 1)])
            t = [BC_INTERIOR] * 4
            if j == 0:
                t[0] = tags[0]
            if i == nx - 1:
                t[1] = tags[1]
            if j == ny - 1:
                t[2] = tags[2]
            if i == 0:
                t[3] = tags[3]
            bc.append(t)
    return dict(node_xy=node_xy, elem_nodes=np.asarray(elems, np.int32),
                node_topo=np.arange(node_xy.shape[0], dtype=np.int32),
                elem_face_bc=np.asarray(bc, np.int8))


def ogrid_ratio_for_outer(n_r, first, outer_gap):
    """Geometric ratio q with first*(q**n_r - 1)/(q - 1) == outer_gap (bisection)."""
    lo, hi = 1.0 + 1e-12, 4.0
    for _ in range(200):
        q = 0.5 * (lo + hi)
        if first * (q ** n_r - 1.0) / (q - 1.0) > outer_gap:
            hi = q
        else:
            lo = q
    return 0.5 * (lo + hi)


def cylinder_ogrid(n_theta, n_r, radius=0.5, first=1e-4, ratio=1.15):
    """Structured O-grid around a cylinder of diameter 2*radius.

    Ring j sits at radius + first*(ratio**j - 1)/(ratio - 1).  Element (i, j)
    spans rings j..j+1 and angles i..i+1; its local vertex order is
    (r_j, t_i), (r_j+1, t_i), (r_j+1, t_i+1), (r_j, t_i+1), which is
    counter-clockwise, so local edge 3 is on the inner ring (the wall when
    j == 0) and local edge 1 on the outer ring (far field when j == n_r-1).
    Elements are numbered ring by ring from the wall outwards.
    """
    j = np.arange(n_r + 1)
    if ratio == 1.0:
        r = radius + first * j
    else:
        r = radius + first * (ratio ** j - 1.0) / (ratio - 1.0)
    t = 2.0 * np.pi * np.arange(n_theta) / n_theta
    R, T = np.meshgrid(r, t)                    # [i][j]
    node_xy = np.stack([(R * np.cos(T)).ravel(), (R * np.sin(T)).ravel()],
                       axis=1).astype(np.float64)
    nid = lambda i, jj: (i % n_theta) * (n_r + 1) + jj
    elems, bc = [], []
    for jj in range(n_r):
        for i in range(n_theta):
            elems.append([nid(i, jj), nid(i, jj + 1), nid(i + 1, jj + 1),
                          nid(i + 1, jj)])
            tags = [BC_INTERIOR] * 4
            if jj == 0:
                tags[3] = BC_WALL
            if jj == n_r - 1:
                tags[1] = BC_FARFIELD
            bc.append(tags)
    return dict(node_xy=node_xy, elem_nodes=np.asarray(elems, np.int32),
                node_topo=np.arange(node_xy.shape[0], dtype=np.int32),
                elem_face_bc=np.asarray(bc, np.int8))


def concat_meshes(descs):
    """Several independent meshes as one description: node ids offset, the
    element lists and boundary tags concatenated, and ``elem_instance`` /
    ``n_instances`` naming each element's source mesh."""
    xy, en, topo, bc, inst = [], [], [], [], []
    off = 0
    for i, d in enumerate(descs):
        n = len(d["node_xy"])
        xy.append(np.asarray(d["node_xy"], np.float64))
        en.append(np.asarray(d["elem_nodes"], np.int64) + off)
        t = d.get("node_topo")
        topo.append((np.arange(n) if t is None else np.asarray(t, np.int64)) + off)
        bc.append(np.asarray(d.get("elem_face_bc",
                                   np.zeros((len(d["elem_nodes"]), 4))), np.int8))
        inst.append(np.full(len(d["elem_nodes"]), i, np.int32))
        off += n
    return dict(node_xy=np.concatenate(xy), elem_nodes=np.concatenate(en).astype(np.int32),
                node_topo=np.concatenate(topo).astype(np.int32),
                elem_face_bc=np.concatenate(bc), elem_instance=np.concatenate(inst),
                n_instances=len(descs))
