"""Pins of the oracle's mesh, skeleton, partition and trace map (Section 2
skeleton and mapping, Section 3.2 surjective trace map of eq:assembly,
Section 4 partition, Section 5 stiffness indicator)."""
import json
import os

import numpy as np
import pytest

import fr_inputs as fi
import oracle
from oracle.mesh import MeshError, FACE_TRACE
from oracle.residual import face_values
from tests.oracle_cases import c1_mesh

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_c1_counts_match_hand_count():
    gold = json.load(open(os.path.join(GOLD, "c1_mesh_counts.json")))
    m = c1_mesh(p=gold["p"])
    c = m.counts()
    for k, v in gold.items():
        if k.startswith("_") or k == "p":
            continue
        assert c[k] == v, k


def test_trace_map_is_surjective_two_to_one():
    m = c1_mesh(p=3, perturb=0.2, seed=7)
    tm = m.trace_map[m.trace_map >= 0]
    counts = np.bincount(tm, minlength=m.Ntp)
    assert np.all(counts == 2)


def test_flux_points_coincide_across_faces():
    """Point q of the owner and the neighbour's mapped point are the same
    physical point (orientation reversal along the shared edge)."""
    m = c1_mesh(p=3, perturb=0.2, seed=3)
    xy = np.stack([m.x, m.y], axis=-1)
    xf = face_values(m.ops, xy)                       # (Ne,4,P,2)
    for f in range(m.Nf):
        (e0, e1), (l0, l1) = m.face_e[f], m.face_l[f]
        a = xf[e0, l0]
        b = xf[e1, l1][::-1]
        # periodic faces differ by a lattice translation of the box
        d = a - b
        assert np.allclose(d, d[0], atol=1e-12)
        assert np.allclose(np.mod(d[0] + 1e-9, 10.0), 1e-9, atol=1e-8)


def test_face_normals_opposite_and_geometric():
    m = c1_mesh(p=2, perturb=0.25, seed=11)
    for f in range(m.Nf):
        (e0, e1), (l0, l1) = m.face_e[f], m.face_l[f]
        own = m.S_own[e0, l0]
        nb_own_geom = m.S_own[e1, l1][::-1]
        assert np.allclose(own, -nb_own_geom, atol=1e-13)
    # straight edges: |S| * 2 = edge length, constant along the face
    L = np.hypot(m.vert_x[:, 1] - m.vert_x[:, 0], m.vert_y[:, 1] - m.vert_y[:, 0])
    assert np.allclose(2 * np.hypot(*m.S_own[:, 0, 0].T), L, atol=1e-13)


def test_stiffness_indicator_unit_square_and_cutoff():
    d = fi.periodic_quad_mesh(4, 4, 0.0, 4.0, 0.0, 4.0)
    m = oracle.QuadMesh(d, 1)
    assert np.allclose(m.Es, 0.25)          # area 1 / perimeter 4
    d2 = fi.cylinder_ogrid(16, 8, first=1e-3, ratio=1.3)
    m2 = oracle.QuadMesh(d2, 1, es_cutoff=0.0)
    es = m2.Es.reshape(8, 16)
    assert np.all(np.diff(es.mean(axis=1)) > 0)      # grows away from wall
    cut = 0.5 * (es[2].max() + es[3].min())
    m3 = oracle.QuadMesh(d2, 1, es_cutoff=cut, uinf=fi.freestream_state())
    assert m3.Nim == 3 * 16


def test_clockwise_and_unmatched_rejected():
    d = fi.periodic_quad_mesh(4, 4)
    bad = dict(d)
    bad["elem_nodes"] = d["elem_nodes"][:, ::-1].copy()
    with pytest.raises(MeshError):
        oracle.QuadMesh(bad, 1)
    d2 = fi.cylinder_ogrid(8, 3)
    d2 = dict(d2)
    d2["elem_face_bc"] = np.zeros_like(d2["elem_face_bc"])
    with pytest.raises(MeshError):
        oracle.QuadMesh(d2, 1)
