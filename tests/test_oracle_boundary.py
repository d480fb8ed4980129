"""Pins of the oracle's boundary path: ghost states, the standard FR
boundary flux of explicit elements (Rusanov against the ghost, Section 2.1),
the hybridized boundary flux of implicit elements (eq:hfrriemann against the
boundary trace of the F^BC reading, eq:hfr2 / eq:hfrimex), free-stream
preservation on a non-periodic box, the discrete conservation identity on
the cylinder with the boundary fluxes as its only boundary terms, and a
brute-force stage solve that keeps the boundary traces as unknowns."""
import numpy as np
import pytest

import fr_inputs as fi
import oracle
from oracle import residual as res, newton as nw, boundary_trace as bt
from oracle.physics import (Euler, EDAC, BC_WALL, BC_FARFIELD, rusanov,
                            boundary_flux, hfr_boundary_flux, boundary_trace)

G = 1.4


def _euler_states(rng, k):
    rho = 0.5 + rng.random(k)
    vx, vy = rng.normal(size=k), rng.normal(size=k)
    p = 0.5 + rng.random(k)
    E = p / (G - 1) + 0.5 * rho * (vx * vx + vy * vy)
    return np.stack([rho, rho * vx, rho * vy, E], axis=-1)


def _normals(rng, k):
    th = rng.uniform(0, 2 * np.pi, k)
    mag = 0.1 + rng.random(k)
    return np.stack([mag * np.cos(th), mag * np.sin(th)], axis=-1)


def test_wall_ghost_closed_form():
    """Slip wall: density, energy and tangential momentum kept, normal
    momentum negated; far field returns the free stream."""
    rng = np.random.default_rng(1)
    u = _euler_states(rng, 50)
    S = _normals(rng, 50)
    n = S / np.linalg.norm(S, axis=1)[:, None]
    t = np.stack([-n[:, 1], n[:, 0]], axis=1)
    ph = Euler(G)
    uinf = np.array([1.0, 0.3, -0.2, 3.0])
    ug = ph.ghost(u, n[:, 0], n[:, 1], np.full(50, BC_WALL), uinf)
    m, mg = u[:, 1:3], ug[:, 1:3]
    assert np.array_equal(ug[:, 0], u[:, 0]) and np.array_equal(ug[:, 3], u[:, 3])
    assert np.allclose((mg * n).sum(1), -(m * n).sum(1), rtol=0, atol=1e-14)
    assert np.allclose((mg * t).sum(1), (m * t).sum(1), rtol=0, atol=1e-14)
    uf = ph.ghost(u, n[:, 0], n[:, 1], np.full(50, BC_FARFIELD), uinf)
    assert np.array_equal(uf, np.broadcast_to(uinf, u.shape))


def test_explicit_wall_flux_closed_form():
    """Rusanov against the mirrored state: no mass or energy crosses the
    wall, and the momentum flux is p S + (m.n)(v.S + s|S|) n with
    s = |v.n| + c, n the unit normal."""
    rng = np.random.default_rng(2)
    u = _euler_states(rng, 40)
    S = _normals(rng, 40)
    ph = Euler(G)
    F = boundary_flux(ph, u, S, np.full(40, BC_WALL), None)
    magS = np.linalg.norm(S, axis=1)
    n = S / magS[:, None]
    rho, m = u[:, 0], u[:, 1:3]
    v = m / rho[:, None]
    p = (G - 1) * (u[:, 3] - 0.5 * rho * (v * v).sum(1))
    c = np.sqrt(G * p / rho)
    mn = (m * n).sum(1)
    s = np.abs((v * n).sum(1)) + c
    mom = p[:, None] * S + (mn * ((v * S).sum(1) + s * magS))[:, None] * n
    assert np.abs(F[:, 0]).max() < 1e-14 * np.abs(F).max()
    assert np.abs(F[:, 3]).max() < 1e-14 * np.abs(F).max()
    assert np.allclose(F[:, 1:3], mom, rtol=1e-13, atol=1e-13)


def test_implicit_wall_trace_and_flux_closed_form():
    """Boundary trace of the F^BC reading at a slip wall: (rho, m - (m.n) n,
    E), tangential to the wall; the hybridized flux against it carries no
    mass or energy, and its momentum is p(uhat) S + c(uhat) |S| (m.n) n."""
    rng = np.random.default_rng(3)
    u = _euler_states(rng, 40)
    S = _normals(rng, 40)
    ph = Euler(G)
    tags = np.full(40, BC_WALL)
    uh = boundary_trace(ph, u, S, tags, None)
    magS = np.linalg.norm(S, axis=1)
    n = S / magS[:, None]
    mn = (u[:, 1:3] * n).sum(1)
    want = u.copy()
    want[:, 1:3] -= mn[:, None] * n
    assert np.allclose(uh, want, rtol=0, atol=1e-14)
    F = hfr_boundary_flux(ph, u, S, tags, None)
    rho = uh[:, 0]
    ph_ = (G - 1) * (uh[:, 3] - 0.5 * (uh[:, 1] ** 2 + uh[:, 2] ** 2) / rho)
    ch = np.sqrt(G * ph_ / rho)
    mom = ph_[:, None] * S + (ch * magS * mn)[:, None] * n
    assert np.abs(F[:, [0, 3]]).max() < 1e-13 * np.abs(F).max()
    assert np.allclose(F[:, 1:3], mom, rtol=1e-13, atol=1e-13)


def test_edac_wall_fluxes_closed_form():
    """EDAC slip wall (normal velocity mirrored): no volume flux (first
    component) for either boundary flux; the momentum flux is normal."""
    rng = np.random.default_rng(4)
    u = np.stack([rng.normal(size=30), rng.normal(size=30), rng.normal(size=30),
                  rng.normal(size=30)], axis=-1)
    S = _normals(rng, 30)
    n = S / np.linalg.norm(S, axis=1)[:, None]
    ph = EDAC(theta=20.0)
    tags = np.full(30, BC_WALL)
    for F in (boundary_flux(ph, u, S, tags, None),
              hfr_boundary_flux(ph, u, S, tags, None)):
        assert np.abs(F[:, 0]).max() < 1e-13 * np.abs(F).max()
        tang = F[:, 1] * -n[:, 1] + F[:, 2] * n[:, 0]
        assert np.abs(tang).max() < 1e-13 * np.abs(F).max()
        assert np.abs(F[:, 3]).max() < 1e-13 * np.abs(F).max()


@pytest.mark.parametrize("phys", ["euler", "edac"])
def test_farfield_fluxes_at_freestream(phys):
    """At u = u_inf both boundary fluxes reduce to the physical flux F(u_inf).S
    and the boundary trace is u_inf."""
    rng = np.random.default_rng(5)
    ph = Euler(G) if phys == "euler" else EDAC(theta=30.0)
    uinf = fi.freestream_state(0.3, angle=0.4) if phys == "euler" else \
        fi.edac_freestream(0.4)
    S = _normals(rng, 20)
    u = np.broadcast_to(uinf, (20, 4)).copy()
    Fx, Fy = ph.flux(u)
    phys_flux = Fx * S[:, :1] + Fy * S[:, 1:]
    tags = np.full(20, BC_FARFIELD)
    assert np.allclose(boundary_flux(ph, u, S, tags, uinf), phys_flux,
                       rtol=1e-14, atol=1e-13)
    assert np.allclose(hfr_boundary_flux(ph, u, S, tags, uinf), phys_flux,
                       rtol=1e-14, atol=1e-13)
    assert np.array_equal(boundary_trace(ph, u, S, tags, uinf), u)


def _box(p, mask_kind, perturb=0.25, seed=7):
    d = fi.box_quad_mesh(5, 4, -1.0, 1.5, -1.0, 0.8, perturb=perturb, seed=seed)
    cx = d["node_xy"][d["elem_nodes"], 0].mean(axis=1)
    mask = {"none": cx < -9, "all": cx > -9, "half": cx < 0.2}[mask_kind]
    uinf = fi.freestream_state(0.4, angle=0.3)
    return oracle.QuadMesh(d, p, implicit_mask=mask, uinf=uinf), uinf


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_box_farfield_freestream_preserved(p):
    """A perturbed non-periodic box tagged far field on every side keeps the
    free stream: FR residual, hybridized residuals (trace = u_inf) and a
    stage solve that needs no Newton iteration, for every partition."""
    for kind in ("none", "all", "half"):
        m, uinf = _box(p, kind)
        u = np.broadcast_to(uinf, (m.Ne, m.P, m.P, 4)).copy()
        ph = Euler(G)
        # round-off scale of a residual: flux magnitude over the cell size
        Fx, Fy = ph.flux(uinf)
        tol = 1e-14 * np.abs(np.concatenate([Fx, Fy])).max() / m.Es.min() * m.P
        assert np.abs(res.fr_residual(m, ph, u)).max() < tol
        if m.Nim:
            uhat = np.broadcast_to(uinf, (m.Ntp, 4)).copy()
            R, g = res.hfr_residual(m, ph, u, uhat)
            assert np.abs(R).max() < tol
            assert g.size == 0 or np.abs(g).max() < tol
            u_im, uh, it = nw.solve_stage(m, ph, u, u[m.imp_elems], 0.05,
                                          tol=1e-12)
            assert it == 0


def _weights(m):
    return np.outer(m.ops.w, m.ops.w)[None] * m.J


def _cylinder(p, n_impl_rings):
    d = fi.cylinder_ogrid(12, 4, first=0.05, ratio=1.3)
    ring = np.arange(12 * 4) // 12
    uinf = fi.freestream_state(0.3)
    return oracle.QuadMesh(d, p, implicit_mask=ring < n_impl_rings, uinf=uinf), uinf


def _boundary_terms(m, u, implicit_side):
    """Sum over boundary flux points of w_q F_bc . S, with the wall fluxes
    written in their closed forms and the far field as Rusanov against u_inf
    (explicit) or the hybridized flux against (u + u_inf)/2 (implicit)."""
    ph = Euler(G)
    uf = res.face_values(m.ops, u)
    tot = np.zeros(4)
    for e in range(m.Ne):
        for lf in range(4):
            tag = m.elem_face_bc[e, lf]
            if tag == 0:
                continue
            S = m.S_face[e, lf]
            a = uf[e, lf]
            magS = np.linalg.norm(S, axis=1)
            n = S / magS[:, None]
            if tag == BC_WALL:
                rho, mm = a[:, 0], a[:, 1:3]
                mn = (mm * n).sum(1)
                F = np.zeros_like(a)
                if m.implicit[e]:
                    uh = a.copy()
                    uh[:, 1:3] -= mn[:, None] * n
                    pw = (G - 1) * (uh[:, 3] - 0.5 * (uh[:, 1:3] ** 2).sum(1) / rho)
                    cw = np.sqrt(G * pw / rho)
                    F[:, 1:3] = pw[:, None] * S + (cw * magS * mn)[:, None] * n
                else:
                    v = mm / rho[:, None]
                    pw = (G - 1) * (a[:, 3] - 0.5 * rho * (v * v).sum(1))
                    s = np.abs((v * n).sum(1)) + np.sqrt(G * pw / rho)
                    F[:, 1:3] = pw[:, None] * S + \
                        (mn * ((v * S).sum(1) + s * magS))[:, None] * n
            else:
                ub = np.broadcast_to(m.uinf, a.shape)
                if m.implicit[e]:
                    from oracle.physics import hfr_flux
                    F = hfr_flux(ph, a, 0.5 * (a + ub), S)
                else:
                    F = rusanov(ph, a, ub, S)
            tot += (m.ops.w[:, None] * F).sum(0)
    return tot


@pytest.mark.parametrize("p", [1, 3])
def test_cylinder_conservation_identity(p):
    """sum_k sum_i w_i J_i R_i = -sum_trace g - sum_boundary w_q F_bc . S on
    the cylinder O-grid: interior explicit and Upsilon fluxes cancel, and
    the wall and far-field fluxes (written in closed form here) are the only
    boundary terms.  All-explicit, and with two implicit rings."""
    for rings in (0, 2):
        m, uinf = _cylinder(p, rings)
        u = fi.perturb_state(np.broadcast_to(uinf, (m.Ne, m.P, m.P, 4)), 0.05, 11)
        ph = Euler(G)
        R = res.fr_residual(m, ph, u)
        gsum = np.zeros(4)
        if m.Nim:
            uhat = fi.perturb_state(res.trace_average(m, u), 0.01, 12)
            Ri, g = res.hfr_residual(m, ph, u, uhat)
            R[m.imp_elems] = Ri
            gsum = g.sum(0)
        tot = np.einsum("eji,ejiv->v", _weights(m), R)
        want = -gsum - _boundary_terms(m, u, rings > 0)
        scale = np.einsum("eji,ejiv->v", _weights(m), np.abs(R)) + np.abs(want)
        assert np.all(np.abs(tot - want) < 1e-13 * scale), (tot, want)


@pytest.mark.parametrize("phys,p,rings", [("euler", 1, 2), ("euler", 2, 1),
                                          ("edac", 1, 2)])
def test_boundary_traces_as_unknowns_give_the_same_stage(phys, p, rings):
    """Keeping a trace unknown at every boundary flux point of the implicit
    elements (transmission with the ghost's hybridized flux, solved by a
    dense complex-step Newton over all unknowns) yields the stage that the
    closed-form boundary trace gives through condensation and the direct
    trace solve; the boundary trace converges to (u + u_g)/2."""
    d = fi.cylinder_ogrid(6, 3, first=0.05, ratio=1.4)
    ring = np.arange(6 * 3) // 6
    # rings + 1 implicit rings; all three make the far field implicit too
    if phys == "euler":
        uinf = fi.freestream_state(0.3)
        ph = Euler(G)
    else:
        uinf = fi.edac_freestream(0.0)
        ph = EDAC(theta=20.0)
    d["elem_face_bc"][ring == 2, 1] = 2
    m = oracle.QuadMesh(d, p, implicit_mask=ring < rings + 1, uinf=uinf)
    u = fi.perturb_state(np.broadcast_to(uinf, (m.Ne, m.P, m.P, 4)), 0.03, 21)
    if phys == "edac":
        u = u + 0.02 * np.random.default_rng(22).normal(size=u.shape)
    ustar = fi.perturb_state(u[m.imp_elems], 0.01, 23)
    a = 0.005
    u_c, uh_c, _ = nw.solve_stage(m, ph, u, ustar, a, tol=1e-13)
    u_b, uh_b, uhb, _ = bt.solve_stage(m, ph, u, ustar, a, tol=1e-13)
    sc = np.abs(u_c).max(axis=(0, 1, 2))
    assert np.all(np.abs(u_b - u_c).max(axis=(0, 1, 2)) <= 1e-11 * sc)
    assert np.abs(uh_b - uh_c).max() <= 1e-11 * np.abs(uh_c).max()
    bmask = m.elem_face_kind[m.imp_elems] == oracle.FACE_BOUNDARY
    uf = res.face_values(m.ops, u_c)[bmask]
    S = m.S_face[m.imp_elems][bmask]
    tags = np.broadcast_to(m.elem_face_bc[m.imp_elems][bmask][:, None],
                           uf.shape[:-1])
    assert np.abs(uhb - boundary_trace(ph, uf, S, tags, uinf)).max() <= \
        1e-11 * np.abs(uhb).max()
