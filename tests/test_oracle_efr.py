"""Pins of the oracle's interior-embedded FR (EFR) trace: GLL nodes and
interpolation, node numbering and continuity, the EFR residual, its
Jacobian blocks, static condensation and the Newton stage (Section 2.3
trace spaces and the EFR choice; Sections 3.1, 3.2, 4)."""
import numpy as np

import fr_inputs as fi
import oracle
from oracle import efr
from oracle.newton import trace_solve
from oracle.physics import Euler
from tests.oracle_cases import c1_mesh


def _inputs(m, tr, seed=0, amp=0.02):
    u = fi.perturb_state(fi.isentropic_vortex(m.x, m.y), amp, seed)
    ustar = fi.perturb_state(u[m.imp_elems], amp, seed + 1)
    U = fi.perturb_state(efr.node_average(m, tr, u), 0.01, seed + 2)
    return u, ustar, U


def test_gll_points_closed_forms():
    assert np.allclose(efr.gll_points(2), [-1, 1], atol=1e-15)
    assert np.allclose(efr.gll_points(3), [-1, 0, 1], atol=1e-15)
    s = 1 / np.sqrt(5)
    assert np.allclose(efr.gll_points(4), [-1, -s, s, 1], atol=1e-15)
    s = np.sqrt(3 / 7)
    assert np.allclose(efr.gll_points(5), [-1, -s, 0, s, 1], atol=1e-15)


def test_gll_to_gauss_interpolation_exact_on_degree_p():
    for p in range(1, 6):
        m = c1_mesh(p=p, n=4)
        tr = efr.EfrTrace(m)
        xq, xg = m.ops.x, tr.xg
        for k in range(p + 1):
            assert np.allclose(tr.I @ xg ** k, xq ** k, atol=1e-13)
            assert np.allclose(tr.Jg @ xq ** k, xg ** k, atol=1e-13)
        # degree p+1 is not reproduced (the node set is degree p)
        assert np.abs(tr.I @ xg ** (p + 1) - xq ** (p + 1)).max() > 1e-6


def test_node_count_and_continuity_8x8():
    """Hand count for the 8x8 periodic case with the x < 0 half implicit:
    56 trace faces (24 vertical between the four implicit columns, 32
    horizontal) carry one interior GLL node each at p = 2, and the trace
    faces touch 5 x 8 = 40 distinct vertices: 96 nodes."""
    m = c1_mesh(p=2)
    tr = efr.EfrTrace(m)
    assert m.Ntf == 56 and tr.Nn == 96
    # the two sides of every trace face see the same nodes, reversed
    for t, f in enumerate(m.trace_faces):
        (e0, e1), (l0, l1) = m.face_e[f], m.face_l[f]
        k0, k1 = m.elem_to_imp[e0], m.elem_to_imp[e1]
        assert np.array_equal(tr.elem_nodes[k0, l0], tr.elem_nodes[k1, l1][::-1])
    # every node is used; an interior vertex of the implicit block is shared
    # by four trace faces, a vertex on the Upsilon line by one
    inc = np.bincount(tr.face_nodes[:, [0, -1]].ravel(), minlength=tr.Nn)
    vert = inc > 0
    assert set(np.unique(inc[vert])) == {1, 4}
    assert np.sum(inc == 4) == 3 * 8 and np.sum(inc == 1) == 2 * 8


def test_freestream_preserved():
    m = c1_mesh(p=3, perturb=0.2, seed=9)
    tr = efr.EfrTrace(m)
    ph = Euler()
    uinf = np.array([1.0, 0.4, -0.3, 3.0])
    u = np.broadcast_to(uinf, (m.Ne, m.P, m.P, 4)).copy()
    U = np.broadcast_to(uinf, (tr.Nn, 4)).copy()
    R, g = efr.efr_residual(m, tr, ph, u, U)
    assert np.abs(R).max() < 1e-12
    assert np.abs(g).max() < 1e-12


def test_global_conservation_identity():
    """With every element implicit on a periodic mesh,
    sum_k sum_i w_i J_i R_i + sum_nodes g = 0 for any state and trace (the
    GLL basis is a partition of unity, so the nodal transmission residual
    sums to the face integrals of the flux jumps)."""
    d = fi.periodic_quad_mesh(4, 4, -5, 5, -5, 5, perturb=0.2, seed=5)
    m = oracle.QuadMesh(d, 3, implicit_mask=np.ones(16, bool))
    tr = efr.EfrTrace(m)
    ph = Euler()
    u = fi.perturb_state(fi.isentropic_vortex(m.x, m.y), 0.03, 2)
    U = fi.perturb_state(efr.node_average(m, tr, u), 0.05, 4)
    R, g = efr.efr_residual(m, tr, ph, u, U)
    W = np.outer(m.ops.w, m.ops.w)
    tot = np.einsum("ji,eji,ejiv->v", W, m.J[m.imp_elems], R)
    assert np.allclose(tot, -g.sum(axis=0), rtol=0, atol=1e-12 * np.abs(g).sum())


def test_blocks_match_central_differences():
    """B and D (per trace node, after summing face slots) and C against
    central differences of the EFR residual."""
    m = c1_mesh(p=2, n=4, perturb=0.15, seed=2)
    tr = efr.EfrTrace(m)
    ph = Euler()
    u, ustar, U = _inputs(m, tr)
    a = 0.07
    sysd = efr.condense(m, tr, ph, u, U, ustar, a)
    im = m.imp_elems
    rng = np.random.default_rng(1)
    for k in rng.choice(len(im), 3, replace=False):
        glob = sysd["idx"][k]
        for c in rng.choice(len(glob), 4, replace=False):
            node, v = divmod(int(glob[c]), 4)
            hstep = 1e-6
            Up, Um = U.copy(), U.copy()
            Up[node, v] += hstep
            Um[node, v] -= hstep
            Rp, gp = efr.efr_residual(m, tr, ph, u, Up)
            Rm, gm = efr.efr_residual(m, tr, ph, u, Um)
            dh = (-a * (Rp - Rm) / (2 * hstep))[k].ravel()
            assert np.abs(sysd["B"][k][:, c] - dh).max() < 1e-7 * max(1, np.abs(dh).max())
            # D_k is the element's share; the full dg/dU also holds the
            # neighbours' shares, so compare the assembled column
            dg = ((gp - gm) / (2 * hstep)).ravel()
            col = np.zeros_like(dg)
            for kk in range(len(im)):
                gl = sysd["idx"][kk]
                hit = np.nonzero(gl == glob[c])[0]
                if len(hit):
                    col[gl] += sysd["D"][kk][:, hit[0]]
            assert np.abs(col - dg).max() < 1e-7 * max(1, np.abs(dg).max())


def test_condensation_equals_dense_full_solve():
    m = c1_mesh(p=2, n=4, perturb=0.1, seed=3)
    tr = efr.EfrTrace(m)
    ph = Euler()
    u, ustar, U = _inputs(m, tr, seed=4)
    K, rhs, sysd = efr.dense_full_system(m, tr, ph, u, U, ustar, 0.06)
    x = np.linalg.solve(K, rhs)
    E, n = len(m.imp_elems), m.P * m.P * 4
    dU = trace_solve(sysd["L"], sysd["t"])
    du = efr.recover(sysd, dU)
    assert np.abs(dU - x[E * n:]).max() < 1e-10 * max(1, np.abs(x).max())
    assert np.abs(du.ravel() - x[:E * n]).max() < 1e-10 * max(1, np.abs(x).max())


def test_newton_quadratic():
    m = c1_mesh(p=2, perturb=0.1, seed=7)
    tr = efr.EfrTrace(m)
    ph = Euler()
    u, ustar, _ = _inputs(m, tr, seed=8)
    hist = []
    efr.solve_stage(m, tr, ph, u, ustar, 0.08, tol=1e-13, history=hist)
    assert hist[-1] < 1e-12
    # quadratic: each reduction at least squares the previous ratio
    assert len(hist) <= 6
    assert hist[2] / hist[1] < 0.1 * hist[1] / hist[0] or hist[2] < 1e-10


def test_efr_stage_equals_unhybridized_brute_force():
    """Solving h = 0, g = 0 jointly in (u, U) by a dense Newton with a
    finite-difference Jacobian gives the condensed Newton's stage."""
    m = c1_mesh(p=1, n=4)
    tr = efr.EfrTrace(m)
    ph = Euler()
    u, ustar, _ = _inputs(m, tr, seed=6)
    a = 0.08
    u_im, Uc, _ = efr.solve_stage(m, tr, ph, u, ustar, a)
    im = m.imp_elems
    E, n, Nt = len(im), m.P * m.P * 4, tr.Nn * 4

    def F(x):
        uu = u.copy()
        uu[im] = x[:E * n].reshape(u[im].shape)
        R, g = efr.efr_residual(m, tr, ph, uu, x[E * n:].reshape(-1, 4))
        return np.concatenate([(uu[im] - ustar - a * R).ravel(), g.ravel()])
    x = np.concatenate([u[im].ravel(), efr.node_average(m, tr, u).ravel()])
    for _ in range(12):
        f = F(x)
        if np.abs(f).max() < 1e-13:
            break
        Jm = np.zeros((E * n + Nt, E * n + Nt))
        for k in range(E * n + Nt):
            h = 1e-7 * max(1.0, abs(x[k]))
            xp = x.copy()
            xp[k] += h
            Jm[:, k] = (F(xp) - f) / h
        x = x - np.linalg.solve(Jm, f)
    assert np.abs(F(x)).max() < 1e-12
    assert np.abs(x[:E * n] - u_im.ravel()).max() < 1e-11 * np.abs(x).max()
    assert np.abs(x[E * n:] - Uc.ravel()).max() < 1e-11 * np.abs(x).max()


def test_efr_imex_step_conserves_mass():
    """HIMEX2C (b_bar = b) with the EFR trace: at Newton convergence the
    nodal transmission residual vanishes, so the total of every conserved
    variable over a periodic mesh is unchanged by a step (to the Newton
    tolerance)."""
    m = c1_mesh(p=2, n=6, perturb=0.15, seed=11)
    tr = efr.EfrTrace(m)
    ph = Euler()
    u = fi.perturb_state(fi.isentropic_vortex(m.x, m.y), 0.02, 3)
    W = np.outer(m.ops.w, m.ops.w)
    tot0 = np.einsum("ji,eji,ejiv->v", W, m.J, u)
    u1, recs = oracle.imex.imex_step(m, ph, oracle.imex.himex2c(), u, 0.05,
                                     tol=1e-13, trace=tr)
    tot1 = np.einsum("ji,eji,ejiv->v", W, m.J, u1)
    assert all(r["newton_its"] >= 1 for r in recs)
    assert np.abs(tot1 - tot0).max() < 1e-11 * np.abs(tot0).max()
