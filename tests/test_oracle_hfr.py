"""Pins of the oracle's hybridized residual, Jacobian blocks, static
condensation and Newton stage solve (Sections 2.2, 3.1, 3.2; eq:hfrriemann,
eq:hfr2, eq:localproblems, eq:assembly)."""
import numpy as np
import pytest

import fr_inputs as fi
import oracle
from oracle import residual as res, newton as nw
from oracle.physics import Euler, Advection
from tests.oracle_cases import c1_mesh


def _stage_inputs(m, seed=0, amp=0.02):
    u = fi.perturb_state(fi.isentropic_vortex(m.x, m.y), amp, seed)
    ustar = fi.perturb_state(u[m.imp_elems], amp, seed + 1)
    return u, ustar


def test_jacobian_blocks_match_central_differences():
    m = c1_mesh(p=2, n=4, perturb=0.15, seed=2)
    ph = Euler()
    u, _ = _stage_inputs(m)
    uhat = fi.perturb_state(res.trace_average(m, u), 0.01, 5)
    outer = res.implicit_outer(m, u, uhat)
    u_im = u[m.imp_elems]
    a = 0.07
    A, B, C, D = nw.element_blocks(m, ph, u_im, outer, a)
    E, P = u_im.shape[0], m.P
    n, M = P * P * 4, 4 * P * 4

    def hg(ui, oi):
        R, gk = res.hfr_local(m, ph, ui, oi)
        return (ui - a * R).reshape(E, n), gk.reshape(E, M)
    rng = np.random.default_rng(0)
    for col in rng.choice(n, 6, replace=False):
        eps = 1e-6 * max(1.0, np.abs(u_im.reshape(E, n)[:, col]).max())
        up, um = u_im.copy(), u_im.copy()
        up.reshape(E, n)[:, col] += eps
        um.reshape(E, n)[:, col] -= eps
        (hp, gp), (hm, gm) = hg(up, outer), hg(um, outer)
        fdA, fdC = (hp - hm) / (2 * eps), (gp - gm) / (2 * eps)
        assert np.abs(fdA - A[:, :, col]).max() < 1e-6 * max(1, np.abs(A).max())
        assert np.abs(fdC - C[:, :, col]).max() < 1e-6 * max(1, np.abs(C).max())
    for col in rng.choice(M, 6, replace=False):
        eps = 1e-6
        op, om = outer.copy(), outer.copy()
        op.reshape(E, M)[:, col] += eps
        om.reshape(E, M)[:, col] -= eps
        (hp, gp), (hm, gm) = hg(u_im, op), hg(u_im, om)
        assert np.abs((hp - hm) / (2 * eps) - B[:, :, col]).max() < 1e-6 * max(1, np.abs(B).max())
        assert np.abs((gp - gm) / (2 * eps) - D[:, :, col]).max() < 1e-6 * max(1, np.abs(D).max())


def test_condensation_equals_dense_full_solve():
    """Schur complement + direct trace solve + back-substitution gives the
    same Newton update as a dense solve of the full [A B; C D] system."""
    m = c1_mesh(p=2, n=4, perturb=0.1, seed=4)
    ph = Euler()
    u, ustar = _stage_inputs(m, seed=3)
    uhat = fi.perturb_state(res.trace_average(m, u), 0.01, 9)
    K, rhs, sysd = nw.dense_full_system(m, ph, u, uhat, ustar, 0.1)
    x = np.linalg.solve(K, rhs)
    E, n = len(m.imp_elems), m.P * m.P * 4
    duhat = nw.trace_solve(sysd["L"], sysd["t"])
    du = nw.recover(sysd, duhat)
    assert np.abs(x[E * n:] - duhat).max() < 1e-12 * max(1, np.abs(duhat).max())
    assert np.abs(x[:E * n] - du.ravel()).max() < 1e-12 * max(1, np.abs(du).max())


def test_newton_quadratic_and_closed_form_trace():
    m = c1_mesh(p=2)
    ph = Euler()
    u, ustar = _stage_inputs(m, seed=1)
    hist = []
    u_im, uhat, its = nw.solve_stage(m, ph, u, ustar, 0.05, history=hist)
    assert its >= 2
    # quadratic: e_{k+1} <= K e_k^2 with modest K once in the basin
    for e0, e1 in zip(hist[:-1], hist[1:]):
        if e0 < 1e-2 and e1 > 1e-13:
            assert e1 <= 50.0 * e0 * e0
    uu = u.copy()
    uu[m.imp_elems] = u_im
    # inviscid HFR with collocated transmission: trace = average of sides
    assert np.abs(res.trace_average(m, uu) - uhat).max() < 1e-12


def test_hfr_stage_equals_unhybridized_brute_force():
    """Eliminating the trace in closed form (average of the two sides) turns
    the hybridized stage into a standard FR stage with common flux
    F(u_bar).n + s(u_bar)(u_- - u_+)/2; solving that system by a dense
    Newton with a finite-difference Jacobian must give the same stage."""
    m = c1_mesh(p=2, n=4)
    ph = Euler()
    u, ustar = _stage_inputs(m, seed=6)
    a = 0.08
    u_im, uhat, _ = nw.solve_stage(m, ph, u, ustar, a)
    im = m.imp_elems
    E, n = len(im), m.P * m.P * 4

    def F(x):
        uu = u.copy()
        uu[im] = x.reshape(u[im].shape)
        R, _ = res.hfr_residual(m, ph, uu, res.trace_average(m, uu))
        return (uu[im] - ustar - a * R).ravel()
    x = u[im].ravel().copy()
    for _ in range(12):
        f = F(x)
        if np.abs(f).max() < 1e-13:
            break
        Jm = np.zeros((E * n, E * n))
        for k in range(E * n):
            h = 1e-7 * max(1.0, abs(x[k]))
            xp = x.copy()
            xp[k] += h
            Jm[:, k] = (F(xp) - f) / h
        x = x - np.linalg.solve(Jm, f)
    assert np.abs(F(x)).max() < 1e-12
    assert np.abs(x - u_im.ravel()).max() < 1e-12 * np.abs(x).max()


def test_linear_advection_hfr_equals_fr():
    """For linear advection the hybridized method with s = |a.n| reproduces
    standard FR with the upwind flux (the trace is the average of the sides),
    both as a residual and as an implicit stage."""
    m = c1_mesh(p=3, n=4, perturb=0.2, seed=8)
    ph = Advection(1.0, 0.6)
    rng = np.random.default_rng(3)
    u = rng.normal(size=(m.Ne, m.P, m.P, 1))
    R_h, _ = res.hfr_residual(m, ph, u, res.trace_average(m, u))
    R_f = res.fr_residual(m, ph, u)[m.imp_elems]
    assert np.abs(R_h - R_f).max() < 1e-12 * np.abs(R_f).max()
    ustar = u[m.imp_elems] + 0.1 * rng.normal(size=u[m.imp_elems].shape)
    a = 0.3
    u_im, _, _ = nw.solve_stage(m, ph, u, ustar, a)
    # FR stage: linear system (I - a dR/du) x = ustar + a R(0 inside, u ex)
    im = m.imp_elems
    E, n = len(im), m.P * m.P

    def G(x):
        uu = u.copy()
        uu[im] = x.reshape(E, m.P, m.P, 1)
        return (uu[im] - ustar - a * res.fr_residual(m, ph, uu)[im]).ravel()
    g0 = G(np.zeros(E * n))
    Jm = np.stack([G(np.eye(E * n)[k]) - g0 for k in range(E * n)], axis=1)
    x = np.linalg.solve(Jm, -g0)
    assert np.abs(x - u_im.ravel()).max() < 1e-11 * np.abs(x).max()


def test_spatial_conservation_identity():
    """sum_k sum_i w_i J_i R_i over all elements equals minus the sum of the
    transmission residual over all trace points (explicit and Upsilon
    fluxes cancel; periodic mesh)."""
    m = c1_mesh(p=3, perturb=0.2, seed=12)
    ph = Euler()
    u = fi.perturb_state(fi.isentropic_vortex(m.x, m.y), 0.03, 2)
    uhat = fi.perturb_state(res.trace_average(m, u), 0.02, 4)
    R_im, g = res.hfr_residual(m, ph, u, uhat)
    R_ex = res.fr_residual(m, ph, u)[m.exp_elems]
    W = np.outer(m.ops.w, m.ops.w)
    tot = np.einsum("ji,eji,ejiv->v", W, m.J[m.imp_elems], R_im) + \
        np.einsum("ji,eji,ejiv->v", W, m.J[m.exp_elems], R_ex)
    assert np.allclose(tot, -g.sum(axis=0), rtol=0, atol=1e-12 * np.abs(g).sum())


def test_upsilon_flux_bitwise_single_valued():
    m = c1_mesh(p=2, perturb=0.2, seed=1)
    ph = Euler()
    u = fi.perturb_state(fi.isentropic_vortex(m.x, m.y), 0.05, 3)
    uf = res.face_values(m.ops, u)
    ups = np.nonzero(m.face_kind == oracle.FACE_UPSILON)[0]
    for f in ups:
        (e0, e1), (l0, l1) = m.face_e[f], m.face_l[f]
        a = oracle.physics.rusanov(ph, uf[e0, l0], uf[e1, l1][::-1], m.S_face[e0, l0])
        b = oracle.physics.rusanov(ph, uf[e1, l1], uf[e0, l0][::-1], m.S_face[e1, l1])
        assert np.array_equal(a, -b[::-1])


def test_damped_newton_takes_full_steps_when_they_are_admissible():
    """The damping only halves a step that leaves a non-finite residual:
    where every full step is admissible the damped and the plain Newton
    iterations are the same, and the result solves the stage."""
    m = c1_mesh(p=2, n=4, perturb=0.1, seed=4)
    ph = Euler()
    u, ustar = _stage_inputs(m, seed=3)
    a = 0.05
    h1, h2 = [], []
    r1 = nw.solve_stage(m, ph, u, ustar, a, tol=1e-13, history=h1)
    r2 = nw.solve_stage(m, ph, u, ustar, a, tol=1e-13, history=h2, damping=True)
    assert r1[2] == r2[2] and np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])
    assert h1 == h2
