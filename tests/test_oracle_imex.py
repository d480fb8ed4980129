"""Pins of the oracle's IMEX step (Section 3.1 SDIRK2 tableau, Section 4
alg:imex, eq:explicitimex, eq:hfrimex, final update)."""
import os

import numpy as np
import pytest

import fr_inputs as fi
import oracle
from oracle import imex, residual as res
from oracle.physics import Euler
from tests.oracle_cases import c1_mesh

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden_tableau():
    vals = {}
    s2 = np.sqrt(2.0)
    for line in open(os.path.join(GOLD, "sdirk2_tableau.txt")):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            vals[k.strip()] = eval(v, {"s2": s2})
    return vals


def test_sdirk2_matches_paper_tableau():
    g = _read_golden_tableau()
    A, b = imex.sdirk2()
    assert np.allclose(A, [[g["a11"], 0], [g["a21"], g["a22"]]], atol=1e-15)
    assert np.allclose(b, [g["b1"], g["b2"]], atol=1e-15)
    assert np.allclose(A.sum(axis=1), [g["c1"], g["c2"]], atol=1e-15)


def _scalar_ark(tab, lam_e, lam_i, y0, T, nsteps):
    """alg:imex for y' = lam_e y + lam_i y (explicit f, implicit g)."""
    dt = T / nsteps
    y = y0
    s = tab.s
    for _ in range(nsteps):
        Rb = [lam_e * y]
        Ri = []
        for i in range(s):
            known = y + dt * sum(tab.A[i, j] * Ri[j] for j in range(i)) + \
                dt * sum(tab.Abar[i + 1, j] * Rb[j] for j in range(i + 1))
            ui = known / (1.0 - dt * tab.A[i, i] * lam_i)
            Ri.append(lam_i * ui)
            Rb.append(lam_e * ui)
        y = y + dt * sum(tab.b[j] * Ri[j] for j in range(s)) + \
            dt * sum(tab.bbar[j] * Rb[j] for j in range(s + 1))
    return y


@pytest.mark.parametrize("name", ["HIMEX2C", "ARS222"])
def test_ark_second_order_on_split_ode(name):
    tab = imex.TABLEAUS[name]()
    lam_e, lam_i = -0.7 + 0.4j, -3.0
    errs = []
    for n in (20, 40, 80, 160):
        y = _scalar_ark(tab, lam_e, lam_i, 1.0, 1.0, n)
        errs.append(abs(y - np.exp(lam_e + lam_i)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates[1:] - 2.0) < 0.1), rates


def _mass(m, u, elems):
    W = np.outer(m.ops.w, m.ops.w)
    return np.einsum("ji,eji,ejiv->v", W, m.J[elems], u)


def test_step_conservative_with_equal_weights():
    m = c1_mesh(p=2, perturb=0.1, seed=3)
    ph = Euler()
    u = fi.isentropic_vortex(m.x, m.y)
    dt = 0.05
    u1, recs = imex.imex_step(m, ph, imex.himex2c(), u, dt)
    all_e = np.arange(m.Ne)
    dM = _mass(m, u1, all_e) - _mass(m, u, all_e)
    scale = _mass(m, np.abs(u), all_e)
    assert np.all(np.abs(dM) < 1e-13 * scale), dM


def test_ars222_upsilon_mass_defect_closed_form():
    """With b_bar != b the step leaves a mass defect across Upsilon equal to
    dt [ d Phi_0 + Phi_1 - g Phi_2 ], Phi_j the net Upsilon flux into the
    explicit region at stage state j (d = 1 - 1/(2g), g = 1 - sqrt(2)/2)."""
    m = c1_mesh(p=2, perturb=0.1, seed=3)
    ph = Euler()
    u = fi.isentropic_vortex(m.x, m.y)
    dt = 0.05
    tab = imex.ars222()
    u1, recs = imex.imex_step(m, ph, tab, u, dt)
    ex = m.exp_elems
    Phi = [_mass(m, res.fr_residual(m, ph, u)[ex], ex)] + \
        [_mass(m, r["Rbar"], ex) for r in recs]
    g = imex.GAMMA
    d = 1 - 1 / (2 * g)
    pred = dt * (d * Phi[0] + Phi[1] - g * Phi[2])
    all_e = np.arange(m.Ne)
    dM = _mass(m, u1, all_e) - _mass(m, u, all_e)
    scale = _mass(m, np.abs(u), all_e)
    assert np.abs(pred).max() > 1e-8 * scale.max()      # the defect is real
    assert np.all(np.abs(dM - pred) < 1e-13 * scale)


def test_freestream_through_imex_step():
    m = c1_mesh(p=3, perturb=0.25, seed=9)
    ph = Euler()
    u = np.broadcast_to(fi.freestream_state(0.5, angle=0.7), (m.Ne, m.P, m.P, 4)).copy()
    u1, recs = imex.imex_step(m, ph, imex.himex2c(), u, 0.1)
    assert np.abs(u1 - u).max() < 1e-12
    assert all(r["newton_its"] == 0 for r in recs)


def test_all_explicit_limit_is_explicit_rk():
    d = fi.periodic_quad_mesh(4, 4)
    m = oracle.QuadMesh(d, 2)
    ph = Euler()
    tab = imex.himex2c()
    u = fi.isentropic_vortex(m.x, m.y)
    dt = 0.02
    u1, _ = imex.imex_step(m, ph, tab, u, dt)
    k = [res.fr_residual(m, ph, u)]
    for i in range(1, 3):
        k.append(res.fr_residual(m, ph, u + dt * sum(tab.Abar[i, j] * k[j] for j in range(i))))
    ref = u + dt * sum(tab.bbar[j] * k[j] for j in range(3))
    assert np.abs(u1 - ref).max() < 1e-14 * np.abs(u).max()


def test_imex_vortex_temporal_order():
    m = c1_mesh(p=2, n=6)
    ph = Euler()
    u0 = fi.isentropic_vortex(m.x, m.y)
    T = 0.16

    def run(n):
        u = u0
        for _ in range(n):
            u, _ = imex.imex_step(m, ph, imex.himex2c(), u, T / n)
        return u
    ref = run(32)
    errs = [np.abs(run(n) - ref).max() for n in (2, 4, 8)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)
