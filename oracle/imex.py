"""Additive IMEX Runge-Kutta step with an element partition.

Section 3.1 (the two-stage SDIRK tableau), Section 4 (padded implicit
tableau, table:butcherimex; alg:imex; explicit stage update
eq:explicitimex; implicit stage with the augmented transmission condition
eq:galdkjad / eq:hfrimex; final update).

The paper's tableau appendix is not available, so the explicit partner of the
paper's SDIRK2 is constructed here from the order conditions:
  * HIMEX2C (default): c_bar = [0, c], A_bar row 2 = (g, 0, 0), row 3 =
    (d, 1-d, 0) with d = 1 - 1/(2g), and b_bar = padded b.  Equal weights
    make the fluxes exchanged across Upsilon cancel in the step.
  * ARS222: the same stages with b_bar = (d, 1-d, 0) (the classical
    Ascher-Ruuth-Spiteri 2-stage, 2nd-order pair).
Stage residuals R_i are re-evaluated as R^im(u_i, u_hat_i) after Newton.
"""
import numpy as np

from .residual import fr_residual, hfr_residual
from .newton import solve_stage

GAMMA = 1.0 - np.sqrt(2.0) / 2.0


class Tableau:
    def __init__(self, name, A, b, Abar, bbar):
        self.name = name
        self.A = np.asarray(A, np.float64)        # s x s implicit (unpadded)
        self.b = np.asarray(b, np.float64)
        self.c = self.A.sum(axis=1)
        self.Abar = np.asarray(Abar, np.float64)  # (s+1) x (s+1) explicit
        self.bbar = np.asarray(bbar, np.float64)
        self.cbar = self.Abar.sum(axis=1)
        self.s = len(self.b)


def sdirk2():
    g = GAMMA
    return np.array([[g, 0.0], [1.0 - g, g]]), np.array([1.0 - g, g])


def himex2c():
    g = GAMMA
    d = 1.0 - 1.0 / (2.0 * g)
    A, b = sdirk2()
    Abar = np.array([[0, 0, 0], [g, 0, 0], [d, 1 - d, 0]], np.float64)
    return Tableau("HIMEX2C", A, b, Abar, np.concatenate([[0.0], b]))


def ars222():
    g = GAMMA
    d = 1.0 - 1.0 / (2.0 * g)
    A, b = sdirk2()
    Abar = np.array([[0, 0, 0], [g, 0, 0], [d, 1 - d, 0]], np.float64)
    return Tableau("ARS222", A, b, Abar, np.array([d, 1 - d, 0.0]))


TABLEAUS = {"HIMEX2C": himex2c, "ARS222": ars222}


def imex_step(mesh, phys, tab, u_n, dt, tol=1e-13, maxit=25, stats=None,
              trace=None):
    """One step u_n -> u_{n+1} (alg:imex with eq:explicitimex).

    ``trace``: None for the HFR trace, or an ``efr.EfrTrace`` for EFR.
    Returns (u_{n+1}, per-stage records).  Each record holds the stage state
    u_i (all elements), the trace u_hat_i, R_i (implicit) and
    R_bar_{i+1} (explicit)."""
    from . import efr
    im, ex = mesh.imp_elems, mesh.exp_elems
    s = tab.s
    Rbar = [fr_residual(mesh, phys, u_n)[ex]]
    R = []
    recs = []
    u_stage = u_n.copy()
    for i in range(s):
        u_stage[ex] = u_n[ex] + dt * sum(tab.Abar[i + 1, j] * Rbar[j]
                                         for j in range(i + 1))
        ustar = u_n[im] + dt * sum((tab.A[i, j] * R[j] for j in range(i)),
                                   np.zeros_like(u_n[im]))
        aii_dt = dt * tab.A[i, i]
        its = 0
        uhat = None
        if len(im) and trace is not None:
            u_im, uhat, its = efr.solve_stage(mesh, trace, phys, u_stage, ustar,
                                              aii_dt, tol=tol, maxit=maxit)
            u_stage[im] = u_im
            Ri, _ = efr.efr_residual(mesh, trace, phys, u_stage, uhat)
        elif len(im):
            u_im, uhat, its = solve_stage(mesh, phys, u_stage, ustar, aii_dt,
                                          tol=tol, maxit=maxit)
            u_stage[im] = u_im
            Ri, _ = hfr_residual(mesh, phys, u_stage, uhat)
        else:
            Ri = np.zeros_like(u_n[im])
        R.append(Ri)
        Rbar.append(fr_residual(mesh, phys, u_stage)[ex])
        recs.append(dict(u=u_stage.copy(), uhat=uhat, R=Ri, Rbar=Rbar[-1],
                         newton_its=its))
    u_next = u_n.copy()
    u_next[ex] = u_n[ex] + dt * sum(tab.bbar[j] * Rbar[j]
                                    for j in range(s + 1))
    u_next[im] = u_n[im] + dt * sum((tab.b[j] * R[j] for j in range(s)),
                                    np.zeros_like(u_n[im]))
    if stats is not None:
        stats.extend(recs)
    return u_next, recs


def solution_points(mesh):
    return mesh.x, mesh.y
