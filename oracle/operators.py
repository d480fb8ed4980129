"""One-dimensional reference operators for tensor-product quadrilaterals.

Section 2 (nodal solution and flux, eq:frsolution, eq:frfluxd; correction
functions eq:fluxcorrection, eq:dsklnf) and the end of Section 2.2 (solution
points at the Gauss-Legendre quadrature points).
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def lagrange_matrix(nodes, x):
    """V[a, j] = l_j(x_a) for the Lagrange basis on ``nodes`` (eq:frsolution)."""
    x = np.atleast_1d(np.asarray(x, np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                V[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return V


def lagrange_derivative_matrix(nodes):
    """D[i, j] = d l_j / dx at nodes[i] (the reference gradient of the nodal
    basis in eq:freq1), from the product rule applied to l_j."""
    n = len(nodes)
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            s = 0.0
            for m in range(n):
                if m == j:
                    continue
                prod = 1.0 / (nodes[j] - nodes[m])
                for l in range(n):
                    if l == j or l == m:
                        continue
                    prod *= (nodes[i] - nodes[l]) / (nodes[j] - nodes[l])
                s += prod
            D[i, j] = s
    return D


def radau_correction(p):
    """Left/right 1D correction polynomials g_L, g_R of the DG-recovering
    (right/left Radau) family, as numpy Legendre series.

    The paper only fixes the property eq:dsklnf (unit normal component at its
    own flux point, zero at the others) and does not name the family; the
    reading taken is the family that makes FR the nodal DG method:
    g_L = (-1)^p/2 (P_p - P_{p+1}),  g_R = 1/2 (P_p + P_{p+1}).
    """
    Pp = npleg.Legendre.basis(p)
    Pq = npleg.Legendre.basis(p + 1)
    gL = ((-1) ** p) * 0.5 * (Pp - Pq)
    gR = 0.5 * (Pp + Pq)
    return gL, gR


class RefOps:
    """Reference operators for degree p: P = p+1 Gauss-Legendre points."""

    def __init__(self, p):
        self.p = p
        self.P = P = p + 1
        self.x, self.w = npleg.leggauss(P)
        self.D = lagrange_derivative_matrix(self.x)
        self.lm = lagrange_matrix(self.x, [-1.0])[0]     # l_j(-1)
        self.lp = lagrange_matrix(self.x, [1.0])[0]      # l_j(+1)
        gL, gR = radau_correction(p)
        # divergence of the correction field of a flux point, per face side:
        # left (xi=-1, outward normal -1): -g_L'(xi_i); right: +g_R'(xi_i)
        self.dgL = gL.deriv()(self.x)
        self.dgR = gR.deriv()(self.x)
        self.corr_left = -self.dgL
        self.corr_right = self.dgR
