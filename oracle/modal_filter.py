"""Modal filter of the airfoil workload (Appendix B, modal filtering).
Test infrastructure only, like the rest of this package.

F = V Lambda* V^-1 per element and conserved variable, with V the
Vandermonde matrix of the orthonormal Legendre basis at the solution points
(tensor product Psi_a(xi) Psi_b(eta) in 2D) and Lambda diagonal with
sigma(eta) for a mode whose leading term has exponent sum eta = a + b:
    sigma = 1                                             eta <  eta_c
    sigma = exp(-alpha ((eta - eta_c)/(eta_max - eta_c))^s) eta_c <= eta <= eta_max
    sigma = 0                                             eta >  eta_max
with eta_max = 2p, the largest exponent sum of the basis.

Reading: the paper normalises Lambda to be independent of the time step
by reference to another work without giving the formula; here
Lambda* = Lambda^kappa with a user exponent kappa (1 by default: the filter
as written, applied once per step).
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def orthonormal_legendre(k, x):
    """Psi_k(x) = sqrt((2k+1)/2) P_k(x), orthonormal on [-1, 1]."""
    return np.sqrt((2 * k + 1) / 2.0) * npleg.legval(x, [0] * k + [1])


def sigma(eta, p, alpha, s, eta_c):
    eta_max = 2 * p
    eta = np.asarray(eta, np.float64)
    out = np.ones_like(eta)
    mid = (eta >= eta_c) & (eta <= eta_max)
    if eta_max > eta_c:
        out[mid] = np.exp(-alpha * ((eta[mid] - eta_c) / (eta_max - eta_c)) ** s)
    else:
        out[mid] = 1.0
    out[eta > eta_max] = 0.0
    return out


def filter_matrix(ops, alpha, s, eta_c, kappa=1.0):
    """Np x Np operator on element values ordered [j, i] (i fastest)."""
    P = ops.P
    p = P - 1
    V1 = np.stack([orthonormal_legendre(k, ops.x) for k in range(P)], axis=1)
    V = np.kron(V1, V1)            # rows (j, i), columns (b, a)
    a = np.tile(np.arange(P), P)
    b = np.repeat(np.arange(P), P)
    lam = sigma(a + b, p, alpha, s, eta_c) ** kappa
    return V @ np.diag(lam) @ np.linalg.inv(V)


def apply(mesh, u, alpha, s, eta_c, kappa=1.0):
    """Filter every element of u (Ne, P, P, nv)."""
    F = filter_matrix(mesh.ops, alpha, s, eta_c, kappa)
    E, P, _, nv = u.shape
    return np.einsum("pq,eqv->epv", F, u.reshape(E, P * P, nv)).reshape(u.shape)
