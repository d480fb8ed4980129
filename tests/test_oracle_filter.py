"""Pins of the oracle's modal filter (Appendix B)."""
import numpy as np

import fr_inputs as fi
from oracle import modal_filter as mf
from oracle.operators import RefOps
from tests.oracle_cases import c1_mesh


def test_orthonormal_basis_under_gauss_quadrature():
    ops = RefOps(4)
    V1 = np.stack([mf.orthonormal_legendre(k, ops.x) for k in range(ops.P)], axis=1)
    assert np.allclose(V1.T @ np.diag(ops.w) @ V1, np.eye(ops.P), atol=1e-13)


def test_sigma_closed_forms():
    p = 3
    assert np.allclose(mf.sigma([0, 1, 2], p, 100.0, 1.0, 3), 1.0)
    assert np.isclose(mf.sigma([6], p, 100.0, 1.0, 3)[0], np.exp(-100.0))
    assert np.isclose(mf.sigma([4], p, 2.0, 2.0, 3)[0], np.exp(-2.0 / 9.0))
    assert mf.sigma([7], p, 1.0, 1.0, 3)[0] == 0.0


def test_identity_cases_and_polynomial_preservation():
    m = c1_mesh(p=3, perturb=0.1, seed=2)
    u = fi.perturb_state(fi.isentropic_vortex(m.x, m.y), 0.05, 1)
    assert np.allclose(mf.apply(m, u, 0.0, 1.0, 1), u, atol=1e-12)
    assert np.allclose(mf.apply(m, u, 50.0, 1.0, 7), u, atol=1e-12)
    # a reference-space polynomial with exponent sum < eta_c is untouched,
    # one with exponent sum 2p is scaled by exp(-alpha) in its top mode
    xi = m.ops.x[None, :]
    et = m.ops.x[:, None]
    low = (1 + 2 * xi + 3 * et * xi + et ** 2) * np.ones((1, 1))
    U = np.broadcast_to(low[None, :, :, None], (m.Ne, m.P, m.P, 1)).copy()
    assert np.allclose(mf.apply(m, U, 80.0, 1.0, 3), U, atol=1e-12)
    top = mf.orthonormal_legendre(3, xi) * mf.orthonormal_legendre(3, et)
    T = np.broadcast_to(top[None, :, :, None], (m.Ne, m.P, m.P, 1)).copy()
    assert np.allclose(mf.apply(m, T, 5.0, 1.0, 2), np.exp(-5.0) * T, atol=1e-12)


def test_filter_conserves_cell_means():
    """The mean mode (exponent sum 0) is never damped, so the element
    integrals of affine elements are unchanged."""
    m = c1_mesh(p=2, perturb=0.0)
    u = fi.perturb_state(fi.isentropic_vortex(m.x, m.y), 0.05, 3)
    W = np.outer(m.ops.w, m.ops.w)
    f = mf.apply(m, u, 30.0, 2.0, 1)
    assert np.allclose(np.einsum("ji,ejiv->ev", W, f), np.einsum("ji,ejiv->ev", W, u),
                       atol=1e-12)
