"""Pins of the reference operators (Section 2: nodal basis, Gauss-Legendre
solution points, correction functions with the property eq:dsklnf)."""
import numpy as np
import pytest

from oracle.operators import RefOps, lagrange_matrix, radau_correction


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_gauss_exactness(p):
    ops = RefOps(p)
    for k in range(2 * p + 2):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs(np.sum(ops.w * ops.x ** k) - exact) < 1e-14
    # degree 2p+2 is not integrated exactly (checks the point count)
    k = 2 * p + 2
    assert abs(np.sum(ops.w * ops.x ** k) - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_lagrange_and_derivative(p):
    ops = RefOps(p)
    xs = np.linspace(-1, 1, 7)
    V = lagrange_matrix(ops.x, xs)
    assert np.allclose(V.sum(axis=1), 1.0, atol=1e-14)
    assert np.allclose(lagrange_matrix(ops.x, ops.x), np.eye(p + 1), atol=1e-14)
    for k in range(p + 1):
        exact = k * ops.x ** (k - 1) if k else 0 * ops.x
        assert np.allclose(ops.D @ ops.x ** k, exact, atol=1e-12)
    assert np.allclose(ops.lm @ ops.x ** p, (-1.0) ** p, atol=1e-13)
    assert np.allclose(ops.lp @ ops.x ** p, 1.0, atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_radau_correction_properties(p):
    gL, gR = radau_correction(p)
    # eq:dsklnf in 1D: unit value at its own end, zero at the other
    assert abs(gL(-1.0) - 1.0) < 1e-14 and abs(gL(1.0)) < 1e-14
    assert abs(gR(1.0) - 1.0) < 1e-14 and abs(gR(-1.0)) < 1e-14
    ops = RefOps(p)
    # integrals of the derivatives: -1 (left), +1 (right)
    assert abs(np.sum(ops.w * ops.dgL) + 1.0) < 1e-13
    assert abs(np.sum(ops.w * ops.dgR) - 1.0) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_correction_is_dg_lifting(p):
    """With Gauss solution points the Radau correction reproduces the DG
    lifting M^-1 l(+-1) (Huynh's equivalence): corr_right_i = l_i(1)/w_i and
    corr_left_i = l_i(-1)/w_i."""
    ops = RefOps(p)
    assert np.allclose(ops.corr_right, ops.lp / ops.w, atol=1e-12)
    assert np.allclose(ops.corr_left, ops.lm / ops.w, atol=1e-12)
