"""Pins of the oracle's EDAC physics (Appendix A, inviscid part, with the
hybridized stabilisation the paper gives for it): eigenstructure of the
normal flux Jacobian, the stabilisation's closed form, flux consistency,
free-stream preservation, discrete conservation, the FR residual against
the analytic divergence of a resolved field, the slip-wall ghost, and the
hybridized stage (condensation against a dense solve, Newton, the trace as
the average of the two sides)."""
import numpy as np

import fr_inputs as fi
from oracle import residual as res, newton as nw
from oracle.physics import EDAC, rusanov, hfr_flux, BC_WALL
from tests.oracle_cases import c1_mesh


def _jac(ph, u, nx, ny):
    J = np.zeros((4, 4))
    for k in range(4):
        up = u.astype(complex)
        up[k] += 1e-30j
        F, G = ph.flux(up)
        J[:, k] = (F * nx + G * ny).imag / 1e-30
    return J


def test_edac_flux_jacobian_eigenvalues():
    """Eigenvalues of d(F nx + G ny)/du are v.n (twice) and
    3/2 v.n -+ sqrt((v.n)^2/4 + P + theta); max_speed is the largest modulus."""
    rng = np.random.default_rng(1)
    for theta in (4.0, 100.0):
        ph = EDAC(theta)
        for _ in range(5):
            u = np.array([rng.normal(), rng.normal(), rng.normal(), rng.normal()])
            th = rng.uniform(0, 2 * np.pi)
            nx, ny = np.cos(th), np.sin(th)
            ev = np.sort(np.linalg.eigvals(_jac(ph, u, nx, ny)).real)
            vn = u[1] * nx + u[2] * ny
            d = np.sqrt(0.25 * vn * vn + u[0] + theta)
            assert np.allclose(ev, np.sort([vn, vn, 1.5 * vn - d, 1.5 * vn + d]), atol=1e-9)
            assert np.isclose(ph.max_speed(u, nx, ny), np.abs(ev).max())


def test_edac_hfr_speed_closed_form():
    """s = 3/2 |v| + sqrt(|v|^2/4 + P + theta): 7.5 + sqrt(18.25) for
    P = 2, v = (3, 4, 0), theta = 10, whatever the normal; never below the
    largest wave speed along any normal."""
    ph = EDAC(10.0)
    u = np.array([2.0, 3.0, 4.0, 0.0])
    for th in np.linspace(0, 2 * np.pi, 13):
        s = ph.hfr_speed(u, np.cos(th), np.sin(th))
        assert np.isclose(s, 7.5 + np.sqrt(18.25), rtol=0, atol=1e-14)
        assert s >= ph.max_speed(u, np.cos(th), np.sin(th)) - 1e-14
    u3 = np.array([0.5, 1.0, 2.0, 2.0])           # |v| = 3 with v_z
    assert np.isclose(ph.hfr_speed(u3, 1.0, 0.0), 4.5 + np.sqrt(2.25 + 0.5 + 10.0))


def test_edac_flux_consistency():
    ph = EDAC(25.0)
    rng = np.random.default_rng(2)
    u = rng.normal(size=(7, 4))
    S = rng.normal(size=(7, 2))
    F, G = ph.flux(u)
    FS = F * S[:, :1] + G * S[:, 1:]
    assert np.allclose(rusanov(ph, u, u, S), FS, atol=1e-13)
    assert np.allclose(hfr_flux(ph, u, u, S), FS, atol=1e-13)


def test_edac_wall_ghost():
    ph = EDAC(9.0)
    u = np.array([[0.3, 1.0, 2.0, -0.5]])
    nx, ny = np.array([0.6]), np.array([0.8])
    g = ph.ghost(u, nx, ny, np.array([BC_WALL]), None)
    vn, vt = 1.0 * 0.6 + 2.0 * 0.8, -1.0 * 0.8 + 2.0 * 0.6
    assert np.isclose(g[0, 0], 0.3) and np.isclose(g[0, 3], -0.5)
    assert np.isclose(g[0, 1] * 0.6 + g[0, 2] * 0.8, -vn)
    assert np.isclose(-g[0, 1] * 0.8 + g[0, 2] * 0.6, vt)


def test_edac_freestream_and_conservation():
    ph = EDAC(50.0)
    for p in (1, 3):
        m = c1_mesh(p=p, perturb=0.3, seed=p)
        u = np.broadcast_to(fi.edac_freestream(0.4) + np.array([0.3, 0, 0, 0.2]),
                            (m.Ne, m.P, m.P, 4)).copy()
        assert np.abs(res.fr_residual(m, ph, u)).max() < 1e-11
    m = c1_mesh(p=3, perturb=0.2, seed=5)
    u = fi.perturb_state(fi.edac_vortex(m.x, m.y), 0.05, 1)
    R = res.fr_residual(m, ph, u)
    W = np.outer(m.ops.w, m.ops.w)
    tot = np.einsum("ji,eji,ejiv->v", W, m.J, R)
    scale = np.einsum("ji,eji,ejiv->v", W, m.J, np.abs(R))
    assert np.all(np.abs(tot) < 1e-12 * scale)


def test_edac_residual_is_minus_divergence():
    """On a resolved smooth field the FR residual approaches -div F, written
    out by hand: R_P = -(v.grad P + (P + theta) div v), R_vx = -(d(vx^2 + P)/dx
    + d(vx vy)/dy), R_vy = -(d(vx vy)/dx + d(vy^2 + P)/dy),
    R_vz = -(d(vx vz)/dx + d(vy vz)/dy)."""
    theta = 4.0
    ph = EDAC(theta)
    m = c1_mesh(p=5, n=8, perturb=0.0)
    k = np.pi / 5.0
    x, y = m.x, m.y
    P, Px, Py = 0.3 * np.sin(k * x), 0.3 * k * np.cos(k * x), 0 * x
    vx, vxx, vxy = 1 + 0.2 * np.cos(k * y), 0 * x, -0.2 * k * np.sin(k * y)
    vy, vyx, vyy = 0.1 * np.sin(k * x) * np.cos(k * y), 0.1 * k * np.cos(k * x) * np.cos(k * y), \
        -0.1 * k * np.sin(k * x) * np.sin(k * y)
    vz, vzx, vzy = 0.5 * np.cos(k * x), -0.5 * k * np.sin(k * x), 0 * x
    u = np.stack([P, vx, vy, vz], axis=-1)
    R = res.fr_residual(m, ph, u)
    exact = np.stack([
        -(vx * Px + vy * Py + (P + theta) * (vxx + vyy)),
        -(2 * vx * vxx + Px + vxy * vy + vx * vyy),
        -(vyx * vx + vy * vxx + 2 * vy * vyy + Py),
        -(vxx * vz + vx * vzx + vyy * vz + vy * vzy)], axis=-1)
    err = np.abs(R - exact).max(axis=(0, 1, 2))
    assert np.all(err < 2e-4 * np.abs(exact).max()), err


def test_edac_hfr_stage():
    """Condensation equals a dense solve of the full system, Newton converges
    quadratically, and the converged trace is the average of the two sides."""
    ph = EDAC(20.0)
    m = c1_mesh(p=2, n=4, perturb=0.1, seed=4)
    u = fi.perturb_state(fi.edac_vortex(m.x, m.y), 0.02, 3)
    ustar = fi.perturb_state(u[m.imp_elems], 0.02, 4)
    uhat = fi.perturb_state(res.trace_average(m, u), 0.01, 9)
    K, rhs, sysd = nw.dense_full_system(m, ph, u, uhat, ustar, 0.1)
    x = np.linalg.solve(K, rhs)
    E, n = len(m.imp_elems), m.P * m.P * 4
    duhat = nw.trace_solve(sysd["L"], sysd["t"])
    du = nw.recover(sysd, duhat)
    assert np.abs(x[E * n:] - duhat).max() < 1e-11 * max(1, np.abs(duhat).max())
    assert np.abs(x[:E * n] - du.ravel()).max() < 1e-11 * max(1, np.abs(du).max())
    m = c1_mesh(p=2)
    u = fi.perturb_state(fi.edac_vortex(m.x, m.y), 0.02, 1)
    ustar = fi.perturb_state(u[m.imp_elems], 0.02, 2)
    hist = []
    u_im, uhat, its = nw.solve_stage(m, ph, u, ustar, 0.05, history=hist)
    assert its >= 2
    for e0, e1 in zip(hist[:-1], hist[1:]):
        if e0 < 1e-2 and e1 > 1e-13:
            assert e1 <= 50.0 * e0 * e0
    uu = u.copy()
    uu[m.imp_elems] = u_im
    assert np.abs(res.trace_average(m, uu) - uhat).max() < 1e-12
