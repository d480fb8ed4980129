"""Physics of the conservation law (Section 2, first equation) and the two
common fluxes the method uses: the Rusanov / local Lax-Friedrichs flux of
standard FR (Section 2.1) and the single-sided hybridized flux (eq:hfrriemann).

All functions accept real or complex arrays, so the oracle can take exact
derivatives by the complex step.  |x| and max(a, b) are evaluated on the real
part (|x| -> x when Re x >= 0, max -> a when Re a >= Re b), which gives the
one-sided derivative of the branch taken.

Flux-point convention: ``S`` is the scaled outward normal J_f n (eq:8923i);
every returned flux is the transformed normal flux F_hat . S.
"""
import numpy as np

BC_WALL = 1
BC_FARFIELD = 2


def rabs(x):
    return np.where(np.real(x) >= 0, x, -x)


def rmax(a, b):
    return np.where(np.real(a) >= np.real(b), a, b)


class Euler:
    """Two-dimensional Euler equations, u = (rho, rho u, rho v, E)."""
    nv = 4

    def __init__(self, gamma=1.4):
        self.gamma = gamma

    def pressure(self, u):
        return (self.gamma - 1.0) * (u[..., 3] - 0.5 * (
            u[..., 1] * u[..., 1] + u[..., 2] * u[..., 2]) / u[..., 0])

    def flux(self, u):
        """Physical fluxes (F, G) along x and y."""
        rho, mx, my, E = u[..., 0], u[..., 1], u[..., 2], u[..., 3]
        p = self.pressure(u)
        vx, vy = mx / rho, my / rho
        F = np.stack([mx, mx * vx + p, my * vx, (E + p) * vx], axis=-1)
        G = np.stack([my, mx * vy, my * vy + p, (E + p) * vy], axis=-1)
        return F, G

    def max_speed(self, u, nx, ny):
        """|v . n| + c, the largest eigenvalue modulus of the normal flux
        Jacobian (the 'maximum local wave speed' of Section 2.1)."""
        rho = u[..., 0]
        vn = (u[..., 1] * nx + u[..., 2] * ny) / rho
        c = np.sqrt(self.gamma * self.pressure(u) / rho)
        return rabs(vn) + c

    def ghost(self, u, nx, ny, tag, uinf):
        """Exterior state of a boundary flux point: slip wall mirrors the
        normal momentum (density, energy and tangential momentum kept), far
        field is the free stream.  Explicit elements take the standard FR
        flux against it; implicit elements the hybridized flux against the
        boundary trace it determines (``hfr_boundary_flux``)."""
        mn = u[..., 1] * nx + u[..., 2] * ny
        wall = np.stack([u[..., 0], u[..., 1] - 2.0 * mn * nx,
                         u[..., 2] - 2.0 * mn * ny, u[..., 3]], axis=-1)
        far = np.broadcast_to(np.asarray(uinf if uinf is not None
                                         else np.zeros(4)), u.shape)
        return np.where((tag == BC_WALL)[..., None], wall, far)


class EDAC:
    """Entropically damped artificial compressibility equations (Appendix A),
    inviscid part, u = (P, v_x, v_y, v_z).

    Reading: the paper's state is three-dimensional; on a two-dimensional
    mesh the fields are taken independent of z, so the z fluxes vanish and
    v_z is carried as a passive scalar.  theta = 1/M^2 (artificial Mach
    number M).  Fluxes along x_i: (v_i (P + theta), v_i v_x + P delta_ix,
    v_i v_y + P delta_iy, v_i v_z)."""
    nv = 4

    def __init__(self, theta=100.0):
        self.theta = theta

    def flux(self, u):
        P, vx, vy, vz = u[..., 0], u[..., 1], u[..., 2], u[..., 3]
        Pt = P + self.theta
        F = np.stack([vx * Pt, vx * vx + P, vx * vy, vx * vz], axis=-1)
        G = np.stack([vy * Pt, vy * vx, vy * vy + P, vy * vz], axis=-1)
        return F, G

    def max_speed(self, u, nx, ny):
        """Largest eigenvalue modulus of the normal flux Jacobian: the
        eigenvalues are v_n (twice) and 3/2 v_n +- sqrt(v_n^2/4 + P + theta)."""
        vn = u[..., 1] * nx + u[..., 2] * ny
        return 1.5 * rabs(vn) + np.sqrt(0.25 * vn * vn + u[..., 0] + self.theta)

    def hfr_speed(self, u, nx, ny):
        """Stabilisation of the hybridized flux given for EDAC (Section 5,
        the airfoil case): s = 3/2 |v| + d, d^2 = |v|^2/4 + P + theta, with
        |v| the speed over all components (isotropic, s I)."""
        vv = u[..., 1] * u[..., 1] + u[..., 2] * u[..., 2] + u[..., 3] * u[..., 3]
        return 1.5 * np.sqrt(vv) + np.sqrt(0.25 * vv + u[..., 0] + self.theta) + 0.0 * nx

    def ghost(self, u, nx, ny, tag, uinf):
        """Slip wall mirrors the normal velocity (P and v_z kept); far field
        is the free stream."""
        vn = u[..., 1] * nx + u[..., 2] * ny
        wall = np.stack([u[..., 0], u[..., 1] - 2.0 * vn * nx,
                         u[..., 2] - 2.0 * vn * ny, u[..., 3]], axis=-1)
        far = np.broadcast_to(np.asarray(uinf if uinf is not None
                                         else np.zeros(4)), u.shape)
        return np.where((tag == BC_WALL)[..., None], wall, far)


class Advection:
    """Scalar linear advection with constant velocity (ax, ay)."""
    nv = 1

    def __init__(self, ax=1.0, ay=0.5):
        self.a = (ax, ay)

    def flux(self, u):
        return self.a[0] * u, self.a[1] * u

    def max_speed(self, u, nx, ny):
        return rabs(self.a[0] * nx + self.a[1] * ny + 0.0 * u[..., 0])

    def ghost(self, u, nx, ny, tag, uinf):
        raise NotImplementedError("advection runs on periodic meshes only")


def _unit(S):
    mag = np.sqrt(S[..., 0] * S[..., 0] + S[..., 1] * S[..., 1])
    return S[..., 0] / mag, S[..., 1] / mag, mag


def rusanov(phys, a, b, S):
    """Standard FR common flux (Section 2.1) times J_f:
    1/2 (F(a) + F(b)) . S + 1/2 s |S| (a - b),  s = max wave speed of a, b."""
    nx, ny, mag = _unit(S)
    Fa, Ga = phys.flux(a)
    Fb, Gb = phys.flux(b)
    cen = 0.5 * ((Fa + Fb) * S[..., 0, None] + (Ga + Gb) * S[..., 1, None])
    s = rmax(phys.max_speed(a, nx, ny), phys.max_speed(b, nx, ny))
    return cen + 0.5 * (s * mag)[..., None] * (a - b)


def hfr_flux(phys, u, uhat, S):
    """Hybridized common flux (eq:hfrriemann) times J_f:
    F(uhat) . S + s(uhat) |S| (u - uhat).

    The paper leaves s to 'the physics'; the reading taken for Euler is the
    largest wave speed at the trace, s = |vhat . n| + chat, applied as a
    scalar (isotropic, like the paper's EDAC choice); a physics that states
    its own s (EDAC) provides hfr_speed."""
    nx, ny, mag = _unit(S)
    F, G = phys.flux(uhat)
    s = getattr(phys, "hfr_speed", phys.max_speed)(uhat, nx, ny)
    return (F * S[..., 0, None] + G * S[..., 1, None]
            + (s * mag)[..., None] * (u - uhat))


def boundary_flux(phys, u, S, tag, uinf):
    """Standard FR flux on a boundary face (Section 2.1): Rusanov against the
    ghost state of the boundary condition."""
    nx, ny, _ = _unit(S)
    return rusanov(phys, u, phys.ghost(u, nx, ny, tag, uinf), S)


def boundary_trace(phys, u, S, tag, uinf):
    """Boundary trace of a hybridized element face, solved in closed form.

    The transmission condition (eq:hfr2, eq:hfrimex) has a boundary term
    F^BC that the paper does not define.  Reading: the jump of the
    hybridized flux across the boundary, with the ghost state of the
    boundary condition on the outside,
        F^BC = F_hat(u, uhat) . S + F_hat(u_g, uhat) . (-S)
             = s(uhat) |S| (u + u_g - 2 uhat),
    the trace fluxes F(uhat) . S cancelling.  With s > 0 it vanishes at one
    point only, uhat = (u + u_g)/2, so the boundary trace is a local
    function of the element's own face state and never enters the global
    trace system."""
    nx, ny, _ = _unit(S)
    return 0.5 * (u + phys.ghost(u, nx, ny, tag, uinf))


def hfr_boundary_flux(phys, u, S, tag, uinf):
    """Hybridized flux (eq:hfrriemann) on a boundary face of an implicit
    element, against the boundary trace of ``boundary_trace``."""
    return hfr_flux(phys, u, boundary_trace(phys, u, S, tag, uinf), S)
