"""Point-wise initial states as functions of physical coordinates: the 2D
Euler equations (conserved variables rho, rho*u, rho*v, E) and the EDAC
equations (P, v_x, v_y, v_z), plus seeded perturbations.  Consumers evaluate
these at their own solution points."""
import numpy as np

EULER_GAMMA = 1.4


def isentropic_vortex(x, y, beta=5.0, gamma=EULER_GAMMA, mach=0.5,
                      x0=0.0, y0=0.0):
    """Shu-type isentropic vortex on a uniform stream along +x.

    Free stream rho = p = 1 (so c = sqrt(gamma)); stream speed mach*c.
    Returns an array of shape x.shape + (4,).
    """
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    uinf = mach * np.sqrt(gamma)
    dx, dy = x - x0, y - y0
    r2 = dx * dx + dy * dy
    e = np.exp(0.5 * (1.0 - r2))
    du = -beta / (2.0 * np.pi) * dy * e
    dv = beta / (2.0 * np.pi) * dx * e
    T = 1.0 - (gamma - 1.0) * beta ** 2 / (8.0 * gamma * np.pi ** 2) * e * e
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    u = uinf + du
    v = dv
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E], axis=-1)


def freestream_state(mach=0.2, gamma=EULER_GAMMA, angle=0.0):
    """Uniform stream with rho = 1, |v| = 1 and p = 1/(gamma*M^2)."""
    p = 1.0 / (gamma * mach * mach)
    u, v = np.cos(angle), np.sin(angle)
    E = p / (gamma - 1.0) + 0.5 * (u * u + v * v)
    return np.array([1.0, u, v, E], np.float64)


def edac_vortex(x, y, beta=2.0, speed=1.0, vz_amp=0.1, x0=0.0, y0=0.0):
    """State (P, v_x, v_y, v_z) of the EDAC equations: a Gaussian vortex of
    strength beta on a uniform stream along +x, with the pressure of the
    incompressible vortex, P = -(beta/(2 pi))^2 exp(1 - r^2) / 2, and a smooth
    passive v_z.  Returns an array of shape x.shape + (4,)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    dx, dy = x - x0, y - y0
    e = np.exp(0.5 * (1.0 - (dx * dx + dy * dy)))
    k = beta / (2.0 * np.pi)
    P = -0.5 * k * k * e * e
    vx = speed - k * dy * e
    vy = k * dx * e
    vz = vz_amp * np.sin(0.2 * np.pi * x) * np.cos(0.2 * np.pi * y)
    return np.stack([P, vx, vy, vz], axis=-1)


def edac_freestream(angle=0.0):
    """Uniform EDAC stream: P = 0, |v| = 1 at the given angle, v_z = 0."""
    return np.array([0.0, np.cos(angle), np.sin(angle), 0.0], np.float64)


def perturb_state(u, amp, seed):
    """Multiply every entry by (1 + amp*U(-1,1)), seeded."""
    rng = np.random.default_rng(seed)
    return u * (1.0 + amp * rng.uniform(-1.0, 1.0, size=u.shape))
