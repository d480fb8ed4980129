// Device physics: fluxes, the standard FR Rusanov flux (Section 2.1), the
// hybridized single-sided flux (eq:hfrriemann), boundary ghost states, and
// the analytic derivatives of each needed by the element blocks of
// Section 3.2, for two systems with four unknowns per point:
//   - the two-dimensional Euler equations, u = (rho, rho u, rho v, E), with
//     the hybridized stabilisation s = |vhat.n| + chat;
//   - the EDAC equations of Appendix A (inviscid part), u = (P, v_x, v_y,
//     v_z) with theta = 1/M^2, on a two-dimensional mesh (fields independent
//     of z, v_z passive), with the stabilisation the paper gives for them,
//     s = 3/2 |vhat| + sqrt(|vhat|^2/4 + Phat + theta) (isotropic).
//
// Every common flux returned is the transformed normal flux F_hat . S with
// S = J_f n the scaled outward normal (eq:8923i).
#pragma once

#include <hip/hip_runtime.h>

namespace hfr {

struct Prim {
    double rho, vx, vy, p, c;
};

__device__ __forceinline__ Prim prim(const double u[4], double g) {
    Prim q;
    q.rho = u[0];
    double ir = 1.0 / u[0];
    q.vx = u[1] * ir;
    q.vy = u[2] * ir;
    q.p = (g - 1.0) * (u[3] - 0.5 * (u[1] * q.vx + u[2] * q.vy));
    q.c = sqrt(g * q.p * ir);
    return q;
}

// normal flux F.S (S not normalised)
__device__ __forceinline__ void flux_n(const double u[4], const Prim& q,
                                       double sx, double sy, double out[4]) {
    double vn = q.vx * sx + q.vy * sy;
    out[0] = u[0] * vn;
    out[1] = u[1] * vn + q.p * sx;
    out[2] = u[2] * vn + q.p * sy;
    out[3] = (u[3] + q.p) * vn;
}

// transformed fluxes at a solution point: f~ = y_eta F - x_eta G,
// g~ = -y_xi F + x_xi G, i.e. normal fluxes along (y_eta,-x_eta) and
// (-y_xi, x_xi)
__device__ __forceinline__ void flux_xy(const double u[4], const Prim& q,
                                        double F[4], double G[4]) {
    F[0] = u[1];
    F[1] = u[1] * q.vx + q.p;
    F[2] = u[2] * q.vx;
    F[3] = (u[3] + q.p) * q.vx;
    G[0] = u[2];
    G[1] = u[1] * q.vy;
    G[2] = u[2] * q.vy + q.p;
    G[3] = (u[3] + q.p) * q.vy;
}

// largest wave speed |v.n| + c along the unit normal (nx, ny)
__device__ __forceinline__ double wave_speed(const Prim& q, double nx,
                                             double ny) {
    double vn = q.vx * nx + q.vy * ny;
    return fabs(vn) + q.c;
}

// ghost state of a boundary flux point: the slip wall mirrors the normal
// momentum (Euler) or velocity (EDAC), both stored in u[1], u[2]; the far
// field is the free stream
__device__ __forceinline__ void ghost_state(const double u[4], double nx,
                                            double ny, bool wall,
                                            const double uinf[4],
                                            double out[4]) {
    if (wall) {
        double mn = u[1] * nx + u[2] * ny;
        out[0] = u[0];
        out[1] = u[1] - 2.0 * mn * nx;
        out[2] = u[2] - 2.0 * mn * ny;
        out[3] = u[3];
    } else {
        for (int v = 0; v < 4; ++v) out[v] = uinf[v];
    }
}

// Rusanov: 1/2 (F(a)+F(b)).S + 1/2 max(la, lb) |S| (a - b)
__device__ __forceinline__ void rusanov(const double a[4], const double b[4],
                                        double sx, double sy, double g,
                                        double out[4]) {
    Prim qa = prim(a, g), qb = prim(b, g);
    double mag = sqrt(sx * sx + sy * sy);
    double nx = sx / mag, ny = sy / mag;
    double fa[4], fb[4];
    flux_n(a, qa, sx, sy, fa);
    flux_n(b, qb, sx, sy, fb);
    double la = wave_speed(qa, nx, ny), lb = wave_speed(qb, nx, ny);
    double s = la >= lb ? la : lb;
    double d = 0.5 * s * mag;
    for (int v = 0; v < 4; ++v) out[v] = 0.5 * (fa[v] + fb[v]) + d * (a[v] - b[v]);
}

// hybridized flux: F(uh).S + s(uh) |S| (u - uh)
__device__ __forceinline__ void hfr_flux(const double u[4], const double uh[4],
                                         double sx, double sy, double g,
                                         double out[4]) {
    Prim q = prim(uh, g);
    double mag = sqrt(sx * sx + sy * sy);
    double f[4];
    flux_n(uh, q, sx, sy, f);
    double s = wave_speed(q, sx / mag, sy / mag);
    double d = s * mag;
    for (int v = 0; v < 4; ++v) out[v] = f[v] + d * (u[v] - uh[v]);
}

// ---- derivatives -------------------------------------------------------

// d(F.S)/du, row-major 4x4 (S not normalised)
__device__ __forceinline__ void dflux_n(const double u[4], const Prim& q,
                                        double sx, double sy, double g,
                                        double A[16]) {
    double vn = q.vx * sx + q.vy * sy;
    double k2 = 0.5 * (g - 1.0) * (q.vx * q.vx + q.vy * q.vy);
    double H = (u[3] + q.p) / u[0];
    double gm = g - 1.0;
    A[0] = 0.0;
    A[1] = sx;
    A[2] = sy;
    A[3] = 0.0;
    A[4] = k2 * sx - q.vx * vn;
    A[5] = vn + q.vx * sx - gm * q.vx * sx;
    A[6] = q.vx * sy - gm * q.vy * sx;
    A[7] = gm * sx;
    A[8] = k2 * sy - q.vy * vn;
    A[9] = q.vy * sx - gm * q.vx * sy;
    A[10] = vn + q.vy * sy - gm * q.vy * sy;
    A[11] = gm * sy;
    A[12] = (k2 - H) * vn;
    A[13] = H * sx - gm * q.vx * vn;
    A[14] = H * sy - gm * q.vy * vn;
    A[15] = g * vn;
}

// d(|v.n| + c)/du along the unit normal (sign(0) taken as +1)
__device__ __forceinline__ void dwave_speed(const double u[4], const Prim& q,
                                            double nx, double ny, double g,
                                            double ds[4]) {
    double ir = 1.0 / u[0];
    double vn = q.vx * nx + q.vy * ny;
    double sg = vn >= 0.0 ? 1.0 : -1.0;
    double gm = g - 1.0;
    double dp0 = gm * 0.5 * (q.vx * q.vx + q.vy * q.vy);
    double kc = g / (2.0 * q.c * u[0]);
    // dc = kc (dp - p/rho drho)
    ds[0] = sg * (-vn * ir) + kc * (dp0 - q.p * ir);
    ds[1] = sg * (nx * ir) + kc * (-gm * q.vx);
    ds[2] = sg * (ny * ir) + kc * (-gm * q.vy);
    ds[3] = kc * gm;
}

// Rusanov derivatives: Ja = d/da, Jb = d/db (ties of the max go to a)
__device__ __forceinline__ void drusanov(const double a[4], const double b[4],
                                         double sx, double sy, double g,
                                         double Ja[16], double Jb[16]) {
    Prim qa = prim(a, g), qb = prim(b, g);
    double mag = sqrt(sx * sx + sy * sy);
    double nx = sx / mag, ny = sy / mag;
    dflux_n(a, qa, sx, sy, g, Ja);
    dflux_n(b, qb, sx, sy, g, Jb);
    double la = wave_speed(qa, nx, ny), lb = wave_speed(qb, nx, ny);
    bool takea = la >= lb;
    double s = takea ? la : lb;
    double ds[4];
    if (takea) dwave_speed(a, qa, nx, ny, g, ds);
    else dwave_speed(b, qb, nx, ny, g, ds);
    for (int k = 0; k < 16; ++k) {
        Ja[k] *= 0.5;
        Jb[k] *= 0.5;
    }
    double hs = 0.5 * s * mag;
    for (int v = 0; v < 4; ++v) {
        Ja[5 * v] += hs;
        Jb[5 * v] -= hs;
        double dv = 0.5 * mag * (a[v] - b[v]);
        for (int w = 0; w < 4; ++w) {
            if (takea) Ja[4 * v + w] += dv * ds[w];
            else Jb[4 * v + w] += dv * ds[w];
        }
    }
}

// hybridized flux derivatives: Ju = d/du = s|S| I, Jh = d/duhat
__device__ __forceinline__ void dhfr_flux(const double u[4], const double uh[4],
                                          double sx, double sy, double g,
                                          double* su, double Jh[16]) {
    Prim q = prim(uh, g);
    double mag = sqrt(sx * sx + sy * sy);
    double nx = sx / mag, ny = sy / mag;
    dflux_n(uh, q, sx, sy, g, Jh);
    double s = wave_speed(q, nx, ny);
    double ds[4];
    dwave_speed(uh, q, nx, ny, g, ds);
    *su = s * mag;
    for (int v = 0; v < 4; ++v) {
        Jh[5 * v] -= s * mag;
        double dv = mag * (u[v] - uh[v]);
        for (int w = 0; w < 4; ++w) Jh[4 * v + w] += dv * ds[w];
    }
}

// ---- EDAC ----------------------------------------------------------------

__device__ __forceinline__ void edac_flux_n(const double u[4], double th, double sx,
                                            double sy, double out[4]) {
    const double vn = u[1] * sx + u[2] * sy;
    out[0] = vn * (u[0] + th);
    out[1] = vn * u[1] + u[0] * sx;
    out[2] = vn * u[2] + u[0] * sy;
    out[3] = vn * u[3];
}

__device__ __forceinline__ void edac_flux_xy(const double u[4], double th, double F[4],
                                             double G[4]) {
    const double Pt = u[0] + th;
    F[0] = u[1] * Pt;
    F[1] = u[1] * u[1] + u[0];
    F[2] = u[1] * u[2];
    F[3] = u[1] * u[3];
    G[0] = u[2] * Pt;
    G[1] = u[2] * u[1];
    G[2] = u[2] * u[2] + u[0];
    G[3] = u[2] * u[3];
}

// largest eigenvalue modulus of the normal flux Jacobian along the unit
// normal: 3/2 |v.n| + sqrt((v.n)^2/4 + P + theta)
__device__ __forceinline__ double edac_wave_speed(const double u[4], double th,
                                                  double nx, double ny) {
    const double vn = u[1] * nx + u[2] * ny;
    return 1.5 * fabs(vn) + sqrt(0.25 * vn * vn + u[0] + th);
}

// hybridized stabilisation 3/2 |v| + sqrt(|v|^2/4 + P + theta)
__device__ __forceinline__ double edac_hfr_speed(const double u[4], double th) {
    const double vv = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
    return 1.5 * sqrt(vv) + sqrt(0.25 * vv + u[0] + th);
}

// d(F.S)/du, row-major 4x4
__device__ __forceinline__ void edac_dflux_n(const double u[4], double th, double sx,
                                             double sy, double A[16]) {
    const double vn = u[1] * sx + u[2] * sy, Pt = u[0] + th;
    A[0] = vn;
    A[1] = Pt * sx;
    A[2] = Pt * sy;
    A[3] = 0.0;
    A[4] = sx;
    A[5] = vn + u[1] * sx;
    A[6] = u[1] * sy;
    A[7] = 0.0;
    A[8] = sy;
    A[9] = u[2] * sx;
    A[10] = vn + u[2] * sy;
    A[11] = 0.0;
    A[12] = 0.0;
    A[13] = u[3] * sx;
    A[14] = u[3] * sy;
    A[15] = vn;
}

// d(wave speed)/du along the unit normal (sign(0) taken as +1)
__device__ __forceinline__ void edac_dwave_speed(const double u[4], double th, double nx,
                                                 double ny, double ds[4]) {
    const double vn = u[1] * nx + u[2] * ny;
    const double d = sqrt(0.25 * vn * vn + u[0] + th);
    const double kv = (vn >= 0.0 ? 1.5 : -1.5) + vn / (4.0 * d);
    ds[0] = 0.5 / d;
    ds[1] = kv * nx;
    ds[2] = kv * ny;
    ds[3] = 0.0;
}

// d(stabilisation)/du; d|v|/dv at v = 0 taken as 0
__device__ __forceinline__ void edac_dhfr_speed(const double u[4], double th, double ds[4]) {
    const double vv = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
    const double vm = sqrt(vv), d = sqrt(0.25 * vv + u[0] + th);
    ds[0] = 0.5 / d;
    for (int c = 1; c < 4; ++c) ds[c] = (vm > 0.0 ? 1.5 * u[c] / vm : 0.0) + u[c] / (4.0 * d);
}

__device__ __forceinline__ void edac_rusanov(const double a[4], const double b[4],
                                             double sx, double sy, double th, double out[4]) {
    const double mag = sqrt(sx * sx + sy * sy);
    const double nx = sx / mag, ny = sy / mag;
    double fa[4], fb[4];
    edac_flux_n(a, th, sx, sy, fa);
    edac_flux_n(b, th, sx, sy, fb);
    const double la = edac_wave_speed(a, th, nx, ny), lb = edac_wave_speed(b, th, nx, ny);
    const double d = 0.5 * (la >= lb ? la : lb) * mag;
    for (int v = 0; v < 4; ++v) out[v] = 0.5 * (fa[v] + fb[v]) + d * (a[v] - b[v]);
}

__device__ __forceinline__ void edac_drusanov(const double a[4], const double b[4],
                                              double sx, double sy, double th,
                                              double Ja[16], double Jb[16]) {
    const double mag = sqrt(sx * sx + sy * sy);
    const double nx = sx / mag, ny = sy / mag;
    edac_dflux_n(a, th, sx, sy, Ja);
    edac_dflux_n(b, th, sx, sy, Jb);
    const double la = edac_wave_speed(a, th, nx, ny), lb = edac_wave_speed(b, th, nx, ny);
    const bool takea = la >= lb;
    const double s = takea ? la : lb;
    double ds[4];
    edac_dwave_speed(takea ? a : b, th, nx, ny, ds);
    for (int k = 0; k < 16; ++k) {
        Ja[k] *= 0.5;
        Jb[k] *= 0.5;
    }
    const double hs = 0.5 * s * mag;
    for (int v = 0; v < 4; ++v) {
        Ja[5 * v] += hs;
        Jb[5 * v] -= hs;
        const double dv = 0.5 * mag * (a[v] - b[v]);
        for (int w = 0; w < 4; ++w) {
            if (takea) Ja[4 * v + w] += dv * ds[w];
            else Jb[4 * v + w] += dv * ds[w];
        }
    }
}

__device__ __forceinline__ void edac_hfr_flux(const double u[4], const double uh[4],
                                              double sx, double sy, double th, double out[4]) {
    const double mag = sqrt(sx * sx + sy * sy);
    double f[4];
    edac_flux_n(uh, th, sx, sy, f);
    const double d = edac_hfr_speed(uh, th) * mag;
    for (int v = 0; v < 4; ++v) out[v] = f[v] + d * (u[v] - uh[v]);
}

__device__ __forceinline__ void edac_dhfr_flux(const double u[4], const double uh[4],
                                               double sx, double sy, double th, double* su,
                                               double Jh[16]) {
    const double mag = sqrt(sx * sx + sy * sy);
    edac_dflux_n(uh, th, sx, sy, Jh);
    const double s = edac_hfr_speed(uh, th);
    double ds[4];
    edac_dhfr_speed(uh, th, ds);
    *su = s * mag;
    for (int v = 0; v < 4; ++v) {
        Jh[5 * v] -= s * mag;
        const double dv = mag * (u[v] - uh[v]);
        for (int w = 0; w < 4; ++w) Jh[4 * v + w] += dv * ds[w];
    }
}

// ---- choice of system -----------------------------------------------------
enum PhysKind : int { PHYS_EULER = 0, PHYS_EDAC = 1 };

struct PhysK {
    int kind;
    double gam, th;
};

__device__ __forceinline__ void phys_flux_xy(const PhysK& k, const double u[4], double F[4],
                                             double G[4]) {
    if (k.kind == PHYS_EDAC) {
        edac_flux_xy(u, k.th, F, G);
    } else {
        const Prim q = prim(u, k.gam);
        flux_xy(u, q, F, G);
    }
}
// the two transformed-flux Jacobians of a solution point
__device__ __forceinline__ void phys_dflux_pair(const PhysK& k, const double u[4], double ax,
                                                double ay, double bx, double by, double A[16],
                                                double B[16]) {
    if (k.kind == PHYS_EDAC) {
        edac_dflux_n(u, k.th, ax, ay, A);
        edac_dflux_n(u, k.th, bx, by, B);
    } else {
        const Prim q = prim(u, k.gam);
        dflux_n(u, q, ax, ay, k.gam, A);
        dflux_n(u, q, bx, by, k.gam, B);
    }
}
__device__ __forceinline__ void phys_rusanov(const PhysK& k, const double a[4],
                                             const double b[4], double sx, double sy,
                                             double out[4]) {
    if (k.kind == PHYS_EDAC) edac_rusanov(a, b, sx, sy, k.th, out);
    else rusanov(a, b, sx, sy, k.gam, out);
}
__device__ __forceinline__ void phys_drusanov(const PhysK& k, const double a[4],
                                              const double b[4], double sx, double sy,
                                              double Ja[16], double Jb[16]) {
    if (k.kind == PHYS_EDAC) edac_drusanov(a, b, sx, sy, k.th, Ja, Jb);
    else drusanov(a, b, sx, sy, k.gam, Ja, Jb);
}
__device__ __forceinline__ void phys_hfr_flux(const PhysK& k, const double u[4],
                                              const double uh[4], double sx, double sy,
                                              double out[4]) {
    if (k.kind == PHYS_EDAC) edac_hfr_flux(u, uh, sx, sy, k.th, out);
    else hfr_flux(u, uh, sx, sy, k.gam, out);
}
__device__ __forceinline__ void phys_dhfr_flux(const PhysK& k, const double u[4],
                                               const double uh[4], double sx, double sy,
                                               double* su, double Jh[16]) {
    if (k.kind == PHYS_EDAC) edac_dhfr_flux(u, uh, sx, sy, k.th, su, Jh);
    else dhfr_flux(u, uh, sx, sy, k.gam, su, Jh);
}

}  // namespace hfr
