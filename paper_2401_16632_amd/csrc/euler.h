// Device physics of the two-dimensional Euler equations: fluxes, the
// standard FR Rusanov flux (Section 2.1), the hybridized single-sided flux
// (eq:hfrriemann) with s = |vhat.n| + chat, boundary ghost states, and the
// analytic derivatives of each needed by the element blocks of Section 3.2.
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

__device__ __forceinline__ void ghost_state(const double u[4], double nx,
                                            double ny, int role,
                                            const double uinf[4],
                                            double out[4]) {
    if (role == 2) {  // slip wall: mirror the normal momentum
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

}  // namespace hfr
