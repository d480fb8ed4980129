// Element residual kernel: standard FR (eq:freq1) for explicit elements and
// the hybridized element equation (eq:hfr1) with the transmission shares of
// eq:hfr2 / eq:hfrimex for implicit elements.
//
// Launch: a workgroup of 256 lanes holds EPB = 256 / Np elements, one lane
// per solution point.  Phase 1 evaluates the transformed flux at the
// solution points into LDS; phase 2 evaluates every flux point of the batch
// (own face value and discontinuous normal flux from LDS, the neighbour's
// face value from global memory, then the common flux) into LDS; phase 3
// forms the divergence plus corrections.  Each interior flux point is
// evaluated once from each side with the face-owned normal (negated on the
// neighbour), so both sides see exactly opposite fluxes without atomics.
#include "euler.h"
#include "internal.h"

namespace hfr {

template <int P>
__device__ __forceinline__ void face_interp_global(const double* __restrict__ u,
                                                   size_t plane, int e, int lf,
                                                   int q, const RefOps& o,
                                                   double out[4]) {
    constexpr int NP = P * P;
    const double* base = u + size_t(e) * NP;
    double acc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int l = 0; l < P; ++l) {
        int pt;
        double wgt;
        if (lf == 0) { pt = l * P + q; wgt = o.lm[l]; }
        else if (lf == 1) { pt = q * P + l; wgt = o.lp[l]; }
        else if (lf == 2) { pt = l * P + (P - 1 - q); wgt = o.lp[l]; }
        else { pt = (P - 1 - q) * P + l; wgt = o.lm[l]; }
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += wgt * base[v * plane + pt];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) out[v] = acc[v];
}

template <int P>
__global__ __launch_bounds__(256) void k_residual(ResidualLaunch a, RefOps og) {
    constexpr int NP = P * P;
    constexpr int EPB = 256 / NP;
    constexpr int NFP = 4 * P;
    __shared__ RefOps o;
    if (a.gate && *a.gate == 0) return;           // uniform over the grid
    copy_ref_ops(o, og);
    __syncthreads();
    __shared__ double s_u[EPB][NP][4];
    __shared__ double s_f[EPB][NP][4];
    __shared__ double s_g[EPB][NP][4];
    __shared__ double s_H[EPB][NFP][4];

    const int t = threadIdx.x;
    const int slot = t / NP, pt = t % NP;
    const int li = blockIdx.x * EPB + slot;
    const bool act = (slot < EPB) && (li < a.nlist);
    const size_t plane = size_t(a.Ne) * NP;
    const PhysK pk{a.phys.kind, a.phys.gamma, a.phys.theta};
    int e = 0;
    double J = 1.0, uloc[4] = {0, 0, 0, 0};
    if (act) {
        e = a.list[li];
        const int i = pt % P, j = pt / P;
        const double xi = o.x[i], et = o.x[j];
        const double* vx = a.verts + size_t(e) * 8;
        const double* vy = vx + 4;
        const double x_xi = 0.25 * ((vx[1] - vx[0]) * (1 - et) + (vx[2] - vx[3]) * (1 + et));
        const double y_xi = 0.25 * ((vy[1] - vy[0]) * (1 - et) + (vy[2] - vy[3]) * (1 + et));
        const double x_et = 0.25 * ((vx[3] - vx[0]) * (1 - xi) + (vx[2] - vx[1]) * (1 + xi));
        const double y_et = 0.25 * ((vy[3] - vy[0]) * (1 - xi) + (vy[2] - vy[1]) * (1 + xi));
        J = x_xi * y_et - x_et * y_xi;
#pragma unroll
        for (int v = 0; v < 4; ++v) uloc[v] = a.u[v * plane + size_t(e) * NP + pt];
        double F[4], G[4];
        phys_flux_xy(pk, uloc, F, G);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            s_u[slot][pt][v] = uloc[v];
            s_f[slot][pt][v] = y_et * F[v] - x_et * G[v];
            s_g[slot][pt][v] = -y_xi * F[v] + x_xi * G[v];
        }
    }
    __syncthreads();

    for (int idx = t; idx < EPB * NFP; idx += blockDim.x) {
        const int sl = idx / NFP, fp = idx % NFP;
        const int f = fp / P, q = fp % P;
        const int l2 = blockIdx.x * EPB + sl;
        if (l2 >= a.nlist) continue;
        const int e2 = a.list[l2];
        double uf[4] = {0, 0, 0, 0}, fdn[4] = {0, 0, 0, 0};
#pragma unroll
        for (int l = 0; l < P; ++l) {
            int p2;
            double wgt;
            if (f == 0) { p2 = l * P + q; wgt = o.lm[l]; }
            else if (f == 1) { p2 = q * P + l; wgt = o.lp[l]; }
            else if (f == 2) { p2 = l * P + (P - 1 - q); wgt = o.lp[l]; }
            else { p2 = (P - 1 - q) * P + l; wgt = o.lm[l]; }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                uf[v] += wgt * s_u[sl][p2][v];
                double fl = (f == 0 || f == 2) ? s_g[sl][p2][v] : s_f[sl][p2][v];
                fdn[v] += wgt * fl;
            }
        }
        if (f == 0 || f == 3) {
#pragma unroll
            for (int v = 0; v < 4; ++v) fdn[v] = -fdn[v];
        }
        const FaceInfo fi = a.finfo[size_t(e2) * 4 + f];
        const double2 S = a.fS[size_t(e2) * 4 + f];
        double com[4], outer[4];
        if (fi.role == ROLE_HFR) {
            const int tf = fi.trace >> 1, side = fi.trace & 1;
            if (a.efr_fnodes) {
                // interior-embedded trace: GLL nodes interpolated to the
                // flux point (element counter-clockwise order)
#pragma unroll
                for (int v = 0; v < 4; ++v) outer[v] = 0.0;
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    const int nd = a.efr_fnodes[size_t(tf) * P + (side ? P - 1 - i : i)];
                    const double wgt = o.gi[q * P + i];
#pragma unroll
                    for (int v = 0; v < 4; ++v) outer[v] += wgt * a.uhat[size_t(nd) * 4 + v];
                }
            } else {
                const int tp = tf * P + (side ? P - 1 - q : q);
#pragma unroll
                for (int v = 0; v < 4; ++v) outer[v] = a.uhat[size_t(tp) * 4 + v];
            }
            phys_hfr_flux(pk, uf, outer, S.x, S.y, com);
            if (a.gk) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    a.gk[((size_t(l2) * 4 + f) * P + q) * 4 + v] = o.w[q] * com[v];
            }
        } else {
            if (fi.role == ROLE_RUSANOV) {
                face_interp_global<P>(a.u, plane, fi.nb_e, fi.nb_lf, P - 1 - q, o, outer);
            } else {
                const double mag = sqrt(S.x * S.x + S.y * S.y);
                ghost_state(uf, S.x / mag, S.y / mag, role_is_wall(fi.role), a.phys.uinf,
                            outer);
            }
            if (role_is_boundary_trace(fi.role)) {
                // boundary trace of an implicit element: the mean of the
                // face state and its ghost, closed-form root of the
                // boundary transmission condition
#pragma unroll
                for (int v = 0; v < 4; ++v) outer[v] = 0.5 * (uf[v] + outer[v]);
                phys_hfr_flux(pk, uf, outer, S.x, S.y, com);
            } else {
                phys_rusanov(pk, uf, outer, S.x, S.y, com);
            }
            if (a.gk) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    a.gk[((size_t(l2) * 4 + f) * P + q) * 4 + v] = 0.0;
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) s_H[sl][fp][v] = com[v] - fdn[v];
    }
    __syncthreads();

    if (!act) return;
    const int i = pt % P, j = pt / P;
    double div[4] = {0, 0, 0, 0};
#pragma unroll
    for (int l = 0; l < P; ++l) {
        const double di = o.D[i * P + l], dj = o.D[j * P + l];
#pragma unroll
        for (int v = 0; v < 4; ++v)
            div[v] += di * s_f[slot][j * P + l][v] + dj * s_g[slot][l * P + i][v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        div[v] += o.cr[i] * s_H[slot][1 * P + j][v] +
                  o.cl[i] * s_H[slot][3 * P + (P - 1 - j)][v] +
                  o.cl[j] * s_H[slot][0 * P + i][v] +
                  o.cr[j] * s_H[slot][2 * P + (P - 1 - i)][v];
    }
    const size_t oplane = size_t(a.nlist) * NP;
    const size_t oidx = size_t(li) * NP + pt;
    const double iJ = 1.0 / J;
    const double adt = a.dtscale ? a.aii_dt * a.dtscale[e] : a.aii_dt;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const double R = -div[v] * iJ;
        if (a.R) a.R[v * oplane + oidx] = R;
        if (a.h) a.h[v * oplane + oidx] = uloc[v] - a.ustar[v * oplane + oidx] - adt * R;
    }
}

template <int P>
static hipError_t launch_residual_p(const RefOps& o, const ResidualLaunch& a,
                                    hipStream_t st) {
    constexpr int EPB = 256 / (P * P);
    int grid = (a.nlist + EPB - 1) / EPB;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_residual<P>, dim3(grid), dim3(256), 0, st, a, o);
    return hipGetLastError();
}

hipError_t launch_residual(const RefOps& o, const ResidualLaunch& a,
                           hipStream_t st) {
    switch (o.P) {
        case 2: return launch_residual_p<2>(o, a, st);
        case 3: return launch_residual_p<3>(o, a, st);
        case 4: return launch_residual_p<4>(o, a, st);
        case 5: return launch_residual_p<5>(o, a, st);
        case 6: return launch_residual_p<6>(o, a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hfr
