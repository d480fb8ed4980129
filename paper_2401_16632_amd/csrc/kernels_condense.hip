// Element blocks and static condensation (Section 3.2).
//
// For implicit element k with n = 4 Np element unknowns and m = 16 P trace
// unknowns (all four faces; a face off the trace gets an identity row and
// zero coupling), the element tableau
//      [ A  B ]
//      [ C  D ]
// is built from analytic flux Jacobians (the exact derivatives of h and of
// the element's share of g) and swept by n Jordan exchanges on the columns
// of A (block Gauss-Jordan elimination with partial pivoting inside the A
// rows).  The swept tableau holds A^-1, A^-1 B, C A^-1 and the element
// Schur complement L^k = D - C A^-1 B of eq:assembly; recovery
// (eq:localproblems) and the condensed right-hand side t^k = s - C A^-1 r
// then reduce to matrix-vector products, the latter accumulated in FP64.
//
// Element-local ordering: u index = point*4 + var (point j*P+i), trace
// index = (face*P + q)*4 + var with q counter-clockwise along the element.
#include "euler.h"
#include "internal.h"
#include "wave_ops.h"

namespace hfr {

template <int P>
struct CondShared {
    static constexpr int NP = P * P;
    double Af[NP][16];
    double Ag[NP][16];
    double c[NP];
    double Fu[4 * P][16];
    double Fh[4 * P][16];
    int tr[4];
};

template <int P>
__device__ void element_linearisation(const CondenseLaunch& a, const RefOps& o,
                                      int k, CondShared<P>& sh) {
    constexpr int NP = P * P;
    const int t = threadIdx.x;
    const int e = a.imp_list[k];
    const size_t plane = size_t(a.Ne) * NP;
    const PhysK pk{a.phys.kind, a.phys.gamma, a.phys.theta};
    const double* vx = a.verts + size_t(e) * 8;
    const double* vy = vx + 4;
    if (t < NP) {
        const int i = t % P, j = t / P;
        const double xi = o.x[i], et = o.x[j];
        const double x_xi = 0.25 * ((vx[1] - vx[0]) * (1 - et) + (vx[2] - vx[3]) * (1 + et));
        const double y_xi = 0.25 * ((vy[1] - vy[0]) * (1 - et) + (vy[2] - vy[3]) * (1 + et));
        const double x_et = 0.25 * ((vx[3] - vx[0]) * (1 - xi) + (vx[2] - vx[1]) * (1 + xi));
        const double y_et = 0.25 * ((vy[3] - vy[0]) * (1 - xi) + (vy[2] - vy[1]) * (1 + xi));
        const double J = x_xi * y_et - x_et * y_xi;
        double uu[4];
        for (int v = 0; v < 4; ++v) uu[v] = a.u[v * plane + size_t(e) * NP + t];
        phys_dflux_pair(pk, uu, y_et, -x_et, -y_xi, x_xi, sh.Af[t], sh.Ag[t]);
        sh.c[t] = (a.dtscale ? a.aii_dt * a.dtscale[e] : a.aii_dt) / J;
    }
    if (t < 4) sh.tr[t] = (a.finfo[size_t(e) * 4 + t].role == ROLE_HFR);
    // the face terms on the second wave, concurrently with the point terms
    // (the face states are interpolated from u directly)
    const int tq = t - 64;
    if (tq >= 0 && tq < 4 * P) {
        const int f = tq / P, q = tq % P;
        const double* ue = a.u + size_t(e) * NP;
        double uf[4] = {0, 0, 0, 0};
        for (int l = 0; l < P; ++l) {
            int p2;
            double wgt;
            if (f == 0) { p2 = l * P + q; wgt = o.lm[l]; }
            else if (f == 1) { p2 = q * P + l; wgt = o.lp[l]; }
            else if (f == 2) { p2 = l * P + (P - 1 - q); wgt = o.lp[l]; }
            else { p2 = (P - 1 - q) * P + l; wgt = o.lm[l]; }
            for (int v = 0; v < 4; ++v) uf[v] += wgt * ue[v * plane + p2];
        }
        const FaceInfo fi = a.finfo[size_t(e) * 4 + f];
        const double2 S = a.fS[size_t(e) * 4 + f];
        double* Fu = sh.Fu[tq];
        double* Fh = sh.Fh[tq];
        for (int z = 0; z < 16; ++z) Fh[z] = 0.0;
        if (fi.role == ROLE_HFR) {
            const int tf = fi.trace >> 1, side = fi.trace & 1;
            double uh[4];
            if (a.efr_fnodes) {
                for (int v = 0; v < 4; ++v) uh[v] = 0.0;
                for (int i = 0; i < P; ++i) {
                    const int nd = a.efr_fnodes[size_t(tf) * P + (side ? P - 1 - i : i)];
                    for (int v = 0; v < 4; ++v) uh[v] += o.gi[q * P + i] * a.uhat[size_t(nd) * 4 + v];
                }
            } else {
                const int tp = tf * P + (side ? P - 1 - q : q);
                for (int v = 0; v < 4; ++v) uh[v] = a.uhat[size_t(tp) * 4 + v];
            }
            double su;
            phys_dhfr_flux(pk, uf, uh, S.x, S.y, &su, Fh);
            for (int z = 0; z < 16; ++z) Fu[z] = 0.0;
            for (int v = 0; v < 4; ++v) Fu[5 * v] = su;
        } else {
            double outer[4], Jb[16];
            const double mag = sqrt(S.x * S.x + S.y * S.y);
            const double nx = S.x / mag, ny = S.y / mag;
            if (fi.role == ROLE_RUSANOV) {
                const double* base = a.u + size_t(fi.nb_e) * NP;
                const int qn = P - 1 - q, lf = fi.nb_lf;
                for (int v = 0; v < 4; ++v) outer[v] = 0.0;
                for (int l = 0; l < P; ++l) {
                    int p2;
                    double wgt;
                    if (lf == 0) { p2 = l * P + qn; wgt = o.lm[l]; }
                    else if (lf == 1) { p2 = qn * P + l; wgt = o.lp[l]; }
                    else if (lf == 2) { p2 = l * P + (P - 1 - qn); wgt = o.lp[l]; }
                    else { p2 = (P - 1 - qn) * P + l; wgt = o.lm[l]; }
                    for (int v = 0; v < 4; ++v) outer[v] += wgt * base[v * plane + p2];
                }
                phys_drusanov(pk, uf, outer, S.x, S.y, Fu, Jb);
            } else {
                const bool wall = role_is_wall(fi.role);
                ghost_state(uf, nx, ny, wall, a.phys.uinf, outer);
                // d ghost / d u: the mirror I - 2 n n^T on the two middle
                // rows at a wall, zero in the far field
                const double R[16] = {1, 0, 0, 0, 0, 1 - 2 * nx * nx, -2 * nx * ny, 0,
                                      0, -2 * nx * ny, 1 - 2 * ny * ny, 0, 0, 0, 0, 1};
                if (role_is_boundary_trace(fi.role)) {
                    // F_hat(u, uhat_b(u)), uhat_b = (u + ghost(u))/2:
                    // dF/du = s|S| I + (dF/duhat) (I + dghost/du)/2
                    for (int v = 0; v < 4; ++v) outer[v] = 0.5 * (uf[v] + outer[v]);
                    double su;
                    phys_dhfr_flux(pk, uf, outer, S.x, S.y, &su, Jb);
                    for (int v = 0; v < 4; ++v)
                        for (int w = 0; w < 4; ++w) {
                            double acc = 0.5 * Jb[4 * v + w];
                            if (wall)
                                for (int z = 0; z < 4; ++z) acc += 0.5 * Jb[4 * v + z] * R[4 * z + w];
                            Fu[4 * v + w] = acc + (v == w ? su : 0.0);
                        }
                } else {
                    phys_drusanov(pk, uf, outer, S.x, S.y, Fu, Jb);
                    if (wall) {
                        for (int v = 0; v < 4; ++v)
                            for (int w = 0; w < 4; ++w) {
                                double acc = 0.0;
                                for (int z = 0; z < 4; ++z) acc += Jb[4 * v + z] * R[4 * z + w];
                                Fu[4 * v + w] += acc;
                            }
                    }
                }
            }
        }
    }
    __syncthreads();
}

// ---- block Gauss-Jordan sweep ----------------------------------------------
// The tableau T = [A B; C D] (N = n + m rows and columns) is swept with n
// Jordan exchanges, one per column k of A, pivoting on the unused A row of
// largest magnitude in that column.  Exchange (p, k) solves equation p for
// the variable of column k:
//      T'[p][k] = 1/T[p][k],  T'[p][j] = -T[p][j]/T[p][k],
//      T'[i][k] = T[i][k]/T[p][k],  T'[i][j] = T[i][j] - T'[i][k] T[p][j].
// With p_k the pivot row of step k, the swept tableau holds
//      T[p_k][j] = A^-1[k][p_j],   T[p_k][n+b] = -(A^-1 B)[k][b],
//      T[n+i][j] = (C A^-1)[i][p_j],  T[n+i][n+b] = (D - C A^-1 B)[i][b],
// i.e. the element inverse used by recovery (eq:localproblems) and the
// element Schur complement of eq:assembly.
//
// Register layout: a workgroup of W waves per element; lane l holds rows
// l + 64 s (s < RPL) and wave w the columns w, w + W, w + 2W, ... (NCW of
// them at most).  A
// pivot row is left unscaled in registers with its factor -1/T[p][k] kept
// per row (applied on the way out), so every step is one rank-1 update
// T[i][j] -= g_i u_j with g_p = 0.  The wave that owns column k finds the
// pivot and the multipliers and passes them to the other waves through LDS
// (one barrier per step); each wave reads its own segment of the pivot row
// from the lane that holds it.  The result is stored column-major, (N x N)
// per element.
// Register shape of the sweep.  Columns of a wave are held as vectors of
// CH values (CH in {4, 8, 16}, the one that pads the wave's column count
// least) so that the column addressed by the wave-uniform step index is
// reached by VGPR indexing.  W, the waves per element, is the smallest
// power of two (at most 16) that keeps the tableau share of a lane within
// about 72 VGPRs: more waves shorten the per-element critical path and
// raise occupancy.
constexpr int sweep_ch(int ncw) {
    int best = 16, pad = (ncw + 15) / 16 * 16;
    for (int c = 8; c >= 4; c /= 2)
        if ((ncw + c - 1) / c * c < pad) { best = c; pad = (ncw + c - 1) / c * c; }
    return best;
}
constexpr int sweep_regs(int rpl, int N, int w, int words) {
    const int ncw = (N + w - 1) / w, ch = sweep_ch(ncw);
    return rpl * ((ncw + ch - 1) / ch * ch) * words;
}
constexpr int sweep_waves(int rpl, int N, int words) {
    int w = 1;
    while (sweep_regs(rpl, N, w, words) > 72 && w < 16) w *= 2;
    return w;
}

// SCHUR: the Schur-only instance holds the rows of A and B only (the rows
// of C and D are not swept: the element Schur complement is formed
// afterwards from C's structure, k_schur_lift)
template <int P, typename T, bool SCHUR>
struct SweepShape {
    static constexpr int NP = P * P, n = 4 * NP, m = 16 * P, N = n + m;
    static constexpr int R = SCHUR ? n : N;          // rows held
    static constexpr int RPL = (R + 63) / 64;
    static constexpr int W = sweep_waves(RPL, N, int(sizeof(T) / 4));
    static constexpr int NCW = (N + W - 1) / W;
    static constexpr int CH = sweep_ch(NCW);
    static constexpr int NCH = (NCW + CH - 1) / CH;
    // occupancy the register budget is held to: the tableau share of a lane
    // plus about 48 registers of the step's working set
    static constexpr int TREGS = RPL * NCH * CH * int(sizeof(T) / 4);
    static constexpr int WPE = TREGS <= 40 ? 6 : TREGS <= 56 ? 5 : TREGS <= 80 ? 4 : 2;
};

// ---- fill of the element tableau ------------------------------------------
// One workgroup per implicit element forms the element linearisation in LDS
// and writes [A B; C D] (exact derivatives, FP64, rounded to T) to the
// element's tableau slot, column-major, one 4x4 point block per thread:
// rows of an element point (or trace point) against the columns of another.
// Consecutive threads take consecutive row blocks of one block column, so
// every 16- or 32-byte store of a block column is contiguous.
template <int P>
__device__ __forceinline__ void block_column(int br, int bc, int cc, const RefOps& o,
                                             const CondShared<P>& sh, double out[4]) {
    // column cc of the 4x4 point block (br, bc): out[v] = E[v][cc]
    constexpr int NP = P * P;
#pragma unroll
    for (int v = 0; v < 4; ++v) out[v] = 0.0;
    if (br < NP) {
        const int i = br % P, j = br / P;
        const double cij = sh.c[br];
        if (bc < NP) {
            const int l = bc % P, kk = bc / P;
            // d(R)/du contributions of the row line (kk == j) and the column
            // line (l == i) through the volume derivative and the lifted
            // face corrections
            double a1 = 0, b1 = 0, c1 = 0, a2 = 0, b2 = 0, c2 = 0;
            if (kk == j) {
                b1 = o.cr[i] * o.lp[l];
                c1 = o.cl[i] * o.lm[l];
                a1 = o.D[i * P + l] - b1 + c1;
            }
            if (l == i) {
                b2 = o.cl[j] * o.lm[kk];
                c2 = o.cr[j] * o.lp[kk];
                a2 = o.D[j * P + kk] + b2 - c2;
            }
            if (kk == j || l == i) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int z = v * 4 + cc;
                    double acc = 0.0;
                    if (kk == j)
                        acc += a1 * sh.Af[bc][z] + b1 * sh.Fu[1 * P + j][z] +
                               c1 * sh.Fu[3 * P + (P - 1 - j)][z];
                    if (l == i)
                        acc += a2 * sh.Ag[bc][z] + b2 * sh.Fu[0 * P + i][z] +
                               c2 * sh.Fu[2 * P + (P - 1 - i)][z];
                    out[v] = cij * acc;
                }
            }
            if (bc == br) out[cc] += 1.0;
        } else {
            const int tb = bc - NP, f2 = tb / P, q2 = tb % P;
            if (!sh.tr[f2]) return;
            double coef = 0.0;
            if (f2 == 1) { if (q2 == j) coef = o.cr[i]; }
            else if (f2 == 3) { if (q2 == P - 1 - j) coef = o.cl[i]; }
            else if (f2 == 0) { if (q2 == i) coef = o.cl[j]; }
            else { if (q2 == P - 1 - i) coef = o.cr[j]; }
            if (coef == 0.0) return;
#pragma unroll
            for (int v = 0; v < 4; ++v) out[v] = cij * coef * sh.Fh[tb][v * 4 + cc];
        }
    } else {
        const int ta = br - NP, f = ta / P, q = ta % P;
        if (!sh.tr[f]) {
            if (bc == br) out[cc] = 1.0;
            return;
        }
        const double wq = o.w[q];
        if (bc < NP) {
            const int l = bc % P, kk = bc / P;
            double coef = 0.0;
            if (f == 1) { if (kk == q) coef = o.lp[l]; }
            else if (f == 3) { if (kk == P - 1 - q) coef = o.lm[l]; }
            else if (f == 0) { if (l == q) coef = o.lm[kk]; }
            else { if (l == P - 1 - q) coef = o.lp[kk]; }
            if (coef == 0.0) return;
#pragma unroll
            for (int v = 0; v < 4; ++v) out[v] = wq * coef * sh.Fu[ta][v * 4 + cc];
        } else if (bc == br) {
#pragma unroll
            for (int v = 0; v < 4; ++v) out[v] = wq * sh.Fh[ta][v * 4 + cc];
        }
    }
}

template <int P>
__device__ __forceinline__ void block_entries(int br, int bc, const RefOps& o,
                                              const CondShared<P>& sh,
                                              double E[4][4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double col[4];
        block_column<P>(br, bc, c, o, sh, col);
#pragma unroll
        for (int v = 0; v < 4; ++v) E[v][c] = col[v];
    }
}

// AB: only the rows of A and B are written (the Schur-only sweep's input);
// the face-point flux Jacobians from which C and D are formed go to a.lin
// ([Nim][2][4P][16] FP64: d F_hat / d u, then d F_hat / d uhat, zero off
// the trace) for k_schur_lift.
template <int P, typename T, bool AB>
__global__ __launch_bounds__(256) void k_tableau_fill(CondenseLaunch a, RefOps og) {
    constexpr int NP = P * P, n = 4 * NP, m = 16 * P, N = n + m, NB = NP + 4 * P;
    constexpr int NBR = AB ? NP : NB;         // block rows written
    __shared__ CondShared<P> sh;
    __shared__ RefOps o;
    if (a.go && *a.go == 0) return;            // uniform over the grid
    const int k = blockIdx.x;
    copy_ref_ops(o, og);
    __syncthreads();
    element_linearisation<P>(a, o, k, sh);
    T* G = reinterpret_cast<T*>(a.M) + size_t(k) * N * N;
    double* bcopy = a.blocks_copy ? a.blocks_copy + size_t(k) * N * N : nullptr;
    if constexpr (AB) {
        double* lin = a.lin + size_t(k) * 2 * 4 * P * 16;
        for (int i = threadIdx.x; i < 4 * P * 16; i += blockDim.x) {
            lin[i] = sh.Fu[i >> 4][i & 15];
            lin[4 * P * 16 + i] = sh.Fh[i >> 4][i & 15];
        }
        if (bcopy) {                           // inspection copy: all blocks
            for (int blk = threadIdx.x; blk < NB * NB; blk += blockDim.x) {
                const int bc = blk / NB, br = blk - bc * NB;
                double E[4][4];
                block_entries<P>(br, bc, o, sh, E);
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        bcopy[size_t(4 * br + v) * N + 4 * bc + c] = E[v][c];
            }
            bcopy = nullptr;
        }
    }
    for (int blk = threadIdx.x; blk < NB * NBR; blk += blockDim.x) {
        const int bc = blk / NBR, br = blk - bc * NBR;
        double E[4][4];
        block_entries<P>(br, bc, o, sh, E);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            // four rows of one column, 16-byte aligned (N is a multiple of 4)
            T* dst = G + size_t(4 * bc + c) * N + 4 * br;
            if constexpr (sizeof(T) == 4) {
                *reinterpret_cast<float4*>(dst) =
                    make_float4(float(E[0][c]), float(E[1][c]), float(E[2][c]), float(E[3][c]));
            } else {
                reinterpret_cast<double2*>(dst)[0] = make_double2(E[0][c], E[1][c]);
                reinterpret_cast<double2*>(dst)[1] = make_double2(E[2][c], E[3][c]);
            }
        }
        if (bcopy) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    bcopy[size_t(4 * br + v) * N + 4 * bc + c] = E[v][c];
        }
    }
}

template <int P, typename T, bool SCHUR>
__global__ __launch_bounds__((64 * SweepShape<P, T, SCHUR>::W))
__attribute__((amdgpu_waves_per_eu(SweepShape<P, T, SCHUR>::WPE))) void k_condense_sweep(
    CondenseLaunch a, RefOps og) {
    using S = SweepShape<P, T, SCHUR>;
    constexpr int n = S::n, N = S::N, R = S::R, RPL = S::RPL, W = S::W, NCW = S::NCW;
    __shared__ T gbuf[2][RPL * 64];
    __shared__ T ibuf[2];
    __shared__ int pbuf[2];
    // right-hand side epilogue of the full sweep: pivot rows, permuted -h,
    // per-wave row sums
    constexpr int NRW = W < n ? W : n;          // waves owning columns of A
    __shared__ short pl[SCHUR ? 1 : n];
    __shared__ double sr[SCHUR ? 1 : n];
    __shared__ double racc[SCHUR ? 1 : NRW][SCHUR ? 1 : RPL * 64];
    const int lane = threadIdx.x & 63;
    // wave index, uniform (so that indices derived from it address
    // registers by index mode rather than by per-lane selects)
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int k = blockIdx.x;

    // ---- load this wave's columns of the filled tableau (column-major)
    constexpr int CH = S::CH, NCH = S::NCH;
    constexpr int SPN = (n + 63) / 64;      // row slots that can hold pivot rows
    typedef T VT __attribute__((ext_vector_type(CH)));
    // columns are dealt round-robin: wave w holds columns w, w + W, ...
    // (local index j is column w + W j), so the owner of the next pivot
    // column, which also searches for its pivot, changes every step
    T* G = reinterpret_cast<T*>(a.M) + size_t(k) * N * N;
    VT t[RPL][NCH];
    T sig[RPL];
    bool used[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int row = lane + 64 * s;
        sig[s] = T(1);
        used[s] = false;
#pragma unroll
        for (int j = 0; j < NCH * CH; ++j) {
            const int col = w + W * j;
            // clamped address: the load stays inside this element's slot
            const T v = G[size_t(min(col, N - 1)) * N + min(row, R - 1)];
            t[s][j / CH][j % CH] = (j < NCW && row < R && col < N) ? v : T(0);
        }
    }
    // Schur-only sweep: the right-hand side [h; 0] rides along as an FP64
    // column on the last wave (after the exchanges it holds -A^-1 h in the
    // pivot rows, unscaled like them, and -C A^-1 h in the rows of C)
    constexpr bool schur = SCHUR;
    constexpr int RW = W - 1;
    double rhs[schur ? RPL : 1];
#pragma unroll
    for (int s = 0; s < (schur ? RPL : 1); ++s) {
        const int row = lane + 64 * s;
        rhs[s] = 0.0;
        if (schur && w == RW && row < n) {
            constexpr int NP = P * P;
            rhs[s] = a.h[size_t(row & 3) * a.nimp * NP + size_t(k) * NP + (row >> 2)];
        }
    }
    // ---- n Jordan exchanges ---------------------------------------------------
    // The wave that owns column k+1 updates that column first and finds the
    // pivot of step k+1 (look-ahead) before its full rank-1 update of step
    // k, so the other waves rarely wait at the step barrier.
    int* pivk = a.piv + size_t(k) * n;
    T gs[RPL];
    T ipv = T(0);
    int p = -1;
    // pivot search: 32-bit keys (n <= 144 < 256 candidate rows)
    static_assert(n <= 256, "pivot rows must fit the 8-bit row field");
    auto find_pivot = [&](const T (&col)[RPL], int step, T (&g)[RPL], T& ip, int& pp) {
        unsigned key = 0;
#pragma unroll
        for (int s = 0; s < SPN; ++s) {
            const int row = lane + 64 * s;
            const unsigned ks = pivot_key32(float(fabs(col[s])), row);
            if (row < n && !used[s] && ks > key) key = ks;
        }
        key = wave_max_u32(key);
        pp = -1;
        ip = T(0);
        if (key != 0) {
            pp = 255 - int(key & 0xffu);
            const int sp = pp >> 6, lp = pp & 63;
            T pv = T(1);
#pragma unroll
            for (int s = 0; s < SPN; ++s)
                if (SPN == 1 || s == sp) pv = lane_value(col[s], lp);
            // FP32: the hardware reciprocal (1 ulp) instead of the
            // correctly rounded division sequence on the critical path
            if constexpr (sizeof(T) == 4) ip = __builtin_amdgcn_rcpf(pv);
            else ip = T(1) / pv;
        }
#pragma unroll
        for (int s = 0; s < RPL; ++s)
            g[s] = (lane + 64 * s == pp) ? T(0) : col[s] * ip;
        const int buf = step & 1;
        if (W > 1) {
#pragma unroll
            for (int s = 0; s < RPL; ++s) gbuf[buf][lane + 64 * s] = g[s];
            if (lane == 0) { pbuf[buf] = pp; ibuf[buf] = ip; }
        }
        if (lane == 0 && pp >= 0) pivk[step] = pp;
    };
    if (w == 0) {
        T col0[RPL];
#pragma unroll
        for (int s = 0; s < RPL; ++s) col0[s] = t[s][0][0];
        find_pivot(col0, 0, gs, ipv, p);
    }
    for (int kk = 0; kk < n; ++kk) {
        const int ow = kk % W, jk = kk / W, buf = kk & 1;
        if (W > 1) {
            __syncthreads();
            if (w != ow) {
                p = __builtin_amdgcn_readfirstlane(pbuf[buf]);
                ipv = ibuf[buf];
#pragma unroll
                for (int s = 0; s < RPL; ++s) gs[s] = gbuf[buf][lane + 64 * s];
            }
        }
        if (p < 0) {
            if (threadIdx.x == 0) *a.pivot_fail = 1;
            return;                                // uniform over the workgroup
        }
        if (!schur && threadIdx.x == 0) pl[kk] = short(p);
        const int sp = p >> 6, lp = p & 63;
#pragma unroll
        for (int s = 0; s < RPL; ++s)
            if (lane + 64 * s == p) { used[s] = true; sig[s] = -ipv; }
        // look-ahead: the owner of column k+1 forms it and picks its pivot
        T gn[RPL];
        T ipn = T(0);
        int pn = -1;
        const int k1 = kk + 1;
        const bool ahead = (k1 < n && w == k1 % W);
        if (ahead) {
            const int j1 = k1 / W, c1 = j1 / CH, e1 = j1 - c1 * CH;
            T cpre[RPL];
#pragma unroll
            for (int s = 0; s < RPL; ++s) cpre[s] = T(0);
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (c == c1) {
#pragma unroll
                    for (int s = 0; s < RPL; ++s) cpre[s] = t[s][c][e1];
                }
            T u1 = T(0);
#pragma unroll
            for (int s = 0; s < SPN; ++s)
                if (SPN == 1 || s == sp) u1 = lane_value(cpre[s], lp);
            T col1[RPL];
#pragma unroll
            for (int s = 0; s < RPL; ++s) col1[s] = fma(-gs[s], u1, cpre[s]);
            find_pivot(col1, k1, gn, ipn, pn);
        }
        // rank-1 update of this wave's columns, two at a time; the pivot
        // row segment comes from the lane holding row p (uniform lane and
        // slot).  In a Schur-only sweep a group whose columns have all been
        // exchanged already (global index <= kk) is skipped.
        constexpr int GJ = 2, NGJ = (NCW + GJ - 1) / GJ;
#pragma unroll
        for (int gq = 0; gq < NGJ; ++gq) {
            const int jlast = (GJ * gq + GJ < NCW ? GJ * gq + GJ : NCW) - 1;
            if (!schur || w + W * jlast > kk) {    // uniform
                T u[GJ];
#pragma unroll
                for (int jj = 0; jj < GJ; ++jj) {
                    const int j = GJ * gq + jj;
                    if (j < NCW) {
                        T src = t[0][j / CH][j % CH];
#pragma unroll
                        for (int s0 = 1; s0 < SPN; ++s0)
                            src = (sp == s0) ? t[s0][j / CH][j % CH] : src;
                        u[jj] = lane_value(src, lp);
                    }
                }
#pragma unroll
                for (int jj = 0; jj < GJ; ++jj) {
                    const int j = GJ * gq + jj;
                    if (j < NCW) {
#pragma unroll
                        for (int s = 0; s < RPL; ++s)
                            t[s][j / CH][j % CH] = fma(-gs[s], u[jj], t[s][j / CH][j % CH]);
                    }
                }
            }
        }
        if constexpr (schur) if (w == RW) {       // uniform
            double ur = rhs[0];
#pragma unroll
            for (int s0 = 1; s0 < SPN; ++s0) ur = (sp == s0) ? rhs[s0] : ur;
            ur = lane_value(ur, lp);
#pragma unroll
            for (int s = 0; s < RPL; ++s) rhs[s] = fma(-double(gs[s]), ur, rhs[s]);
        }
        // column k: multipliers for the other rows, -1 in the pivot row
        if (w == ow) {
            const int ck = jk / CH, ek = jk - ck * CH;
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (c == ck) {
#pragma unroll
                    for (int s = 0; s < RPL; ++s)
                        t[s][c][ek] = (lane + 64 * s == p) ? T(-1) : gs[s];
                }
        }
        if (ahead) {
            p = pn;
            ipv = ipn;
#pragma unroll
            for (int s = 0; s < RPL; ++s) gs[s] = gn[s];
        }
    }

    // ---- FP64 right-hand side (as launch_rhs64): the Schur-only sweep holds
    // A^-1 r in its extra column (scaled here like the pivot rows; C A^-1 r
    // is formed by k_schur_lift); the full sweep forms
    // yr/z[row] = sum_{j<n} T(sig*t)[row][j] * (-h[p_j]) from the registers,
    // each wave over its columns of A, the waves' sums added in a fixed order
    if constexpr (schur) {
        if (w == RW) {
#pragma unroll
            for (int s = 0; s < RPL; ++s) {
                const int row = lane + 64 * s;
                if (row < n) a.yr[size_t(k) * n + row] = double(sig[s]) * rhs[s];
            }
        }
    } else if (a.yr) {
        constexpr int NP = P * P, m = N - n;
        __syncthreads();                           // pl complete
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const int row = pl[j];
            sr[j] = -a.h[size_t(row & 3) * a.nimp * NP + size_t(k) * NP + (row >> 2)];
        }
        __syncthreads();
        if (w < n) {                               // uniform over the wave
            double acc[RPL];
#pragma unroll
            for (int s = 0; s < RPL; ++s) acc[s] = 0.0;
#pragma unroll
            for (int j = 0; j < NCW; ++j) {
                const int col = w + W * j;
                if (col < n) {
                    const double rj = sr[col];
#pragma unroll
                    for (int s = 0; s < RPL; ++s)
                        acc[s] = fma(double(T(sig[s] * t[s][j / CH][j % CH])), rj, acc[s]);
                }
            }
#pragma unroll
            for (int s = 0; s < RPL; ++s) racc[w][lane + 64 * s] = acc[s];
        }
        __syncthreads();
        for (int row = threadIdx.x; row < N; row += blockDim.x) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < NRW; ++q) v += racc[q][row];
            if (row < n) a.yr[size_t(k) * n + row] = v;
            else a.z[size_t(k) * m + row - n] = v;
        }
    }

    // ---- store column-major, pivot rows scaled (a Schur-only sweep stores
    // the rows of A in the columns of B only: -A^-1 B)
#pragma unroll
    for (int j = 0; j < NCW; ++j) {
        const int col = w + W * j;
        if (col >= N) break;
        if (schur && col < n) continue;           // uniform
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            const int row = lane + 64 * s;
            if (row < R) G[size_t(col) * N + row] = sig[s] * t[s][j / CH][j % CH];
        }
    }
}

// ---- element Schur complement from the structure of C (Section 3.2) --------
// After the Schur-only sweep the rows of A in the columns of B hold
// X = -A^-1 B (row p_k: unknown k) and yr[p_k] = (A^-1 r)[k].  The rows of C
// are sparse: face point (f, q), variable v, couples only to the P solution
// points on the grid line through it, with the face-interpolation weight of
// each point times the flux Jacobian d F_hat / d u at the face point (times
// w_q), and D is 4x4 block diagonal (w_q d F_hat / d uhat).  So
//    L^k = D + C X,   z = C A^-1 r,
// each row an interpolation of X along one line followed by a 4x4 product,
// accumulated in FP64 and stored in the rows of D (the assembly's input).
// Faces off the trace keep identity rows of L and zero z.
template <int P, typename T>
__global__ __launch_bounds__(256) void k_schur_lift(CondenseLaunch a, RefOps og) {
    constexpr int NP = P * P, n = 4 * NP, m = 16 * P, N = n + m, NF = 4 * P;
    constexpr int LDX = n + 1;
    __shared__ RefOps o;
    __shared__ T xs[m * LDX];                  // X in unknown order, by column
    __shared__ double ys[n];
    __shared__ double fu[NF][16], fh[NF][16];
    __shared__ short kinv[n];
    __shared__ int tr[4];
    const int k = blockIdx.x, t = threadIdx.x;
    copy_ref_ops(o, og);
    const int* pk = a.piv + size_t(k) * n;
    for (int j = t; j < n; j += blockDim.x) kinv[pk[j]] = short(j);
    const double* lin = a.lin + size_t(k) * 2 * NF * 16;
    for (int i = t; i < NF * 16; i += blockDim.x) {
        fu[i >> 4][i & 15] = lin[i];
        fh[i >> 4][i & 15] = lin[NF * 16 + i];
    }
    if (t < 4) tr[t] = (a.finfo[size_t(a.imp_list[k]) * 4 + t].role == ROLE_HFR);
    __syncthreads();
    T* G = reinterpret_cast<T*>(a.M) + size_t(k) * N * N;
    // X: consecutive rows of a column per thread group, eight loads in
    // flight per thread before the permuted LDS stores
    constexpr int NX = n * m, PASS = 8;
    for (int i0 = t; i0 < NX; i0 += PASS * 256) {
        T v[PASS];
#pragma unroll
        for (int q = 0; q < PASS; ++q) {
            const int idx = min(i0 + q * 256, NX - 1);
            const int b = idx / n, r = idx - b * n;
            v[q] = G[size_t(n + b) * N + r];
        }
#pragma unroll
        for (int q = 0; q < PASS; ++q) {
            const int idx = i0 + q * 256;
            if (idx < NX) {
                const int b = idx / n, r = idx - b * n;
                xs[b * LDX + kinv[r]] = v[q];
            }
        }
    }
    for (int r = t; r < n; r += blockDim.x) ys[kinv[r]] = a.yr[size_t(k) * n + r];
    __syncthreads();
    // one (face point, column) pair per thread and pass: the four rows of
    // the face point in that column (16-byte store, consecutive face points
    // of a column contiguous)
    for (int idx = t; idx < NF * (m + 1); idx += blockDim.x) {
        const int fq = idx % NF, b = idx / NF;    // b == m: the z column
        const int f = fq / P, q = fq - f * P;
        double out[4];
        if (!tr[f]) {
#pragma unroll
            for (int v = 0; v < 4; ++v) out[v] = (b == fq * 4 + v) ? 1.0 : 0.0;
        } else {
            double sw[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int l = 0; l < P; ++l) {
                int pt;
                double c;
                if (f == 0) { pt = l * P + q; c = o.lm[l]; }
                else if (f == 1) { pt = q * P + l; c = o.lp[l]; }
                else if (f == 2) { pt = l * P + (P - 1 - q); c = o.lp[l]; }
                else { pt = (P - 1 - q) * P + l; c = o.lm[l]; }
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    sw[w] += c * (b < m ? double(xs[b * LDX + pt * 4 + w]) : ys[pt * 4 + w]);
            }
            const double wq = o.w[q];
            const bool diag = (b >> 2) == fq;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double acc = diag ? fh[fq][v * 4 + (b & 3)] : 0.0;
#pragma unroll
                for (int w = 0; w < 4; ++w) acc += fu[fq][v * 4 + w] * sw[w];
                out[v] = wq * acc;
            }
        }
        if (b < m) {
            T* dst = a.compact_schur
                         ? G + schur_offset(4 * P, f, b / (4 * P), 4 * q, b % (4 * P))
                         : G + size_t(n + b) * N + n + fq * 4;
            if constexpr (sizeof(T) == 4) {
                *reinterpret_cast<float4*>(dst) = make_float4(float(out[0]), float(out[1]),
                                                              float(out[2]), float(out[3]));
            } else {
                reinterpret_cast<double2*>(dst)[0] = make_double2(out[0], out[1]);
                reinterpret_cast<double2*>(dst)[1] = make_double2(out[2], out[3]);
            }
        } else {
            double* zz = a.z + size_t(k) * m + fq * 4;
#pragma unroll
            for (int v = 0; v < 4; ++v) zz[v] = tr[f] ? out[v] : 0.0;
        }
    }
}

// ---- blocked elimination of the rows of A on the matrix cores --------------
// The Schur-only elimination of the sweep above, in panels of 16 columns of
// A: for panel K (columns 16j..16j+15, pivot rows P chosen by partial
// pivoting among the rows not used yet, in column order),
//      G = T[:, K] T[P, K]^-1   (rows of P: T[P, K]^-1 itself),
//      T[P, L] <- 0,   T[:, L] <- T[:, L] - G U,   U = T[P, L] (before)
// over the live columns L (the columns of A not eliminated yet, those of B,
// and the right-hand side).  A row of P then holds -T[P,K]^-1 U: the
// expression of the panel's unknowns in the remaining ones, and every
// later panel updates it like any other row, so after the last panel row
// p_k holds -(A^-1 B)[k] in the columns of B -- the sweep's result, with
// piv[k] = p_k -- and the right-hand side column A^-1 h.  G comes from 16
// Jordan exchanges on the panel alone, by the wave that owns it, with the
// panel in a lane-per-row layout; the update G U is a product with K = 16
// on 16x16x4 matrix-core tiles.  Clearing the pivot rows before the product
// forms them without cancellation.  Rows and columns of A are padded to a
// multiple of 16 with decoupled identity unknowns.
//
// Layout: W waves per element; wave w holds the 16-column tiles
// c = w, w + W, ... of [A | pad | B] for all rows, as 16x16 accumulator
// tiles (lane 16 g + i: column i; rows 4g + r (FP32) or g + 4r (FP64) of
// register r).  The owner of panel j + 1 applies panel j to that tile
// first, factors it, and applies panel j to its other tiles only in the
// next period, before panel j + 1, so a period lasts one tile update and
// one factorisation; the panel buffers rotate over three slots for that.
// -G is kept in LDS with the columns of each row in the order
// (c mod 4, c div 4) and U column by column in the same order, so the four
// operands a lane feeds the four products of K = 16 are adjacent (one
// 16-byte read per row tile in FP32).  A 128-bit mask of the panel's pivot
// rows lets every wave skip the row tiles and register slots that hold no
// pivot row when it extracts U.
template <int P, typename T, int WSEL = 0>
struct BlockShape {
    static constexpr int NP = P * P, n = 4 * NP, m = 16 * P, N = n + m;
    static constexpr int NPAD = (n + 15) / 16 * 16;
    static constexpr int RT = NPAD / 16;                 // row tiles = panels
    static constexpr int NCT = RT + m / 16;              // column tiles
    static constexpr int words = int(sizeof(T) / 4);
    static constexpr int pick_w() {
        int w = 4;
        while (RT * ((NCT + w - 1) / w) * 4 * words > 112 && w < 16) w *= 2;
        return w;
    }
    // waves per element: WSEL, or the smallest of 4, 8, 16 whose tiles fit
    // about 112 registers
    static constexpr int W = WSEL > 0 ? WSEL : pick_w();
    static constexpr int CTW = (NCT + W - 1) / W;        // column tiles per wave
    static constexpr int TREGS = RT * CTW * 4 * words;   // accumulator registers
    static constexpr int RPL = (NPAD + 63) / 64;         // panel rows per lane
    static constexpr int LDP = 17;                       // panel row stride
    static constexpr int LDG = words == 1 ? 20 : 18;     // -G row / U column stride
    static constexpr int NB = 3;                         // panel buffer slots
    static constexpr int MW = (NPAD + 31) / 32;          // pivot-mask words
    // waves per SIMD the register budget is held to (512 registers): the
    // tiles, the owner's panel rows and about 48 registers of the rest
    static constexpr int WPE = TREGS + 48 + 8 * RPL * words <= 168 ? 3 : 2;
    // LDS of the elimination (-G slots, U per wave, the panel), reused by
    // the Schur lift of the epilogue (flux Jacobians, A^-1 r, X)
    // X in the lift: column-major with a row stride of n + 4 (16-byte
    // aligned rows of four unknowns of a point)
    static constexpr int NF = 4 * P, LDX = n + 4;
    static constexpr size_t ELIM_BYTES =
        sizeof(T) * (size_t(NB) * NPAD * LDG + size_t(W) * 16 * LDG + size_t(NPAD) * LDP);
    static constexpr size_t LIFT_BYTES =
        sizeof(double) * (2 * NF * 16 + n) + sizeof(T) * size_t(m) * LDX;
    // and before the panels, by the element linearisation (operator
    // table and flux Jacobians) the tiles are formed from
    static constexpr bool FUSE = blocked_fuses_fill(P, words == 1 ? HFR_PREC_FP32 : HFR_PREC_FP64);
    static constexpr size_t OPS_BYTES = (sizeof(RefOps) + 15) / 16 * 16;
    static constexpr size_t FILL_BYTES = OPS_BYTES + sizeof(CondShared<P>);
    static constexpr size_t SMEM0 = ELIM_BYTES > LIFT_BYTES ? ELIM_BYTES : LIFT_BYTES;
    static constexpr size_t SMEM = FUSE && FILL_BYTES > SMEM0 ? FILL_BYTES : SMEM0;
    // fused: the face-point flux Jacobians kept from the linearisation to
    // the lift in LDS past everything else (no round trip through memory)
    static constexpr size_t LINR_BYTES = FUSE ? sizeof(double) * 2 * NF * 16 : 0;
    static constexpr size_t SMEM_ALL = SMEM + LINR_BYTES;
};

template <typename T> struct MTile;
template <> struct MTile<float> {
    typedef float V __attribute__((ext_vector_type(4)));
    __device__ static int row(int g, int r) { return 4 * g + r; }
    // bits of a row tile's 16-bit mask held in register r by some lane
    __device__ static unsigned rbits(int r) { return 0x1111u << r; }
    __device__ static V mfma(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static void load4(const float* p, float (&v)[4]) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    }
    __device__ static void store4(float* p, float a, float b, float c, float d) {
        *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
    }
};
template <> struct MTile<double> {
    typedef double V __attribute__((ext_vector_type(4)));
    __device__ static int row(int g, int r) { return g + 4 * r; }
    __device__ static unsigned rbits(int r) { return 0xfu << (4 * r); }
    __device__ static V mfma(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static void load4(const double* p, double (&v)[4]) {
        const double2 q0 = reinterpret_cast<const double2*>(p)[0];
        const double2 q1 = reinterpret_cast<const double2*>(p)[1];
        v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
    }
    __device__ static void store4(double* p, double a, double b, double c, double d) {
        reinterpret_cast<double2*>(p)[0] = make_double2(a, b);
        reinterpret_cast<double2*>(p)[1] = make_double2(c, d);
    }
};
// a wave-uniform double kept in scalar registers
__device__ __forceinline__ double uniform(double x) {
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x)),
                            __builtin_amdgcn_readfirstlane(__double2loint(x)));
}
// the value of lane l (per lane)
__device__ __forceinline__ float lane_shfl(float v, int l) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(4 * l, __float_as_int(v)));
}
__device__ __forceinline__ double lane_shfl(double v, int l) {
    const int lo = __builtin_amdgcn_ds_bpermute(4 * l, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(4 * l, __double2hiint(v));
    return __hiloint2double(hi, lo);
}
// slot of panel column (or U row) c in the operand order (c mod 4, c div 4)
__device__ __forceinline__ int operand_slot(int c) { return (c & 3) * 4 + (c >> 2); }

template <int P, typename T, int WSEL>
__global__ __launch_bounds__((64 * BlockShape<P, T, WSEL>::W))
__attribute__((amdgpu_waves_per_eu(BlockShape<P, T, WSEL>::WPE))) void k_condense_blocked(
    CondenseLaunch a, RefOps og) {
    using S = BlockShape<P, T, WSEL>;
    using M = MTile<T>;
    using V = typename M::V;
    constexpr int n = S::n, N = S::N, NPAD = S::NPAD, RT = S::RT, NCT = S::NCT;
    constexpr int W = S::W, CTW = S::CTW, RPL = S::RPL, LDP = S::LDP, LDG = S::LDG;
    constexpr int NB = S::NB, MW = S::MW;
    constexpr int NP = P * P;
    __shared__ __align__(16) unsigned char smem[S::SMEM_ALL];
    // -G of the last three panels, U of one tile per wave, the panel in row
    // layout
    T (*gbuf)[NPAD * LDG] = reinterpret_cast<T (*)[NPAD * LDG]>(smem);
    T (*ubuf)[16 * LDG] = reinterpret_cast<T (*)[16 * LDG]>(
        smem + sizeof(T) * size_t(NB) * NPAD * LDG);
    T* pbuf = reinterpret_cast<T*>(smem + sizeof(T) * (size_t(NB) * NPAD * LDG +
                                                       size_t(W) * 16 * LDG));
    __shared__ int pivs[NB][16];
    __shared__ short kinv[NPAD];                      // row -> its unknown
    __shared__ int trf[4];                            // faces on the trace
    __shared__ unsigned pmask[NB][MW];                // pivot rows of the panel
    // per row: 1 + its position among the panel's pivots, 0 if none
    __shared__ __align__(4) unsigned char posb[NB][NPAD];
    __shared__ unsigned char used[NPAD];
    __shared__ double rhol[NPAD];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, i = lane & 15;
    const int k = blockIdx.x;
    // a launch queued ahead of the host's Newton test returns at entry when
    // the device flag says the iterate has converged
    if (a.go && *a.go == 0) return;                    // uniform over the grid
    T* G = reinterpret_cast<T*>(a.M) + size_t(k) * N * N;

    // ---- the element linearisation in LDS (the region the panels take
    // later), then tile (t, c) of [A | pad | B] straight from it: the rows of
    // A and B of the tableau fill, entry for entry, formed in registers
    // (dummy unknowns: identity); the face-point flux Jacobians go to a.lin
    // for the lift at the end
    V acc[CTW][RT];
    if constexpr (S::FUSE) {
    {
        RefOps& os = *reinterpret_cast<RefOps*>(smem);
        copy_ref_ops(os, og);
    }
    __syncthreads();
    const RefOps& os = *reinterpret_cast<const RefOps*>(smem);
    CondShared<P>& sh = *reinterpret_cast<CondShared<P>*>(smem + S::OPS_BYTES);
    element_linearisation<P>(a, os, k, sh);            // ends with a barrier
    {
        double* lin = reinterpret_cast<double*>(smem + S::SMEM);
        for (int e2 = threadIdx.x; e2 < 4 * P * 16; e2 += blockDim.x) {
            lin[e2] = sh.Fu[e2 >> 4][e2 & 15];
            lin[4 * P * 16 + e2] = sh.Fh[e2 >> 4][e2 & 15];
        }
    }
#pragma unroll
    for (int q = 0; q < CTW; ++q) {
        const int c = w + W * q;
        const int ci = 16 * c + i;                     // internal column
        const bool dcol = ci >= n && ci < NPAD;
        // block column and component of the global column (A or B)
        const int bc = ci < n ? ci >> 2 : NP + ((ci - NPAD) >> 2);
        const int cc = (ci < n ? ci : ci - NPAD) & 3;
        if constexpr (sizeof(T) == 4) {
        if (c < RT) {                                  // uniform: columns of A
            // the lane's column point (l, kk) couples to the row points of
            // its row line (j == kk) and column line (i == l) only, so the
            // operand blocks of both (column cc) are the same for every row
            // tile: the terms of block_column with them loaded once
            const bool real = ci < n;
            const int bq = real ? bc : 0;
            const int l = bq % P, kk = bq / P;
            double af[4], ag[4], fr1[4], fl1[4], fb2[4], ft2[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int z = v * 4 + cc;
                af[v] = sh.Af[bq][z];
                ag[v] = sh.Ag[bq][z];
                fr1[v] = sh.Fu[1 * P + kk][z];
                fl1[v] = sh.Fu[3 * P + (P - 1 - kk)][z];
                fb2[v] = sh.Fu[0 * P + l][z];
                ft2[v] = sh.Fu[2 * P + (P - 1 - l)][z];
            }
            const double lpl = os.lp[l], lml = os.lm[l], lpk = os.lp[kk], lmk = os.lm[kk];
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                // rows 4g + r: the four variables of point br = 4t + g
                const int br = 4 * t + g;
                double col[4] = {0.0, 0.0, 0.0, 0.0};
                if (real && br < NP) {
                    const int pi = br % P, pj = br / P;
                    const bool rl = kk == pj, cl = l == pi;
                    if (rl || cl) {
                        const double cij = sh.c[br];
                        double a1 = 0, b1 = 0, c1 = 0, a2 = 0, b2 = 0, c2 = 0;
                        if (rl) {
                            b1 = os.cr[pi] * lpl;
                            c1 = os.cl[pi] * lml;
                            a1 = os.D[pi * P + l] - b1 + c1;
                        }
                        if (cl) {
                            b2 = os.cl[pj] * lmk;
                            c2 = os.cr[pj] * lpk;
                            a2 = os.D[pj * P + kk] + b2 - c2;
                        }
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            double s2 = 0.0;
                            if (rl) s2 += a1 * af[v] + b1 * fr1[v] + c1 * fl1[v];
                            if (cl) s2 += a2 * ag[v] + b2 * fb2[v] + c2 * ft2[v];
                            col[v] = cij * s2;
                        }
                    }
                    if (bc == br) col[cc] += 1.0;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * t + M::row(g, r);
                    T v = T(col[r]);
                    if (row >= n && dcol && row == ci) v = T(1);
                    acc[q][t][r] = v;
                }
            }
            continue;
        }
        if (c < NCT) {                                 // uniform: columns of B
            // the lane's trace column (face f2, point q2): a row point couples
            // to it only on the grid line through q2 normal to face f2, with
            // the lifting weight of its side; face flux Jacobian column cc
            // loaded once, the coupling test and weight by selects (no
            // branches per lane)
            const int tb = bc - NP, f2 = tb / P, q2 = tb - f2 * P;
            const bool tr = sh.tr[f2] != 0;
            double fh[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) fh[v] = sh.Fh[tb][v * 4 + cc];
            const bool right = f2 == 1 || f2 == 2;       // cr (else cl)
            const bool by_i = f2 == 1 || f2 == 3;        // weight of point i (else j)
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int br = 4 * t + g;
                const bool rowok = br < NP;
                const int brc = rowok ? br : 0;
                const int pi = brc % P, pj = brc / P;
                const bool on = tr && rowok &&
                                ((f2 == 1 && q2 == pj) || (f2 == 3 && q2 == P - 1 - pj) ||
                                 (f2 == 0 && q2 == pi) || (f2 == 2 && q2 == P - 1 - pi));
                const int wi = by_i ? pi : pj;
                const double cw = right ? os.cr[wi] : os.cl[wi];
                const double f = on ? sh.c[brc] * cw : 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[q][t][r] = T(f * fh[r]);
            }
            continue;
        }
        }
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            if constexpr (sizeof(T) == 4) {
                // rows 4g + r: the four variables of point 4t + g
                const int br = 4 * t + g;
                double col[4] = {0.0, 0.0, 0.0, 0.0};
                if (c < NCT && !dcol && 16 * t + 4 * g < n) block_column<P>(br, bc, cc, os, sh, col);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * t + M::row(g, r);
                    T v = T(col[r]);
                    if (c < NCT && row >= n && dcol && row == ci) v = T(1);
                    acc[q][t][r] = v;
                }
            } else {
                // rows g + 4r: variable g of point 4t + r
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * t + M::row(g, r);
                    double col[4] = {0.0, 0.0, 0.0, 0.0};
                    if (c < NCT && !dcol && row < n) block_column<P>(row >> 2, bc, cc, os, sh, col);
                    T v = T(col[g]);
                    if (c < NCT && row >= n && dcol && row == ci) v = T(1);
                    acc[q][t][r] = v;
                }
            }
        }
    }
    } else {
    // the rows of A and B as the tableau fill wrote them (column-major)
#pragma unroll
    for (int q = 0; q < CTW; ++q) {
        const int c = w + W * q;
        const int ci = 16 * c + i;                     // internal column
        const bool dcol = ci >= n && ci < NPAD;
        const int gc = ci < n ? ci : n + (ci - NPAD);  // global column (A or B)
#pragma unroll
        for (int t = 0; t < RT; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * t + M::row(g, r);
                T v = T(0);
                if (c < NCT) {
                    if (row < n && !dcol) v = G[size_t(min(gc, N - 1)) * N + row];
                    else if (row >= n && dcol && row == ci) v = T(1);
                }
                acc[q][t][r] = v;
            }
        }
    }
    }
    for (int r = threadIdx.x; r < NPAD; r += blockDim.x) used[r] = 0;
    // right-hand side h (FP64), one value per row, updated by wave 0
    for (int row = threadIdx.x; row < NPAD; row += blockDim.x)
        rhol[row] = row < n ? a.h[size_t(row & 3) * a.nimp * NP + size_t(k) * NP + (row >> 2)]
                            : 0.0;
    __syncthreads();

    auto wave_sync = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // accumulator tiles of one column tile -> LDS rows (the owner's panel)
    auto to_panel = [&](const V (&tile)[RT]) {
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                pbuf[(16 * t + M::row(g, r)) * LDP + i] = tile[t][r];
    };
    // ---- panel factorisation by its owner (panel in pbuf): 16 Jordan
    // exchanges on the panel's columns; -G, pivots, positions and the pivot
    // mask to slot j mod 3
    auto factor = [&](int j) {
        wave_sync();
        T x[RPL][16];
        bool usd[RPL];
        T sig[RPL];
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            const int row = lane + 64 * s;
            usd[s] = row >= NPAD || used[min(row, NPAD - 1)];
            sig[s] = T(1);
#pragma unroll
            for (int cc = 0; cc < 16; ++cc)
                x[s][cc] = row < NPAD ? pbuf[min(row, NPAD - 1) * LDP + cc] : T(0);
        }
        int pos[RPL];
#pragma unroll
        for (int s = 0; s < RPL; ++s) pos[s] = 0;
        int pvv = 0;                                   // lane cc: pivot row of exchange cc
        bool fail = false;
        T ipv = T(0);                                  // lane cc: 1 / pivot of exchange cc
        // The padding columns of the last panel (n .. NPAD-1) are identity
        // columns whose only nonzero is their own padding row, decoupled from
        // the element's rows and columns: the exchange of each pivots on that
        // row with factor 1 and changes nothing else, so its outcome is
        // written here and the loop below skips it.
        constexpr int NR = n - 16 * (RT - 1);          // real columns, last panel
        const bool pad = NR < 16 && j == RT - 1;       // uniform
        if (pad) {
#pragma unroll
            for (int s = 0; s < RPL; ++s) {
                const int row = lane + 64 * s;
                if (row >= n && row < NPAD) {
                    usd[s] = true;
                    pos[s] = row - 16 * j + 1;
                }
#pragma unroll
                for (int cc = NR; cc < 16; ++cc)
                    if (row == 16 * j + cc) x[s][cc] = T(-1);
            }
            if (lane >= NR && lane < 16) {
                pvv = 16 * j + lane;
                ipv = T(1);
            }
        }
        // pivot search of one column: some row is always unused, so the
        // maximum names one; a zero pivot is flagged and its exchange
        // leaves the tableau as it is (the result is discarded)
        auto column_key = [&](int c) {
            unsigned key = 0;
#pragma unroll
            for (int s = 0; s < RPL; ++s) {
                const unsigned ks = pivot_key32z(float(fabs(x[s][c])), lane + 64 * s);
                if (!usd[s] && ks > key) key = ks;
            }
            return wave_max_u32(key);
        };
        unsigned key = column_key(0);
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
            if (cc >= NR && pad) continue;             // uniform: written above
            const int p = 255 - int(key & 0xffu);
            const bool bad = key < 0x200u;
            fail = fail || bad;
            const int sp = p >> 6, lp = p & 63;
            // the pivot row into scalar registers: one read per column from
            // the pivot's slot, chosen by a uniform branch
            T u[16];
#pragma unroll
            for (int s0 = 0; s0 < RPL; ++s0)
                if (sp == s0)
#pragma unroll
                    for (int c2 = 0; c2 < 16; ++c2) u[c2] = lane_value(x[s0][c2], lp);
            T ip;
            if constexpr (sizeof(T) == 4) ip = __builtin_amdgcn_rcpf(u[cc]);
            else ip = T(1) / u[cc];
            ip = bad ? T(0) : ip;
            ipv = lane == cc ? ip : ipv;
            asm volatile("" : "+v"(ipv));              // keep the select here
            pvv = lane == cc ? p : pvv;
            asm volatile("" : "+v"(pvv));
            T gsv[RPL];
            bool me[RPL];
#pragma unroll
            for (int s = 0; s < RPL; ++s) {
                me[s] = lane + 64 * s == p;
                gsv[s] = me[s] ? T(0) : x[s][cc] * ip;
                usd[s] = usd[s] || me[s];
            }
            // the next pivot column first, and its search, ahead of the
            // other columns of this exchange
            if (cc + 1 < 16) {
#pragma unroll
                for (int s = 0; s < RPL; ++s) x[s][cc + 1] = fma(-gsv[s], u[cc + 1], x[s][cc + 1]);
                key = column_key(cc + 1);
            }
#pragma unroll
            for (int c2 = 0; c2 < 16; ++c2) {
                if (c2 == cc || c2 == cc + 1) continue;
#pragma unroll
                for (int s = 0; s < RPL; ++s) x[s][c2] = fma(-gsv[s], u[c2], x[s][c2]);
            }
#pragma unroll
            for (int s = 0; s < RPL; ++s) {
                x[s][cc] = me[s] ? T(-1) : gsv[s];
                pos[s] = me[s] ? cc + 1 : pos[s];
                asm volatile("" : "+v"(pos[s]));
            }
        }
        if (fail && lane == 0) *a.pivot_fail = 1;
        // -G: pivot rows scaled by their factors; the rows of P hold
        // T[P,K]^-1, the others T[:,K] T[P,K]^-1
        const int jb = j % NB;
        T* gb = gbuf[jb];
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            // every lane takes part in the permute: a lane outside the
            // exchange mask would supply 0
            const T ipl = lane_shfl(ipv, max(pos[s] - 1, 0));
            sig[s] = pos[s] ? -ipl : T(1);
        }
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            const int row = lane + 64 * s;
            if (row < NPAD) {
                const T f = -sig[s];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    M::store4(gb + row * LDG + 4 * q, f * x[s][q], f * x[s][4 + q],
                              f * x[s][8 + q], f * x[s][12 + q]);
                if (usd[s]) used[row] = 1;
                posb[jb][row] = (unsigned char)pos[s];
            }
            const unsigned long long bm = __ballot(pos[s] != 0);
            if (lane == 0) {
                if (2 * s < MW) pmask[jb][2 * s] = unsigned(bm);
                if (2 * s + 1 < MW) pmask[jb][2 * s + 1] = unsigned(bm >> 32);
            }
        }
        if (lane < 16) {
            pivs[jb][lane] = pvv;
            const int col = 16 * j + lane;
            if (col < n) {
                a.piv[size_t(k) * n + col] = pvv;
                kinv[pvv] = short(col);
            }
        }
    };

    // one tile and panel slot b: the tile's pivot rows to LDS (U) and
    // cleared, then tile += (-G) U
    auto update_tile = [&](int b, V (&tile)[RT]) {
        T* ub = ubuf[w];
        unsigned pm[MW];
#pragma unroll
        for (int q = 0; q < MW; ++q) pm[q] = __builtin_amdgcn_readfirstlane(pmask[b][q]);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const unsigned msk = (pm[(16 * t) >> 5] >> ((16 * t) & 31)) & 0xffffu;
            if (msk == 0) continue;                    // uniform
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if ((msk & M::rbits(r)) == 0) continue;  // uniform
                const int rl = M::row(g, r);
                if ((msk >> rl) & 1u) {
                    const int u = posb[b][16 * t + rl] - 1;
                    ub[i * LDG + operand_slot(u)] = tile[t][r];
                    tile[t][r] = T(0);
                }
            }
        }
        wave_sync();
        T bop[4];
        M::load4(ub + i * LDG + 4 * g, bop);
        const T* gb = gbuf[b];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            T aop[4];
            M::load4(gb + (16 * t + i) * LDG + 4 * g, aop);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) tile[t] = M::mfma(aop[kk], bop[kk], tile[t]);
        }
        wave_sync();                                   // ub free for the next tile
    };

    // Period j: panel j is published (none in period -1); the owner of
    // panel j + 1 brings that panel's tile up to date and factors it.  One
    // inlined copy of the factorisation and one tile update per register
    // tile keep the code small enough for the instruction cache, which the
    // elements resident on a CU share at different points of the kernel.
    for (int j = -1; j < RT; ++j) {
        if (j >= 0) __syncthreads();                   // panel j published
        const int b = (j + NB) % NB;
        const int j1 = j + 1;
        const bool ahead = j1 < RT && w == j1 % W;     // uniform
        const bool late = j > 0 && w == j % W;         // deferred panel j - 1
#pragma unroll
        for (int q = 0; q < CTW; ++q) {
            const int c = w + W * q;
            // panels this tile takes now (e = 0: j - 1, e = 1: j): the
            // owner of panel j + 1 updates only that panel's tile and
            // leaves panel j to the next period for its other tiles
            int e0 = 2;
            if (j >= 0 && c > j && c < NCT) e0 = ahead ? (c == j1 ? 1 : 2) : (late ? 0 : 1);
#pragma unroll 1
            for (int e = e0; e < 2; ++e) update_tile(e == 0 ? (j + NB - 1) % NB : b, acc[q]);
            if (ahead && c == j1) to_panel(acc[q]);
        }
        if (ahead) factor(j1);
        if (j < 0) continue;
        if (w == 0) {                                  // right-hand side
            double rp[16];
#pragma unroll
            for (int cc = 0; cc < 16; ++cc) rp[cc] = uniform(rhol[pivs[b][cc]]);
            wave_sync();
            const T* gb = gbuf[b];
#pragma unroll
            for (int s = 0; s < RPL; ++s) {
                const int row = lane + 64 * s;
                if (row < NPAD) {
                    double v = posb[b][row] ? 0.0 : rhol[row];
#pragma unroll
                    for (int cc = 0; cc < 16; ++cc)
                        v = fma(double(gb[row * LDG + operand_slot(cc)]), rp[cc], v);
                    rhol[row] = v;
                }
            }
        }
    }

    // ---- store: rows of A in the columns of B (-A^-1 B at row p_k), and
    // A^-1 h at the same rows
#pragma unroll
    for (int q = 0; q < CTW; ++q) {
        const int c = w + W * q;
        if (c < RT || c >= NCT) continue;              // uniform
        const int col = n + 16 * (c - RT) + i;
        T* xc = a.compact_schur ? G + schur_x_offset(4 * P) + size_t(col - n) * n
                                : G + size_t(col) * N;
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * t + M::row(g, r);
                if (row < n) xc[row] = acc[q][t][r];
            }
    }
    __syncthreads();
    for (int row = threadIdx.x; row < n; row += blockDim.x) a.yr[size_t(k) * n + row] = rhol[row];

    // ---- the Schur lift (k_schur_lift, in place of its launch): X and
    // A^-1 r in unknown order and the face-point flux Jacobians to the LDS
    // the elimination has finished with, then L = D + C X and z = C A^-1 r
    constexpr int NF = S::NF, LDX = S::LDX, m = S::m;
    // fused: the flux Jacobians are in LDS already (past the regions the
    // elimination and the lift use); else from the fill's copy in memory
    double* fu = S::FUSE ? reinterpret_cast<double*>(smem + S::SMEM)
                         : reinterpret_cast<double*>(smem);
    double* fh = fu + NF * 16;
    double* ys = S::FUSE ? reinterpret_cast<double*>(smem) : fh + NF * 16;
    T* xs = reinterpret_cast<T*>(ys + n);
    {
        if constexpr (!S::FUSE) {
            const double* lin = a.lin + size_t(k) * 2 * NF * 16;
            for (int e = threadIdx.x; e < NF * 16; e += blockDim.x) {
                fu[e] = lin[e];
                fh[e] = lin[NF * 16 + e];
            }
        }
        if (threadIdx.x < 4)
            trf[threadIdx.x] = a.finfo[size_t(a.imp_list[k]) * 4 + threadIdx.x].role == ROLE_HFR;
        for (int row = threadIdx.x; row < n; row += blockDim.x) ys[kinv[row]] = rhol[row];
#pragma unroll
        for (int q = 0; q < CTW; ++q) {
            const int c = w + W * q;
            if (c < RT || c >= NCT) continue;          // uniform
            const int b = 16 * (c - RT) + i;
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * t + M::row(g, r);
                    if (row < n) xs[b * LDX + kinv[row]] = acc[q][t][r];
                }
        }
    }
    __syncthreads();
    // each thread one face point fq and the columns b = b0, b0 + GF, ... (b
    // == m: the z column): the face point's flux Jacobian, line points and
    // interpolation weights stay in registers, the four rows of a line point
    // in a column come in one 16-byte (FP32) read, and the four rows of the
    // face point go out in one store
    constexpr int GF = 64 * W / NF;                  // threads per face point
    if (threadIdx.x < GF * NF) {
        const int fq = threadIdx.x % NF, b0 = threadIdx.x / NF;
        const int f = fq / P, q = fq - f * P;
        const bool tr = trf[f] != 0;
        const double wq = og.w[q];
        int pt[P];
        double cl[P];
#pragma unroll
        for (int l = 0; l < P; ++l) {
            if (f == 0) { pt[l] = l * P + q; cl[l] = og.lm[l]; }
            else if (f == 1) { pt[l] = q * P + l; cl[l] = og.lp[l]; }
            else if (f == 2) { pt[l] = l * P + (P - 1 - q); cl[l] = og.lp[l]; }
            else { pt[l] = (P - 1 - q) * P + l; cl[l] = og.lm[l]; }
        }
        double fr[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) fr[e] = fu[fq * 16 + e];
    for (int b = b0; b <= m; b += GF) {
        double out[4];
        if (!tr) {
#pragma unroll
            for (int v = 0; v < 4; ++v) out[v] = (b == fq * 4 + v) ? 1.0 : 0.0;
        } else {
            double sw[4] = {0.0, 0.0, 0.0, 0.0};
            if (b < m) {
#pragma unroll
                for (int l = 0; l < P; ++l) {
                    T xv[4];
                    M::load4(xs + b * LDX + pt[l] * 4, xv);
#pragma unroll
                    for (int v = 0; v < 4; ++v) sw[v] += cl[l] * double(xv[v]);
                }
            } else {
#pragma unroll
                for (int l = 0; l < P; ++l)
#pragma unroll
                    for (int v = 0; v < 4; ++v) sw[v] += cl[l] * ys[pt[l] * 4 + v];
            }
            const bool diag = (b >> 2) == fq;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double acc2 = diag ? fh[fq * 16 + v * 4 + (b & 3)] : 0.0;
#pragma unroll
                for (int w2 = 0; w2 < 4; ++w2) acc2 += fr[v * 4 + w2] * sw[w2];
                out[v] = wq * acc2;
            }
        }
        if (b < m) {
            T* dst = a.compact_schur
                         ? G + schur_offset(4 * P, f, b / (4 * P), 4 * q, b % (4 * P))
                         : G + size_t(n + b) * N + n + fq * 4;
            if constexpr (sizeof(T) == 4) {
                *reinterpret_cast<float4*>(dst) = make_float4(float(out[0]), float(out[1]),
                                                              float(out[2]), float(out[3]));
            } else {
                reinterpret_cast<double2*>(dst)[0] = make_double2(out[0], out[1]);
                reinterpret_cast<double2*>(dst)[1] = make_double2(out[2], out[3]);
            }
        } else {
            double* zz = a.z + size_t(k) * m + fq * 4;
#pragma unroll
            for (int v = 0; v < 4; ++v) zz[v] = tr ? out[v] : 0.0;
        }
    }
    }
}

template <int P, typename T>
static hipError_t launch_sweep(const RefOps& o, const CondenseLaunch& a,
                               hipStream_t st) {
    if (a.schur_only && a.yr) {
        // the blocked kernels end with the Schur lift themselves
        if (a.blocked == 2) {
            hipLaunchKernelGGL((k_condense_blocked<P, T, 8>), dim3(a.nimp),
                               dim3(64 * BlockShape<P, T, 8>::W), 0, st, a, o);
        } else if (a.blocked) {
            hipLaunchKernelGGL((k_condense_blocked<P, T, 0>), dim3(a.nimp),
                               dim3(64 * BlockShape<P, T, 0>::W), 0, st, a, o);
        } else {
            hipLaunchKernelGGL((k_condense_sweep<P, T, true>), dim3(a.nimp),
                               dim3(64 * SweepShape<P, T, true>::W), 0, st, a, o);
            hipLaunchKernelGGL((k_schur_lift<P, T>), dim3(a.nimp), dim3(256), 0, st, a, o);
        }
    } else {
        hipLaunchKernelGGL((k_condense_sweep<P, T, false>), dim3(a.nimp),
                           dim3(64 * SweepShape<P, T, false>::W), 0, st, a, o);
    }
    return hipGetLastError();
}

// FP64 right-hand side from the swept tableau (FP64 or FP32 entries): with
// r = -h and r'_j = r[p_j],
//      y~ = T[0:n][0:n] r'  (A^-1 r in pivot-row order: y~[p_k] = (A^-1 r)[k])
//      z  = T[n:N][0:n] r'  (C A^-1 r)
// accumulated in FP64.  The element shares of g are large and cancel
// between the two sides of a trace face, so they never pass through the
// factor precision; only C A^-1 r does, which is proportional to the
// (small) residual h.  One wave per element, four per workgroup.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_rhs64(int nimp, const T* M,
                                               const int* piv, const double* h,
                                               double* yr, double* z) {
    constexpr int NP = P * P, n = 4 * NP, m = 16 * P, N = n + m;
    __shared__ double sr[4][n];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int k = blockIdx.x * 4 + wv;
    if (k >= nimp) return;
    const int* pk = piv + size_t(k) * n;
    for (int j = lane; j < n; j += 64) {
        const int row = pk[j];
        sr[wv][j] = -h[size_t(row & 3) * nimp * NP + size_t(k) * NP + (row >> 2)];
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const T* Mk = M + size_t(k) * N * N;
    for (int row = lane; row < N; row += 64) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += double(Mk[size_t(j) * N + row]) * sr[wv][j];
        if (row < n) yr[size_t(k) * n + row] = acc;
        else z[size_t(k) * m + row - n] = acc;
    }
}

template <typename T>
static hipError_t launch_rhs64_t(int P, int nimp, const T* M, const int* piv,
                                 const double* h, double* yr, double* z,
                                 hipStream_t st) {
    const dim3 grid((nimp + 3) / 4), blk(256);
    switch (P) {
        case 2: hipLaunchKernelGGL((k_rhs64<T, 2>), grid, blk, 0, st, nimp, M, piv, h, yr, z); break;
        case 3: hipLaunchKernelGGL((k_rhs64<T, 3>), grid, blk, 0, st, nimp, M, piv, h, yr, z); break;
        case 4: hipLaunchKernelGGL((k_rhs64<T, 4>), grid, blk, 0, st, nimp, M, piv, h, yr, z); break;
        case 5: hipLaunchKernelGGL((k_rhs64<T, 5>), grid, blk, 0, st, nimp, M, piv, h, yr, z); break;
        case 6: hipLaunchKernelGGL((k_rhs64<T, 6>), grid, blk, 0, st, nimp, M, piv, h, yr, z); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rhs64(int P, int nimp, const void* M, int precision,
                        const int* piv, const double* h, double* yr,
                        double* z, hipStream_t st) {
    if (nimp == 0) return hipSuccess;
    if (precision == HFR_PREC_FP64)
        return launch_rhs64_t(P, nimp, reinterpret_cast<const double*>(M), piv, h, yr, z, st);
    return launch_rhs64_t(P, nimp, reinterpret_cast<const float*>(M), piv, h, yr, z, st);
}

template <int P>
static hipError_t launch_condense_p(const RefOps& o, const CondenseLaunch& a,
                                    hipStream_t st) {
    if (a.nimp == 0) return hipSuccess;
    if (a.precision == HFR_PREC_FP64) return launch_sweep<P, double>(o, a, st);
    return launch_sweep<P, float>(o, a, st);
}

template <int P>
static hipError_t launch_fill_p(const RefOps& o, const CondenseLaunch& a,
                                hipStream_t st) {
    if (a.nimp == 0) return hipSuccess;
    const bool ab = a.schur_only != 0;
    if (a.precision == HFR_PREC_FP64) {
        if (ab) hipLaunchKernelGGL((k_tableau_fill<P, double, true>), dim3(a.nimp), dim3(256), 0, st, a, o);
        else hipLaunchKernelGGL((k_tableau_fill<P, double, false>), dim3(a.nimp), dim3(256), 0, st, a, o);
    } else {
        if (ab) hipLaunchKernelGGL((k_tableau_fill<P, float, true>), dim3(a.nimp), dim3(256), 0, st, a, o);
        else hipLaunchKernelGGL((k_tableau_fill<P, float, false>), dim3(a.nimp), dim3(256), 0, st, a, o);
    }
    return hipGetLastError();
}

hipError_t launch_tableau_fill(const RefOps& o, const CondenseLaunch& a,
                               hipStream_t st) {
    switch (o.P) {
        case 2: return launch_fill_p<2>(o, a, st);
        case 3: return launch_fill_p<3>(o, a, st);
        case 4: return launch_fill_p<4>(o, a, st);
        case 5: return launch_fill_p<5>(o, a, st);
        case 6: return launch_fill_p<6>(o, a, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_condense(const RefOps& o, const CondenseLaunch& a,
                           hipStream_t st) {
    switch (o.P) {
        case 2: return launch_condense_p<2>(o, a, st);
        case 3: return launch_condense_p<3>(o, a, st);
        case 4: return launch_condense_p<4>(o, a, st);
        case 5: return launch_condense_p<5>(o, a, st);
        case 6: return launch_condense_p<6>(o, a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hfr
