// Element blocks and static condensation (Section 3.2).
//
// For implicit element k with n = 4 Np element unknowns and m = 16 P trace
// unknowns (all four faces; a face off the trace gets an identity row and
// zero coupling), the augmented matrix
//      [ A  B  r ]        r = -h,  s = -g^(k)
//      [ C  D  s ]
// is built from analytic flux Jacobians (the exact derivatives of h and of
// the element's share of g), then LU elimination of the first n columns
// with partial pivoting inside the A rows turns it into
//      [ L\U    L^-1 P B     L^-1 P r   ]
//      [ C U^-1  D - C A^-1 B  s - C A^-1 r ] = [ .  L^k  t^k ]
// which holds the recovery factors of eq:localproblems (back substitution
// with U) and the element Schur complement of eq:assembly in place.  The
// right-hand side used by Newton is recomputed in FP64 by k_rhs64 from the
// stored factors (the r, s columns here are not used downstream).
//
// Element-local ordering: u index = point*4 + var (point j*P+i), trace
// index = (face*P + q)*4 + var with q counter-clockwise along the element.
#include "euler.h"
#include "internal.h"

namespace hfr {

template <int P>
struct CondShared {
    static constexpr int NP = P * P;
    double Af[NP][16];
    double Ag[NP][16];
    double c[NP];
    double u[NP][4];
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
    const double gam = a.phys.gamma;
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
        for (int v = 0; v < 4; ++v) {
            uu[v] = a.u[v * plane + size_t(e) * NP + t];
            sh.u[t][v] = uu[v];
        }
        Prim q = prim(uu, gam);
        dflux_n(uu, q, y_et, -x_et, gam, sh.Af[t]);
        dflux_n(uu, q, -y_xi, x_xi, gam, sh.Ag[t]);
        sh.c[t] = a.aii_dt / J;
    }
    if (t < 4) sh.tr[t] = (a.finfo[size_t(e) * 4 + t].role == ROLE_HFR);
    __syncthreads();
    if (t < 4 * P) {
        const int f = t / P, q = t % P;
        double uf[4] = {0, 0, 0, 0};
        for (int l = 0; l < P; ++l) {
            int p2;
            double wgt;
            if (f == 0) { p2 = l * P + q; wgt = o.lm[l]; }
            else if (f == 1) { p2 = q * P + l; wgt = o.lp[l]; }
            else if (f == 2) { p2 = l * P + (P - 1 - q); wgt = o.lp[l]; }
            else { p2 = (P - 1 - q) * P + l; wgt = o.lm[l]; }
            for (int v = 0; v < 4; ++v) uf[v] += wgt * sh.u[p2][v];
        }
        const FaceInfo fi = a.finfo[size_t(e) * 4 + f];
        const double2 S = a.fS[size_t(e) * 4 + f];
        double* Fu = sh.Fu[t];
        double* Fh = sh.Fh[t];
        for (int z = 0; z < 16; ++z) Fh[z] = 0.0;
        if (fi.role == ROLE_HFR) {
            const int tf = fi.trace >> 1, side = fi.trace & 1;
            const int tp = tf * P + (side ? P - 1 - q : q);
            double uh[4];
            for (int v = 0; v < 4; ++v) uh[v] = a.uhat[size_t(tp) * 4 + v];
            double su;
            dhfr_flux(uf, uh, S.x, S.y, gam, &su, Fh);
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
                drusanov(uf, outer, S.x, S.y, gam, Fu, Jb);
            } else {
                ghost_state(uf, nx, ny, fi.role, a.phys.uinf, outer);
                drusanov(uf, outer, S.x, S.y, gam, Fu, Jb);
                if (fi.role == ROLE_WALL) {
                    // d ghost / d u: identity except momentum rows I - 2 n n^T
                    double R[16] = {1, 0, 0, 0, 0, 1 - 2 * nx * nx, -2 * nx * ny, 0,
                                    0, -2 * nx * ny, 1 - 2 * ny * ny, 0, 0, 0, 0, 1};
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
    __syncthreads();
}

// value of entry (r, c) of the augmented matrix
template <int P>
__device__ __forceinline__ double aug_entry(int r, int c, int k,
                                            const CondenseLaunch& a,
                                            const RefOps& o,
                                            const CondShared<P>& sh) {
    constexpr int NP = P * P;
    constexpr int n = 4 * NP, m = 16 * P;
    if (r < n) {
        const int pr = r >> 2, v = r & 3;
        const int i = pr % P, j = pr / P;
        const double cij = sh.c[pr];
        if (c < n) {
            const int pc = c >> 2, w = c & 3;
            const int l = pc % P, kk = pc / P;
            double acc = 0.0;
            if (kk == j) {
                const double af = sh.Af[pc][v * 4 + w];
                acc += o.D[i * P + l] * af;
                acc += o.cr[i] * o.lp[l] * (sh.Fu[1 * P + j][v * 4 + w] - af);
                acc += o.cl[i] * o.lm[l] * (sh.Fu[3 * P + (P - 1 - j)][v * 4 + w] + af);
            }
            if (l == i) {
                const double ag = sh.Ag[pc][v * 4 + w];
                acc += o.D[j * P + kk] * ag;
                acc += o.cl[j] * o.lm[kk] * (sh.Fu[0 * P + i][v * 4 + w] + ag);
                acc += o.cr[j] * o.lp[kk] * (sh.Fu[2 * P + (P - 1 - i)][v * 4 + w] - ag);
            }
            return (r == c ? 1.0 : 0.0) + cij * acc;
        } else if (c < n + m) {
            const int b = c - n;
            const int f = b / (4 * P), q = (b >> 2) % P, w = b & 3;
            if (!sh.tr[f]) return 0.0;
            double coef;
            if (f == 1 && q == j) coef = o.cr[i];
            else if (f == 3 && q == P - 1 - j) coef = o.cl[i];
            else if (f == 0 && q == i) coef = o.cl[j];
            else if (f == 2 && q == P - 1 - i) coef = o.cr[j];
            else return 0.0;
            return cij * coef * sh.Fh[f * P + q][v * 4 + w];
        } else {
            return -a.h[size_t(v) * a.nimp * NP + size_t(k) * NP + pr];
        }
    } else {
        const int b = r - n;
        const int f = b / (4 * P), q = (b >> 2) % P, v = b & 3;
        if (!sh.tr[f]) {
            if (c >= n && c < n + m) return (c - n == b) ? 1.0 : 0.0;
            return 0.0;
        }
        const double wq = o.w[q];
        if (c < n) {
            const int pc = c >> 2, w = c & 3;
            const int l = pc % P, kk = pc / P;
            double coef = 0.0;
            if (f == 1) { if (kk == q) coef = o.lp[l]; }
            else if (f == 3) { if (kk == P - 1 - q) coef = o.lm[l]; }
            else if (f == 0) { if (l == q) coef = o.lm[kk]; }
            else { if (l == P - 1 - q) coef = o.lp[kk]; }
            return wq * coef * sh.Fu[f * P + q][v * 4 + w];
        } else if (c < n + m) {
            const int b2 = c - n;
            if ((b2 >> 2) != (b >> 2)) return 0.0;
            return wq * sh.Fh[f * P + q][v * 4 + (b2 & 3)];
        } else {
            return -a.gk[((size_t(k) * 4 + f) * P + q) * 4 + v];
        }
    }
}

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaVec;
template <> struct MfmaVec<float> { typedef floatx4 type; };
template <> struct MfmaVec<double> { typedef doublex4 type; };

// D(16x16) += A(16x4) B(4x16); lane l supplies A[l%16][l/16] and
// B[l/16][l%16].  Element r of lane l holds D[i][l%16] with
// i = 4*(l/16) + r for the FP32 instruction and i = l/16 + 4*r for the
// FP64 one (measured on gfx950).
__device__ __forceinline__ floatx4 mfma16(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma16(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename T> __device__ __forceinline__ int mfma_row(int lk, int q);
template <> __device__ __forceinline__ int mfma_row<float>(int lk, int q) { return 4 * lk + q; }
template <> __device__ __forceinline__ int mfma_row<double>(int lk, int q) { return lk + 4 * q; }

constexpr int kPanel = 16;

// Right-looking LU of the first n columns of the rows x ld matrix M
// (row-major, leading dimension ld) with partial pivoting restricted to the
// first n rows; rows n.. are eliminated but never chosen as pivots.  After
// the call: rows 0..n-1 hold L\U and L^-1 P [B r]; rows n.. hold C U^-1 and
// the Schur complement [D - C A^-1 B | s - C A^-1 r].  Panel of 16 columns:
// unblocked factorisation of the panel, forward substitution for the pivot
// rows' trailing part, then a rank-16 trailing update on MFMA tiles.
template <typename T>
__device__ bool lu_condense(T* M, int n, int rows, int ld, int* s_piv,
                            T* s_val, int* piv_out) {
    typedef typename MfmaVec<T>::type vec4;
    const int t = threadIdx.x, nt = blockDim.x;
    const int lane = t & 63, wave = t >> 6, nwaves = nt >> 6;
    for (int k0 = 0; k0 < n; k0 += kPanel) {
        const int k1 = min(n, k0 + kPanel);
        // ---- panel factorisation -----------------------------------------
        for (int kk = k0; kk < k1; ++kk) {
            if (wave == 0) {
                T best = T(-1);
                int bi = kk;
                for (int r = kk + lane; r < n; r += 64) {
                    const T v = fabs(M[size_t(r) * ld + kk]);
                    if (v > best) { best = v; bi = r; }
                }
                for (int off = 32; off > 0; off >>= 1) {
                    const T ob = __shfl_xor(best, off, 64);
                    const int oi = __shfl_xor(bi, off, 64);
                    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
                }
                if (lane == 0) { *s_piv = bi; *s_val = best; }
            }
            __syncthreads();
            const int piv = *s_piv;
            if (!(*s_val > T(0))) return false;
            if (t == 0) piv_out[kk] = piv;
            if (piv != kk) {
                for (int c = t; c < ld; c += nt) {
                    const T x = M[size_t(kk) * ld + c];
                    M[size_t(kk) * ld + c] = M[size_t(piv) * ld + c];
                    M[size_t(piv) * ld + c] = x;
                }
                __syncthreads();
            }
            const T inv = T(1) / M[size_t(kk) * ld + kk];
            for (int r = kk + 1 + t; r < rows; r += nt) M[size_t(r) * ld + kk] *= inv;
            __syncthreads();
            const int w = k1 - kk - 1;
            if (w > 0) {
                const int tot = (rows - kk - 1) * w;
                for (int idx = t; idx < tot; idx += nt) {
                    const int r = kk + 1 + idx / w, c = kk + 1 + idx % w;
                    M[size_t(r) * ld + c] -= M[size_t(r) * ld + kk] * M[size_t(kk) * ld + c];
                }
                __syncthreads();
            }
        }
        if (k1 >= ld) break;
        // ---- U12 = L11^-1 A12 (pivot rows, trailing columns) ---------------
        for (int c = k1 + t; c < ld; c += nt) {
            for (int i = k0 + 1; i < k1; ++i) {
                T acc = M[size_t(i) * ld + c];
                for (int j = k0; j < i; ++j) acc -= M[size_t(i) * ld + j] * M[size_t(j) * ld + c];
                M[size_t(i) * ld + c] = acc;
            }
        }
        __syncthreads();
        // ---- A22 -= L21 U12 on 16x16 MFMA tiles ------------------------------
        const int R0 = k1, C0 = k1;
        const int TR = (rows - R0 + 15) / 16, TC = (ld - C0 + 15) / 16;
        const int kw = k1 - k0;             // multiple of 4
        const int li = lane & 15, lk = lane >> 4;
        for (int tile = wave; tile < TR * TC; tile += nwaves) {
            const int tr = tile % TR, tc = tile / TR;
            const int r0 = R0 + 16 * tr, c0 = C0 + 16 * tc;
            vec4 acc;
            const int cc = c0 + li;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rr = r0 + mfma_row<T>(lk, q);
                acc[q] = (rr < rows && cc < ld) ? M[size_t(rr) * ld + cc] : T(0);
            }
            for (int kq = 0; kq < kw; kq += 4) {
                const int ra = r0 + li;
                const T av = (ra < rows) ? -M[size_t(ra) * ld + k0 + kq + lk] : T(0);
                const T bv = (cc < ld) ? M[size_t(k0 + kq + lk) * ld + cc] : T(0);
                acc = mfma16(av, bv, acc);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rr = r0 + mfma_row<T>(lk, q);
                if (rr < rows && cc < ld) M[size_t(rr) * ld + cc] = acc[q];
            }
        }
        __syncthreads();
    }
    return true;
}

// One workgroup per implicit element.  kLDS: the augmented matrix is built
// and factored in LDS and copied out once; otherwise it stays in the
// solver workspace.
template <int P, typename T, bool kLDS>
__global__ __launch_bounds__(256) void k_condense_lu(CondenseLaunch a, RefOps o) {
    constexpr int NP = P * P;
    constexpr int n = 4 * NP, m = 16 * P, rows = n + m, ld = n + m + 1;
    __shared__ CondShared<P> sh;
    __shared__ int s_piv;
    __shared__ T s_val;
    extern __shared__ double dyn_lds[];
    const int k = blockIdx.x;
    const int t = threadIdx.x;
    element_linearisation<P>(a, o, k, sh);
    T* G = reinterpret_cast<T*>(a.M) + size_t(k) * rows * ld;
    T* M = kLDS ? reinterpret_cast<T*>(dyn_lds) : G;
    for (int idx = t; idx < rows * ld; idx += blockDim.x) {
        const int r = idx / ld, c = idx % ld;
        const double val = aug_entry<P>(r, c, k, a, o, sh);
        M[idx] = T(val);
        if (a.blocks_copy && c < rows)
            a.blocks_copy[size_t(k) * rows * rows + size_t(r) * rows + c] = val;
    }
    __syncthreads();
    const bool ok = lu_condense<T>(M, n, rows, ld, &s_piv, &s_val,
                                   a.piv + size_t(k) * n);
    if (!ok) {
        if (t == 0) *a.pivot_fail = 1;
        return;
    }
    if (kLDS) {
        for (int idx = t; idx < rows * ld; idx += blockDim.x) G[idx] = M[idx];
    }
}

template <int P, typename T>
static hipError_t launch_lu(const RefOps& o, const CondenseLaunch& a,
                            hipStream_t st) {
    constexpr int NP = P * P;
    constexpr int n = 4 * NP, m = 16 * P, rows = n + m, ld = n + m + 1;
    constexpr size_t bytes = size_t(rows) * ld * sizeof(T);
    constexpr size_t kMaxDyn = 160 * 1024 - sizeof(CondShared<P>) - 256;
    if (bytes <= kMaxDyn) {
        static bool attr = false;
        if (!attr) {
            hipError_t e = hipFuncSetAttribute(
                reinterpret_cast<const void*>(&k_condense_lu<P, T, true>),
                hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
            if (e != hipSuccess) return e;
            attr = true;
        }
        hipLaunchKernelGGL((k_condense_lu<P, T, true>), dim3(a.nimp), dim3(256),
                           bytes, st, a, o);
    } else {
        hipLaunchKernelGGL((k_condense_lu<P, T, false>), dim3(a.nimp), dim3(256),
                           0, st, a, o);
    }
    return hipGetLastError();
}

// FP64 right-hand side with the stored factors (FP64 or FP32): the
// element shares of g are large and cancel between the two sides of a
// trace face, so they never pass through the factor precision; only
// C A^-1 r does, which is proportional to the (small) residual h.
// one wave per element; row i of the element lives in lane i % 64, slot
// i / 64 (NS slots); cross-lane values move by readlane-style shuffles
template <int NS>
__device__ __forceinline__ double slot_get(const double (&y)[NS], int s) {
    double r = y[0];
#pragma unroll
    for (int i = 1; i < NS; ++i) r = (s == i) ? y[i] : r;
    return r;
}

template <typename T, int P>
__global__ __launch_bounds__(256) void k_rhs64(int nimp, const T* M,
                                               const int* piv, const double* h,
                                               double* yr, double* z) {
    constexpr int NP = P * P, n = 4 * NP, m = 16 * P, ld = n + m + 1;
    constexpr int NS = (n + 63) / 64;
    __shared__ double sy[4][n];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int k = blockIdx.x * 4 + wv;
    if (k >= nimp) return;
    const T* Mk = M + size_t(k) * (n + m) * ld;
    double y[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int row = lane + 64 * s;
        y[s] = row < n ? -h[size_t(row & 3) * nimp * NP + size_t(k) * NP + (row >> 2)] : 0.0;
    }
    // row interchanges of the factorisation, in order
    const int* pk = piv + size_t(k) * n;
    for (int kk = 0; kk < n; ++kk) {
        const int p = pk[kk];
        if (p == kk) continue;
        const double a = __shfl(slot_get<NS>(y, kk >> 6), kk & 63, 64);
        const double b = __shfl(slot_get<NS>(y, p >> 6), p & 63, 64);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int row = lane + 64 * s;
            if (row == kk) y[s] = b;
            if (row == p) y[s] = a;
        }
    }
    // forward substitution with the unit lower factor
    for (int j = 0; j < n - 1; ++j) {
        const double yj = __shfl(slot_get<NS>(y, j >> 6), j & 63, 64);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int row = lane + 64 * s;
            if (row > j && row < n) y[s] -= double(Mk[size_t(row) * ld + j]) * yj;
        }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int row = lane + 64 * s;
        if (row < n) {
            yr[size_t(k) * n + row] = y[s];
            sy[wv][row] = y[s];
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int b = lane; b < m; b += 64) {
        const T* cr = Mk + size_t(n + b) * ld;
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += double(cr[j]) * sy[wv][j];
        z[size_t(k) * m + b] = acc;
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
    if (a.precision == HFR_PREC_FP64) return launch_lu<P, double>(o, a, st);
    return launch_lu<P, float>(o, a, st);
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
