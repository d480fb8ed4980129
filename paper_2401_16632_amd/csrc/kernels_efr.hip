// Interior-embedded trace (Section 2.3: the continuous trace of the EFR
// choice after eq:hfrspaces).  The element kernels are shared with HFR:
// they evaluate the trace at the Gauss flux points by the GLL-to-Gauss
// interpolation Q of every face, so the element blocks of the nodal trace
// are B Q, Q^T C and Q^T D Q, and the element Schur complement and
// right-hand side are Q^T L^k Q and Q^T z^k of the flux-point ones.  This
// file holds the kernels that differ: the nodal transmission residual, the
// in-place Q^T L Q of every element, the node-block assembly and the
// initial nodal trace.
//
// Slot numbering: slot (imp*4 + lf)*P + i is GLL node i, in the element's
// counter-clockwise order, of local face lf of implicit element imp.
#include "internal.h"

namespace hfr {

namespace {
constexpr int kThreads = 256;
int blocks_for(long work) { return int((work + kThreads - 1) / kThreads); }
}  // namespace

// g[node][v] = sum over slots of the node of sum_q phi_i(x_q) gk[imp][lf][q][v]
__global__ void k_efr_gather_g(RefOps og, int nnodes, const int* inc_ptr,
                               const int* inc, const double* gk, double* g) {
    __shared__ double gi[kMaxP * kMaxP];
    for (int t = threadIdx.x; t < kMaxP * kMaxP; t += blockDim.x) gi[t] = og.gi[t];
    __syncthreads();
    const int P = og.P;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nnodes * 4) return;
    const int nd = idx >> 2, v = idx & 3;
    double acc = 0.0;
    for (int c = inc_ptr[nd]; c < inc_ptr[nd + 1]; ++c) {
        const int s = inc[c];
        const int kf = s / P, i = s - kf * P;
        const double* gq = gk + size_t(kf) * P * 4 + v;
        for (int q = 0; q < P; ++q) acc += gi[q * P + i] * gq[q * 4];
    }
    g[idx] = acc;
}

hipError_t launch_efr_gather_g(const RefOps& ops, int nnodes, const int* inc_ptr,
                               const int* inc, const double* gk, double* g,
                               hipStream_t st) {
    if (nnodes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_efr_gather_g, dim3(blocks_for(4L * nnodes)), dim3(kThreads),
                       0, st, ops, nnodes, inc_ptr, inc, gk, g);
    return hipGetLastError();
}

__device__ __forceinline__ void load4_aligned(const float* p, float (&q)[4]) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    q[0] = x.x; q[1] = x.y; q[2] = x.z; q[3] = x.w;
}
__device__ __forceinline__ void load4_aligned(const double* p, double (&q)[4]) {
    const double2 x = reinterpret_cast<const double2*>(p)[0];
    const double2 y = reinterpret_cast<const double2*>(p)[1];
    q[0] = x.x; q[1] = x.y; q[2] = y.x; q[3] = y.y;
}
__device__ __forceinline__ void store4_aligned(float* p, const float (&q)[4]) {
    *reinterpret_cast<float4*>(p) = make_float4(q[0], q[1], q[2], q[3]);
}
__device__ __forceinline__ void store4_aligned(double* p, const double (&q)[4]) {
    reinterpret_cast<double2*>(p)[0] = make_double2(q[0], q[1]);
    reinterpret_cast<double2*>(p)[1] = make_double2(q[2], q[3]);
}

// In place on the Schur block of element blockIdx.x (rows/columns n..n+m of
// the column-major N x N tableau, N = n + m): first every row's P values of
// a (face, variable) column group become sum_q' L[r][(f,q',w)] phi_i'(x_q'),
// then every column's P values of a (face, variable) row group likewise.
template <typename T>
__global__ void k_efr_transform(RefOps og, int nimp, T* M, int n, int m) {
    __shared__ double gi[kMaxP * kMaxP];
    for (int t = threadIdx.x; t < kMaxP * kMaxP; t += blockDim.x) gi[t] = og.gi[t];
    __syncthreads();
    const int P = og.P, N = n + m;
    const int k = blockIdx.x;
    T* L = M + size_t(k) * N * N + size_t(n) * N + n;   // L[r][c] = L[c*N + r]
    const int groups = m / P;                            // (face, variable) groups
    double x[kMaxP], y[kMaxP];
    // columns: thread per (row, column group)
    for (int t = threadIdx.x; t < m * groups; t += blockDim.x) {
        const int r = t % m, gc = t / m;
        const int f = gc >> 2, w = gc & 3;
        for (int q = 0; q < P; ++q) x[q] = double(L[size_t((f * P + q) * 4 + w) * N + r]);
        for (int i = 0; i < P; ++i) {
            double acc = 0.0;
            for (int q = 0; q < P; ++q) acc += x[q] * gi[q * P + i];
            y[i] = acc;
        }
        for (int i = 0; i < P; ++i) L[size_t((f * P + i) * 4 + w) * N + r] = T(y[i]);
    }
    __syncthreads();
    // rows: thread per (column, row group)
    for (int t = threadIdx.x; t < m * groups; t += blockDim.x) {
        const int gr = t % groups, c = t / groups;
        const int f = gr >> 2, v = gr & 3;
        for (int q = 0; q < P; ++q) x[q] = double(L[size_t(c) * N + (f * P + q) * 4 + v]);
        for (int i = 0; i < P; ++i) {
            double acc = 0.0;
            for (int q = 0; q < P; ++q) acc += gi[q * P + i] * x[q];
            y[i] = acc;
        }
        for (int i = 0; i < P; ++i) L[size_t(c) * N + (f * P + i) * 4 + v] = T(y[i]);
    }
}

// The same two passes on a copy of the Schur block in LDS (row stride
// m + 4): the block is read and written once, as 16-byte pieces.  The order
// is fixed at compile time, so a thread's P values stay in registers.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_efr_transform_lds(RefOps og, int nimp, T* M) {
    constexpr int n = 4 * P * P, m = 16 * P, N = n + m, S = m + 4, m4 = m / 4;
    extern __shared__ __align__(16) unsigned char efr_dyn[];
    T* sL = reinterpret_cast<T*>(efr_dyn);
    __shared__ double gi[P * P];
    for (int t = threadIdx.x; t < P * P; t += blockDim.x) gi[t] = og.gi[t];
    const int k = blockIdx.x;
    T* L = M + size_t(k) * N * N + size_t(n) * N + n;   // L[r][c] = L[c*N + r]
    for (int t = threadIdx.x; t < m * m4; t += blockDim.x) {
        const int c = t / m4, r = (t - c * m4) * 4;
        T q[4];
        load4_aligned(L + size_t(c) * N + r, q);
        store4_aligned(sL + c * S + r, q);
    }
    __syncthreads();
    constexpr int groups = m / P;                        // (face, variable) groups
    double x[P], y[P];
    // columns: thread per (row, column group)
    for (int t = threadIdx.x; t < m * groups; t += blockDim.x) {
        const int r = t % m, gc = t / m;
        const int f = gc >> 2, w = gc & 3;
#pragma unroll
        for (int q = 0; q < P; ++q) x[q] = double(sL[((f * P + q) * 4 + w) * S + r]);
#pragma unroll
        for (int i = 0; i < P; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < P; ++q) acc += x[q] * gi[q * P + i];
            y[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < P; ++i) sL[((f * P + i) * 4 + w) * S + r] = T(y[i]);
    }
    __syncthreads();
    // rows: thread per (column, row group)
    for (int t = threadIdx.x; t < m * groups; t += blockDim.x) {
        const int gr = t % groups, c = t / groups;
        const int f = gr >> 2, v = gr & 3;
#pragma unroll
        for (int q = 0; q < P; ++q) x[q] = double(sL[c * S + (f * P + q) * 4 + v]);
#pragma unroll
        for (int i = 0; i < P; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < P; ++q) acc += gi[q * P + i] * x[q];
            y[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < P; ++i) sL[c * S + (f * P + i) * 4 + v] = T(y[i]);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < m * m4; t += blockDim.x) {
        const int c = t / m4, r = (t - c * m4) * 4;
        T q[4];
        load4_aligned(sL + c * S + r, q);
        store4_aligned(L + size_t(c) * N + r, q);
    }
}

template <typename T>
static hipError_t launch_efr_transform_lds(const RefOps& ops, int nimp, T* M, size_t lds,
                                           hipStream_t st) {
#define HFR_ET(PP) hipLaunchKernelGGL((k_efr_transform_lds<T, PP>), dim3(nimp), dim3(kThreads), \
                                      lds, st, ops, nimp, M); break;
    switch (ops.P) {
        case 2: HFR_ET(2)
        case 3: HFR_ET(3)
        case 4: HFR_ET(4)
        case 5: HFR_ET(5)
        case 6: HFR_ET(6)
        default: return hipErrorInvalidValue;
    }
#undef HFR_ET
    return hipGetLastError();
}

hipError_t launch_efr_transform(const RefOps& ops, int nimp, void* M,
                                int precision, int n, int m, hipStream_t st) {
    if (nimp == 0) return hipSuccess;
    const size_t sc = precision == HFR_PREC_FP64 ? 8 : 4;
    const size_t lds = sc * size_t(m) * (m + 4);
    if (lds <= 64 * 1024 && n == 4 * ops.P * ops.P && m == 16 * ops.P) {
        if (precision == HFR_PREC_FP64)
            return launch_efr_transform_lds(ops, nimp, reinterpret_cast<double*>(M), lds, st);
        return launch_efr_transform_lds(ops, nimp, reinterpret_cast<float*>(M), lds, st);
    }
    if (precision == HFR_PREC_FP64)
        hipLaunchKernelGGL(k_efr_transform<double>, dim3(nimp), dim3(kThreads), 0, st,
                           ops, nimp, reinterpret_cast<double*>(M), n, m);
    else
        hipLaunchKernelGGL(k_efr_transform<float>, dim3(nimp), dim3(kThreads), 0, st,
                           ops, nimp, reinterpret_cast<float*>(M), n, m);
    return hipGetLastError();
}


// node blocks (4x4, column-major) of L from the transformed element Schur
// blocks, then t = -g - sum over node slots of sum_q phi_i(x_q) z
template <typename T>
__global__ void k_efr_assemble(RefOps og, EfrAssembleLaunch a) {
    __shared__ double gi[kMaxP * kMaxP];
    for (int t = threadIdx.x; t < kMaxP * kMaxP; t += blockDim.x) gi[t] = og.gi[t];
    __syncthreads();
    const int N = a.n + a.m, P = a.P;
    const T* M = reinterpret_cast<const T*>(a.M);
    // one thread per node block: each contribution is a 4x4 sub-block of an
    // element's Schur block, four columns of four adjacent entries (16-byte
    // aligned: N, n and the slot offsets are multiples of 4)
    for (long b = blockIdx.x * long(blockDim.x) + threadIdx.x; b < a.nblocks;
         b += long(gridDim.x) * blockDim.x) {
        double val[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) val[e] = 0.0;
        for (int c = a.cptr[b]; c < a.cptr[b + 1]; ++c) {
            const int* ct = a.contrib + 3 * size_t(c);
            const T* src = M + size_t(ct[0]) * N * N + size_t(a.n + ct[2] * 4) * N +
                           a.n + ct[1] * 4;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                T q[4];
                load4_aligned(src + size_t(w) * N, q);
#pragma unroll
                for (int v = 0; v < 4; ++v) val[4 * w + v] += double(q[v]);
            }
        }
        if (a.L64) {
#pragma unroll
            for (int e = 0; e < 16; e += 2)
                *reinterpret_cast<double2*>(a.L64 + 16 * b + e) = make_double2(val[e], val[e + 1]);
        }
        if (a.L32) {
#pragma unroll
            for (int e = 0; e < 16; e += 4)
                *reinterpret_cast<float4*>(a.L32 + 16 * b + e) =
                    make_float4(float(val[e]), float(val[e + 1]), float(val[e + 2]),
                                float(val[e + 3]));
        }
    }
    const long nt = long(a.nnodes) * 4;
    for (long idx = blockIdx.x * long(blockDim.x) + threadIdx.x; idx < nt;
         idx += long(gridDim.x) * blockDim.x) {
        const int nd = int(idx >> 2), v = int(idx & 3);
        double zs = 0.0;
        for (int c = a.inc_ptr[nd]; c < a.inc_ptr[nd + 1]; ++c) {
            const int s = a.inc[c];
            const int kf = s / P, i = s - kf * P;            // kf = imp*4 + lf
            const int k = kf >> 2, lf = kf & 3;
            const double* zq = a.z + size_t(k) * a.m + (lf * P) * 4 + v;
            for (int q = 0; q < P; ++q) zs += gi[q * P + i] * zq[q * 4];
        }
        a.t[idx] = -a.g[idx] - zs;
    }
}

hipError_t launch_efr_assemble(const RefOps& ops, const EfrAssembleLaunch& a,
                               hipStream_t st) {
    long work = std::max(long(a.nblocks), long(a.nnodes) * 4);
    if (work == 0) return hipSuccess;
    int grid = std::min(blocks_for(work), 65536);
    if (a.precision == HFR_PREC_FP64)
        hipLaunchKernelGGL(k_efr_assemble<double>, dim3(grid), dim3(kThreads), 0, st, ops, a);
    else
        hipLaunchKernelGGL(k_efr_assemble<float>, dim3(grid), dim3(kThreads), 0, st, ops, a);
    return hipGetLastError();
}

// uhat[node] = mean over the node's slots of the element state at the node:
// face values at the Gauss flux points (from the solution points), then the
// Gauss-point basis at the GLL node
__global__ void k_efr_trace_average(RefOps og, int nnodes, int Ne, const int* inc_ptr,
                                    const int* inc, const int* imp_list,
                                    const double* u, double* uhat) {
    __shared__ RefOps o;
    copy_ref_ops(o, og);
    __syncthreads();
    const int P = o.P, Np = P * P;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nnodes * 4) return;
    const int nd = idx >> 2, v = idx & 3;
    const size_t plane = size_t(Ne) * Np;
    double acc = 0.0;
    const int c0 = inc_ptr[nd], c1 = inc_ptr[nd + 1];
    for (int c = c0; c < c1; ++c) {
        const int s = inc[c];
        const int kf = s / P, i = s - kf * P;
        const int k = kf >> 2, lf = kf & 3;
        const double* base = u + size_t(v) * plane + size_t(imp_list[k]) * Np;
        double val = 0.0;
        for (int q = 0; q < P; ++q) {
            double uf = 0.0;
            for (int l = 0; l < P; ++l) {
                int pt;
                double wgt;
                if (lf == 0) { pt = l * P + q; wgt = o.lm[l]; }
                else if (lf == 1) { pt = q * P + l; wgt = o.lp[l]; }
                else if (lf == 2) { pt = l * P + (P - 1 - q); wgt = o.lp[l]; }
                else { pt = (P - 1 - q) * P + l; wgt = o.lm[l]; }
                uf += wgt * base[pt];
            }
            val += o.gj[i * P + q] * uf;
        }
        acc += val;
    }
    uhat[idx] = c1 > c0 ? acc / double(c1 - c0) : 0.0;
}

hipError_t launch_efr_trace_average(const RefOps& ops, int nnodes, int Ne,
                                    const int* inc_ptr, const int* inc,
                                    const int* imp_list, const double* u,
                                    double* uhat, hipStream_t st) {
    if (nnodes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_efr_trace_average, dim3(blocks_for(4L * nnodes)), dim3(kThreads),
                       0, st, ops, nnodes, Ne, inc_ptr, inc, imp_list, u, uhat);
    return hipGetLastError();
}

}  // namespace hfr
