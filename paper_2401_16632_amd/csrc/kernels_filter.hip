// Modal filter (Appendix B): every (variable, element) column of Np values
// is multiplied by F = V Lambda V^-1, V the Vandermonde matrix of the
// tensor-product orthonormal Legendre basis at the Gauss solution points
// and Lambda the diagonal of sigma over each mode's exponent sum.  Gauss
// quadrature with P points integrates the product of two basis functions of
// degree below P exactly, so V^-1 = V^T W with W the quadrature weights:
//     F[k][l] = w_l sum_m V[k][m] sigma(m) V[l][m].
// The [4][Ne][Np] state is a 4 Ne x Np row-major matrix of columns (one per
// variable and element), filtered in place.
#include "internal.h"

namespace hfr {

namespace {
constexpr int kRows = 64;              // columns per block: one per lane of a wave
constexpr int kWaves = 4;              // each wave forms a quarter of the outputs
constexpr int kThreads = kRows * kWaves;

// Barrier for LDS traffic only: it waits for this wave's LDS operations,
// not for its global loads in flight.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
}  // namespace

// Block b filters columns 64b .. 64b+63.  The tile's coalesced global loads
// are issued first; F is built in LDS while they are in flight, through
//   G[b][i][ii] = sum_a psi_a(x_i) psi_a(x_ii) sigma(a + b)
//   F[(j,i)][(jj,ii)] = w_jj w_ii sum_b psi_b(x_j) psi_b(x_jj) G[b][i][ii].
// Lane r of every wave takes column r of the padded LDS tile into
// registers; wave q forms outputs k = qK .. qK+K-1 of it, reading F as LDS
// broadcasts (the whole wave reads one entry).  The tile goes back to HBM
// through LDS with coalesced stores.
template <int P>
__global__ __launch_bounds__(kThreads) void k_modal_filter(FilterLaunch f, long nrows,
                                                           double* u) {
    constexpr int Np = P * P, LD = Np + 1;     // odd row stride: fewer bank conflicts
    constexpr int K = (Np + kWaves - 1) / kWaves;
    constexpr int NL = (kRows * Np + kThreads - 1) / kThreads;   // loads per thread
    __shared__ double V1[P * P], W[P], S[2 * P - 1];
    __shared__ double G[P * P * P];
    __shared__ double F[Np * Np];              // F[k*Np+l]
    __shared__ double U[kRows * LD];
    const int tid = threadIdx.x, lane = tid % kRows, q = tid / kRows;
    const long r0 = long(blockIdx.x) * kRows;
    const int nv = int(min(long(kRows), nrows - r0)) * Np;
    double* base = u + r0 * Np;
    double v[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c) {
        const int t = tid + c * kThreads;
        v[c] = t < nv ? base[t] : 0.0;
    }
    if (tid == 0) {                            // uniform (scalar) argument loads
#pragma unroll
        for (int c = 0; c < P * P; ++c) V1[c] = f.v1[c];
#pragma unroll
        for (int c = 0; c < P; ++c) W[c] = f.w[c];
#pragma unroll
        for (int c = 0; c < 2 * P - 1; ++c) S[c] = f.sig[c];
    }
    lds_barrier();
    for (int t = tid; t < P * P * P; t += kThreads) {
        const int b = t / (P * P), i = (t / P) % P, ii = t % P;
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < P; ++a) acc += V1[i * P + a] * V1[ii * P + a] * S[a + b];
        G[t] = acc;
    }
    lds_barrier();
    for (int t = tid; t < Np * Np; t += kThreads) {
        const int k = t / Np, l = t - k * Np;
        const int j = k / P, i = k - j * P, jj = l / P, ii = l - jj * P;
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < P; ++b)
            acc += V1[j * P + b] * V1[jj * P + b] * G[(b * P + i) * P + ii];
        F[t] = acc * W[jj] * W[ii];
    }
#pragma unroll
    for (int c = 0; c < NL; ++c) {
        const int t = tid + c * kThreads;
        if (t < kRows * Np) {
            const int r = t / Np, l = t - r * Np;
            U[r * LD + l] = v[c];
        }
    }
    lds_barrier();
    double x[Np];
#pragma unroll
    for (int l = 0; l < Np; ++l) x[l] = U[lane * LD + l];
    double y[K];
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
        const int k = q * K + kk;
        double acc = 0.0;
        if (k < Np) {
#pragma unroll
            for (int l = 0; l < Np; ++l) acc += F[k * Np + l] * x[l];
        }
        y[kk] = acc;
    }
    lds_barrier();                             // every wave has read its column
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
        const int k = q * K + kk;
        if (k < Np) U[lane * LD + k] = y[kk];
    }
    lds_barrier();
#pragma unroll
    for (int c = 0; c < NL; ++c) {
        const int t = tid + c * kThreads;
        if (t < nv) {
            const int r = t / Np, l = t - r * Np;
            base[t] = U[r * LD + l];
        }
    }
}

hipError_t launch_modal_filter(const FilterLaunch& f, long nrows, double* u,
                               hipStream_t st) {
    if (nrows <= 0) return hipSuccess;
    const dim3 grid(unsigned((nrows + kRows - 1) / kRows)), block(kThreads);
    switch (f.P) {
        case 2: hipLaunchKernelGGL(k_modal_filter<2>, grid, block, 0, st, f, nrows, u); break;
        case 3: hipLaunchKernelGGL(k_modal_filter<3>, grid, block, 0, st, f, nrows, u); break;
        case 4: hipLaunchKernelGGL(k_modal_filter<4>, grid, block, 0, st, f, nrows, u); break;
        case 5: hipLaunchKernelGGL(k_modal_filter<5>, grid, block, 0, st, f, nrows, u); break;
        case 6: hipLaunchKernelGGL(k_modal_filter<6>, grid, block, 0, st, f, nrows, u); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hfr
