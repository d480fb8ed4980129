// Restarted GMRES for the condensed trace system L du_hat = t (Section 3.2;
// the paper does not name its global solver).
//
// Right block-Jacobi preconditioning is folded into the matrix once per
// linearisation: Lt = L Dinv (Dinv = inverse of each trace face's diagonal
// block), so an Arnoldi step is one block-sparse product.  One Arnoldi step
// is three kernels and no host synchronisation:
//   A: v_j = w / |w| (own rows), y = Lt w / |w|, partial dots V_i . y
//   B: w = y - sum h1_i V_i, partial dots V_i . w        (Gram-Schmidt, 1)
//   C: w -= sum h2_i V_i, partial |w|^2; Givens update  (Gram-Schmidt, 2)
// Each workgroup owns the rows of FPB consecutive trace faces.  The last
// workgroup to finish a kernel (device-scope fence + counter) reduces the
// partial sums in a fixed order, so results are deterministic.  Once the
// cycle has converged every later kernel of the cycle returns at entry.
#include "internal.h"
#include "gmres.h"

namespace hfr {

namespace {

__device__ __forceinline__ double wsum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// reduce k values per thread (vals[i] for i < k, computed by f(i)) to one
// partial per i for this block: out[i] (block-level, written by thread 0..k-1)
template <class F>
__device__ void block_partials(int k, F f, double* red, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < k; ++i) {
        const double s = wsum(f(i));
        if (lane == 0) red[i * nw + wave] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[i * nw + w];
        out[i] = s;
    }
}

// returns true in every thread of the last block to arrive
__device__ bool last_block(unsigned* counter) {
    __shared__ bool amlast;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = atomicAdd(counter, 1u);
        amlast = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (amlast) __threadfence();
    return amlast;
}

// fixed-order sum over blocks of partial[b*ld + i] for i < k -> out[i]
__device__ void reduce_partials(int k, int nb, const double* partial, int ld,
                                double* out, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    for (int i = wave; i < k; i += nw) {
        double s = 0.0;
        for (int b = lane; b < nb; b += 64) s += partial[size_t(b) * ld + i];
        s = wsum(s);
        if (lane == 0) red[i] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += blockDim.x) out[i] = red[i];
    __syncthreads();
}

__device__ __forceinline__ double spmv_row(const GmresArgs& a, const double* x,
                                           int F, int aa) {
    const int bs = a.bs;
    double acc = 0.0;
    for (int p = a.rowptr[F]; p < a.rowptr[F + 1]; ++p) {
        const size_t base = size_t(p) * bs * bs + aa;
        const double* xb = x + size_t(a.col[p]) * bs;
        if (a.Lt64) {
            for (int b = 0; b < bs; ++b) acc += a.Lt64[base + size_t(b) * bs] * xb[b];
        } else {
            for (int b = 0; b < bs; ++b) acc += double(a.Lt32[base + size_t(b) * bs]) * xb[b];
        }
    }
    return acc;
}

}  // namespace

// ---- A: scale, product, first projection ---------------------------------
__global__ __launch_bounds__(256) void k_arnoldi_a(GmresArgs a, int j,
                                                   const double* wcur,
                                                   double* wnxt) {
    GmresState* gs = a.gs;
    if (gs->done) return;
    __shared__ double red[kGmresMaxK * 4];
    __shared__ double fin[kGmresMaxK];
    const int fpb = a.fpb, bs = a.bs;
    const int F = blockIdx.x * fpb + threadIdx.x / bs;
    const int aa = threadIdx.x % bs;
    const bool act = (threadIdx.x < fpb * bs) && (F < a.ntf);
    const size_t r = size_t(F) * bs + aa;
    const double inv = gs->inv_norm;
    double y = 0.0;
    if (act) {
        a.V[size_t(j) * a.ldv + r] = wcur[r] * inv;
        y = spmv_row(a, wcur, F, aa) * inv;
        wnxt[r] = y;
    }
    __syncthreads();
    block_partials(j + 1, [&](int i) {
        return act ? a.V[size_t(i) * a.ldv + r] * y : 0.0;
    }, red, a.part + size_t(blockIdx.x) * kGmresMaxK);
    if (last_block(a.counters + 0)) {
        reduce_partials(j + 1, gridDim.x, a.part, kGmresMaxK, fin, red);
        for (int i = threadIdx.x; i <= j; i += blockDim.x) gs->h1[i] = fin[i];
        if (threadIdx.x == 0) a.counters[0] = 0u;
    }
}

// ---- B: first orthogonalisation, second projection ------------------------
__global__ __launch_bounds__(256) void k_arnoldi_b(GmresArgs a, int j,
                                                   double* w) {
    GmresState* gs = a.gs;
    if (gs->done) return;
    __shared__ double red[kGmresMaxK * 4];
    __shared__ double fin[kGmresMaxK];
    __shared__ double h[kGmresMaxK];
    for (int i = threadIdx.x; i <= j; i += blockDim.x) h[i] = gs->h1[i];
    __syncthreads();
    const int fpb = a.fpb, bs = a.bs;
    const int F = blockIdx.x * fpb + threadIdx.x / bs;
    const bool act = (threadIdx.x < fpb * bs) && (F < a.ntf);
    const size_t r = size_t(F) * bs + threadIdx.x % bs;
    double x = 0.0;
    if (act) {
        x = w[r];
        for (int i = 0; i <= j; ++i) x -= h[i] * a.V[size_t(i) * a.ldv + r];
        w[r] = x;
    }
    __syncthreads();
    block_partials(j + 1, [&](int i) {
        return act ? a.V[size_t(i) * a.ldv + r] * x : 0.0;
    }, red, a.part + size_t(blockIdx.x) * kGmresMaxK);
    if (last_block(a.counters + 1)) {
        reduce_partials(j + 1, gridDim.x, a.part, kGmresMaxK, fin, red);
        for (int i = threadIdx.x; i <= j; i += blockDim.x) gs->h2[i] = fin[i];
        if (threadIdx.x == 0) a.counters[1] = 0u;
    }
}

// ---- C: second orthogonalisation, norm, Givens rotation -------------------
__global__ __launch_bounds__(256) void k_arnoldi_c(GmresArgs a, int j,
                                                   double* w) {
    GmresState* gs = a.gs;
    if (gs->done) return;
    __shared__ double red[kGmresMaxK * 4];
    __shared__ double fin[kGmresMaxK];
    __shared__ double h[kGmresMaxK];
    for (int i = threadIdx.x; i <= j; i += blockDim.x) h[i] = gs->h2[i];
    __syncthreads();
    const int fpb = a.fpb, bs = a.bs;
    const int F = blockIdx.x * fpb + threadIdx.x / bs;
    const bool act = (threadIdx.x < fpb * bs) && (F < a.ntf);
    const size_t r = size_t(F) * bs + threadIdx.x % bs;
    double x = 0.0;
    if (act) {
        x = w[r];
        for (int i = 0; i <= j; ++i) x -= h[i] * a.V[size_t(i) * a.ldv + r];
        w[r] = x;
    }
    __syncthreads();
    block_partials(1, [&](int) { return x * x; }, red,
                   a.part2 + size_t(blockIdx.x) * 2);
    if (last_block(a.counters + 2)) {
        reduce_partials(1, gridDim.x, a.part2, 2, fin, red);
        if (threadIdx.x == 0) {
            const int R = a.restart;
            double* hc = gs->H + size_t(j) * (R + 1);
            const double hn = sqrt(fin[0]);
            for (int i = 0; i <= j; ++i) hc[i] = gs->h1[i] + gs->h2[i];
            hc[j + 1] = hn;
            for (int i = 0; i < j; ++i) {
                const double t0 = gs->cs[i] * hc[i] + gs->sn[i] * hc[i + 1];
                hc[i + 1] = -gs->sn[i] * hc[i] + gs->cs[i] * hc[i + 1];
                hc[i] = t0;
            }
            const double den = sqrt(hc[j] * hc[j] + hc[j + 1] * hc[j + 1]);
            const double c = den > 0.0 ? hc[j] / den : 1.0;
            const double s = den > 0.0 ? hc[j + 1] / den : 0.0;
            gs->cs[j] = c;
            gs->sn[j] = s;
            hc[j] = den;
            hc[j + 1] = 0.0;
            gs->g[j + 1] = -s * gs->g[j];
            gs->g[j] = c * gs->g[j];
            gs->jlast = j;
            gs->iters += 1;
            gs->inv_norm = hn > 0.0 ? 1.0 / hn : 0.0;
            const double res = fabs(gs->g[j + 1]);
            if (res <= gs->target || !(hn > 0.0) || j == R - 1 || !(res == res))
                gs->done = 1;
            a.counters[2] = 0u;
        }
    }
}

// ---- end of a cycle: y = H^-1 g, x += Dinv (V y) --------------------------
__global__ void k_gmres_update(GmresArgs a, double* x) {
    GmresState* gs = a.gs;
    __shared__ double y[kGmresMaxK];
    __shared__ double z[256];
    const int jl = gs->jlast;
    if (threadIdx.x == 0) {
        const int R = a.restart;
        for (int i = jl; i >= 0; --i) {
            double acc = gs->g[i];
            for (int k = i + 1; k <= jl; ++k) acc -= gs->H[size_t(k) * (R + 1) + i] * y[k];
            y[i] = acc / gs->H[size_t(i) * (R + 1) + i];
        }
    }
    __syncthreads();
    const int fpb = a.fpb, bs = a.bs;
    const int fl = threadIdx.x / bs, aa = threadIdx.x % bs;
    const int F = blockIdx.x * fpb + fl;
    const bool act = (threadIdx.x < fpb * bs) && (F < a.ntf);
    const size_t r = size_t(F) * bs + aa;
    double zz = 0.0;
    if (act && jl >= 0)
        for (int i = 0; i <= jl; ++i) zz += y[i] * a.V[size_t(i) * a.ldv + r];
    z[threadIdx.x] = zz;
    __syncthreads();
    if (!act || jl < 0) return;
    double acc = 0.0;
    const size_t base = size_t(F) * bs * bs + aa;
    for (int b = 0; b < bs; ++b) {
        double dv;
        if (a.pc == HFR_PC_FP64) dv = reinterpret_cast<const double*>(a.Dinv)[base + size_t(b) * bs];
        else if (a.pc == HFR_PC_FP32) dv = double(reinterpret_cast<const float*>(a.Dinv)[base + size_t(b) * bs]);
        else dv = double(__uint_as_float(uint32_t(reinterpret_cast<const uint16_t*>(a.Dinv)[base + size_t(b) * bs]) << 16));
        acc += dv * z[fl * bs + b];
    }
    x[r] += acc;
}

// ---- restart: r = t - L x (FP64), beta = |r|, w = r, new cycle -----------
__global__ __launch_bounds__(256) void k_gmres_restart(GmresArgs a,
                                                       const double* x,
                                                       double* w, int first) {
    GmresState* gs = a.gs;
    __shared__ double red[4 * 4];
    __shared__ double fin[2];
    const int fpb = a.fpb, bs = a.bs;
    const int F = blockIdx.x * fpb + threadIdx.x / bs;
    const int aa = threadIdx.x % bs;
    const bool act = (threadIdx.x < fpb * bs) && (F < a.ntf);
    const size_t r = size_t(F) * bs + aa;
    double v = 0.0;
    if (act) {
        double lx = 0.0;
        if (!first) {
            for (int p = a.rowptr[F]; p < a.rowptr[F + 1]; ++p) {
                const size_t base = size_t(p) * bs * bs + aa;
                const double* xb = x + size_t(a.col[p]) * bs;
                if (a.L64) {
                    for (int b = 0; b < bs; ++b) lx += a.L64[base + size_t(b) * bs] * xb[b];
                } else {
                    for (int b = 0; b < bs; ++b) lx += double(a.L32[base + size_t(b) * bs]) * xb[b];
                }
            }
        }
        v = a.t[r] - lx;
        w[r] = v;
    }
    __syncthreads();
    block_partials(1, [&](int) { return v * v; }, red,
                   a.part2 + size_t(blockIdx.x) * 2);
    if (last_block(a.counters + 3)) {
        reduce_partials(1, gridDim.x, a.part2, 2, fin, red);
        if (threadIdx.x == 0) {
            const double beta = sqrt(fin[0]);
            if (first) {
                gs->bnorm = beta;
                gs->target = a.rtol * beta;
                gs->iters = 0;
                gs->cycles = 0;
            } else {
                gs->cycles += 1;
            }
            gs->beta = beta;
            gs->g[0] = beta;
            for (int i = 1; i <= a.restart; ++i) gs->g[i] = 0.0;
            gs->inv_norm = beta > 0.0 ? 1.0 / beta : 0.0;
            gs->jlast = -1;
            const bool conv = !(beta > gs->target);
            gs->converged = conv ? 1 : 0;
            gs->done = (conv || !(beta == beta)) ? 1 : 0;
            a.counters[3] = 0u;
        }
    }
}

// ---- Lt = L Dinv (per block: Lt_FG = L_FG Dinv_G) -------------------------
__global__ void k_precondition_matrix(int nblocks, int bs, const int* col,
                                      const double* L64, const float* L32,
                                      int pc, const void* Dinv, double* Lt64,
                                      float* Lt32) {
    const long total = long(nblocks) * bs * bs;
    for (long idx = blockIdx.x * long(blockDim.x) + threadIdx.x; idx < total;
         idx += long(gridDim.x) * blockDim.x) {
        const int p = int(idx / (bs * bs));
        const int rem = int(idx % (bs * bs));
        const int b = rem / bs, aa = rem % bs;
        const size_t lb = size_t(p) * bs * bs;
        const size_t db = size_t(col[p]) * bs * bs;
        double acc = 0.0;
        for (int c = 0; c < bs; ++c) {
            const double lv = L64 ? L64[lb + size_t(c) * bs + aa] : double(L32[lb + size_t(c) * bs + aa]);
            double dv;
            const size_t di = db + size_t(b) * bs + c;
            if (pc == HFR_PC_FP64) dv = reinterpret_cast<const double*>(Dinv)[di];
            else if (pc == HFR_PC_FP32) dv = double(reinterpret_cast<const float*>(Dinv)[di]);
            else dv = double(__uint_as_float(uint32_t(reinterpret_cast<const uint16_t*>(Dinv)[di]) << 16));
            acc += lv * dv;
        }
        if (Lt64) Lt64[idx] = acc;
        else Lt32[idx] = float(acc);
    }
}

hipError_t launch_precondition_matrix(int nblocks, int bs, const int* col,
                                      const double* L64, const float* L32,
                                      int pc, const void* Dinv, double* Lt64,
                                      float* Lt32, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    long total = long(nblocks) * bs * bs;
    int grid = int(std::min<long>((total + 255) / 256, 65536));
    hipLaunchKernelGGL(k_precondition_matrix, dim3(grid), dim3(256), 0, st,
                       nblocks, bs, col, L64, L32, pc, Dinv, Lt64, Lt32);
    return hipGetLastError();
}

hipError_t launch_gmres_restart(const GmresArgs& a, const double* x,
                                double* w, int first, hipStream_t st) {
    hipLaunchKernelGGL(k_gmres_restart, dim3(a.nblk), dim3(256), 0, st, a, x,
                       w, first);
    return hipGetLastError();
}

hipError_t launch_arnoldi(const GmresArgs& a, int j, const double* wcur,
                          double* wnxt, hipStream_t st) {
    hipLaunchKernelGGL(k_arnoldi_a, dim3(a.nblk), dim3(256), 0, st, a, j, wcur, wnxt);
    hipLaunchKernelGGL(k_arnoldi_b, dim3(a.nblk), dim3(256), 0, st, a, j, wnxt);
    hipLaunchKernelGGL(k_arnoldi_c, dim3(a.nblk), dim3(256), 0, st, a, j, wnxt);
    return hipGetLastError();
}

hipError_t launch_gmres_update(const GmresArgs& a, double* x, hipStream_t st) {
    hipLaunchKernelGGL(k_gmres_update, dim3(a.nblk), dim3(256), 0, st, a, x);
    return hipGetLastError();
}

}  // namespace hfr
