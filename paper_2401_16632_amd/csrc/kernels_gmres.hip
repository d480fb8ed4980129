// Restarted GMRES for the condensed trace system L du_hat = t (Section 3.2;
// the paper does not name its global solver).
//
// Right block-Jacobi preconditioning is folded into the matrix once per
// linearisation: Lt = L Dinv (Dinv = inverse of each trace face's diagonal
// block), so an Arnoldi step is one block-sparse product.  One Arnoldi step
// is four kernels and no host synchronisation:
//   A: v_j = w / |w| (own rows), y = Lt w / |w|, partial dots V_i . y
//   B: w = y - sum h1_i V_i, partial dots V_i . w        (Gram-Schmidt, 1)
//   C: w -= sum h2_i V_i, partial |w|^2                  (Gram-Schmidt, 2)
//   D: |w|, Givens rotation, convergence flag
// A fourth, one-workgroup kernel applies the Givens rotation.  Partial sums
// are reduced in a fixed order by the consuming kernel, so results are
// deterministic.  Once the cycle has converged every later kernel of the
// cycle returns at entry.
#include "internal.h"
#include "gmres.h"

namespace hfr {

namespace {

constexpr int kThr = 512;        // threads per workgroup of the vector kernels

__device__ __forceinline__ double wsum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// sum of per-thread values over the block for each i < k -> out[i]
// (written by threads 0..k-1); red needs k * (blockDim/64) doubles
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
    __syncthreads();
}

// fixed-order sum over blocks of partial[b*ld + i] for i < k -> out[i] (LDS);
// every block computes the same values
__device__ void reduce_partials(int k, int nb, const double* partial, int ld,
                                double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    for (int i = wave; i < k; i += nw) {
        double s = 0.0;
        for (int b = lane; b < nb; b += 64) s += partial[size_t(b) * ld + i];
        s = wsum(s);
        if (lane == 0) out[i] = s;
    }
    __syncthreads();
}

// rows of block blockIdx.x: [r0, r1) (whole faces)
__device__ __forceinline__ void block_rows(const GmresArgs& a, int& r0, int& r1) {
    const int f0 = blockIdx.x * a.fpb;
    const int f1 = min(a.ntf, f0 + a.fpb);
    r0 = f0 * a.bs;
    r1 = f1 * a.bs;
}

__device__ __forceinline__ double spmv_row(const GmresArgs& a, const double* x,
                                           int F, int aa) {
    const int bs = a.bs;
    double acc = 0.0;
    const int p1 = a.rowptr[F + 1];
    for (int p = a.rowptr[F]; p < p1; ++p) {
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

// Each workgroup owns the rows of a.fpb consecutive faces (a.nblk <= 256
// workgroups of 512 threads) and loops over them.  Partial sums go to
// a.part[block][i]; the next kernel reduces them in every workgroup (fixed
// order), so no device-scope fences or counters are needed.

constexpr int kRPT = 4;          // rows per thread (<= 2048 rows per block)

// ---- A: scale, product, first projection ---------------------------------
// Own decomposition: a.nblkA workgroups of 256 threads, 64 rows at a time,
// four threads per row (thread group q takes blocks q, q+4, ... of the row).
__global__ __launch_bounds__(256) void k_arnoldi_a(GmresArgs a, int j,
                                                   const double* wcur,
                                                   double* wnxt) {
    GmresState* gs = a.gs;
    if (gs->done) return;
    __shared__ double red[kGmresMaxK * 4];
    __shared__ double sacc[4][64];
    const double inv = gs->inv_norm;
    const int bs = a.bs;
    const int f0 = blockIdx.x * a.fpbA, f1 = min(a.ntf, f0 + a.fpbA);
    const int r0 = f0 * bs, r1 = f1 * bs;
    const int part = threadIdx.x >> 6, lr = threadIdx.x & 63;
    double yv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        yv[q] = 0.0;
        const int rb = r0 + 64 * q;
        if (rb >= r1) continue;                   // uniform
        const int r = rb + lr;
        double acc = 0.0;
        if (r < r1) {
            const int F = r / bs, aa = r - F * bs;
            const int p1 = a.rowptr[F + 1];
            for (int p = a.rowptr[F] + part; p < p1; p += 4) {
                const size_t base = size_t(p) * bs * bs + aa;
                const double* xb = wcur + size_t(a.col[p]) * bs;
                if (a.Lt64) {
                    for (int b = 0; b < bs; ++b) acc += a.Lt64[base + size_t(b) * bs] * xb[b];
                } else {
                    for (int b = 0; b < bs; ++b) acc += double(a.Lt32[base + size_t(b) * bs]) * xb[b];
                }
            }
        }
        sacc[part][lr] = acc;
        __syncthreads();
        if (part == 0 && r < r1) {
            const double y = (sacc[0][lr] + sacc[1][lr] + sacc[2][lr] + sacc[3][lr]) * inv;
            a.V[size_t(j) * a.ldv + r] = wcur[r] * inv;
            wnxt[r] = y;
            yv[q] = y;
        }
        __syncthreads();
    }
    // projections V_i . y over this block's rows (group 0 holds y)
    block_partials(j + 1, [&](int i) {
        double s = 0.0;
        if (part == 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int r = r0 + 64 * q + lr;
                if (r < r1) s += a.V[size_t(i) * a.ldv + r] * yv[q];
            }
        }
        return s;
    }, red, a.part3 + size_t(blockIdx.x) * kGmresMaxK);
}

// ---- A2: reduce the product kernel's partials (one workgroup) ------------
__global__ __launch_bounds__(512) void k_arnoldi_a2(GmresArgs a, int j) {
    GmresState* gs = a.gs;
    if (gs->done) return;
    __shared__ double h[kGmresMaxK];
    reduce_partials(j + 1, a.nblkA, a.part3, kGmresMaxK, h);
    for (int i = threadIdx.x; i <= j; i += blockDim.x) gs->h1[i] = h[i];
}

// ---- B: first orthogonalisation, second projection ------------------------
__global__ __launch_bounds__(kThr) void k_arnoldi_b(GmresArgs a, int j,
                                                    double* w) {
    GmresState* gs = a.gs;
    if (gs->done) return;
    __shared__ double red[kGmresMaxK * (kThr / 64)];
    __shared__ double h[kGmresMaxK];
    const int k = j + 1;
    for (int i = threadIdx.x; i < k; i += blockDim.x) h[i] = gs->h1[i];
    __syncthreads();
    int r0, r1;
    block_rows(a, r0, r1);
    double x[kRPT];
#pragma unroll
    for (int q = 0; q < kRPT; ++q) {
        const int r = r0 + threadIdx.x + kThr * q;
        x[q] = 0.0;
        if (r < r1) {
            double v = w[r];
            for (int i = 0; i < k; ++i) v -= h[i] * a.V[size_t(i) * a.ldv + r];
            w[r] = v;
            x[q] = v;
        }
    }
    block_partials(k, [&](int i) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < kRPT; ++q) {
            const int r = r0 + threadIdx.x + kThr * q;
            if (r < r1) s += a.V[size_t(i) * a.ldv + r] * x[q];
        }
        return s;
    }, red, a.part2 + size_t(blockIdx.x) * kGmresMaxK);
}

// ---- C: second orthogonalisation, norm partials --------------------------
__global__ __launch_bounds__(kThr) void k_arnoldi_c(GmresArgs a, int j,
                                                    double* w) {
    GmresState* gs = a.gs;
    if (gs->done) return;
    __shared__ double red[kGmresMaxK * (kThr / 64)];
    __shared__ double h[kGmresMaxK];
    const int k = j + 1;
    reduce_partials(k, gridDim.x, a.part2, kGmresMaxK, h);
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < k; i += blockDim.x) gs->h2[i] = h[i];
    int r0, r1;
    block_rows(a, r0, r1);
    double nn = 0.0;
    for (int r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        double x = w[r];
        for (int i = 0; i < k; ++i) x -= h[i] * a.V[size_t(i) * a.ldv + r];
        w[r] = x;
        nn += x * x;
    }
    block_partials(1, [&](int) { return nn; }, red, a.part + size_t(blockIdx.x) * kGmresMaxK);
}

// ---- D: norm, Givens rotation, convergence flag (one workgroup) ----------
__global__ __launch_bounds__(kThr) void k_arnoldi_d(GmresArgs a, int j) {
    GmresState* gs = a.gs;
    if (gs->done) return;
    __shared__ double fin[kGmresMaxK];
    reduce_partials(1, a.nblk, a.part, kGmresMaxK, fin);
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
    }
}

// ---- end of a cycle: y = H^-1 g, x += Dinv (V y) --------------------------
__global__ __launch_bounds__(kThr) void k_gmres_update(GmresArgs a, double* x) {
    GmresState* gs = a.gs;
    __shared__ double y[kGmresMaxK];
    __shared__ double z[kThr];
    const int jl = gs->jlast;
    if (jl < 0) return;
    if (threadIdx.x == 0) {
        const int R = a.restart;
        for (int i = jl; i >= 0; --i) {
            double acc = gs->g[i];
            for (int k = i + 1; k <= jl; ++k) acc -= gs->H[size_t(k) * (R + 1) + i] * y[k];
            y[i] = acc / gs->H[size_t(i) * (R + 1) + i];
        }
    }
    __syncthreads();
    const int bs = a.bs;
    const int fps = kThr / bs;                 // faces per sub-chunk
    const int f0 = blockIdx.x * a.fpb, f1 = min(a.ntf, f0 + a.fpb);
    for (int fs = f0; fs < f1; fs += fps) {
        const int fl = threadIdx.x / bs, aa = threadIdx.x - fl * bs;
        const int F = fs + fl;
        const bool act = (fl < fps) && (F < f1);
        const size_t r = size_t(F) * bs + aa;
        double zz = 0.0;
        if (act)
            for (int i = 0; i <= jl; ++i) zz += y[i] * a.V[size_t(i) * a.ldv + r];
        z[threadIdx.x] = zz;
        __syncthreads();
        if (act) {
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
        __syncthreads();
    }
}

// ---- restart: r = t - L x (FP64), partial |r|^2 ---------------------------
__global__ __launch_bounds__(kThr) void k_gmres_residual(GmresArgs a,
                                                         const double* x,
                                                         double* w, int first) {
    __shared__ double red[kThr / 64];
    int r0, r1;
    block_rows(a, r0, r1);
    double nn = 0.0;
    for (int r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const int F = r / a.bs, aa = r - F * a.bs;
        double lx = 0.0;
        if (!first) {
            const int bs = a.bs;
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
        const double v = a.t[r] - lx;
        w[r] = v;
        nn += v * v;
    }
    block_partials(1, [&](int) { return nn; }, red, a.part + size_t(blockIdx.x) * kGmresMaxK);
}

// beta = |r|, new cycle (one workgroup)
__global__ __launch_bounds__(kThr) void k_gmres_restart(GmresArgs a, int first) {
    GmresState* gs = a.gs;
    __shared__ double fin[kGmresMaxK];
    reduce_partials(1, a.nblk, a.part, kGmresMaxK, fin);
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
    }
}

__device__ __forceinline__ double load_pc(const double* d, size_t i) { return d[i]; }
__device__ __forceinline__ double load_pc(const float* d, size_t i) { return double(d[i]); }
__device__ __forceinline__ double load_pc(const uint16_t* d, size_t i) {
    return double(__uint_as_float(uint32_t(d[i]) << 16));     // BF16 -> FP32
}

// ---- Lt = L Dinv (per block: Lt_FG = L_FG Dinv_G) -------------------------
// One wave per block, four blocks per workgroup; both factors staged in LDS
// (FP64), each lane forms BS*BS/64 entries of the product.
template <int BS, typename TL, typename TD>
__global__ __launch_bounds__(256) void k_precondition_matrix(int nblocks, const int* col,
                                                             const TL* L, const TD* Dinv,
                                                             TL* Lt) {
    constexpr int BB = BS * BS;
    __shared__ double sL[4][BB], sD[4][BB];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int p = blockIdx.x * 4 + wv;
    if (p >= nblocks) return;                      // whole wave
    const size_t lb = size_t(p) * BB, db = size_t(col[p]) * BB;
    for (int i = lane; i < BB; i += 64) {
        sL[wv][i] = double(L[lb + i]);
        sD[wv][i] = load_pc(Dinv, db + i);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // entry (a, b) of the column-major product: sum_c L[a][c] Dinv[c][b]
    for (int i = lane; i < BB; i += 64) {
        const int b = i / BS, a = i - b * BS;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < BS; ++c) acc = fma(sL[wv][c * BS + a], sD[wv][b * BS + c], acc);
        Lt[lb + i] = TL(acc);
    }
}

template <int BS, typename TL>
static void launch_pm_t(int nblocks, const int* col, const TL* L, int pc,
                        const void* Dinv, TL* Lt, hipStream_t st) {
    const dim3 grid((nblocks + 3) / 4), blk(256);
    if (pc == HFR_PC_FP64)
        hipLaunchKernelGGL((k_precondition_matrix<BS, TL, double>), grid, blk, 0, st, nblocks, col, L,
                           reinterpret_cast<const double*>(Dinv), Lt);
    else if (pc == HFR_PC_FP32)
        hipLaunchKernelGGL((k_precondition_matrix<BS, TL, float>), grid, blk, 0, st, nblocks, col, L,
                           reinterpret_cast<const float*>(Dinv), Lt);
    else
        hipLaunchKernelGGL((k_precondition_matrix<BS, TL, uint16_t>), grid, blk, 0, st, nblocks, col, L,
                           reinterpret_cast<const uint16_t*>(Dinv), Lt);
}

template <typename TL>
static hipError_t launch_pm(int nblocks, int bs, const int* col, const TL* L, int pc,
                            const void* Dinv, TL* Lt, hipStream_t st) {
    switch (bs) {
        case 4: launch_pm_t<4>(nblocks, col, L, pc, Dinv, Lt, st); break;
        case 8: launch_pm_t<8>(nblocks, col, L, pc, Dinv, Lt, st); break;
        case 12: launch_pm_t<12>(nblocks, col, L, pc, Dinv, Lt, st); break;
        case 16: launch_pm_t<16>(nblocks, col, L, pc, Dinv, Lt, st); break;
        case 20: launch_pm_t<20>(nblocks, col, L, pc, Dinv, Lt, st); break;
        case 24: launch_pm_t<24>(nblocks, col, L, pc, Dinv, Lt, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_precondition_matrix(int nblocks, int bs, const int* col,
                                      const double* L64, const float* L32,
                                      int pc, const void* Dinv, double* Lt64,
                                      float* Lt32, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    if (L64) return launch_pm<double>(nblocks, bs, col, L64, pc, Dinv, Lt64, st);
    return launch_pm<float>(nblocks, bs, col, L32, pc, Dinv, Lt32, st);
}

hipError_t launch_gmres_restart(const GmresArgs& a, const double* x,
                                double* w, int first, hipStream_t st) {
    hipLaunchKernelGGL(k_gmres_residual, dim3(a.nblk), dim3(kThr), 0, st, a, x,
                       w, first);
    hipLaunchKernelGGL(k_gmres_restart, dim3(1), dim3(kThr), 0, st, a, first);
    return hipGetLastError();
}

hipError_t launch_arnoldi_product(const GmresArgs& a, int j, const double* wcur,
                                  double* wnxt, hipStream_t st) {
    hipLaunchKernelGGL(k_arnoldi_a, dim3(a.nblkA), dim3(256), 0, st, a, j, wcur, wnxt);
    hipLaunchKernelGGL(k_arnoldi_a2, dim3(1), dim3(512), 0, st, a, j);
    return hipGetLastError();
}

hipError_t launch_arnoldi_orth(const GmresArgs& a, int j, double* wnxt,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_arnoldi_b, dim3(a.nblk), dim3(kThr), 0, st, a, j, wnxt);
    hipLaunchKernelGGL(k_arnoldi_c, dim3(a.nblk), dim3(kThr), 0, st, a, j, wnxt);
    hipLaunchKernelGGL(k_arnoldi_d, dim3(1), dim3(kThr), 0, st, a, j);
    return hipGetLastError();
}

hipError_t launch_gmres_update(const GmresArgs& a, double* x, hipStream_t st) {
    hipLaunchKernelGGL(k_gmres_update, dim3(a.nblk), dim3(kThr), 0, st, a, x);
    return hipGetLastError();
}

}  // namespace hfr
