// Kernels of the condensed trace system (Section 3.2): deterministic
// element-by-element assembly (eq:assembly / eq:assembly2) into block
// sparse rows (one block row per trace face, block size bs = 4 P), the
// block-sparse product, the block-Jacobi preconditioner, Krylov vector
// kernels, local recovery (eq:localproblems), Newton updates, and the IMEX
// stage combinations (eq:explicitimex and the final update).
#include "internal.h"
#include "wave_ops.h"

namespace hfr {

namespace {

constexpr int kThreads = 256;

inline int blocks_for(long n, int per = kThreads) {
    long b = (n + per - 1) / per;
    return int(b < 1 ? 1 : b);
}

__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < int(blockDim.x >> 6); ++i) s += red[i];
    __syncthreads();
    return s;  // valid in thread 0
}

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return uint16_t(b >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) {
    return __uint_as_float(uint32_t(h) << 16);
}

}  // namespace

// ---- assembly (eq:assembly): every block of L is the sum of at most two
// element Schur sub-blocks, t = -g - sum of the sides' C A^-1 r; a gather
// in a fixed order, no atomics.
// The block order P is fixed at compile time; a thread moves four
// consecutive rows of one block column (one point of a face, its four
// variables), which are contiguous both in the swept tableau and in the
// column-major block, as 16-byte accesses.
template <typename T> struct Vec4;
template <> struct Vec4<float> {
    typedef float4 type;
    __device__ static void get(const float* p, double (&v)[4]) {
        const float4 x = *reinterpret_cast<const float4*>(p);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    }
};
template <> struct Vec4<double> {
    __device__ static void get(const double* p, double (&v)[4]) {
        const double2 x = reinterpret_cast<const double2*>(p)[0];
        const double2 y = reinterpret_cast<const double2*>(p)[1];
        v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
    }
};

template <typename T, int P>
__global__ __launch_bounds__(256) void k_assemble4(AssembleLaunch a) {
    constexpr int bs = 4 * P, bb = bs * bs, per = bs * P;   // 4-row chunks per block
    const size_t N = size_t(a.n + a.m);
    const T* M = reinterpret_cast<const T*>(a.M);
    const long total = long(a.nblocks) * per;
    for (long idx = blockIdx.x * long(blockDim.x) + threadIdx.x; idx < total;
         idx += long(gridDim.x) * blockDim.x) {
        const int bi = int(idx / per);
        const int rem = int(idx - long(bi) * per);
        const int blk = a.blk_list ? a.blk_list[bi] : bi;
        const int b = rem / P, qa = rem - b * P;   // column, point of the rows
        const int qb = b >> 2, wb = b & 3;
        double val[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int* ct = a.blk_contrib + (size_t(blk) * 2 + c) * 3;
            const int imp = ct[0];
            if (imp < 0) continue;
            const int lr = ct[1] >> 1, sr = ct[1] & 1, lc = ct[2] >> 1, sc = ct[2] & 1;
            const int qea = sr ? P - 1 - qa : qa;
            const int qeb = sc ? P - 1 - qb : qb;
            const size_t row = a.n + (lr * P + qea) * 4;
            const size_t col = a.n + (lc * P + qeb) * 4 + wb;
            double v[4];
            Vec4<T>::get(M + size_t(imp) * N * N + col * N + row, v);
#pragma unroll
            for (int r = 0; r < 4; ++r) val[r] += v[r];
        }
        const size_t o = size_t(blk) * bb + size_t(b) * bs + 4 * qa;
        if (a.L64) {
            reinterpret_cast<double2*>(a.L64 + o)[0] = make_double2(val[0], val[1]);
            reinterpret_cast<double2*>(a.L64 + o)[1] = make_double2(val[2], val[3]);
        }
        if (a.L32)
            *reinterpret_cast<float4*>(a.L32 + o) =
                make_float4(float(val[0]), float(val[1]), float(val[2]), float(val[3]));
    }
    const long tt = long(a.ntf) * bs;
    for (long idx = blockIdx.x * long(blockDim.x) + threadIdx.x; idx < tt;
         idx += long(gridDim.x) * blockDim.x) {
        const int F = int(idx / bs), aa = int(idx - long(F) * bs);
        const int q = aa >> 2, v = aa & 3;
        double zs = 0.0;
        for (int s = 0; s < 2; ++s) {
            const int imp = a.tside[(size_t(F) * 2 + s) * 2];
            if (imp < 0) continue;
            const int lf = a.tside[(size_t(F) * 2 + s) * 2 + 1];
            const int qe = s ? P - 1 - q : q;
            zs += a.z[size_t(imp) * a.m + (lf * P + qe) * 4 + v];
        }
        a.t[idx] = -a.g[idx] - zs;
    }
}

template <typename T, int P>
static void launch_assemble4(const AssembleLaunch& a, hipStream_t st) {
    constexpr int bs = 4 * P;
    const long work = std::max(long(a.nblocks) * bs * P, long(a.ntf) * bs);
    int grid = blocks_for(work);
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL((k_assemble4<T, P>), dim3(grid), dim3(kThreads), 0, st, a);
}

template <typename T>
static hipError_t launch_assemble_t(const AssembleLaunch& a, hipStream_t st) {
    switch (a.P) {
        case 2: launch_assemble4<T, 2>(a, st); break;
        case 3: launch_assemble4<T, 3>(a, st); break;
        case 4: launch_assemble4<T, 4>(a, st); break;
        case 5: launch_assemble4<T, 5>(a, st); break;
        case 6: launch_assemble4<T, 6>(a, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_assemble(const AssembleLaunch& a, hipStream_t st) {
    if (a.precision == HFR_PREC_FP64) return launch_assemble_t<double>(a, st);
    return launch_assemble_t<float>(a, st);
}

// ---- block-Jacobi: invert the diagonal block of every trace face -------
// Lane r of a group holds row r of the BS x BS block in registers and BS
// Jordan exchanges with partial pivoting (DPP argmax over the group, pivot
// row through LDS) turn it into the inverse with row and column
// permutations, T[p_k][j] = Inv[k][p_j]; pivot rows are kept unscaled with
// their factor -1/pivot applied at the store.

// Blocks of at most 16 rows: four blocks per wave, one per row of 16 lanes
// (lane r of a row holds row r of its block).  The pivot search is a
// 16-lane DPP maximum; the pivot row is passed through LDS (each row's
// pivot lane writes it, the row's lanes read it back).  Rows of a wave past
// the last block run on the identity and store nothing.
__device__ __forceinline__ unsigned long long row16_max_key(unsigned long long x) {
    x = key_max(x, key_dpp<0xb1, 0xf>(x));      // quad_perm [1,0,3,2]
    x = key_max(x, key_dpp<0x4e, 0xf>(x));      // quad_perm [2,3,0,1]
    x = key_max(x, key_dpp<0x141, 0xf>(x));     // row_half_mirror
    x = key_max(x, key_dpp<0x140, 0xf>(x));     // row_mirror: every lane of the row
    return x;
}

__device__ __forceinline__ unsigned row16_max_u32(unsigned x) {
    x = max(x, key32_dpp<0xb1, 0xf>(x));        // quad_perm [1,0,3,2]
    x = max(x, key32_dpp<0x4e, 0xf>(x));        // quad_perm [2,3,0,1]
    x = max(x, key32_dpp<0x141, 0xf>(x));       // row_half_mirror
    x = max(x, key32_dpp<0x140, 0xf>(x));       // row_mirror: every lane of the row
    return x;
}

// C is the arithmetic of the exchanges: FP64, or FP32 for an inverse that
// is stored in FP32 or BF16 (32-bit pivot keys, hardware reciprocal)
template <int BS, typename C>
__global__ __launch_bounds__(256) void k_block_inverse16(int ntf, const int* diag_blk,
                                                         const double* L64,
                                                         const float* L32, int pc,
                                                         void* out, int* fail) {
    static_assert(BS <= 16, "four blocks per wave need BS <= 16");
    __shared__ C prow[4][4][BS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = lane >> 4, r = lane & 15;
    const int F = (blockIdx.x * 4 + wv) * 4 + grp;
    const bool valid = F < ntf;
    const size_t blk = valid ? size_t(diag_blk[F]) * BS * BS : 0;
    C t[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) {
        const size_t i = blk + size_t(c) * BS + min(r, BS - 1);   // in bounds
        C v = c == r ? C(1) : C(0);
        if (valid) v = L64 ? C(L64[i]) : C(L32[i]);
        t[c] = r < BS ? v : C(0);
    }
    C sig = C(1);
    bool used = r >= BS, bad = false;
    int pos = 0;
    int pj[BS];
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        int p;
        if constexpr (sizeof(C) == 8) {
            const unsigned long long key =
                row16_max_key(used ? 0ull : pivot_key(float(fabs(t[k])), r));
            p = int(0xffffffffu - unsigned(key));
            if ((key >> 32) == 0) {                 // no nonzero candidate
                bad = true;
                p = 0;
            }
        } else {
            const unsigned key =
                row16_max_u32(used ? 0u : pivot_key32(float(fabs(t[k])), r));
            p = 255 - int(key & 0xffu);
            if (key == 0) {                         // no nonzero candidate
                bad = true;
                p = 0;
            }
        }
        pj[k] = p;
        if (r == p) {
#pragma unroll
            for (int j = 0; j < BS; ++j) prow[wv][grp][j] = t[j];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        C u[BS];
#pragma unroll
        for (int j = 0; j < BS; ++j) u[j] = prow[wv][grp][j];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        C ipv;
        if constexpr (sizeof(C) == 8) ipv = bad ? 0.0 : 1.0 / u[k];
        else ipv = bad ? 0.f : __builtin_amdgcn_rcpf(u[k]);
        const C g = (r == p) ? C(0) : t[k] * ipv;
#pragma unroll
        for (int j = 0; j < BS; ++j) t[j] = fma(-g, u[j], t[j]);
        t[k] = (r == p) ? C(-1) : g;
        if (r == p) { used = true; sig = -ipv; pos = k; }
    }
    if (bad && valid && r == 0) *fail = 1;
    if (!valid || r >= BS) return;
    // store column-major: out[F][b][a] = Inv[a][b], Inv[pos][p_j] = sig t[j]
    const size_t o = size_t(F) * BS * BS + pos;
#pragma unroll
    for (int j = 0; j < BS; ++j) {
        const C v = sig * t[j];
        const size_t i = o + size_t(pj[j]) * BS;
        if (pc == HFR_PC_FP64) reinterpret_cast<double*>(out)[i] = double(v);
        else if (pc == HFR_PC_FP32) reinterpret_cast<float*>(out)[i] = float(v);
        else reinterpret_cast<uint16_t*>(out)[i] = f2bf(float(v));
    }
}

// Blocks of 17 to 32 rows: two blocks per wave, one per half of 32 lanes.
// The pivot search is the 16-lane DPP maximum, then row 0 into row 1 and
// row 2 into row 3 (row_bcast:15), read back from lanes 31 and 63; the
// pivot row is passed through LDS as for the 16-row blocks.  These are the
// face blocks of p = 4 and 5, whose L is assembled together with L Dinv
// afterwards: each lane sums its row of the diagonal block from the element
// tableaux (dg) instead of reading an assembled L.
__device__ __forceinline__ unsigned long long half32_max_key(unsigned long long x, int half) {
    x = row16_max_key(x);
    x = key_max(x, key_dpp<0x142, 0xa>(x));     // row_bcast:15 into rows 1, 3
    const int lo = int(unsigned(x)), hi = int(unsigned(x >> 32));
    const unsigned long long a =
        (static_cast<unsigned long long>(unsigned(__builtin_amdgcn_readlane(hi, 31))) << 32) |
        unsigned(__builtin_amdgcn_readlane(lo, 31));
    const unsigned long long b =
        (static_cast<unsigned long long>(unsigned(__builtin_amdgcn_readlane(hi, 63))) << 32) |
        unsigned(__builtin_amdgcn_readlane(lo, 63));
    return half ? b : a;
}
__device__ __forceinline__ unsigned half32_max_u32(unsigned x, int half) {
    x = row16_max_u32(x);
    x = max(x, key32_dpp<0x142, 0xa>(x));       // row_bcast:15 into rows 1, 3
    const unsigned a = unsigned(__builtin_amdgcn_readlane(int(x), 31));
    const unsigned b = unsigned(__builtin_amdgcn_readlane(int(x), 63));
    return half ? b : a;
}

template <int BS, typename C>
__global__ __launch_bounds__(256) void k_block_inverse32(int ntf, const int* diag_blk,
                                                         const double* L64,
                                                         const float* L32, int pc,
                                                         void* out, int* fail,
                                                         DiagGather dg) {
    static_assert(BS > 16 && BS <= 32, "two blocks per wave need 16 < BS <= 32");
    __shared__ C prow[4][2][BS];
    __shared__ __align__(16) double gsh[4][2][BS * BS];   // compact gather
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int half = lane >> 5, r = lane & 31;
    const int F = (blockIdx.x * 4 + wv) * 2 + half;
    const bool valid = F < ntf;
    const size_t blk = valid ? size_t(diag_blk[F]) * BS * BS : 0;
    C t[BS];
    if (dg.compact_schur) {                       // uniform over the grid
        // the element Schur sub-blocks are contiguous: each contribution in
        // 16-byte pieces (four rows of a point in one column, which stay
        // four consecutive trace rows), summed in FP64 into the block in LDS
        // in trace order (0, then the first side, then the second), then
        // each lane takes its row
        constexpr int P = BS / 4, BB = BS * BS;
        const size_t N = size_t(dg.n + dg.m);
        double* gs = &gsh[wv][half][0];
        for (int e = r; e < BB; e += 32) gs[e] = 0.0;
        auto wave_sync = [] {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        wave_sync();
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const int* ct = dg.blk_contrib + (blk / BB * 2 + cc) * 3;
            const int imp = valid ? ct[0] : -1;
            if (imp >= 0) {
                const int lr = ct[1] >> 1, sr = ct[1] & 1, lc = ct[2] >> 1, sc = ct[2] & 1;
                const size_t src = size_t(imp) * N * N + schur_offset(BS, lr, lc, 0, 0);
                for (int e = r; e < BB / 4; e += 32) {
                    const int be = (4 * e) / BS, qe = ((4 * e) % BS) >> 2;   // element column, point
                    const int tr = (sr ? P - 1 - qe : qe) * 4;
                    const int tc = (sc ? P - 1 - (be >> 2) : (be >> 2)) * 4 + (be & 3);
                    double v[4];
                    if (L64) {
                        const double2 x0 = reinterpret_cast<const double2*>(
                            reinterpret_cast<const double*>(dg.M) + src + 4 * e)[0];
                        const double2 x1 = reinterpret_cast<const double2*>(
                            reinterpret_cast<const double*>(dg.M) + src + 4 * e)[1];
                        v[0] = x0.x; v[1] = x0.y; v[2] = x1.x; v[3] = x1.y;
                    } else {
                        const float4 x = *reinterpret_cast<const float4*>(
                            reinterpret_cast<const float*>(dg.M) + src + 4 * e);
                        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
                    }
                    double* d = gs + tc * BS + tr;
#pragma unroll
                    for (int k = 0; k < 4; ++k) d[k] += v[k];
                }
            }
            wave_sync();
        }
        const int rr = min(r, BS - 1);
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            const double a2 = gs[c * BS + rr];
            C v = c == r ? C(1) : C(0);
            if (valid) v = L64 ? C(a2) : C(float(a2));
            t[c] = r < BS ? v : C(0);
        }
    } else {
        // the block summed from the element tableaux as the assembly forms it
        // (FP64 sum rounded to the storage precision of L)
        constexpr int P = BS / 4;
        const size_t N = size_t(dg.n + dg.m);
        const int rr = min(r, BS - 1), qa = rr >> 2;
        double acc[BS];
#pragma unroll
        for (int c = 0; c < BS; ++c) acc[c] = 0.0;
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const int* ct = dg.blk_contrib + (blk / (BS * BS) * 2 + cc) * 3;
            const int imp = valid ? ct[0] : -1;
            if (imp < 0) continue;
            const int lr = ct[1] >> 1, sr = ct[1] & 1, lc = ct[2] >> 1, sc = ct[2] & 1;
            const int ra = (sr ? P - 1 - qa : qa) * 4 + (rr & 3);   // row in face lr
            const size_t row = size_t(dg.n) + lr * 4 * P + ra;
#pragma unroll
            for (int c = 0; c < BS; ++c) {
                const int qb = c >> 2;
                const int cb = (sc ? P - 1 - qb : qb) * 4 + (c & 3);  // column in face lc
                const size_t cl = size_t(dg.n) + lc * 4 * P + cb;
                const size_t o = size_t(imp) * N * N +
                                 (dg.compact_schur ? schur_offset(BS, lr, lc, ra, cb)
                                                   : cl * N + row);
                acc[c] += L64 ? reinterpret_cast<const double*>(dg.M)[o]
                              : double(reinterpret_cast<const float*>(dg.M)[o]);
            }
        }
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            C v = c == r ? C(1) : C(0);
            if (valid) v = L64 ? C(acc[c]) : C(float(acc[c]));
            t[c] = r < BS ? v : C(0);
        }
    }
    C sig = C(1);
    bool used = r >= BS, bad = false;
    int pos = 0;
    int pj[BS];
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        int p;
        if constexpr (sizeof(C) == 8) {
            const unsigned long long key =
                half32_max_key(used ? 0ull : pivot_key(float(fabs(t[k])), r), half);
            p = int(0xffffffffu - unsigned(key));
            if ((key >> 32) == 0) {                 // no nonzero candidate
                bad = true;
                p = 0;
            }
        } else {
            const unsigned key =
                half32_max_u32(used ? 0u : pivot_key32(float(fabs(t[k])), r), half);
            p = 255 - int(key & 0xffu);
            if (key == 0) {                         // no nonzero candidate
                bad = true;
                p = 0;
            }
        }
        pj[k] = p;
        if (r == p) {
#pragma unroll
            for (int j = 0; j < BS; ++j) prow[wv][half][j] = t[j];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        C u[BS];
#pragma unroll
        for (int j = 0; j < BS; ++j) u[j] = prow[wv][half][j];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        C ipv;
        if constexpr (sizeof(C) == 8) ipv = bad ? 0.0 : 1.0 / u[k];
        else ipv = bad ? 0.f : __builtin_amdgcn_rcpf(u[k]);
        const C g = (r == p) ? C(0) : t[k] * ipv;
#pragma unroll
        for (int j = 0; j < BS; ++j) t[j] = fma(-g, u[j], t[j]);
        t[k] = (r == p) ? C(-1) : g;
        if (r == p) { used = true; sig = -ipv; pos = k; }
    }
    if (bad && valid && r == 0) *fail = 1;
    if (!valid || r >= BS) return;
    // store column-major: out[F][b][a] = Inv[a][b], Inv[pos][p_j] = sig t[j]
    const size_t o = size_t(F) * BS * BS + pos;
#pragma unroll
    for (int j = 0; j < BS; ++j) {
        const C v = sig * t[j];
        const size_t i = o + size_t(pj[j]) * BS;
        if (pc == HFR_PC_FP64) reinterpret_cast<double*>(out)[i] = double(v);
        else if (pc == HFR_PC_FP32) reinterpret_cast<float*>(out)[i] = float(v);
        else reinterpret_cast<uint16_t*>(out)[i] = f2bf(float(v));
    }
}

hipError_t launch_block_inverse_impl(int ntf, int bs, const int* diag_blk,
                                     const double* L64, const float* L32,
                                     int pc, void* out, int* fail,
                                     hipStream_t st, const DiagGather* dgp) {
    const DiagGather dg = dgp ? *dgp : DiagGather{};
    // blocks of 20 and 24 rows are gathered from the tableaux, the others
    // read from the assembled L
    if ((bs == 20 || bs == 24) != (dg.M != nullptr)) return hipErrorInvalidValue;
    if (ntf == 0) return hipSuccess;
    const dim3 blk(256);
    const dim3 grid16((ntf + 15) / 16);            // four blocks per wave
    const dim3 grid32((ntf + 7) / 8);              // two blocks per wave
    const bool f64 = pc == HFR_PC_FP64;
#define HFR_INV32(B)                                                                          \
    if (f64) hipLaunchKernelGGL((k_block_inverse32<B, double>), grid32, blk, 0, st, ntf,     \
                                diag_blk, L64, L32, pc, out, fail, dg);                      \
    else hipLaunchKernelGGL((k_block_inverse32<B, float>), grid32, blk, 0, st, ntf,          \
                            diag_blk, L64, L32, pc, out, fail, dg);                          \
    break;
#define HFR_INV16(B)                                                                          \
    if (f64) hipLaunchKernelGGL((k_block_inverse16<B, double>), grid16, blk, 0, st, ntf,     \
                                diag_blk, L64, L32, pc, out, fail);                          \
    else hipLaunchKernelGGL((k_block_inverse16<B, float>), grid16, blk, 0, st, ntf,          \
                            diag_blk, L64, L32, pc, out, fail);                              \
    break;
    switch (bs) {
        case 4: HFR_INV16(4)
        case 8: HFR_INV16(8)
        case 12: HFR_INV16(12)
        case 16: HFR_INV16(16)
        case 20: HFR_INV32(20)
        case 24: HFR_INV32(24)
        default: return hipErrorInvalidValue;
    }
#undef HFR_INV16
#undef HFR_INV32
    return hipGetLastError();
}

// ---- y = yin + alpha * L x  (block sparse, column-major blocks) ---------
__global__ void k_spmv(int nrows, int bs, const int* rowptr, const int* col,
                       const double* L64, const float* L32, const double* x,
                       double* y, double alpha, const double* yin) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const int F = r / bs, aa = r - F * bs;
    double acc = 0.0;
    for (int p = rowptr[F]; p < rowptr[F + 1]; ++p) {
        const size_t base = size_t(p) * bs * bs + aa;
        const double* xb = x + size_t(col[p]) * bs;
        if (L64) {
            for (int b = 0; b < bs; ++b) acc += L64[base + size_t(b) * bs] * xb[b];
        } else {
            for (int b = 0; b < bs; ++b) acc += double(L32[base + size_t(b) * bs]) * xb[b];
        }
    }
    y[r] = (yin ? yin[r] : 0.0) + alpha * acc;
}

hipError_t launch_spmv(int ntf, int bs, const int* rowptr, const int* col,
                       const double* L64, const float* L32, const double* x,
                       double* y, double alpha, const double* yin,
                       hipStream_t st) {
    const int nrows = ntf * bs;
    if (nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_spmv, dim3(blocks_for(nrows)), dim3(kThreads), 0, st,
                       nrows, bs, rowptr, col, L64, L32, x, y, alpha, yin);
    return hipGetLastError();
}

__global__ void k_absmax_partial(int N, const double* x, double* partial) {
    __shared__ double red[kThreads];
    double m = 0.0;
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < N;
         i += long(gridDim.x) * blockDim.x) {
        const double a = fabs(x[i]);
        m = (a > m || a != a) ? a : m;   // NaN propagates
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double o = red[threadIdx.x + s];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_absmax_final(int nblk, const double* partial, double* out) {
    __shared__ double red[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        const double o = partial[i];
        if (o > m || o != o) m = o;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double o = red[threadIdx.x + s];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_absmax(int N, const double* x, double* partial, int nblk,
                         double* out, hipStream_t st) {
    if (N == 0) {
        hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(256), 0, st, 0, partial, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_absmax_partial, dim3(nblk), dim3(kThreads), 0, st, N, x, partial);
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(256), 0, st, nblk, partial, out);
    return hipGetLastError();
}

// Newton residual norms: blocks [0, nbx) take max |x| over [0, Nx), the
// others max |y| over [0, Ny); one partial per block (NaN propagates).
__global__ void k_absmax2_partial(int Nx, const double* x, int nbx, int Ny,
                                  const double* y, double* partial) {
    __shared__ double red[kThreads];
    const bool isx = int(blockIdx.x) < nbx;
    const int N = isx ? Nx : Ny;
    const double* v = isx ? x : y;
    const long b = isx ? blockIdx.x : blockIdx.x - nbx;
    const long nb = isx ? nbx : gridDim.x - nbx;
    double m = 0.0;
    for (long i = b * blockDim.x + threadIdx.x; i < N; i += nb * blockDim.x) {
        const double a = fabs(v[i]);
        m = (a > m || a != a) ? a : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double o = red[threadIdx.x + s];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// both maxima -> out[0], out[1] (host-visible), *go = 0 iff both <= tol,
// either is not finite or the gate is closed; the two failure flags are copied to flags_out.  With
// tol_scale set the test uses tol * max(1, *tol_scale), written to out[2].
__global__ void k_absmax2_final(int nbx, int nby, const double* partial, double tol,
                                const double* tol_scale,
                                double* out, int* go, const int* gate,
                                const int* flags, int* flags_out,
                                long long* seq_out, long long* seq_ctr, Forcing fc) {
    __shared__ double red[2][256];
    double mx = 0.0, my = 0.0;
    for (int i = threadIdx.x; i < nbx; i += blockDim.x) {
        const double o = partial[i];
        if (o > mx || o != o) mx = o;
    }
    for (int i = threadIdx.x; i < nby; i += blockDim.x) {
        const double o = partial[nbx + i];
        if (o > my || o != o) my = o;
    }
    red[0][threadIdx.x] = mx;
    red[1][threadIdx.x] = my;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            for (int c = 0; c < 2; ++c) {
                const double o = red[c][threadIdx.x + s];
                if (o > red[c][threadIdx.x] || o != o) red[c][threadIdx.x] = o;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (tol_scale) tol *= fmax(1.0, *tol_scale);
        out[0] = red[0][0];
        out[1] = red[1][0];
        out[2] = tol;
        const bool open = !gate || *gate != 0;
        // a non-finite residual closes the gate too: the host stops (or
        // damps the step) and no linearisation queued behind may run on it
        const bool fin = isfinite(red[0][0]) && isfinite(red[1][0]);
        *go = (open && fin && !(red[0][0] <= tol && red[1][0] <= tol)) ? 1 : 0;
        if (fc.hist && open) {
            const double r = fmax(red[0][0], red[1][0]);
            const double rp = fc.hist[0];
            double eta = fc.hi;
            if (!fc.first && r > 0.0 && rp > 0.0 && r < rp) {
                const double q = r / rp;
                eta = fmin(fc.hi, fmax(fc.lo, 0.1 * fmax(r * q * q, tol) / r));
            }
            fc.hist[0] = r;
            fc.hist[1] = eta;
        }
        if (flags_out) {
            flags_out[0] = flags[0];
            flags_out[1] = flags[1];
        }
        if (seq_out) {                    // published after the values above
            const long long seq = *seq_ctr + 1;
            *seq_ctr = seq;
            __threadfence_system();
            *reinterpret_cast<volatile long long*>(seq_out) = seq;
        }
    }
}

hipError_t launch_newton_norms(int Nx, const double* x, int Ny, const double* y,
                               double* partial, double tol, const double* tol_scale,
                               double* out, int* go,
                               const int* gate, const int* flags, int* flags_out,
                               long long* seq_out, long long* seq_ctr, hipStream_t st,
                               Forcing fc) {
    const int nbx = std::min(1024, std::max(1, (Nx + kThreads - 1) / kThreads));
    const int nby = std::min(1024, std::max(1, (Ny + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(k_absmax2_partial, dim3(nbx + nby), dim3(kThreads), 0, st, Nx, x,
                       nbx, Ny, y, partial);
    hipLaunchKernelGGL(k_absmax2_final, dim3(1), dim3(256), 0, st, nbx, nby, partial, tol,
                       tol_scale, out, go, gate, flags, flags_out, seq_out, seq_ctr, fc);
    return hipGetLastError();
}

// ---- recovery (eq:localproblems) from the swept element tableau:
// du[k] = (A^-1 r)[k] - (A^-1 B duhat_loc)[k] = y~[p_k] + T[p_k][n:N] duhat_loc
// with y~ from the FP64 right-hand-side pass (pivot-row order).  One
// workgroup per element: thread (c, g) takes rows 4g .. 4g+3 of the columns
// c, c + CS, ... of T[:, n:N] as 16-byte reads, the CS partial sums meet in
// LDS, and thread r forms unknown r from pivot row p_r.  With nu set the
// same launch also applies the Newton update: every element adds du to its
// state in u, and the workgroups past the elements' add duhat to uhat
// (neither u nor uhat is read by the recovery).
struct NewtonUpdate {
    double* u;              // [4][Ne][Np] state (null: recovery only)
    const int* imp_list;
    int Ne;
    int ntp4;               // trace unknowns
    double* uhat;
};
template <typename T, int P>
__global__ __launch_bounds__(256) void k_recover(RefOps o, int efr, int nimp,
                                                 const T* M, const int* piv,
                                                 const double* yr,
                                                 const int* trace_map,
                                                 const double* duhat,
                                                 double* du, const int* gate,
                                                 NewtonUpdate nu, int compact) {
    constexpr int NP = P * P, n = 4 * NP, m = 16 * P, N = n + m;
    constexpr int RG = NP;                          // groups of four rows
    constexpr int CS = (256 / RG < m ? 256 / RG : m);   // column sets
    __shared__ double sloc[m];
    __shared__ double part[CS][n];
    if (gate && *gate == 0) return;               // uniform over the grid
    if (int(blockIdx.x) >= nimp) {                // trace part of the update
        const long i = (long(blockIdx.x) - nimp) * blockDim.x + threadIdx.x;
        if (i < nu.ntp4) nu.uhat[i] += duhat[i];
        return;                                   // uniform over the workgroup
    }
    const int k = blockIdx.x, t = threadIdx.x;
    if (t < m) {
        const int b = t;
        const int f = b / (4 * P), q = (b >> 2) % P, w = b & 3;
        const int* tm = trace_map + (size_t(k) * 4 + f) * P;
        double v = 0.0;
        if (efr) {
            // trace at the flux point from the face's GLL nodes
            if (tm[0] >= 0)
                for (int i = 0; i < P; ++i) v += o.gi[q * P + i] * duhat[size_t(tm[i]) * 4 + w];
        } else if (tm[q] >= 0) {
            v = duhat[size_t(tm[q]) * 4 + w];
        }
        sloc[b] = v;
    }
    __syncthreads();
    if (t < RG * CS) {
        const int c = t / RG, g = t - c * RG;
        // -A^-1 B: the columns n.. of the tableau, or compact after the
        // element's Schur sub-blocks
        const size_t ldx = compact ? size_t(n) : N;
        const T* Mk = M + size_t(k) * N * N + (compact ? schur_x_offset(4 * P) : size_t(n) * N) +
                      4 * g;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int b = c; b < m; b += CS) {
            double x[4];
            Vec4<T>::get(Mk + size_t(b) * ldx, x);
            const double s = sloc[b];
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] += x[r] * s;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) part[c][4 * g + r] = acc[r];
    }
    __syncthreads();
    for (int row = t; row < n; row += blockDim.x) {
        const int pr = piv[size_t(k) * n + row];
        double acc = yr[size_t(k) * n + pr];
        for (int c = 0; c < CS; ++c) acc += part[c][pr];
        du[size_t(row & 3) * nimp * NP + size_t(k) * NP + (row >> 2)] = acc;
        if (nu.u)
            nu.u[size_t(row & 3) * nu.Ne * NP + size_t(nu.imp_list[k]) * NP + (row >> 2)] += acc;
    }
}

template <typename T>
static hipError_t launch_recover_t(const RefOps& o, int efr, int nimp, const T* M,
                                   const int* piv, const double* yr,
                                   const int* trace_map, const double* duhat,
                                   double* du, const int* gate, const NewtonUpdate& nu,
                                   hipStream_t st, bool compact) {
    const int nbt = nu.u ? int((nu.ntp4 + 255) / 256) : 0;
    const dim3 grid(nimp + nbt), blk(256);
#define HFR_RC(PP) hipLaunchKernelGGL((k_recover<T, PP>), grid, blk, 0, st, o, efr, nimp, M, piv, yr, trace_map, duhat, du, gate, nu, compact ? 1 : 0); break;
    switch (o.P) {
        case 2: HFR_RC(2)
        case 3: HFR_RC(3)
        case 4: HFR_RC(4)
        case 5: HFR_RC(5)
        case 6: HFR_RC(6)
        default: return hipErrorInvalidValue;
    }
#undef HFR_RC
    return hipGetLastError();
}

hipError_t launch_recover(const RefOps& ops, bool efr, int nimp, const void* M,
                          int precision, const int* piv, const double* yr,
                          const int* trace_map, const double* duhat, double* du,
                          hipStream_t st, const int* gate, bool compact) {
    if (nimp == 0) return hipSuccess;
    const NewtonUpdate nu{nullptr, nullptr, 0, 0, nullptr};
    if (precision == HFR_PREC_FP64)
        return launch_recover_t(ops, efr ? 1 : 0, nimp, reinterpret_cast<const double*>(M),
                                piv, yr, trace_map, duhat, du, gate, nu, st, compact);
    return launch_recover_t(ops, efr ? 1 : 0, nimp, reinterpret_cast<const float*>(M),
                            piv, yr, trace_map, duhat, du, gate, nu, st, compact);
}

hipError_t launch_recover_update(const RefOps& ops, bool efr, int nimp, const void* M,
                                 int precision, const int* piv, const double* yr,
                                 const int* trace_map, const double* duhat, double* du,
                                 int Ne, const int* imp_list, double* u, int ntp4,
                                 double* uhat, hipStream_t st, const int* gate,
                                 bool compact) {
    if (nimp == 0)
        return launch_newton_update(0, 0, Ne, imp_list, du, u, ntp4, duhat, uhat, st, gate);
    const NewtonUpdate nu{u, imp_list, Ne, ntp4, uhat};
    if (precision == HFR_PREC_FP64)
        return launch_recover_t(ops, efr ? 1 : 0, nimp, reinterpret_cast<const double*>(M),
                                piv, yr, trace_map, duhat, du, gate, nu, st, compact);
    return launch_recover_t(ops, efr ? 1 : 0, nimp, reinterpret_cast<const float*>(M),
                            piv, yr, trace_map, duhat, du, gate, nu, st, compact);
}

// ---- Newton update: u_im += du (scatter), uhat += duhat -----------------
__global__ void k_newton_update(int Np, int nimp, int Ne, const int* imp_list,
                                const double* du, double* u, int ntp4,
                                const double* duhat, double* uhat, const int* gate,
                                double th) {
    if (gate && *gate == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = nimp * Np;
    const int nu = 4 * per;
    if (i < nu) {
        const int v = i / per;
        const int rem = i - v * per;
        const int k = rem / Np, pt = rem - k * Np;
        u[size_t(v) * Ne * Np + size_t(imp_list[k]) * Np + pt] += th * du[i];
    } else if (i - nu < ntp4) {
        uhat[i - nu] += th * duhat[i - nu];
    }
}

hipError_t launch_newton_update(int Np, int nimp, int Ne, const int* imp_list,
                                const double* du, double* u, int ntp4,
                                const double* duhat, double* uhat,
                                hipStream_t st, const int* gate, double theta) {
    const long n = 4L * nimp * Np + ntp4;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_newton_update, dim3(blocks_for(n)), dim3(kThreads), 0,
                       st, Np, nimp, Ne, imp_list, du, u, ntp4, duhat, uhat, gate, theta);
    return hipGetLastError();
}

// ---- transmission residual: sum of the two sides' shares -----------------
__global__ void k_gather_g(int ntp, const int* tpside, const double* gk,
                           double* g) {
    const long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i >= 4L * ntp) return;
    const int tp = int(i >> 2), v = int(i & 3);
    const int s0 = tpside[2 * tp], s1 = tpside[2 * tp + 1];
    g[i] = gk[size_t(s0) * 4 + v] + gk[size_t(s1) * 4 + v];
}

// The transmission residual g (as k_gather_g) together with the partial
// maxima of the Newton test: workgroups [0, nbx) take |x| over a grid
// stride, the others form g and take |g|, each writing its maximum to
// partial[blockIdx.x] (the layout k_absmax2_final reads)
__global__ void k_gather_g_absmax(int ntp, const int* tpside, const double* gk,
                                  double* g, int Nx, const double* x, int nbx,
                                  double* partial) {
    __shared__ double red[kThreads];
    double mx = 0.0;
    if (int(blockIdx.x) < nbx) {
        for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < Nx;
             i += long(nbx) * blockDim.x) {
            const double a = fabs(x[i]);
            mx = (a > mx || a != a) ? a : mx;
        }
    } else {
        const long nby = long(gridDim.x) - nbx;
        for (long i = (long(blockIdx.x) - nbx) * blockDim.x + threadIdx.x; i < 4L * ntp;
             i += nby * blockDim.x) {
            const int tp = int(i >> 2), v = int(i & 3);
            const int s0 = tpside[2 * tp], s1 = tpside[2 * tp + 1];
            const double gv = gk[size_t(s0) * 4 + v] + gk[size_t(s1) * 4 + v];
            g[i] = gv;
            const double a = fabs(gv);
            mx = (a > mx || a != a) ? a : mx;
        }
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double o = red[threadIdx.x + s];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

hipError_t launch_gather_g_norms(int ntp, const int* tpside, const double* gk, double* g,
                                 int Nx, const double* x, double* partial, double tol,
                                 const double* tol_scale, double* out, int* go,
                                 const int* gate, const int* flags,
                                 int* flags_out, long long* seq_out, long long* seq_ctr,
                                 hipStream_t st, Forcing fc) {
    const int nbx = std::min(1024, std::max(1, (Nx + kThreads - 1) / kThreads));
    const int nby = std::min(1024, std::max(1, (4 * ntp + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(k_gather_g_absmax, dim3(nbx + nby), dim3(kThreads), 0, st, ntp,
                       tpside, gk, g, Nx, x, nbx, partial);
    hipLaunchKernelGGL(k_absmax2_final, dim3(1), dim3(256), 0, st, nbx, nby, partial, tol,
                       tol_scale, out, go, gate, flags, flags_out, seq_out, seq_ctr, fc);
    return hipGetLastError();
}

hipError_t launch_trace_gather_g(int ntp, int P, const int* tpside,
                                 const double* gk, double* g, hipStream_t st) {
    (void)P;
    if (ntp == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_g, dim3(blocks_for(4L * ntp)), dim3(kThreads),
                       0, st, ntp, tpside, gk, g);
    return hipGetLastError();
}

// ---- initial trace: average of both sides' interpolated states ---------
struct Lagr {
    double lm[kMaxP], lp[kMaxP];
};

__global__ void k_trace_average_v(int ntp, int P, int Ne, const int* tpside,
                                  const int* imp_list, Lagr L, const double* u,
                                  double* uhat) {
    const long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i >= 4L * ntp) return;
    const int tp = int(i >> 2), v = int(i & 3);
    const int NP = P * P;
    double acc = 0.0;
    for (int s = 0; s < 2; ++s) {
        const int code = tpside[2 * tp + s];
        const int q = code % P, lf = (code / P) & 3, k = code / (4 * P);
        const double* base = u + size_t(v) * Ne * NP + size_t(imp_list[k]) * NP;
        double val = 0.0;
        for (int l = 0; l < P; ++l) {
            int pt;
            double w;
            if (lf == 0) { pt = l * P + q; w = L.lm[l]; }
            else if (lf == 1) { pt = q * P + l; w = L.lp[l]; }
            else if (lf == 2) { pt = l * P + (P - 1 - q); w = L.lp[l]; }
            else { pt = (P - 1 - q) * P + l; w = L.lm[l]; }
            val += w * base[pt];
        }
        acc += val;
    }
    uhat[i] = 0.5 * acc;
}

hipError_t launch_trace_average_ops(const RefOps& o, int ntp, int Ne,
                                    const int* tpside, const int* imp_list,
                                    const double* u, double* uhat,
                                    hipStream_t st) {
    if (ntp == 0) return hipSuccess;
    Lagr L{};
    for (int l = 0; l < o.P; ++l) {
        L.lm[l] = o.lm[l];
        L.lp[l] = o.lp[l];
    }
    hipLaunchKernelGGL(k_trace_average_v, dim3(blocks_for(4L * ntp)),
                       dim3(kThreads), 0, st, ntp, o.P, Ne, tpside, imp_list,
                       L, u, uhat);
    return hipGetLastError();
}

// ---- stage combinations ---------------------------------------------------
struct Combo {
    const double* base;      // full [4][Ne][Np], gathered through list
    const double* terms[6];  // compact [4][nlist][Np]
    double coef[6];
    int nterm;
    double* out;             // full (scatter) or compact
    int scatter;
    const double* dtscale;   // [Ne] factor of every coefficient, or null
};

__global__ void k_combine(int nlist, int Np, int Ne, const int* list, Combo c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = nlist * Np;
    if (i >= 4 * per) return;
    const int v = i / per;
    const int rem = i - v * per;
    const int li = rem / Np, pt = rem - li * Np;
    const size_t full = size_t(v) * Ne * Np + size_t(list[li]) * Np + pt;
    double acc = 0.0;
    for (int t = 0; t < c.nterm; ++t) acc += c.coef[t] * c.terms[t][i];
    acc = c.base[full] + (c.dtscale ? c.dtscale[list[li]] : 1.0) * acc;
    if (c.scatter) c.out[full] = acc;
    else c.out[i] = acc;
}

hipError_t launch_combine(int nlist, int Np, int Ne, const int* list,
                          const double* base, int nterm,
                          const double* const* terms, const double* coefs,
                          double* out, int scatter, const double* dtscale,
                          hipStream_t st) {
    if (nlist == 0) return hipSuccess;
    if (nterm > 6) return hipErrorInvalidValue;
    Combo c{};
    c.base = base;
    c.nterm = nterm;
    for (int t = 0; t < nterm; ++t) {
        c.terms[t] = terms[t];
        c.coef[t] = coefs[t];
    }
    c.out = out;
    c.scatter = scatter;
    c.dtscale = dtscale;
    const long n = 4L * nlist * Np;
    hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(kThreads), 0, st,
                       nlist, Np, Ne, list, c);
    return hipGetLastError();
}

}  // namespace hfr
