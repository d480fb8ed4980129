// Restarted GMRES for the condensed trace system L du_hat = t (Section 3.2;
// the paper does not name its global solver).
//
// Right block-Jacobi preconditioning is folded into the matrix once per
// linearisation: Lt = L Dinv (Dinv = inverse of each trace face's diagonal
// block, Lt stored per block by 16-byte row pieces so that the lanes of a
// block's rows read adjacent pieces), so an Arnoldi step is one block-sparse
// product.  One Arnoldi
// step is two kernels (three with a second Gram-Schmidt pass) and no host
// synchronisation:
//   A: finish column j-1 (norm from the last pass's partials, Givens
//      rotation, convergence test; every workgroup forms the same values,
//      workgroup 0 stores them), v_j = w / |w| (own rows), y = Lt v_j,
//      partial dots V_i . y
//   B: reduce A's partials, w = y - sum h1_i V_i, then partial |w|^2, or
//      with two passes partial dots V_i . w        (classical Gram-Schmidt)
//   C: (two passes only) reduce B's partials, w -= sum h2_i V_i, partial
//      |w|^2
// The last column of a chunk of steps is finished by the update kernel that
// follows the chunk (every workgroup forms it, workgroup 0 stores it) before
// it updates the solution if the cycle has ended.  Partial sums
// are reduced in a fixed order by the consuming kernel, so results are
// deterministic.  Once the cycle has converged every later kernel of the
// cycle returns at entry.
#include <type_traits>

#include "internal.h"
#include "gmres.h"
#include "wave_ops.h"

namespace hfr {

namespace {

constexpr int kThr = 512;        // threads per workgroup of the vector kernels
constexpr int kRPT = 4;          // rows per thread (<= 2048 rows per block)

__device__ __forceinline__ double wsum(double v) { return wave_sum(v); }

// Partial sums are stored value-major: partial[i * nb + b] is block b's
// share of value i, so a reader of value i loads consecutive addresses.

// sum of per-thread values over the block for each i < k -> out[i * stride]
// (written by threads 0..k-1); red needs k * (blockDim/64) doubles
template <class F>
__device__ void block_partials(int k, F f, double* red, double* out, int stride) {
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
        out[size_t(i) * stride] = s;
    }
    __syncthreads();
}

// fixed-order sum over blocks of partial[i * nb + b] for i < k -> out[i]
// (LDS); every block computes the same values.  A lane's loads of a pass
// are all issued before the first addition, so one pass costs one memory
// round trip.
__device__ void reduce_partials(int k, int nb, const double* partial, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    for (int i = wave; i < k; i += nw) {
        const double* p = partial + size_t(i) * nb;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        // sixteen loads per lane in flight (up to 1024 partials per pass)
        for (int b = lane; b < nb; b += 1024) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = b + 64 * u < nb ? p[b + 64 * u] : 0.0;
#pragma unroll
            for (int u = 0; u < 16; u += 4) {
                s0 += v[u];
                s1 += v[u + 1];
                s2 += v[u + 2];
                s3 += v[u + 3];
            }
        }
        const double s = wsum((s0 + s1) + (s2 + s3));
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

// LDS copy of what the Givens step of column jc reads (all threads)
struct GivensStage {
    double hc[kGmresMaxK + 1];
    double cs[kGmresMaxK], sn[kGmresMaxK];
    double gj, target, dec[2];
    double gf;               // output: rotated right-hand side of the column
};

__device__ void stage_givens(const GmresArgs& a, int jc, GivensStage& g) {
    const GmresState* gs = a.gs;
    for (int i = threadIdx.x; i <= jc; i += blockDim.x) {
        g.hc[i] = gs->h1[i] + gs->h2[i];
        if (i < jc) {
            g.cs[i] = gs->cs[i];
            g.sn[i] = gs->sn[i];
        }
    }
    if (threadIdx.x == 0) {
        g.gj = gs->g[jc];
        g.target = gs->target;
    }
}

// Givens step of column jc (thread 0 only, after stage_givens and a
// barrier): H column from the two projections and the norm hn, rotations of
// the earlier columns, the new rotation and the residual estimate.
// gs->g[jc] (the running right-hand side) is only read; the rotated value
// goes to gs->gf[jc] and the new running value to gs->g[jc+1], so workgroups
// that form the same column concurrently never read what the writer stores.
// g.dec[0] = done, g.dec[1] = 1/hn.
__device__ void givens_column(const GmresArgs& a, int jc, double hn, bool write,
                              GivensStage& g) {
    GmresState* gs = a.gs;
    const int R = a.restart;
    double* hc = g.hc;
    hc[jc + 1] = hn;
    for (int i = 0; i < jc; ++i) {
        const double t0 = g.cs[i] * hc[i] + g.sn[i] * hc[i + 1];
        hc[i + 1] = -g.sn[i] * hc[i] + g.cs[i] * hc[i + 1];
        hc[i] = t0;
    }
    const double den = sqrt(hc[jc] * hc[jc] + hc[jc + 1] * hc[jc + 1]);
    const double c = den > 0.0 ? hc[jc] / den : 1.0;
    const double sn = den > 0.0 ? hc[jc + 1] / den : 0.0;
    hc[jc] = den;
    hc[jc + 1] = 0.0;
    const double gnext = -sn * g.gj;
    const double res = fabs(gnext);
    const bool done = res <= g.target || !(hn > 0.0) || jc == R - 1 || !(res == res);
    const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
    if (write) {
        double* H = gs->H + size_t(jc) * (R + 1);
        for (int i = 0; i <= jc + 1; ++i) H[i] = hc[i];
        gs->cs[jc] = c;
        gs->sn[jc] = sn;
        gs->gf[jc] = c * g.gj;
        gs->g[jc + 1] = gnext;
        gs->jlast = jc;
        gs->iters += 1;
        gs->inv_norm = inv;
        gs->est_conv = (res <= g.target) ? 1 : 0;
        if (done) gs->done = 1;
    }
    g.dec[0] = done ? 1.0 : 0.0;
    g.dec[1] = inv;
    g.gf = c * g.gj;
}

// Position of entry (a, b) of a bs x bs block of Lt: rows are cut into
// 16-byte pieces (four FP32 or two FP64 entries) and the block holds piece
// 0 of every row, then piece 1, ...
template <typename T>
__device__ __forceinline__ size_t lt_at(int a, int b, int bs) {
    constexpr int CW = 16 / int(sizeof(T));
    return (size_t(b / CW) * bs + a) * CW + (b % CW);
}

// Block-sparse product over rows [r0, r1) of the block's faces: 64 rows at a
// time (up to 8 passes), thread group `part` takes blocks part, part+4, ...
// of a row, the four shares are added in LDS.  Preconditioned blocks (Lt)
// are stored by 16-byte row pieces, piece-major (lt_at), so the lanes of
// consecutive rows read consecutive pieces; column-major blocks (L) are
// read column by column (consecutive lanes read consecutive rows).
// row aa of block p of Lt times x's segment c, added to acc: all loads
// issued before the first FMA (block size fixed at compile time)
template <int BS, typename T>
__device__ __forceinline__ double row_block(const T* M, const double* x, int c, int p,
                                            int aa, double acc) {
    const double2* x2 = reinterpret_cast<const double2*>(x + size_t(c) * BS);
    const T* blk = M + size_t(p) * BS * BS;
    double2 xv[BS / 2];
#pragma unroll
    for (int b = 0; b < BS / 2; ++b) xv[b] = x2[b];
    if constexpr (sizeof(T) == 8) {
        double2 l[BS / 2];
#pragma unroll
        for (int b = 0; b < BS / 2; ++b) l[b] = reinterpret_cast<const double2*>(blk)[b * BS + aa];
#pragma unroll
        for (int b = 0; b < BS / 2; ++b) {
            acc = fma(l[b].x, xv[b].x, acc);
            acc = fma(l[b].y, xv[b].y, acc);
        }
    } else {
        float4 l[BS / 4];
#pragma unroll
        for (int b = 0; b < BS / 4; ++b) l[b] = reinterpret_cast<const float4*>(blk)[b * BS + aa];
#pragma unroll
        for (int b = 0; b < BS / 4; ++b) {
            acc = fma(double(l[b].x), xv[2 * b].x, acc);
            acc = fma(double(l[b].y), xv[2 * b].y, acc);
            acc = fma(double(l[b].z), xv[2 * b + 1].x, acc);
            acc = fma(double(l[b].w), xv[2 * b + 1].y, acc);
        }
    }
    return acc;
}

// The same share for blocks of Lt of size BS through the padded table
// a.ell of the block rows (trace faces, or trace nodes in EFR): {block
// index, block column} of row F's k-th block at F * kmax + k, {-1, -1} past
// its end, so the block and column indices
// are one load away instead of behind the row pointers.  Group `part` takes
// blocks part, part + 4, ... two per pass, all their loads in flight
// together; the additions are those of one block per pass, in the same
// order.  e1, e2: the row's entries part and part + 4, loaded by the caller.
template <typename T, int BS>
__device__ __forceinline__ double row_share_ell(const GmresArgs& a, const T* M,
                                                const double* x, int r, int2 e1, int2 e2) {
    const int F = r / BS, aa = r - F * BS;
    const int2* ell = reinterpret_cast<const int2*>(a.ell) + size_t(F) * a.kmax;
    double acc = 0.0;
    for (int k = threadIdx.x >> 6; e1.x >= 0;) {
        const bool two = e2.x >= 0;
        const int p2 = two ? e2.x : e1.x, c2 = two ? e2.y : e1.y;
        const double a1 = row_block<BS>(M, x, e1.y, e1.x, aa, acc);
        const double a2 = row_block<BS>(M, x, c2, p2, aa, a1);
        acc = two ? a2 : a1;
        k += 8;
        if (!two || k >= a.kmax) break;
        e1 = ell[k];
        e2 = k + 4 < a.kmax ? ell[k + 4] : make_int2(-1, -1);
    }
    return acc;
}

// entries part and part + 4 of block row F in the padded table
__device__ __forceinline__ void ell_pair(const GmresArgs& a, int F, int2& e1, int2& e2) {
    const int part = threadIdx.x >> 6;
    const int2* ell = reinterpret_cast<const int2*>(a.ell) + size_t(F) * a.kmax;
    e1 = part < a.kmax ? ell[part] : make_int2(-1, -1);
    e2 = part + 4 < a.kmax ? ell[part + 4] : make_int2(-1, -1);
}

template <bool ROW_MAJOR, typename T>
__device__ __forceinline__ double row_share(const GmresArgs& a, const T* M,
                                            const double* x, int r, int pb = -1,
                                            int p1 = -1) {
    const int bs = a.bs;
    const int F = r / bs, aa = r - F * bs;
    const int part = threadIdx.x >> 6;
    if (pb < 0) {                                  // row pointers not preloaded
        pb = a.rowptr[F];
        p1 = a.rowptr[F + 1];
    }
    double acc = 0.0;
    for (int p = pb + part; p < p1; p += 4) {
        const double2* x2 = reinterpret_cast<const double2*>(x + size_t(a.col[p]) * bs);
        if (ROW_MAJOR) {                           // Lt: 16-byte pieces, piece-major
            const T* blk = M + size_t(p) * bs * bs;
            if constexpr (sizeof(T) == 8) {
                const double2* l2 = reinterpret_cast<const double2*>(blk);
                for (int b = 0; b < bs / 2; ++b) {
                    const double2 l = l2[b * bs + aa], xv = x2[b];
                    acc = fma(double(l.x), xv.x, acc);
                    acc = fma(double(l.y), xv.y, acc);
                }
            } else {
                const float4* l4 = reinterpret_cast<const float4*>(blk);
                for (int b = 0; b < bs / 4; ++b) {
                    const float4 l = l4[b * bs + aa];
                    const double2 x0 = x2[2 * b], x1 = x2[2 * b + 1];
                    acc = fma(double(l.x), x0.x, acc);
                    acc = fma(double(l.y), x0.y, acc);
                    acc = fma(double(l.z), x1.x, acc);
                    acc = fma(double(l.w), x1.y, acc);
                }
            }
        } else {
            const T* blk = M + size_t(p) * bs * bs + aa;
            const double* xb = x + size_t(a.col[p]) * bs;
            for (int b = 0; b < bs; ++b) acc = fma(double(blk[size_t(b) * bs]), xb[b], acc);
        }
    }
    return acc;
}

}  // namespace

// Each vector-kernel workgroup owns the rows of a.fpb consecutive faces
// (a.nblk <= 256 workgroups of 512 threads).  Product kernels use their own
// decomposition: a.nblkA workgroups of 256 threads owning a.fpbA faces.
// Partial sums go to a partial buffer; the next kernel reduces them in
// every workgroup (fixed order), so no device-scope fences or counters are
// needed.

// ---- A: finish column j-1, scale, product, first projection --------------
// fin_prev: column j-1 was finished by D or by the restart (first step of a
// chunk); otherwise this kernel finishes it.  The product does not depend on
// the scale, so it is formed first.
// TL: the precision of Lt; BS: the face block size (0: a.bs at run time)
template <typename TL, int BS>
__global__ __launch_bounds__(256) void k_arnoldi_a(GmresArgs a, int j, int fin_prev,
                                                   const double* wcur,
                                                   double* wnxt) {
    GmresState* gs = a.gs;
    const int bs = BS > 0 ? BS : a.bs;
    const int f0 = blockIdx.x * a.fpbA, f1 = min(a.ntf, f0 + a.fpbA);
    const int r0 = f0 * bs, r1 = f1 * bs;
    const int part = threadIdx.x >> 6, lr = threadIdx.x & 63;
    // the first pass's table entries (or row pointers) are loaded together
    // with the flag
    int pb0 = 0, pe0 = 0;
    int2 e1 = make_int2(-1, -1), e2 = make_int2(-1, -1);
    if (r0 + lr < r1) {
        const int F0 = (r0 + lr) / bs;
        if constexpr (BS > 0) {
            ell_pair(a, F0, e1, e2);
        } else {
            pb0 = a.rowptr[F0];
            pe0 = a.rowptr[F0 + 1];
        }
    }
    if (gs->done) return;
    __shared__ double red[1];                     // |w| of column j-1
    __shared__ double sacc[8][4][64];
    __shared__ GivensStage gv;
    // the inputs of column j-1's Givens step (its projections, rotations and
    // norm partials) are loaded before the product so that their latency
    // overlaps the product's loads; they are staged in LDS after it
    const int jc = j - 1;
    double ph = 0.0, pcs = 0.0, psn = 0.0, pgj = 0.0, ptg = 0.0;
    double pn[4] = {0.0, 0.0, 0.0, 0.0};
    if (!fin_prev) {
        const int t = threadIdx.x;
        if (t <= jc) {
            ph = gs->h1[t] + gs->h2[t];
            if (t < jc) {
                pcs = gs->cs[t];
                psn = gs->sn[t];
            }
        }
        if (t == 0) {
            pgj = gs->g[jc];
            ptg = gs->target;
        }
        if (part == 0) {                           // wave 0: the norm partials
            int b = lr, q = 0;
            for (; b < a.nblk; b += 64, q = (q + 1) & 3) pn[q] += a.part[b];
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int r = r0 + 64 * q + lr;
        if (r0 + 64 * q >= r1) break;             // uniform
        double acc = 0.0;
        if (r < r1) {
            const TL* Lt;
            if constexpr (sizeof(TL) == 8) Lt = a.Lt64;
            else Lt = a.Lt32;
            if constexpr (BS > 0) {
                if (q > 0) ell_pair(a, r / BS, e1, e2);
                acc = row_share_ell<TL, BS>(a, Lt, wcur, r, e1, e2);
            } else {
                acc = row_share<true>(a, Lt, wcur, r, q == 0 ? pb0 : -1, pe0);
            }
        }
        sacc[q][part][lr] = acc;
    }
    double inv;
    if (fin_prev) {
        inv = gs->inv_norm;
        __syncthreads();
    } else {
        const int t = threadIdx.x;
        if (t <= jc) {
            gv.hc[t] = ph;
            if (t < jc) {
                gv.cs[t] = pcs;
                gv.sn[t] = psn;
            }
        }
        if (t == 0) {
            gv.gj = pgj;
            gv.target = ptg;
        }
        if (part == 0) {
            const double sn = wave_sum((pn[0] + pn[1]) + (pn[2] + pn[3]));
            if (lr == 0) red[0] = sn;
        }
        __syncthreads();
        if (threadIdx.x == 0) givens_column(a, j - 1, sqrt(red[0]), blockIdx.x == 0, gv);
        __syncthreads();
        if (gv.dec[0] != 0.0) return;             // same decision in every workgroup
        inv = gv.dec[1];
    }
    __shared__ double ysh[8][64];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int r = r0 + 64 * q + lr;
        if (part == 0 && r < r1) {
            const double y = (sacc[q][0][lr] + sacc[q][1][lr] + sacc[q][2][lr] +
                              sacc[q][3][lr]) * inv;
            a.V[size_t(j) * a.ldv + r] = wcur[r] * inv;
            wnxt[r] = y;
            ysh[q][lr] = y;
        }
    }
    __syncthreads();
    // projections V_i . y over this block's rows: wave w forms i = w, w + 4,
    // ..., two values per pass so that two loads are in flight, each value
    // a single wave's sum (rows in order, then the wave sum), written to the
    // value-major partials directly
    double* out = a.part3 + blockIdx.x;
    const int ldp = gridDim.x;
    for (int i = part; i <= j; i += 8) {
        const bool two = i + 4 <= j;                  // uniform
        const double* v0 = a.V + size_t(i) * a.ldv;
        const double* v1 = a.V + size_t(two ? i + 4 : i) * a.ldv;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int r = r0 + 64 * q + lr;
            if (r0 + 64 * q >= r1) break;             // uniform
            if (r < r1) {
                const double y = ysh[q][lr];
                s0 += v0[r] * y;
                s1 += v1[r] * y;
            }
        }
        s0 = wsum(s0);
        s1 = wsum(s1);
        if (lr == 0) {
            out[size_t(i) * ldp] = s0;
            if (two) out[size_t(i + 4) * ldp] = s1;
        }
    }
}

// ---- y = Lt x alone: the block-row product of the Arnoldi kernel A (same
// decomposition, padded table, pass structure and order of additions),
// without the Givens step, scaling and projections (inspection) ---------------
template <typename TL, int BS>
__global__ __launch_bounds__(256) void k_block_product(GmresArgs a, const double* x,
                                                       double* y) {
    const int f0 = blockIdx.x * a.fpbA, f1 = min(a.ntf, f0 + a.fpbA);
    const int r0 = f0 * BS, r1 = f1 * BS;
    const int part = threadIdx.x >> 6, lr = threadIdx.x & 63;
    __shared__ double sacc[8][4][64];
    const TL* Lt;
    if constexpr (sizeof(TL) == 8) Lt = a.Lt64;
    else Lt = a.Lt32;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int r = r0 + 64 * q + lr;
        if (r0 + 64 * q >= r1) break;             // uniform
        double acc = 0.0;
        if (r < r1) {
            int2 e1, e2;
            ell_pair(a, r / BS, e1, e2);
            acc = row_share_ell<TL, BS>(a, Lt, x, r, e1, e2);
        }
        sacc[q][part][lr] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int r = r0 + 64 * q + lr;
        if (part == 0 && r < r1)
            y[r] = sacc[q][0][lr] + sacc[q][1][lr] + sacc[q][2][lr] + sacc[q][3][lr];
    }
}

// ---- B: first orthogonalisation, second projection ------------------------
__global__ __launch_bounds__(kThr) void k_arnoldi_b(GmresArgs a, int j,
                                                    double* w) {
    GmresState* gs = a.gs;
    const int k = j + 1;
    int r0, r1;
    block_rows(a, r0, r1);
    // the first row's w and up to NPF basis entries are loaded before the
    // flag and the reduction of the projections, which they do not need
    constexpr int NPF = 8;
    const int rf = r0 + threadIdx.x;
    double wf = 0.0, vf[NPF];
#pragma unroll
    for (int i = 0; i < NPF; ++i) vf[i] = 0.0;
    if (rf < r1) {
        wf = w[rf];
#pragma unroll
        for (int i = 0; i < NPF; ++i)
            if (i < k) vf[i] = a.V[size_t(i) * a.ldv + rf];
    }
    const int done = gs->done;
    if (blockIdx.x == 0 && threadIdx.x == 0) gs->done_pre = done;
    if (done) return;
    __shared__ double red[kGmresMaxK * (kThr / 64)];
    __shared__ double h[kGmresMaxK];
    reduce_partials(k, a.nblkA, a.part3, h);
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < k; i += blockDim.x) gs->h1[i] = h[i];
    double x[kRPT];
#pragma unroll
    for (int q = 0; q < kRPT; ++q) {
        const int r = r0 + threadIdx.x + kThr * q;
        x[q] = 0.0;
        if (r < r1) {
            double v;
            int i = 0;
            if (q == 0) {
                v = wf;
#pragma unroll
                for (; i < NPF; ++i)
                    if (i < k) v -= h[i] * vf[i];
                i = k < NPF ? k : NPF;
            } else {
                v = w[r];
            }
            for (; i < k; ++i) v -= h[i] * a.V[size_t(i) * a.ldv + r];
            w[r] = v;
            x[q] = v;
        }
    }
    if (a.passes == 1) {
        // one pass: the norm partials of w here, no second projection
        if (blockIdx.x == 0)
            for (int i = threadIdx.x; i < k; i += blockDim.x) gs->h2[i] = 0.0;
        double nn = 0.0;
#pragma unroll
        for (int q = 0; q < kRPT; ++q) nn += x[q] * x[q];
        block_partials(1, [&](int) { return nn; }, red, a.part + blockIdx.x, gridDim.x);
        return;
    }
    block_partials(k, [&](int i) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < kRPT; ++q) {
            const int r = r0 + threadIdx.x + kThr * q;
            if (r < r1) s += a.V[size_t(i) * a.ldv + r] * x[q];
        }
        return s;
    }, red, a.part2 + blockIdx.x, gridDim.x);
}

// ---- C: second orthogonalisation, norm partials --------------------------
__global__ __launch_bounds__(kThr) void k_arnoldi_c(GmresArgs a, int j,
                                                    double* w) {
    GmresState* gs = a.gs;
    if (gs->done) return;
    __shared__ double red[kGmresMaxK * (kThr / 64)];
    __shared__ double h[kGmresMaxK];
    const int k = j + 1;
    reduce_partials(k, gridDim.x, a.part2, h);
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
    block_partials(1, [&](int) { return nn; }, red, a.part + blockIdx.x, gridDim.x);
}

// ---- end of a chunk: finish its last column; at the end of a cycle
// y = H^-1 g, x += Dinv (V y) ---------------------------------------------------
// jfin >= 0: column jfin (the chunk's last step) is finished first, unless
// the cycle had already ended at an earlier step (gs->done_pre, written by
// the last orthogonalisation kernel: gs->done itself may be set during this
// launch by workgroup 0).  Every workgroup forms the column's Givens step,
// workgroup 0 stores it, and the others take the column and its rotated
// right-hand side from their own copy, not from gs.
// cond: only when the cycle has ended, else return after the column
__global__ __launch_bounds__(kThr) void k_gmres_update(GmresArgs a, double* x, int cond,
                                                       int jfin) {
    GmresState* gs = a.gs;
    __shared__ double y[kGmresMaxK];
    __shared__ double z[kThr];
    __shared__ double Hs[kGmresMaxK * kGmresMaxK];
    __shared__ double fin[kGmresMaxK];
    __shared__ GivensStage gv;
    int done, jl;
    bool own = false;                              // column jl formed here
    if (jfin >= 0 && gs->done_pre == 0) {          // uniform
        stage_givens(a, jfin, gv);
        reduce_partials(1, a.nblk, a.part, fin);   // ends with a barrier
        if (threadIdx.x == 0) givens_column(a, jfin, sqrt(fin[0]), blockIdx.x == 0, gv);
        __syncthreads();
        done = gv.dec[0] != 0.0 ? 1 : 0;
        jl = jfin;
        own = true;
    } else {
        done = gs->done;                           // not written by this launch
        jl = gs->jlast;
    }
    if (cond && !done) return;
    if (jl < 0) return;
    const int R = a.restart;
    const int n = jl + 1;
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
        const int k = t / n, i = t - k * n;       // column k, row i
        Hs[t] = (own && k == jl) ? gv.hc[i] : gs->H[size_t(k) * (R + 1) + i];
    }
    for (int t = threadIdx.x; t < n; t += blockDim.x)
        y[t] = (own && t == jl) ? gv.gf : gs->gf[t];
    __syncthreads();
    // back substitution H y = gf on wave 0 (n <= 64), column by column from
    // the last: lane k finishes y[k], which is broadcast, and every lane
    // t < k subtracts H[t][k] y[k]
    if (threadIdx.x < 64) {
        const int t = threadIdx.x;
        double yt = t <= jl ? y[t] : 0.0;
        for (int k = jl; k >= 0; --k) {
            const double yk = lane_value(yt / Hs[k * n + k], k);
            if (t == k) yt = yk;
            else if (t < k) yt = fma(-Hs[k * n + t], yk, yt);
        }
        if (t <= jl) y[t] = yt;
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
        if (act) {
            // four basis vectors per pass, their loads issued together
            int i = 0;
            for (; i + 3 <= jl; i += 4) {
                const double* v = a.V + size_t(i) * a.ldv + r;
                const double v0 = v[0], v1 = v[a.ldv], v2 = v[2 * a.ldv], v3 = v[3 * a.ldv];
                zz += y[i] * v0;
                zz += y[i + 1] * v1;
                zz += y[i + 2] * v2;
                zz += y[i + 3] * v3;
            }
            for (; i <= jl; ++i) zz += y[i] * a.V[size_t(i) * a.ldv + r];
        }
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

// (L x)_r summed from the element Schur sub-blocks: every block (F, G) of
// row F as the assembly forms it (the one or two element contributions,
// each side's points in its own order), the part-th blocks of the row
__device__ __forceinline__ double row_share_elem(const GmresArgs& a, const double* x, int r) {
    const int bs = a.bs, P = bs / 4;
    const int F = r / bs, aa = r - F * bs, qa = aa >> 2;
    const int part = threadIdx.x >> 6;
    const size_t N = size_t(a.nloc + a.mloc);
    double acc = 0.0;
    for (int p = a.rowptr[F] + part; p < a.rowptr[F + 1]; p += 4) {
        const double* xg = x + size_t(a.col[p]) * bs;
        for (int c = 0; c < 2; ++c) {
            const int* ct = a.econtrib + (size_t(p) * 2 + c) * 3;
            const int imp = ct[0];
            if (imp < 0) continue;
            const int lr = ct[1] >> 1, sr = ct[1] & 1, lc = ct[2] >> 1, sc = ct[2] & 1;
            const int ra = (sr ? P - 1 - qa : qa) * 4 + (aa & 3);
            const size_t base = size_t(imp) * N * N + schur_offset(bs, lr, lc, ra, 0);
            for (int cc = 0; cc < bs; ++cc) {
                const int qb = cc >> 2;
                const size_t o = base + size_t((sc ? P - 1 - qb : qb) * 4 + (cc & 3)) * bs;
                const double v = a.el64 ? reinterpret_cast<const double*>(a.Mel)[o]
                                        : double(reinterpret_cast<const float*>(a.Mel)[o]);
                acc = fma(v, xg[cc], acc);
            }
        }
    }
    return acc;
}

// ---- restart: r = t - L x (FP64), partial |r|^2 ---------------------------
// Product decomposition of A (a.nblkA workgroups of 256 threads).
// first: x is zeroed here (the solve starts from zero), r = t
__global__ __launch_bounds__(256) void k_gmres_residual(GmresArgs a,
                                                        double* x,
                                                        double* w, int first, int cond) {
    if (cond && !a.gs->done) return;
    if (cond && !a.verify && a.gs->est_conv) return;  // the estimate is trusted
    __shared__ double red[4];
    __shared__ double sacc[8][4][64];
    const int bs = a.bs;
    const int f0 = blockIdx.x * a.fpbA, f1 = min(a.ntf, f0 + a.fpbA);
    const int r0 = f0 * bs, r1 = f1 * bs;
    const int part = threadIdx.x >> 6, lr = threadIdx.x & 63;
    if (!first) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int r = r0 + 64 * q + lr;
            if (r0 + 64 * q >= r1) break;         // uniform
            double acc = 0.0;
            if (r < r1)
                acc = a.L64 ? row_share<false>(a, a.L64, x, r)
                      : a.L32 ? row_share<false>(a, a.L32, x, r)
                              : row_share_elem(a, x, r);
            sacc[q][part][lr] = acc;
        }
        __syncthreads();
    }
    double nn = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int r = r0 + 64 * q + lr;
        if (part == 0 && r < r1) {
            const double lx = first ? 0.0 : (sacc[q][0][lr] + sacc[q][1][lr] +
                                             sacc[q][2][lr] + sacc[q][3][lr]);
            const double v = a.t[r] - lx;
            if (first) x[r] = 0.0;
            w[r] = v;
            nn += v * v;
        }
    }
    block_partials(1, [&](int) { return nn; }, red, a.part3 + blockIdx.x, gridDim.x);
}

// beta = |r|, new cycle (one workgroup)
__global__ __launch_bounds__(kThr) void k_gmres_restart(GmresArgs a, int first, int cond,
                                                        int cap) {
    GmresState* gs = a.gs;
    __shared__ double fin[kGmresMaxK];
    const bool act = !cond || gs->done;            // uniform
    if (!act && threadIdx.x == 0) gs->finished = 0;
    if (act && cond && !a.verify && gs->est_conv) {
        // the cycle reached the target by its residual estimate: the solve
        // ends with that estimate as its residual (no true residual formed)
        if (threadIdx.x == 0) {
            gs->cycles += 1;
            gs->beta = fabs(gs->g[gs->jlast + 1]);
            gs->converged = 1;
            gs->done = 1;
            gs->finished = 1;
        }
    } else if (act) {
        reduce_partials(1, a.nblkA, a.part3, fin);
        if (threadIdx.x == 0) {
            const double beta = sqrt(fin[0]);
            if (first) {
                gs->bnorm = beta;
                gs->target = (a.eta ? *a.eta : a.rtol) * beta;
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
            gs->est_conv = 0;
            const bool conv = !(beta > gs->target);
            gs->converged = conv ? 1 : 0;
            gs->done = (conv || !(beta == beta)) ? 1 : 0;
            gs->finished = (conv || cap || !(beta == beta)) ? 1 : 0;
        }
    }
    // the state the host reads after a chunk, in host-visible memory
    if (threadIdx.x == 0 && a.pub) {
        GmresPublish* p = reinterpret_cast<GmresPublish*>(a.pub);
        p->done = gs->done;
        p->converged = gs->converged;
        p->jlast = gs->jlast;
        p->iters = gs->iters;
        p->cycles = gs->cycles;
        p->finished = gs->finished;
        p->inv_norm = gs->inv_norm;
        p->beta = gs->beta;
        p->bnorm = gs->bnorm;
        p->target = gs->target;
        const long long seq = gs->pub_seq + 1;
        gs->pub_seq = seq;
        __threadfence_system();
        *reinterpret_cast<volatile long long*>(&p->seq) = seq;
    }
}

// four consecutive entries as one 16-byte access (FP32) or two (FP64)
template <typename T> struct Vec4Load;
template <> struct Vec4Load<float> {
    __device__ static void get(const float* p, double (&v)[4]) {
        const float4 x = *reinterpret_cast<const float4*>(p);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    }
    __device__ static void put(float* p, const double (&v)[4]) {
        *reinterpret_cast<float4*>(p) = make_float4(float(v[0]), float(v[1]), float(v[2]), float(v[3]));
    }
    __device__ static void copy(float* d, const float* s) {
        *reinterpret_cast<float4*>(d) = *reinterpret_cast<const float4*>(s);
    }
};
template <> struct Vec4Load<double> {
    __device__ static void get(const double* p, double (&v)[4]) {
        const double2 x = reinterpret_cast<const double2*>(p)[0];
        const double2 y = reinterpret_cast<const double2*>(p)[1];
        v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
    }
    __device__ static void put(double* p, const double (&v)[4]) {
        reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
        reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
    }
    __device__ static void copy(double* d, const double* s) {
        reinterpret_cast<double2*>(d)[0] = reinterpret_cast<const double2*>(s)[0];
        reinterpret_cast<double2*>(d)[1] = reinterpret_cast<const double2*>(s)[1];
    }
};

__device__ __forceinline__ double load_pc(const double* d, size_t i) { return d[i]; }
__device__ __forceinline__ double load_pc(const float* d, size_t i) { return double(d[i]); }
__device__ __forceinline__ double load_pc(const uint16_t* d, size_t i) {
    return double(__uint_as_float(uint32_t(d[i]) << 16));     // BF16 -> FP32
}
// four consecutive preconditioner entries (16, 32 or 8 bytes, aligned)
__device__ __forceinline__ void load4_pc(const double* d, double (&v)[4]) {
    Vec4Load<double>::get(d, v);
}
__device__ __forceinline__ void load4_pc(const float* d, double (&v)[4]) {
    Vec4Load<float>::get(d, v);
}
__device__ __forceinline__ void load4_pc(const uint16_t* d, double (&v)[4]) {
    const uint2 x = *reinterpret_cast<const uint2*>(d);
    v[0] = double(__uint_as_float(x.x << 16));
    v[1] = double(__uint_as_float(x.x & 0xffff0000u));
    v[2] = double(__uint_as_float(x.y << 16));
    v[3] = double(__uint_as_float(x.y & 0xffff0000u));
}

// ---- Lt = L Dinv (per block: Lt_FG = L_FG Dinv_G) -------------------------
// One wave per block, four blocks per workgroup; both factors staged in LDS
// (FP64, Dinv transposed), each lane forms BS*BS/64 entries of the product.
// L and Dinv are column-major per block; Lt is written by 16-byte row pieces (lt_at).
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
        const int b = i / BS, c = i - b * BS;     // Dinv entry (c, b)
        sL[wv][i] = double(L[lb + i]);
        sD[wv][c * BS + b] = load_pc(Dinv, db + i);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // entry (a, b) of the product, stored at a*BS + b: sum_c L[a][c] Dinv[c][b]
    for (int i = lane; i < BB; i += 64) {
        const int a = i / BS, b = i - a * BS;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < BS; ++c) acc = fma(sL[wv][c * BS + a], sD[wv][c * BS + b], acc);
        Lt[lb + lt_at<TL>(a, b, BS)] = TL(acc);
    }
}

// bs = 4 (the node blocks of the interior-embedded trace): one thread per
// block row, the same FP64 sums in the same order as k_precondition_matrix;
// the four threads of a block read its 16 entries of L and of Dinv together
// and the row leaves as one 16-byte (FP32) or two (FP64) stores.
template <typename TL, typename TD>
__global__ __launch_bounds__(256) void k_precondition_matrix4(int nblocks, const int* col,
                                                              const TL* L, const TD* Dinv,
                                                              TL* Lt) {
    const long t = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= 4 * long(nblocks)) return;
    const int p = int(t >> 2), a = int(t & 3);
    const size_t lb = size_t(p) * 16, db = size_t(col[p]) * 16;
    double l[4], d[16];
#pragma unroll
    for (int c = 0; c < 4; ++c) l[c] = double(L[lb + 4 * c + a]);
#pragma unroll
    for (int i = 0; i < 16; ++i) d[i] = load_pc(Dinv, db + i);   // Dinv(c, b) at 4 b + c
    double acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        acc[b] = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[b] = fma(l[c], d[4 * b + c], acc[b]);
    }
    if constexpr (sizeof(TL) == 4) {                // one piece: the row
        *reinterpret_cast<float4*>(Lt + lb + lt_at<float>(a, 0, 4)) =
            make_float4(float(acc[0]), float(acc[1]), float(acc[2]), float(acc[3]));
    } else {                                       // pieces (a, 0..1) and (a, 2..3)
        *reinterpret_cast<double2*>(Lt + lb + lt_at<double>(a, 0, 4)) = make_double2(acc[0], acc[1]);
        *reinterpret_cast<double2*>(Lt + lb + lt_at<double>(a, 2, 4)) = make_double2(acc[2], acc[3]);
    }
}

// bs = 16: the same product on 16x16x4 matrix-core tiles, one wave per
// block, K = 16 in four steps.  Operands: lane l = 16 g + i holds
// L(i, 4kk + g) (a contiguous 64-value slice of the column-major block) and
// Dinv(4kk + g, i); the FP32 result holds Lt(4g + r, i) in register r, the
// FP64 result Lt(g + 4r, i).
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));
template <typename TL, typename TD>
__global__ __launch_bounds__(256) void k_precondition_matrix16(int nblocks, const int* col,
                                                               const TL* L, const TD* Dinv,
                                                               TL* Lt) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int p = blockIdx.x * 4 + wv;
    if (p >= nblocks) return;                      // whole wave
    const size_t lb = size_t(p) * 256;
    // the A operands (block p of L) are loaded first: they depend on
    // nothing, while the Dinv block waits for its column index
    TL av[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) av[kk] = L[lb + 64 * kk + lane];
    const size_t db = size_t(col[p]) * 256;
    const int i = lane & 15, g = lane >> 4;
    // the column face's Dinv block, read with consecutive lanes on
    // consecutive entries and staged in LDS with a row stride of 17 (the
    // operand reads below then hit 16 different banks)
    __shared__ TL dsh[4][16 * 17];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = lane + 64 * q, c = e >> 4, r = e & 15;
        dsh[wv][c * 17 + r] = TL(load_pc(Dinv, db + e));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if constexpr (sizeof(TL) == 4) {
        mf4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const float b = dsh[wv][i * 17 + 4 * kk + g];
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk], b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) Lt[lb + lt_at<TL>(4 * g + r, i, 16)] = acc[r];
    } else {
        md4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const double b = dsh[wv][i * 17 + 4 * kk + g];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk], b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) Lt[lb + lt_at<TL>(g + 4 * r, i, 16)] = acc[r];
    }
}

// Assembly and preconditioning in one pass (eq:assembly, then Lt = L Dinv)
// for block sizes 16, 20 and 24: each wave gathers its block of L from the at
// most two element Schur blocks in the tableaux (as the assembly does: four
// rows of one column per 16-byte read, the sum formed in FP64 and rounded
// once), stores it, stages it in LDS and multiplies it by the column face's
// inverse diagonal block on 16x16 tiles (one, or 2 x 2 zero-padded: rows
// and columns 0..15 and 16..BS-1; K = BS in BS/4 steps of 16x16x4), so L is
// read from the tableaux once instead of being written, read back and
// multiplied.  The diagonal blocks and their
// inverses must already exist (assembled and inverted first); their L
// blocks are rewritten with the same values.
template <int BS, int P, typename TL, typename TD, bool CM>
__global__ __launch_bounds__(256) void k_assemble_precondition(AssembleLaunch a, const int* col,
                                                               const TD* Dinv, TL* Lout,
                                                               TL* Lt) {
    static_assert(BS == 4 * P && BS >= 16 && BS <= 32, "one or 2 x 2 tiles of 16");
    constexpr int BB = BS * BS, KC = BS / 4, CH = BS * P;   // 4-row pieces per block
    constexpr int NT = BS > 16 ? 2 : 1;            // 16x16 tiles per block side
    constexpr int Q = BB / 4;                      // 4-entry pieces of a block
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __shared__ __align__(16) TL lsh[4][BB];        // L (column-major), then Lt (row-major)
    __shared__ __align__(16) TL dsh[4][BB];        // Dinv (column-major)
    const int i = lane & 15, g = lane >> 4;
    const size_t N = size_t(a.n + a.m);
    const TL* M = reinterpret_cast<const TL*>(a.M);
    // column mode (a.tcol): the workgroup owns block column G = blockIdx.x,
    // its Dinv staged once in LDS for the four waves, which take the
    // column's blocks k = wv, wv + 4, ...; row mode: one block per wave,
    // the wave stages its column face's Dinv itself
    constexpr bool cm = CM;                         // a.tcol given
    if constexpr (cm) {
        const size_t db = size_t(blockIdx.x) * BB;
        for (int e = threadIdx.x; e < Q; e += blockDim.x) {
            double v[4];
            load4_pc(Dinv + db + 4 * size_t(e), v);
            Vec4Load<TL>::put(&dsh[0][4 * e], v);
        }
        __syncthreads();
    }
    auto one_block = [&](const int p, const int ds) {   // ds: the dsh slot holding Dinv
    const size_t lb = size_t(p) * BB;
    if constexpr (!cm) {
        // the column face's Dinv block does not depend on the gather: issued first
        const size_t db = size_t(col[p]) * BB;
#pragma unroll
        for (int e0 = 0; e0 < Q; e0 += 64) {
            const int e = e0 + lane;
            if (e < Q) {
                double v[4];
                load4_pc(Dinv + db + 4 * size_t(e), v);
                Vec4Load<TL>::put(&dsh[ds][4 * e], v);
            }
        }
    }
    int imp[2], lr[2], sr[2], lc[2], sc[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int* ct = a.blk_contrib + (size_t(p) * 2 + c) * 3;
        imp[c] = ct[0];
        lr[c] = ct[1] >> 1;
        sr[c] = ct[1] & 1;
        lc[c] = ct[2] >> 1;
        sc[c] = ct[2] & 1;
    }
    // piece e: column b = e / P, rows 4 qa .. 4 qa + 3 with qa = e mod P
#pragma unroll
    for (int e0 = 0; e0 < CH; e0 += 64) {
        const int e = e0 + lane;
        if (e < CH) {
            const int b = e / P, qa = e - b * P, qb = b >> 2, wb = b & 3;
            double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (imp[c] < 0) continue;
                const int ra = (sr[c] ? P - 1 - qa : qa) * 4;            // rows in face lr
                const int cb = (sc[c] ? P - 1 - qb : qb) * 4 + wb;       // column in face lc
                const size_t row = size_t(a.n) + lr[c] * 4 * P + ra;
                const size_t cl = size_t(a.n) + lc[c] * 4 * P + cb;
                double w[4];
                Vec4Load<TL>::get(M + size_t(imp[c]) * N * N +
                                      (a.compact_schur ? schur_offset(BS, lr[c], lc[c], ra, cb)
                                                       : cl * N + row),
                                  w);
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] += w[r];
            }
            TL* dst = &lsh[wv][b * BS + 4 * qa];
            if (Lout) Vec4Load<TL>::put(Lout + lb + size_t(b) * BS + 4 * qa, v);
            Vec4Load<TL>::put(dst, v);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // A operands L(16 ti + i, 4 kk + g), B operands Dinv(4 kk + g, 16 tj + i);
    // rows and columns past BS are zero
    TL av[NT][KC], bv[NT][KC];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            const int x = 16 * t + i;
            const TL va = lsh[wv][(4 * kk + g) * BS + min(x, BS - 1)];
            const TL vb = dsh[ds][min(x, BS - 1) * BS + 4 * kk + g];
            av[t][kk] = x < BS ? va : TL(0);
            bv[t][kk] = x < BS ? vb : TL(0);
        }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the product tiles go to LDS row-major and leave as 16-byte pieces
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) {
            if constexpr (sizeof(TL) == 4) {
                mf4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kk = 0; kk < KC; ++kk)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ti][kk], bv[tj][kk], acc, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ar = 16 * ti + 4 * g + r, b = 16 * tj + i;
                    if (ar < BS && b < BS) lsh[wv][ar * BS + b] = acc[r];
                }
            } else {
                md4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < KC; ++kk)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ti][kk], bv[tj][kk], acc, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ar = 16 * ti + g + 4 * r, b = 16 * tj + i;
                    if (ar < BS && b < BS) lsh[wv][ar * BS + b] = acc[r];
                }
            }
        }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // piece e of Lt: 16 bytes of row e mod BS at piece e div BS
    constexpr int CW = 16 / int(sizeof(TL)), QW = BB / CW;
#pragma unroll
    for (int e0 = 0; e0 < QW; e0 += 64) {
        const int e = e0 + lane;
        if (e < QW) {
            const int c = e / BS, ar = e - c * BS;
            *reinterpret_cast<float4*>(Lt + lb + size_t(e) * CW) =
                *reinterpret_cast<const float4*>(&lsh[wv][ar * BS + c * CW]);
        }
    }
    };
    if constexpr (cm) {
        const int* tc = a.tcol + size_t(blockIdx.x) * a.kmax;
        for (int k = wv; k < a.kmax; k += 4) {
            const int p = tc[k];
            if (p < 0) break;                      // uniform over the wave
            one_block(p, 0);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();       // lsh[wv] free for the next block
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    } else {
        const int p = blockIdx.x * 4 + wv;
        if (p < a.nblocks) one_block(p, wv);
    }
}

template <int BS, int P, typename TL, bool CM>
static void launch_ap_pc(const AssembleLaunch& a, dim3 grid, const int* col, int pc,
                         const void* Dinv, TL* Lout, TL* Lt, hipStream_t st) {
    const dim3 blk(256);
    if (pc == HFR_PC_FP64)
        hipLaunchKernelGGL((k_assemble_precondition<BS, P, TL, double, CM>), grid, blk, 0, st,
                           a, col, reinterpret_cast<const double*>(Dinv), Lout, Lt);
    else if (pc == HFR_PC_FP32)
        hipLaunchKernelGGL((k_assemble_precondition<BS, P, TL, float, CM>), grid, blk, 0, st,
                           a, col, reinterpret_cast<const float*>(Dinv), Lout, Lt);
    else
        hipLaunchKernelGGL((k_assemble_precondition<BS, P, TL, uint16_t, CM>), grid, blk, 0,
                           st, a, col, reinterpret_cast<const uint16_t*>(Dinv), Lout, Lt);
}

template <int P, typename TL>
static void launch_ap_t(const AssembleLaunch& a0, const int* col, int pc, const void* Dinv,
                        TL* Lout, TL* Lt, hipStream_t st) {
    constexpr int BS = 4 * P;
    // by block column only for FP32/BF16 L, where the Dinv re-reads are the
    // traffic saved; FP64 L keeps one block per wave (a column's blocks
    // spread unevenly over four waves)
    constexpr bool CM = !std::is_same<TL, double>::value;
    AssembleLaunch a = a0;
    if (!CM) a.tcol = nullptr;
    const dim3 grid(a.tcol ? a.ntf : (a.nblocks + 3) / 4), blk(256);
    if (a.tcol) {
        if constexpr (CM) launch_ap_pc<BS, P, TL, true>(a, grid, col, pc, Dinv, Lout, Lt, st);
    } else {
        launch_ap_pc<BS, P, TL, false>(a, grid, col, pc, Dinv, Lout, Lt, st);
    }
}

bool assemble_precondition_fused(int P) { return P == 4 || P == 5 || P == 6; }

hipError_t launch_assemble_precondition(const AssembleLaunch& a, const int* col, int pc,
                                        const void* Dinv, double* Lt64, float* Lt32,
                                        hipStream_t st) {
    if (a.nblocks == 0) return hipSuccess;
    if (!assemble_precondition_fused(a.P) || a.blk_list) return hipErrorInvalidValue;
    const bool f64 = a.precision == HFR_PREC_FP64;
    // L itself is written only where given (a.L64 / a.L32; Lt always)
    if (f64 ? !Lt64 : !Lt32) return hipErrorInvalidValue;
    if (a.P == 4) {
        if (f64) launch_ap_t<4, double>(a, col, pc, Dinv, a.L64, Lt64, st);
        else launch_ap_t<4, float>(a, col, pc, Dinv, a.L32, Lt32, st);
    } else if (a.P == 5) {
        if (f64) launch_ap_t<5, double>(a, col, pc, Dinv, a.L64, Lt64, st);
        else launch_ap_t<5, float>(a, col, pc, Dinv, a.L32, Lt32, st);
    } else {
        if (f64) launch_ap_t<6, double>(a, col, pc, Dinv, a.L64, Lt64, st);
        else launch_ap_t<6, float>(a, col, pc, Dinv, a.L32, Lt32, st);
    }
    return hipGetLastError();
}

template <int BS, typename TL>
static void launch_pm_t(int nblocks, const int* col, const TL* L, int pc,
                        const void* Dinv, TL* Lt, hipStream_t st) {
    const dim3 grid((nblocks + 3) / 4), blk(256);
    if constexpr (BS == 4) {
        const dim3 g4((4 * long(nblocks) + 255) / 256);
        if (pc == HFR_PC_FP64)
            hipLaunchKernelGGL((k_precondition_matrix4<TL, double>), g4, blk, 0, st, nblocks,
                               col, L, reinterpret_cast<const double*>(Dinv), Lt);
        else if (pc == HFR_PC_FP32)
            hipLaunchKernelGGL((k_precondition_matrix4<TL, float>), g4, blk, 0, st, nblocks,
                               col, L, reinterpret_cast<const float*>(Dinv), Lt);
        else
            hipLaunchKernelGGL((k_precondition_matrix4<TL, uint16_t>), g4, blk, 0, st,
                               nblocks, col, L, reinterpret_cast<const uint16_t*>(Dinv), Lt);
        return;
    }
    if constexpr (BS == 16) {
        if (pc == HFR_PC_FP64)
            hipLaunchKernelGGL((k_precondition_matrix16<TL, double>), grid, blk, 0, st, nblocks,
                               col, L, reinterpret_cast<const double*>(Dinv), Lt);
        else if (pc == HFR_PC_FP32)
            hipLaunchKernelGGL((k_precondition_matrix16<TL, float>), grid, blk, 0, st, nblocks,
                               col, L, reinterpret_cast<const float*>(Dinv), Lt);
        else
            hipLaunchKernelGGL((k_precondition_matrix16<TL, uint16_t>), grid, blk, 0, st,
                               nblocks, col, L, reinterpret_cast<const uint16_t*>(Dinv), Lt);
        return;
    }
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
        // 20 and 24: assembled and preconditioned together
        // (launch_assemble_precondition)
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

hipError_t launch_gmres_restart(const GmresArgs& a, double* x,
                                double* w, int first, int cond, int cap,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_gmres_residual, dim3(a.nblkA), dim3(256), 0, st, a, x,
                       w, first, cond);
    hipLaunchKernelGGL(k_gmres_restart, dim3(1), dim3(kThr), 0, st, a, first, cond, cap);
    return hipGetLastError();
}

hipError_t launch_arnoldi_product(const GmresArgs& a, int j, int fin_prev,
                                  const double* wcur, double* wnxt, hipStream_t st) {
    const bool f64 = a.Lt64 != nullptr;
#define HFR_AA(TL, B)                                                                   \
    hipLaunchKernelGGL((k_arnoldi_a<TL, B>), dim3(a.nblkA), dim3(256), 0, st, a, j,      \
                       fin_prev, wcur, wnxt)
    switch (a.bs) {
        case 4: if (f64) HFR_AA(double, 4); else HFR_AA(float, 4); break;
        case 8: if (f64) HFR_AA(double, 8); else HFR_AA(float, 8); break;
        case 12: if (f64) HFR_AA(double, 12); else HFR_AA(float, 12); break;
        case 16: if (f64) HFR_AA(double, 16); else HFR_AA(float, 16); break;
        case 20: if (f64) HFR_AA(double, 20); else HFR_AA(float, 20); break;
        case 24: if (f64) HFR_AA(double, 24); else HFR_AA(float, 24); break;
        default: if (f64) HFR_AA(double, 0); else HFR_AA(float, 0); break;
    }
#undef HFR_AA
    return hipGetLastError();
}

hipError_t launch_block_product(const GmresArgs& a, const double* x, double* y,
                                hipStream_t st) {
    if (a.ntf == 0) return hipSuccess;
    const bool f64 = a.Lt64 != nullptr;
#define HFR_BP(TL, B)                                                                   \
    hipLaunchKernelGGL((k_block_product<TL, B>), dim3(a.nblkA), dim3(256), 0, st, a, x, y)
    switch (a.bs) {
        case 4: if (f64) HFR_BP(double, 4); else HFR_BP(float, 4); break;
        case 8: if (f64) HFR_BP(double, 8); else HFR_BP(float, 8); break;
        case 12: if (f64) HFR_BP(double, 12); else HFR_BP(float, 12); break;
        case 16: if (f64) HFR_BP(double, 16); else HFR_BP(float, 16); break;
        case 20: if (f64) HFR_BP(double, 20); else HFR_BP(float, 20); break;
        case 24: if (f64) HFR_BP(double, 24); else HFR_BP(float, 24); break;
        default: return hipErrorInvalidValue;
    }
#undef HFR_BP
    return hipGetLastError();
}

hipError_t launch_arnoldi_orth(const GmresArgs& a, int j, double* wnxt,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_arnoldi_b, dim3(a.nblk), dim3(kThr), 0, st, a, j, wnxt);
    if (a.passes != 1)
        hipLaunchKernelGGL(k_arnoldi_c, dim3(a.nblk), dim3(kThr), 0, st, a, j, wnxt);
    return hipGetLastError();
}

hipError_t launch_gmres_update(const GmresArgs& a, double* x, int cond, int jfin,
                               hipStream_t st) {
    // one sub-chunk of faces per workgroup (the update writes no partial
    // sums, so its decomposition is free; it reads a.nblk partials)
    GmresArgs u = a;
    u.fpb = std::max(1, kThr / a.bs);
    const int grid = std::max(1, (a.ntf + u.fpb - 1) / u.fpb);
    hipLaunchKernelGGL(k_gmres_update, dim3(grid), dim3(kThr), 0, st, u, x, cond, jfin);
    return hipGetLastError();
}

}  // namespace hfr
