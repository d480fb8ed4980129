// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include <cstdint>
#include <string>
#include <vector>

#include "hfr_imex.h"

namespace hfr {

constexpr int kMaxP = FR_MAX_ORDER + 1;  // points per direction

// One-dimensional reference operators on P Gauss-Legendre points, passed
// to kernels by value (kernel-argument segment, read through scalar loads).
struct RefOps {
    int P;
    double x[kMaxP], w[kMaxP];
    double D[kMaxP * kMaxP];       // D[i*P+l] = l_l'(x_i)
    double lm[kMaxP], lp[kMaxP];   // l_j(-1), l_j(+1)
    double cl[kMaxP], cr[kMaxP];   // correction divergences (DG lifting)
    // interior-embedded trace: GLL nodes on a face, the GLL basis at the
    // Gauss flux points gi[q*P+i] = phi_i(x_q), and the Gauss-point basis at
    // the GLL nodes gj[i*P+q] = l_q(xg_i)
    double xg[kMaxP];
    double gi[kMaxP * kMaxP], gj[kMaxP * kMaxP];
};

// Copy of the operator table (a kernel argument) into LDS by every thread
// of the workgroup, one 4-byte word each; the caller synchronises.
__device__ __forceinline__ void copy_ref_ops(RefOps& dst, const RefOps& src) {
    const int* s = reinterpret_cast<const int*>(&src);
    int* d = reinterpret_cast<int*>(&dst);
    for (int i = threadIdx.x; i < int(sizeof(RefOps) / 4); i += blockDim.x) d[i] = s[i];
}

// Role of the common flux on one element face.
enum FaceRole : int {
    ROLE_RUSANOV = 0,   // standard FR flux against the neighbour
    ROLE_HFR = 1,       // hybridized flux against the trace
    ROLE_WALL = 2,      // standard FR flux against the slip-wall ghost
    ROLE_FAR = 3,       // standard FR flux against the free stream
    // implicit elements: hybridized flux against the boundary trace, which
    // the boundary transmission condition fixes per flux point as the mean
    // of the face state and its ghost (slip wall, far field)
    ROLE_WALL_T = 4,
    ROLE_FAR_T = 5
};

__host__ __device__ constexpr bool role_is_wall(int r) {
    return r == ROLE_WALL || r == ROLE_WALL_T;
}
__host__ __device__ constexpr bool role_is_boundary_trace(int r) {
    return r == ROLE_WALL_T || r == ROLE_FAR_T;
}

// Per element face: neighbour element, neighbour local face, role, and
// trace encoding (trace_face*2 + side, -1 off the trace).
struct FaceInfo {
    int nb_e, nb_lf, role, trace;
};

struct Physics {
    double gamma;
    double uinf[4];
    int kind;        // FR_PHYS_EULER or FR_PHYS_EDAC
    double theta;    // EDAC: 1/M^2
};

void set_error(const std::string& msg);
fr_status fail(fr_status st, const std::string& msg);
#define HIP_TRY(expr)                                                      \
    do {                                                                   \
        hipError_t _e = (expr);                                            \
        if (_e != hipSuccess)                                              \
            return ::hfr::fail(FR_E_DEVICE, std::string(#expr ": ") +      \
                                                hipGetErrorString(_e));    \
    } while (0)

RefOps make_ref_ops(int P);

// ---- kernel launchers (kernels_*.hip) ---------------------------------
struct ResidualLaunch {
    const int* list;   // element ids
    int nlist;
    const double* u;   // [4][Ne][Np]
    int Ne;
    const double* verts;     // [Ne][8]
    const FaceInfo* finfo;   // [Ne][4]
    const double2* fS;       // [Ne][4] scaled outward normal of the face
    const double* uhat;      // [Ntp][4]
    Physics phys;
    double* R;               // [4][nlist][Np] or null
    double* h;               // [4][nlist][Np] or null
    const double* ustar;     // [4][nlist][Np]
    double aii_dt;
    double* gk;              // [nlist][4][P][4] or null
    const int* efr_fnodes;   // [Ntf][P] trace nodes (interior-embedded trace) or null
    const int* gate;         // if set and *gate == 0 the kernel returns at entry
    const double* dtscale;   // [Ne] factor of aii_dt per element, or null
};
hipError_t launch_residual(const RefOps& ops, const ResidualLaunch& a,
                           hipStream_t st);

// The blocked Schur-only elimination forms the rows of A and B itself
// (no tableau fill) in FP32 up to p = 4; elsewhere its register budget
// leaves no room and it reads the filled tableau.
constexpr bool blocked_fuses_fill(int P, int precision) {
    return precision == HFR_PREC_FP32 && P <= 5;
}

struct CondenseLaunch {
    const int* imp_list;     // implicit element ids
    int nimp;
    const double* u;         // [4][Ne][Np]
    int Ne;
    const double* verts;
    const FaceInfo* finfo;
    const double2* fS;
    const double* uhat;
    Physics phys;
    double aii_dt;
    const double* h;         // [4][Nim][Np]
    const double* gk;        // [Nim][4][P][4]
    int precision;           // HFR_PREC_*
    void* M;                 // per element swept tableau (n+m)^2 column-major, FP64 or FP32
    double* blocks_copy;     // optional (n+m)^2 FP64 copy per element
    int* pivot_fail;         // set to 1 if a zero pivot is met
    int* piv;                // [Nim][n] pivot row p_k of each exchange
    const int* efr_fnodes;   // [Ntf][P] trace nodes (interior-embedded trace) or null
    // optional: the sweep also forms the FP64 right-hand side of
    // launch_rhs64 from its registers (yr [Nim][n], z [Nim][m]) when set
    double* yr;
    double* z;
    // optional: the fill returns at entry when *go == 0 (a fill launched
    // before the host has read the Newton convergence test)
    const int* go;
    // with yr set: keep only what recovery and assembly read (the columns of
    // B and D, and yr, z); the columns of A already exchanged are skipped,
    // so A^-1 and C A^-1 are not stored, and the right-hand side is carried
    // through the sweep as an FP64 column instead of formed afterwards.  The
    // fill then writes the rows of A and B only and the face-point flux
    // Jacobians to lin; the sweep holds the rows of A only, and L^k and z
    // are formed from C's structure afterwards (k_schur_lift)
    int schur_only;
    double* lin;             // [Nim][2][4P][16] (schur_only)
    const double* dtscale;   // [Ne] factor of aii_dt per element, or null
    int blocked;             // schur_only: panels of 16 on the matrix cores
                             // (k_condense_blocked) instead of the sweep;
                             // 1: default waves per element, 2: eight
    int compact_schur;       // blocked: the Schur complement L^k stored as
                             // 4 x 4 contiguous face sub-blocks at the start
                             // of the element's slot (schur_offset), where
                             // the Schur-only path keeps nothing else, and
                             // -A^-1 B after them (schur_x_offset)
};
// compact Schur complement of an element (bs = 4P rows per face): entry
// (row a, column b) of face sub-block (lr, lc), a and b in the element's
// own point order, at this offset in the element's slot
__host__ __device__ __forceinline__ size_t schur_offset(int bs, int lr, int lc, int a, int b) {
    return (size_t(lc * 4 + lr) * bs + b) * bs + a;
}
// and -A^-1 B (n x m, column-major, row p_k holding unknown k) right after
// the 16 face sub-blocks
__host__ __device__ __forceinline__ size_t schur_x_offset(int bs) {
    return size_t(16) * bs * bs;
}
// element linearisation and the tableau [A B; C D] (must precede
// launch_condense, which sweeps the tableau in place)
hipError_t launch_tableau_fill(const RefOps& ops, const CondenseLaunch& a,
                               hipStream_t st);
hipError_t launch_condense(const RefOps& ops, const CondenseLaunch& a,
                           hipStream_t st);
// FP64 right-hand side with the swept tableau: A^-1 (-h) in pivot-row order
// -> yr [Nim][n], C A^-1 (-h) -> z [Nim][m]; the condensed right-hand side
// is then t = -g - sum over the two sides of z (assembled in FP64)
hipError_t launch_rhs64(int P, int nimp, const void* M, int precision,
                        const int* piv, const double* h, double* yr,
                        double* z, hipStream_t st);

struct AssembleLaunch {
    int nblocks;             // BSR blocks (or entries of blk_list)
    const int* blk_contrib;  // [blocks][2][3]: imp, lf_row*2+side_row, lf_col*2+side_col (-1 none)
    const int* blk_list;     // null: blocks 0..nblocks-1; else the blocks assembled
    int ntf;
    const int* tside;        // [Ntf][2][2]: imp, lf*2+side (-1 none) per side
    const void* M;
    int precision;
    int P, n, m;
    double* L64;             // [nblocks][bs][bs] column-major blocks or null
    float* L32;              // same in FP32 or null
    double* t;               // [Ntf*bs]  t = -g - sum_sides z
    const double* g;         // [Ntf*bs]  assembled transmission residual
    const double* z;         // [Nim][m]  C A^-1 r per element
    int compact_schur;       // element Schur blocks at schur_offset
    // fused assembly with L Dinv by block column (null: by block): per trace
    // face G (ntf of them) the ids of the blocks (F, G), kmax per face, -1
    // past the last
    const int* tcol;
    int kmax;
};
hipError_t launch_assemble(const AssembleLaunch& a, hipStream_t st);
// the diagonal blocks of L read by the block-Jacobi inverse straight from
// the element tableaux (blocks of 20 and 24): the block's contributions as
// in AssembleLaunch; M null: read the assembled blocks of L
struct DiagGather {
    const int* blk_contrib;
    const void* M;           // FP64 tableaux when L64 is given, else FP32
    int n, m;
    int compact_schur;       // element Schur blocks at schur_offset
};

hipError_t launch_spmv(int ntf, int bs, const int* rowptr, const int* col,
                       const double* L64, const float* L32, const double* x,
                       double* y, double alpha, const double* yin,
                       hipStream_t st);
// recovery; with efr the trace at the flux points is interpolated from the
// trace nodes of trace_map (GLL basis of ops)
// compact: -A^-1 B at schur_x_offset (CondenseLaunch.compact_schur)
hipError_t launch_recover(const RefOps& ops, bool efr, int nimp, const void* M,
                          int precision, const int* piv, const double* yr,
                          const int* trace_map, const double* duhat, double* du,
                          hipStream_t st, const int* gate = nullptr, bool compact = false);
// recovery and the Newton update (u_im += du, uhat += duhat) in one launch
hipError_t launch_recover_update(const RefOps& ops, bool efr, int nimp, const void* M,
                                 int precision, const int* piv, const double* yr,
                                 const int* trace_map, const double* duhat, double* du,
                                 int Ne, const int* imp_list, double* u, int ntp4,
                                 double* uhat, hipStream_t st, const int* gate = nullptr,
                                 bool compact = false);

// ---- interior-embedded trace (kernels_efr.hip) ------------------------
// g at the trace nodes: sum over each node's incidences (slot
// (imp*4+lf)*P+i) of sum_q phi_i(x_q) gk[imp][lf][q]
hipError_t launch_efr_gather_g(const RefOps& ops, int nnodes, const int* inc_ptr,
                               const int* inc, const double* gk, double* g,
                               hipStream_t st);
// in place on each element's Schur block: L <- Q^T L Q with Q the
// GLL-to-Gauss interpolation on every face (slot space (lf, i))
hipError_t launch_efr_transform(const RefOps& ops, int nimp, void* M,
                                int precision, int n, int m, hipStream_t st);
struct EfrAssembleLaunch {
    int nblocks;              // 4x4 node blocks
    const int* cptr;          // [nblocks+1] contribution lists
    const int* contrib;       // (imp, slot_row, slot_col) triples
    const void* M;
    int precision;
    int n, m;
    double* L64;
    float* L32;
    int nnodes;
    const int* inc_ptr;       // node incidences (slots)
    const int* inc;
    double* t;                // [Nn*4] t = -g - sum Q^T z
    const double* g;
    const double* z;          // [Nim][m]
    int P;
};
hipError_t launch_efr_assemble(const RefOps& ops, const EfrAssembleLaunch& a,
                               hipStream_t st);
// initial trace: at every node the mean over its incidences of the
// element's state interpolated to the node
hipError_t launch_efr_trace_average(const RefOps& ops, int nnodes, int Ne,
                                    const int* inc_ptr, const int* inc,
                                    const int* imp_list, const double* u,
                                    double* uhat, hipStream_t st);
// u_im += theta du (scatter), uhat += theta duhat
hipError_t launch_newton_update(int Np, int nimp, int Ne, const int* imp_list,
                                const double* du, double* u, int ntp4,
                                const double* duhat, double* uhat,
                                hipStream_t st, const int* gate = nullptr,
                                double theta = 1.0);
// Modal filter: orthonormal Legendre basis at the Gauss points
// v1[q*P+a] = psi_a(x_q), the Gauss weights, and sigma (already raised to
// the time-step exponent) per exponent sum a + b = 0 .. 2(P-1).
struct FilterLaunch {
    int P;
    double v1[kMaxP * kMaxP], w[kMaxP];
    double sig[2 * kMaxP - 1];
};
hipError_t launch_modal_filter(const FilterLaunch& f, long nrows, double* u,
                               hipStream_t st);
hipError_t launch_absmax(int N, const double* x, double* partial, int nblk,
                         double* out, hipStream_t st);
// Newton test: out[0] = max |x|, out[1] = max |y| (out may be host memory
// mapped for the device), *go = 1 when the gate (if any) is open and either
// exceeds the tolerance, both being finite, else 0; the tolerance is tol, or
// tol * max(1, *tol_scale) with tol_scale (device memory) set, and is
// written to out[2]; flags[0..1] copied to flags_out (if set); then the
// next number of the device counter *seq_ctr is written to seq_out (if set)
// behind a system-scope fence, so a host that sees it sees the rest;
// partial needs 2048 doubles
// Inexact-Newton forcing (optional, hist null: none): with the norms the
// final kernel forms the relative tolerance of the next trace solve,
// eta = 0.1 max(r_k (r_k / r_{k-1})^2, tol) / r_k clamped to [lo, hi]
// (the quadratic model of the next residual; eta = hi at the first check of
// a stage), r_k = max(|h|inf, |g|inf); hist[0] keeps r_k, hist[1] eta.
struct Forcing {
    double* hist;
    double lo, hi;
    int first;
};
hipError_t launch_newton_norms(int Nx, const double* x, int Ny, const double* y,
                               double* partial, double tol, const double* tol_scale,
                               double* out, int* go,
                               const int* gate, const int* flags, int* flags_out,
                               long long* seq_out, long long* seq_ctr, hipStream_t st,
                               Forcing fc = Forcing{nullptr, 0.0, 0.0, 0});
hipError_t launch_trace_gather_g(int ntp, int P, const int* tpside,
                                 const double* gk, double* g,
                                 hipStream_t st);
// launch_trace_gather_g and launch_newton_norms (x = h, y = g) in two
// launches: the gather also takes the partial maxima
hipError_t launch_gather_g_norms(int ntp, const int* tpside, const double* gk, double* g,
                                 int Nx, const double* x, double* partial, double tol,
                                 const double* tol_scale, double* out, int* go,
                                 const int* gate, const int* flags,
                                 int* flags_out, long long* seq_out, long long* seq_ctr,
                                 hipStream_t st, Forcing fc = Forcing{nullptr, 0.0, 0.0, 0});

}  // namespace hfr
