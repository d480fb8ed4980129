// Device-resident GMRES state and kernel arguments.
#pragma once

#include "internal.h"

namespace hfr {

constexpr int kGmresMaxK = 65;   // restart <= 64

struct GmresState {
    // finished: the solve is over (converged, or ended at the iteration cap)
    int done, converged, jlast, iters, cycles, finished;
    int est_conv;            // the cycle ended with the residual estimate on target
    int done_pre;            // done as the orthogonalisation kernel of the last
                             // step saw it (read by the update kernel, whose
                             // workgroup 0 may set done itself)
    double inv_norm, beta, bnorm, target;
    double nres, eta;        // inexact-Newton forcing: last Newton residual and
                             // the relative tolerance of the next solve
    double h1[kGmresMaxK], h2[kGmresMaxK];
    double cs[kGmresMaxK], sn[kGmresMaxK];
    // publication counters: the restart kernel and the Newton norms kernel
    // number what they publish from these, so a launch recorded once (in a
    // graph) and replayed still publishes a fresh sequence number
    long long pub_seq, norm_seq;
    double g[kGmresMaxK + 1];    // running right-hand side of the least squares
    double gf[kGmresMaxK + 1];   // rotated (final) right-hand side
    double H[(kGmresMaxK + 1) * kGmresMaxK];
};

struct GmresArgs {
    int ntf, bs, fpb, nblk, restart, pc;
    int fpbA, nblkA;         // decomposition of the product kernel
    int passes;              // classical Gram-Schmidt passes per step (1 or 2)
    int verify;              // 0: a cycle whose residual estimate reached the
                             // target ends the solve without the FP64 true
                             // residual (the Newton loop checks its residuals)
    double rtol;
    const double* eta;       // set: the relative tolerance is *eta (the
                             // forcing term of the Newton iteration), not rtol
    size_t ldv;
    const int* rowptr;
    const int* col;
    const int* ell;          // padded block rows: kmax {block, column} pairs
    int kmax;                // per row, {-1, -1} past its end (product kernel)
    const double* L64;       // original matrix (true residual)
    const float* L32;
    // with L64 and L32 null: the true residual's L x from the element Schur
    // sub-blocks (compact layout, schur_offset) and the block contributions
    const void* Mel;
    const int* econtrib;     // [blocks][2][3] as AssembleLaunch.blk_contrib
    int nloc, mloc, el64;    // element block sizes n, m; Mel in FP64
    const double* Lt64;      // preconditioned matrix L Dinv
    const float* Lt32;
    const void* Dinv;
    const double* t;
    double* V;               // restart x ldv
    double* part;            // nblk x kGmresMaxK
    double* part2;           // nblk x kGmresMaxK
    double* part3;           // nblkA x kGmresMaxK (product kernel)
    unsigned* counters;      // 4
    GmresState* gs;
    void* pub;               // host-visible copy of the state prefix (or null)
};

// the prefix of GmresState the host reads after every chunk
struct GmresPublish {
    int done, converged, jlast, iters, cycles, finished;
    double inv_norm, beta, bnorm, target;
    long long seq;           // written last, behind a system-scope fence
};

hipError_t launch_precondition_matrix(int nblocks, int bs, const int* col,
                                      const double* L64, const float* L32,
                                      int pc, const void* Dinv, double* Lt64,
                                      float* Lt32, hipStream_t st);
// L and Lt = L Dinv of every block in one pass from the element tableaux
// (face blocks of 16, 20 and 24: orders with assemble_precondition_fused);
// Dinv must be in place, and a.blk_list null; with a.L64 / a.L32 null only
// Lt is written
bool assemble_precondition_fused(int P);
hipError_t launch_assemble_precondition(const AssembleLaunch& a, const int* col, int pc,
                                        const void* Dinv, double* Lt64, float* Lt32,
                                        hipStream_t st);
// r = t - L x, beta = |r|, new cycle; cond: only if the cycle has ended
// cap: the host ends the solve here (iteration cap)
// (publishes the state with the next number of gs->pub_seq)
hipError_t launch_gmres_restart(const GmresArgs& a, double* x,
                                double* w, int first, int cond, int cap,
                                hipStream_t st);
hipError_t launch_arnoldi_product(const GmresArgs& a, int j, int fin_prev,
                                  const double* wcur, double* wnxt, hipStream_t st);
// y = Lt x with the Arnoldi product's block-row code (face block sizes 4..24)
hipError_t launch_block_product(const GmresArgs& a, const double* x, double* y,
                                hipStream_t st);
hipError_t launch_arnoldi_orth(const GmresArgs& a, int j, double* wnxt,
                               hipStream_t st);
// jfin >= 0: the update first finishes column jfin (the last step of the
// chunk); cond: the update only when the cycle has ended
hipError_t launch_gmres_update(const GmresArgs& a, double* x, int cond, int jfin,
                               hipStream_t st);

}  // namespace hfr
