// Host orchestration of the implicit stage: residuals, condensation and
// assembly (Section 3.2), the Krylov trace solve, local recovery, Newton
// (Section 3.1) and the element-partitioned IMEX step (alg:imex,
// eq:explicitimex, eq:hfrimex and the final update of Section 4).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <functional>
#include <map>
#include <mutex>
#include <array>
#include <string>
#include <vector>

#include "gmres.h"
#include "mesh.h"

namespace hfr {
hipError_t launch_block_inverse_impl(int ntf, int bs, const int* diag_blk,
                                     const double* L64, const float* L32,
                                     int pc, void* out, int* fail,
                                     hipStream_t st, const DiagGather* dg = nullptr);
hipError_t launch_trace_average_ops(const RefOps& o, int ntp, int Ne,
                                    const int* tpside, const int* imp_list,
                                    const double* u, double* uhat,
                                    hipStream_t st);
hipError_t launch_combine(int nlist, int Np, int Ne, const int* list,
                          const double* base, int nterm,
                          const double* const* terms, const double* coefs,
                          double* out, int scatter, const double* dtscale,
                          hipStream_t st);
}  // namespace hfr

using namespace hfr;

struct hfr_solver_s {
    fr_mesh_t mesh = nullptr;
    hfr_opts opts{};
    int n = 0, m = 0, bs = 0, N = 0, restart = 0;
    int nbr = 0;             // block rows of L: trace faces (HFR) or trace nodes (EFR)
    size_t elem_M = 0;       // scalars per element matrix
    int nblocks = 0;
    // device
    void* M = nullptr;
    double* blocks_copy = nullptr;
    double* h = nullptr;     // [4][Nim][Np]
    double* gk = nullptr;    // [Nim][4][P][4]
    double* g = nullptr;     // [Ntp][4]
    double* ustar = nullptr; // [4][Nim][Np]
    double* du = nullptr;    // [4][Nim][Np]
    double* duhat = nullptr; // [N]
    int* rowptr = nullptr;
    int* tcol = nullptr;     // [nbr][kmax] blocks (F, G) of block column G, -1
                             // past the last (null: not every column fits)
    int* col = nullptr;
    int* ell = nullptr;      // rows padded to kmax {block, column} pairs
    int kmax = 0;
    int* contrib = nullptr;
    int* tside = nullptr;
    int* efr_cptr = nullptr;     // node-block contribution lists (EFR)
    int* efr_contrib = nullptr;
    int* diag_blk = nullptr;
    double* L64 = nullptr;
    float* L32 = nullptr;
    double* t = nullptr;
    void* Dinv = nullptr;
    int* flags = nullptr;    // [0] pivot fail, [1] block inverse fail
    double* Lt64 = nullptr;  // L Dinv (right-preconditioned matrix)
    float* Lt32 = nullptr;
    double* W = nullptr;     // 2 x N Arnoldi work vectors
    GmresState* gs = nullptr;
    bool forcing = false;    // inside Newton with hfr_opts.gmres_forcing_max > 0:
                             // each trace solve to the device's forcing term
    double* part = nullptr;
    double* part2 = nullptr;
    double* part3 = nullptr;
    unsigned* counters = nullptr;
    int fpb = 1, gblk = 1, fpbA = 1, gblkA = 1;
    int* piv = nullptr;      // [Nim][n]
    double* lin = nullptr;   // [Nim][2][4P][16] face-point flux Jacobians
    double* yr = nullptr;    // [Nim][n]  L^-1 P r (FP64)
    double* zz = nullptr;    // [Nim][m]  C A^-1 r (FP64)
    bool have_factors = false;
    int last_gmres_iters = 4;
    // Krylov iterations of the k-th trace solve of the last Newton solve
    // (k < 8; 0 unknown): the first chunk of the k-th solve of the next one
    // is sized from it (with a forcing term the counts rise within a stage)
    int newton_solve_iters[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int chunk_hint = 0;      // > 0: the first chunk of the next solve
    // linearisations of the last Newton solve; while an iteration index is
    // below it the condensation of that iteration (blocked elimination) is
    // queued with the checks, gated on the device by their outcome
    // (spec_condensed: one is queued)
    int newton_prev_iters = 0;
    bool spec_condensed = false;
    bool compact = false;    // the last condensation stored the compact layout
                             // (CondenseLaunch.compact_schur): recovery reads it
    bool l_valid = true;     // L (unpreconditioned) formed for the last
                             // linearisation: the compact Newton path forms only
                             // L Dinv, the true residual then sums L x from the
                             // element sub-blocks and hfr_trace_matvec forms L
    bool verbose = false;
    int stage_calls = 0;
    double* V = nullptr;     // (restart+1) x N
    double* scratch = nullptr;  // partials
    int* go = nullptr;       // 1 while the Newton residual is above tolerance
    double* dscale = nullptr;  // max |u*| of the stage solve (scales its tolerance)
    double* hpin = nullptr;  // pinned, device-mapped host buffer (kPinDoubles):
                             // [0..1] Newton norms, [2] their tolerance,
                             // [kPinGmres..] GMRES state
    double* dpin = nullptr;  // the same buffer's device address
    long long seq_norms = 0;     // last sequence number queued for the norms
    long long seq_gmres = 0;     // ... and for the GMRES state
    int ck = -1;             // condensation kernel in use (HFR_CK_*), -1: not chosen
    double tune_ms[3] = {-1.0, -1.0, -1.0};   // measured candidates (sweep,
                                              // blocked, blocked with 8 waves)
    size_t ws_bytes = 0;     // working buffers (one block, carved)
    size_t table_bytes = 0;  // library-owned read-only device tables
    struct WsItem { void** ptr; size_t bytes; };
    std::vector<WsItem> ws_items;
    void* ws_owned = nullptr;   // the block, when the library allocated it
    bool ws_bound = false;
    // event timers (categories in tmask)
    bool timing = false;
    unsigned tmask = 0;
    double tms[HFR_NTIMERS] = {};
    int64_t tcnt[HFR_NTIMERS] = {};
    struct Pend { hipEvent_t a, b; int cat; };
    std::vector<Pend> pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    // graph form of a Newton iteration: one recorded graph per first-chunk
    // length and per stage arguments, replayed on the caller's stream
    hipStream_t cst = nullptr;   // stream the graphs are recorded on
    struct IterGraph {
        int K;
        const double* u;
        const double* uhat;
        const double* ustar;
        double aii_dt;
        const double* R_out;
        hipGraph_t g;
        hipGraphExec_t x;
    };
    std::vector<IterGraph> graphs;
};

namespace {

int tbegin(hfr_solver_s* s, int cat, hipStream_t st) {
    if (!s || !s->timing || !(s->tmask & (1u << cat))) return -1;
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (s->pool.empty()) {
        if (hipEventCreate(&ev.first) != hipSuccess) return -1;
        if (hipEventCreate(&ev.second) != hipSuccess) {
            (void)hipEventDestroy(ev.first);
            return -1;
        }
    } else {
        ev = s->pool.back();
        s->pool.pop_back();
    }
    (void)hipEventRecord(ev.first, st);
    s->pending.push_back({ev.first, ev.second, cat});
    return int(s->pending.size()) - 1;
}

void tend(hfr_solver_s* s, int idx, hipStream_t st) {
    if (idx < 0 || !s) return;
    (void)hipEventRecord(s->pending[idx].b, st);
}

void tflush(hfr_solver_s* s) {
    if (!s) return;
    for (auto& p : s->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess &&
            hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            s->tms[p.cat] += ms;
            s->tcnt[p.cat] += 1;
        }
        s->pool.push_back({p.a, p.b});
    }
    s->pending.clear();
}

}  // namespace

namespace {

template <class T>
fr_status dalloc(T** p, size_t count, size_t& total) {
    *p = nullptr;
    if (count == 0) return FR_OK;
    if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess)
        return fail(FR_E_NOMEM, "hipMalloc of solver workspace failed (" +
                                    std::to_string(count * sizeof(T)) + " bytes)");
    total += count * sizeof(T);
    return FR_OK;
}

void drop_graphs(hfr_solver_s* s) {
    for (auto& g : s->graphs) {
        (void)hipGraphExecDestroy(g.x);
        (void)hipGraphDestroy(g.g);
    }
    s->graphs.clear();
}

void free_solver(hfr_solver_s* s) {
    tflush(s);
    drop_graphs(s);
    if (s->cst) (void)hipStreamDestroy(s->cst);
    s->cst = nullptr;
    if (s->hpin) (void)hipHostFree(s->hpin);
    s->hpin = nullptr;
    for (auto& p : s->pool) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    s->pool.clear();
    void* ptrs[] = {s->rowptr, s->tcol, s->col, s->ell, s->contrib, s->tside, s->diag_blk,
                    s->efr_cptr, s->efr_contrib, s->ws_owned};
    for (void* p : ptrs) (void)hipFree(p);
}

template <class T>
void plan(hfr_solver_s* s, T** p, size_t count) {
    s->ws_items.push_back({reinterpret_cast<void**>(p), count * sizeof(T)});
}

constexpr int kPinDoubles = 64;
constexpr int kPinGmres = 8;

constexpr int kPinNormSeq = 3;    // long long at double slot 3
constexpr int kPinFlags = 4;      // two int32 at double slot 4

constexpr size_t ws_align(size_t b) { return (b + 255) & ~size_t(255); }

// Carves the working buffers from `base` (256-byte aligned pieces in plan
// order) and clears the state the kernels expect to start at zero.
fr_status bind_internal(hfr_solver_s* s, char* base) {
    size_t off = 0;
    for (auto& it : s->ws_items) {
        *it.ptr = it.bytes ? base + off : nullptr;
        off += ws_align(it.bytes);
    }
    if (hipMemset(s->flags, 0, 8) != hipSuccess ||
        hipMemset(s->counters, 0, 16) != hipSuccess ||
        hipMemset(s->gs, 0, sizeof(GmresState)) != hipSuccess)
        return fail(FR_E_DEVICE, "clearing the solver workspace failed");
    // the device publication counters restart from zero, and so do the
    // host's expectations and the published marks
    s->seq_norms = s->seq_gmres = 0;
    if (s->hpin) std::memset(s->hpin, 0, sizeof(double) * kPinDoubles);
    drop_graphs(s);                    // they name the old buffers
    s->have_factors = false;
    s->ws_bound = true;
    return FR_OK;
}

fr_status need_workspace(const hfr_solver_s* s) {
    return s->ws_bound ? FR_OK
                       : fail(FR_E_INVALID, "solver workspace not bound "
                                            "(hfr_solver_bind_workspace)");
}


// Kernels write what the host reads (Newton norms, GMRES state) straight
// into the pinned buffer, a sequence number last behind a system-scope
// fence.  The host spins on the sequence number, so no event record sits in
// the stream between the kernels (work queued after it keeps running).
fr_status wait_seq(hfr_solver_s* s, const void* slot, long long target, hipStream_t st) {
    const volatile long long* p = reinterpret_cast<const volatile long long*>(slot);
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned it = 1;; ++it) {
        if (*p >= target) {
            std::atomic_thread_fence(std::memory_order_acquire);
            return FR_OK;
        }
        if ((it & 4095) == 0) {
            const hipError_t q = hipStreamQuery(st);
            if (q != hipSuccess && q != hipErrorNotReady)
                return fail(FR_E_DEVICE, std::string("device error: ") + hipGetErrorString(q));
            if (q == hipSuccess && *p < target)
                return fail(FR_E_DEVICE, "stream idle but the readback was not published");
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(600))
                return fail(FR_E_DEVICE, "readback wait timed out");
        }
        __builtin_ia32_pause();
    }
}

fr_status sync_check(hipStream_t st) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return fail(FR_E_DEVICE, std::string("device error: ") + hipGetErrorString(e));
    return FR_OK;
}

ResidualLaunch implicit_launch(hfr_solver_s* s, const double* u,
                               const double* uhat) {
    fr_mesh_s* m = s->mesh;
    ResidualLaunch a{};
    a.list = m->d_imp;
    a.nlist = m->Nim;
    a.u = u;
    a.Ne = m->Ne;
    a.verts = m->d_verts;
    a.finfo = m->d_finfo;
    a.fS = m->d_fS;
    a.uhat = uhat;
    a.phys = m->phys;
    a.efr_fnodes = m->efr ? m->d_efr_fnodes : nullptr;
    a.dtscale = m->d_dtscale;
    return a;
}

// h, the element shares g^(k) and the assembled g (internal buffers)
fr_status residual_internal(hfr_solver_s* s, const double* u,
                            const double* uhat, const double* ustar,
                            double aii_dt, double* R_out, hipStream_t st,
                            const int* gate = nullptr, bool gather = true) {
    fr_mesh_s* m = s->mesh;
    if (m->Nim == 0) return FR_OK;
    ResidualLaunch a = implicit_launch(s, u, uhat);
    a.gate = gate;
    a.R = R_out;
    a.h = s->h;
    a.ustar = ustar;
    a.aii_dt = aii_dt;
    a.gk = s->gk;
    int tk = tbegin(s, HFR_T_RESIDUAL, st);
    HIP_TRY(launch_residual(m->ops, a, st));
    tend(s, tk, st);
    if (m->efr)
        HIP_TRY(launch_efr_gather_g(m->ops, m->Ntp, m->d_efr_inc_ptr, m->d_efr_inc,
                                    s->gk, s->g, st));
    else if (gather)
        HIP_TRY(launch_trace_gather_g(m->Ntp, m->P, m->d_tpside, s->gk, s->g, st));
    return FR_OK;
}

// node-block assembly of the interior-embedded trace system (t only when
// with_matrix is false)
fr_status efr_assemble(hfr_solver_s* s, bool with_matrix, hipStream_t st) {
    fr_mesh_s* m = s->mesh;
    EfrAssembleLaunch a{};
    a.nblocks = with_matrix ? s->nblocks : 0;
    a.cptr = s->efr_cptr;
    a.contrib = s->efr_contrib;
    a.M = s->M;
    a.precision = s->opts.precision;
    a.n = s->n;
    a.m = s->m;
    a.L64 = s->L64;
    a.L32 = s->L32;
    a.nnodes = m->Ntp;
    a.inc_ptr = m->d_efr_inc_ptr;
    a.inc = m->d_efr_inc;
    a.t = s->t;
    a.g = s->g;
    a.z = s->zz;
    a.P = m->P;
    HIP_TRY(launch_efr_assemble(m->ops, a, st));
    return FR_OK;
}

CondenseLaunch condense_launch(hfr_solver_s* s, const double* u,
                               const double* uhat, double aii_dt) {
    fr_mesh_s* m = s->mesh;
    CondenseLaunch c{};
    c.imp_list = m->d_imp;
    c.nimp = m->Nim;
    c.u = u;
    c.Ne = m->Ne;
    c.verts = m->d_verts;
    c.finfo = m->d_finfo;
    c.fS = m->d_fS;
    c.uhat = uhat;
    c.phys = m->phys;
    c.aii_dt = aii_dt;
    c.h = s->h;
    c.gk = s->gk;
    c.precision = s->opts.precision;
    c.M = s->M;
    c.blocks_copy = s->blocks_copy;
    c.pivot_fail = s->flags;
    c.piv = s->piv;
    c.efr_fnodes = m->efr ? m->d_efr_fnodes : nullptr;
    c.lin = s->lin;
    c.dtscale = m->d_dtscale;
    const int ck = s->ck > 0 ? s->ck : s->opts.condense_kernel;
    c.blocked = ck == HFR_CK_BLOCKED ? 1 : ck == HFR_CK_BLOCKED_W8 ? 2 : 0;
    return c;
}

// The Schur-only elimination in use forms the rows of A and B itself: no
// tableau fill is queued for it (unless the blocks are kept for inspection,
// which the fill writes).
// The Newton path (Schur-only) with the blocked elimination and face
// blocks of 20 or 24 rows keeps each element Schur complement as contiguous
// face sub-blocks (schur_offset): its only readers are then the gathering
// block inverse and the fused assembly with L Dinv, which read whole
// sub-blocks instead of 4(p+1)-entry column pieces of the tableau.
bool compact_schur(const hfr_solver_s* s) {
    const int ck = s->ck > 0 ? s->ck : s->opts.condense_kernel;
    return !s->mesh->efr && assemble_precondition_fused(s->mesh->P) &&
           (s->bs == 20 || s->bs == 24) && (ck == HFR_CK_BLOCKED || ck == HFR_CK_BLOCKED_W8);
}

bool fused_fill(const hfr_solver_s* s) {
    const int ck = s->ck > 0 ? s->ck : s->opts.condense_kernel;
    return (ck == HFR_CK_BLOCKED || ck == HFR_CK_BLOCKED_W8) &&
           blocked_fuses_fill(s->mesh->P, s->opts.precision) && !s->blocks_copy;
}

// Fill of the element tableaus; with `go`, every workgroup returns at entry
// when the device flag says the Newton iteration has converged.
// schur: the input of the Schur-only sweep (rows of A and B, and the
// face-point flux Jacobians)
fr_status condense_fill(hfr_solver_s* s, const double* u, const double* uhat,
                        double aii_dt, const int* go, hipStream_t st,
                        bool schur = false) {
    fr_mesh_s* m = s->mesh;
    if (m->Nim == 0) return FR_OK;
    CondenseLaunch c = condense_launch(s, u, uhat, aii_dt);
    c.go = go;
    c.schur_only = schur ? 1 : 0;
    const int tk = tbegin(s, HFR_T_FILL, st);
    HIP_TRY(launch_tableau_fill(m->ops, c, st));
    tend(s, tk, st);
    return FR_OK;
}

// Sweep, assembly and preconditioner; fill_done: the fill of (u, uhat) has
// already been queued.
// condensed: the fused condensation of (u, uhat) is already queued (gated
// on the device); only the assembly and the preconditioner follow.
fr_status condense_internal(hfr_solver_s* s, const double* u,
                            const double* uhat, double aii_dt,
                            hipStream_t st, bool fill_done = false,
                            bool schur_only = false, bool condensed = false) {
    fr_mesh_s* m = s->mesh;
    if (m->Nim == 0) return FR_OK;
    if (!condensed) {
        if (!fill_done && !(schur_only && fused_fill(s))) {
            fr_status e = condense_fill(s, u, uhat, aii_dt, nullptr, st, schur_only);
            if (e) return e;
        }
        CondenseLaunch c = condense_launch(s, u, uhat, aii_dt);
        const int tc = tbegin(s, HFR_T_CONDENSE, st);
        c.yr = s->yr;                   // the sweep also forms the FP64 right-hand side
        c.z = s->zz;
        c.schur_only = schur_only ? 1 : 0;
        c.compact_schur = schur_only && compact_schur(s) ? 1 : 0;
        s->compact = c.compact_schur != 0;
        HIP_TRY(launch_condense(m->ops, c, st));
        tend(s, tc, st);
    }
    int tk = -1;
    s->l_valid = true;                  // unless the compact path below skips L
    if (s->nbr == 0) return FR_OK;
    if (m->efr) {
        tk = tbegin(s, HFR_T_ASSEMBLE, st);
        HIP_TRY(launch_efr_transform(m->ops, m->Nim, s->M, s->opts.precision,
                                     s->n, s->m, st));
        fr_status ea = efr_assemble(s, true, st);
        tend(s, tk, st);
        if (ea) return ea;
    }
    // HFR face blocks of 16, 20 and 24: the assembly forms t only (and the
    // diagonal blocks at 16, which the 16-row inverse reads; at 20 and 24
    // the inverse gathers them from the tableaux itself), and L is gathered
    // with Lt = L Dinv after the inverses
    const bool fuse_pc = !m->efr && assemble_precondition_fused(m->P);
    const bool gather_diag = fuse_pc && (s->bs == 20 || s->bs == 24);
    const int cpt = schur_only && compact_schur(s) ? 1 : 0;
    AssembleLaunch a{};
    a.compact_schur = cpt;
    if (!m->efr) {
        a.nblocks = !fuse_pc ? s->nblocks : gather_diag ? 0 : s->nbr;
        a.blk_list = fuse_pc && !gather_diag ? s->diag_blk : nullptr;
        a.blk_contrib = s->contrib;
        a.ntf = m->Ntf;
        a.tside = s->tside;
        a.M = s->M;
        a.precision = s->opts.precision;
        a.P = m->P;
        a.n = s->n;
        a.m = s->m;
        a.L64 = s->L64;
        a.L32 = s->L32;
        a.t = s->t;
        a.g = s->g;
        a.z = s->zz;
        tk = tbegin(s, HFR_T_ASSEMBLE, st);
        HIP_TRY(launch_assemble(a, st));
        tend(s, tk, st);
    }
    tk = tbegin(s, HFR_T_PCSETUP, st);
    const DiagGather dg{s->contrib, s->M, s->n, s->m, cpt};
    HIP_TRY(launch_block_inverse_impl(s->nbr, s->bs, s->diag_blk, s->L64,
                                      s->L64 ? nullptr : s->L32,
                                      s->opts.precond, s->Dinv, s->flags + 1,
                                      st, gather_diag ? &dg : nullptr));
    if (fuse_pc) {
        a.nblocks = s->nblocks;
        a.blk_list = nullptr;
        a.tcol = s->tcol;                // by block column (null: by block)
        a.kmax = s->kmax;
        if (cpt) {                       // Newton reads L only at a restart
            a.L64 = nullptr;
            a.L32 = nullptr;
        }
        HIP_TRY(launch_assemble_precondition(a, s->col, s->opts.precond, s->Dinv,
                                             s->Lt64, s->Lt32, st));
        s->l_valid = !cpt;
    } else {
        HIP_TRY(launch_precondition_matrix(s->nblocks, s->bs, s->col, s->L64,
                                           s->L64 ? nullptr : s->L32,
                                           s->opts.precond, s->Dinv, s->Lt64,
                                           s->Lt32, st));
    }
    tend(s, tk, st);
    return FR_OK;
}

// L of the last linearisation where the compact Newton path formed only
// L Dinv: the fused assembly again, from the element sub-blocks, with L
// (Lt comes out the same)
fr_status form_L(hfr_solver_s* s, hipStream_t st) {
    if (s->l_valid) return FR_OK;
    fr_mesh_s* m = s->mesh;
    AssembleLaunch a{};
    a.nblocks = s->nblocks;
    a.blk_contrib = s->contrib;
    a.ntf = m->Ntf;
    a.tside = s->tside;
    a.M = s->M;
    a.precision = s->opts.precision;
    a.P = m->P;
    a.n = s->n;
    a.m = s->m;
    a.L64 = s->L64;
    a.L32 = s->L32;
    a.t = s->t;
    a.g = s->g;
    a.z = s->zz;
    a.compact_schur = 1;
    a.tcol = s->tcol;
    a.kmax = s->kmax;
    HIP_TRY(launch_assemble_precondition(a, s->col, s->opts.precond, s->Dinv, s->Lt64,
                                         s->Lt32, st));
    s->l_valid = true;
    return FR_OK;
}

// lagged Jacobian: re-condense the right-hand side with the stored factors
fr_status recondense_rhs_internal(hfr_solver_s* s, hipStream_t st) {
    fr_mesh_s* m = s->mesh;
    if (m->Nim == 0) return FR_OK;
    HIP_TRY(launch_rhs64(m->P, m->Nim, s->M, s->opts.precision, s->piv, s->h,
                         s->yr, s->zz, st));
    if (s->nbr == 0) return FR_OK;
    if (m->efr) {
        const int tk = tbegin(s, HFR_T_ASSEMBLE, st);
        fr_status ea = efr_assemble(s, false, st);
        tend(s, tk, st);
        return ea;
    }
    AssembleLaunch a{};
    a.nblocks = 0;            // t only
    a.blk_contrib = s->contrib;
    a.ntf = m->Ntf;
    a.tside = s->tside;
    a.M = s->M;
    a.precision = s->opts.precision;
    a.P = m->P;
    a.n = s->n;
    a.m = s->m;
    a.t = s->t;
    a.g = s->g;
    a.z = s->zz;
    const int tk = tbegin(s, HFR_T_ASSEMBLE, st);
    HIP_TRY(launch_assemble(a, st));
    tend(s, tk, st);
    return FR_OK;
}

GmresArgs gmres_args(hfr_solver_s* s) {
    fr_mesh_s* m = s->mesh;
    GmresArgs a{};
    a.ntf = s->nbr;
    a.bs = s->bs;
    a.fpb = s->fpb;
    a.nblk = s->gblk;
    a.fpbA = s->fpbA;
    a.nblkA = s->gblkA;
    a.passes = s->opts.gmres_cgs_passes == 2 ? 2 : 1;
    a.verify = 1;
    a.restart = s->restart;
    a.pc = s->opts.precond;
    a.rtol = s->opts.gmres_rtol;
    a.eta = s->forcing ? &s->gs->eta : nullptr;
    a.ldv = size_t(s->N);
    a.rowptr = s->rowptr;
    a.col = s->col;
    a.ell = s->ell;
    a.kmax = s->kmax;
    a.L64 = s->l_valid ? s->L64 : nullptr;
    a.L32 = s->l_valid && !s->L64 ? s->L32 : nullptr;
    a.Mel = s->M;
    a.econtrib = s->contrib;
    a.nloc = s->n;
    a.mloc = s->m;
    a.el64 = s->opts.precision == HFR_PREC_FP64 ? 1 : 0;
    a.Lt64 = s->Lt64;
    a.Lt32 = s->Lt64 ? nullptr : s->Lt32;
    a.Dinv = s->Dinv;
    a.t = s->t;
    a.V = s->V;
    a.part = s->part;
    a.part2 = s->part2;
    a.part3 = s->part3;
    a.counters = s->counters;
    a.gs = s->gs;
    a.pub = s->dpin + kPinGmres;
    return a;
}

// Restarted GMRES.  Arnoldi steps are launched in chunks (the first sized
// by the previous solve's iteration count).  Each chunk is followed by the
// end-of-cycle kernels (update, true residual, restart) in their conditional
// form, which act only if the cycle has ended, and by one readback of the
// state: a solve that converges within its first chunk costs one host
// synchronisation.  Within a chunk there are no host round trips, and steps
// after convergence return at entry.
// chain (optional): work queued after every chunk's end-of-cycle kernels,
// gated on the device by the solve's `finished` flag, that records the
// readback mark itself; *chained tells whether it ran for a finished solve.
// pre >= 0: the start and a first chunk of `pre` steps, with its end-of-cycle
// kernels and the chain, are already queued (a replayed iteration graph)
fr_status gmres(hfr_solver_s* s, double* x, hfr_solve_stats* stats,
                hipStream_t st, const std::function<fr_status()>& chain = nullptr,
                bool* chained = nullptr, bool verify = true, int pre = -1) {
    if (chained) *chained = false;
    const int N = s->N;
    hfr_solve_stats loc{};
    if (N == 0) {
        if (stats) *stats = loc;
        return FR_OK;
    }
    GmresArgs a = gmres_args(s);
    a.verify = verify ? 1 : 0;
    const int R = s->restart;
    const int maxit = std::max(1, s->opts.gmres_max_iters);
    double* W0 = s->W;
    double* W1 = s->W + N;
    static_assert(sizeof(GmresPublish) <= (kPinDoubles - kPinGmres) * sizeof(double),
                  "readback size");
    GmresPublish hs{};
    // the restart kernel, last of every chunk's sequence, publishes the state
    auto fetch = [&](bool run_chain) -> fr_status {
        fr_status e = chain && run_chain ? chain() : FR_OK;
        if (e) return e;
        // the chain publishes the norms after the restart kernel's state
        if (chain) e = wait_seq(s, s->hpin + kPinNormSeq, s->seq_norms, st);
        else e = wait_seq(s, &reinterpret_cast<GmresPublish*>(s->hpin + kPinGmres)->seq,
                          s->seq_gmres, st);
        if (e) return e;
        std::memcpy(&hs, s->hpin + kPinGmres, sizeof(hs));
        if (!(hs.beta == hs.beta) || std::isinf(hs.beta))
            return fail(FR_E_NONFINITE, "non-finite trace residual");
        return FR_OK;
    };
    if (pre < 0) {
        HIP_TRY(launch_gmres_restart(a, x, W0, 1, 0, 0, st));
        ++s->seq_gmres;
    }
    int launched = 0;
    int chunk = std::max(2, std::min(R, s->chunk_hint > 0 ? s->chunk_hint
                                                          : s->last_gmres_iters + 1));
    int cycles_seen = 0;
    int j = 0;
    fr_status e;
    for (;;) {
        if (pre >= 0) {                          // the recorded first chunk
            j = launched = pre;
            pre = -1;
            if ((e = fetch(false))) return e;
        } else {
        const int steps = std::max(0, std::min(std::min(chunk, R - j), maxit - launched));
        for (int c = 0; c < steps; ++c, ++j) {
            double* wc = j % 2 ? W1 : W0;
            double* wn = j % 2 ? W0 : W1;
            const int tk = tbegin(s, HFR_T_SPMV, st);
            HIP_TRY(launch_arnoldi_product(a, j, c == 0 ? 1 : 0, wc, wn, st));
            tend(s, tk, st);
            HIP_TRY(launch_arnoldi_orth(a, j, wn, st));
        }
        launched += steps;
        // at the iteration cap the cycle is ended whether or not it is done;
        // the update kernel first finishes the chunk's last column
        const int cap = launched >= maxit ? 1 : 0;
        HIP_TRY(launch_gmres_update(a, x, 1 - cap, steps > 0 ? j - 1 : -1, st));
        HIP_TRY(launch_gmres_restart(a, x, W0, 0, 1 - cap, cap, st));
        ++s->seq_gmres;
        if ((e = fetch(true))) return e;
        }
        if (hs.cycles != cycles_seen) {          // the cycle ended and restarted
            cycles_seen = hs.cycles;
            if (hs.finished) {
                if (chained) *chained = chain != nullptr;
                break;
            }
            j = 0;
            chunk = std::max(2, std::min(R, s->last_gmres_iters + 1));
        } else {
            chunk = 2;
        }
    }
    s->last_gmres_iters = hs.iters;
    loc.iterations = hs.iters;
    loc.restarts = hs.cycles;
    loc.rel_residual = hs.bnorm > 0 ? hs.beta / hs.bnorm : 0.0;
    if (stats) *stats = loc;
    if (!hs.converged) return fail(FR_E_NOT_CONVERGED, "GMRES iteration cap reached");
    return FR_OK;
}

// The start of a solve inside Newton and its first chunk of K steps, as the
// first round of gmres() queues them (estimate-trusting cycles, no iteration
// cap inside the chunk), then the chain: the part of a Newton iteration a
// graph records.
fr_status gmres_first_chunk(hfr_solver_s* s, double* x, int K, hipStream_t q,
                            const std::function<fr_status()>& chain) {
    GmresArgs a = gmres_args(s);
    a.verify = 0;
    double* W0 = s->W;
    double* W1 = s->W + s->N;
    HIP_TRY(launch_gmres_restart(a, x, W0, 1, 0, 0, q));
    ++s->seq_gmres;
    for (int j = 0; j < K; ++j) {
        double* wc = j % 2 ? W1 : W0;
        double* wn = j % 2 ? W0 : W1;
        HIP_TRY(launch_arnoldi_product(a, j, j == 0 ? 1 : 0, wc, wn, q));
        HIP_TRY(launch_arnoldi_orth(a, j, wn, q));
    }
    HIP_TRY(launch_gmres_update(a, x, 1, K - 1, q));
    HIP_TRY(launch_gmres_restart(a, x, W0, 0, 1, 0, q));
    ++s->seq_gmres;
    return chain();
}

// Process-wide choice of the Schur-only condensation kernel per (order,
// precision), measured once on the first linearisation of a Newton solve:
// each candidate is timed with the tableau fill it needs (none for a
// blocked kernel that forms the rows of A and B itself), and the fastest is
// kept for every later solver of that shape.
std::mutex g_tune_mutex;
std::map<std::pair<int, int>, std::pair<int, std::array<double, 3>>> g_tuned;

fr_status tune_condense(hfr_solver_s* s, const double* u, const double* uhat,
                        double aii_dt, hipStream_t st) {
    fr_mesh_s* m = s->mesh;
    const auto key = std::make_pair(m->P, s->opts.precision);
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            s->ck = it->second.first;
            for (int i = 0; i < 3; ++i) s->tune_ms[i] = it->second.second[i];
            return FR_OK;
        }
    }
    const int cand[3] = {HFR_CK_SWEEP, HFR_CK_BLOCKED, HFR_CK_BLOCKED_W8};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(FR_E_DEVICE, "hipEventCreate failed");
    }
    std::array<double, 3> ms{};
    fr_status e = FR_OK;
    for (int c = 0; c < 3 && !e; ++c) {
        s->ck = cand[c];
        float best = 1e30f;
        for (int rep = 0; rep < 2 && !e; ++rep) {   // the first run warms up
            // each candidate timed with the fill it needs
            if (hipEventRecord(e0, st) != hipSuccess) {
                e = fail(FR_E_DEVICE, "condensation tuning launch failed");
                break;
            }
            if (!fused_fill(s) && (e = condense_fill(s, u, uhat, aii_dt, nullptr, st, true)))
                break;
            CondenseLaunch cl = condense_launch(s, u, uhat, aii_dt);
            cl.yr = s->yr;
            cl.z = s->zz;
            cl.schur_only = 1;
            if (launch_condense(m->ops, cl, st) != hipSuccess ||
                hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                e = fail(FR_E_DEVICE, "condensation tuning launch failed");
                break;
            }
            float t = 0.f;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (rep > 0) best = std::min(best, t);
        }
        ms[c] = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e) {
        s->ck = -1;
        return e;
    }
    int bi = 0;
    for (int c = 1; c < 3; ++c)
        if (ms[c] < ms[bi]) bi = c;
    s->ck = cand[bi];
    for (int i = 0; i < 3; ++i) s->tune_ms[i] = ms[i];
    // leave a fresh fill for the linearisation that follows (if it needs one)
    if (!fused_fill(s) && (e = condense_fill(s, u, uhat, aii_dt, nullptr, st, true))) return e;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tuned[key] = std::make_pair(s->ck, ms);
    return FR_OK;
}

// R_out (optional): every check of an iterate also writes R^im(u, uhat)
// there, so on convergence it holds R_i of the converged iterate (the last
// check's, the same kernel on the same arguments as a fresh evaluation)
fr_status newton(hfr_solver_s* s, double* u, double* uhat,
                 const double* ustar, double aii_dt, hfr_newton_stats* stats,
                 hipStream_t st, double* R_out = nullptr) {
    fr_mesh_s* m = s->mesh;
    hfr_newton_stats loc{};
    const int nu = 4 * m->Nim * m->Np;
    // trace solves inside this Newton solve take the forcing term; the
    // per-solve state is cleared however the solve ends
    s->forcing = s->opts.gmres_forcing_max > 0.0;
    struct NewtonScope {
        hfr_solver_s* s;
        ~NewtonScope() {
            s->forcing = false;
            s->chunk_hint = 0;
            s->spec_condensed = false;
        }
    } newton_scope{s};
    // the tolerance newton_tol * max(1, |u*|) is formed on the device by the
    // norms kernel and published with the norms (no readback here)
    HIP_TRY(launch_absmax(nu, ustar, s->scratch, std::min(1024, std::max(1, (nu + 255) / 256)),
                          s->dscale, st));
    const double rtol = s->opts.newton_tol;
    double tol = 0.0;
    fr_status e;
    const int lag = s->opts.jacobian_lag;
    const bool spec = lag <= 0 && m->Nim > 0;
    int* flags_pub = reinterpret_cast<int*>(s->dpin + kPinFlags);
    long long* seq_pub = reinterpret_cast<long long*>(s->dpin + kPinNormSeq);
    // Residual at the current iterate, its norms and the failure flags into
    // the pinned buffer, the readback mark, then (unless the Jacobian is
    // reused) the next linearisation's fill, which the device skips when the
    // norms pass the test or the gate is closed.
    // the stream the chain below is queued on (the caller's, or the one an
    // iteration graph is recorded on)
    hipStream_t qs = st;
    // the forcing term of the next trace solve is formed with the norms
    // (first: the stage's first check, which starts the residual history)
    auto forcing = [&](bool first) {
        return s->forcing ? Forcing{&s->gs->nres, s->opts.gmres_rtol,
                                    s->opts.gmres_forcing_max, first ? 1 : 0}
                          : Forcing{nullptr, 0.0, 0.0, 0};
    };
    // index of the Newton iteration the checks queued next would precede
    int it_next = 0;
    // the condensation of the next iteration (the blocked kernel; its fill is
    // queued above where it is not fused) queued right behind the checks
    // (the device skips it when they pass or fail), so the host's
    // reading of the norms does not leave the device idle: only while the
    // last Newton solve suggests another iteration, and never with timers
    // (they would time the skipped launches), recorded graphs or damping
    auto speculate = [&]() {
        const int ck = s->ck > 0 ? s->ck : s->opts.condense_kernel;
        return spec && (ck == HFR_CK_BLOCKED || ck == HFR_CK_BLOCKED_W8) && !s->blocks_copy &&
               !s->timing && !s->opts.iteration_graph && !s->opts.newton_damping &&
               s->nbr > 0 && it_next < s->newton_prev_iters &&
               it_next < s->opts.newton_max_iters;   // never one the cap would leave unused
    };
    auto queue_checks = [&](const int* gate, bool first = false) -> fr_status {
        // the HFR gather of g also takes the norms' partial maxima
        fr_status e2 = residual_internal(s, u, uhat, ustar, aii_dt, R_out, qs, gate,
                                         m->efr);
        if (e2) return e2;
        if (m->efr)
            HIP_TRY(launch_newton_norms(nu, s->h, 4 * m->Ntp, s->g, s->scratch, rtol,
                                        s->dscale, s->dpin, s->go, gate, s->flags, flags_pub,
                                        seq_pub, &s->gs->norm_seq, qs, forcing(first)));
        else
            HIP_TRY(launch_gather_g_norms(m->Ntp, m->d_tpside, s->gk, s->g, nu, s->h,
                                          s->scratch, rtol, s->dscale, s->dpin, s->go, gate,
                                          s->flags,
                                          flags_pub, seq_pub, &s->gs->norm_seq, qs,
                                          forcing(first)));
        ++s->seq_norms;
        if (spec && !fused_fill(s) &&
            (e2 = condense_fill(s, u, uhat, aii_dt, s->go, qs, true)))
            return e2;
        if (speculate()) {
            CondenseLaunch c = condense_launch(s, u, uhat, aii_dt);
            c.yr = s->yr;
            c.z = s->zz;
            c.schur_only = 1;
            c.compact_schur = compact_schur(s) ? 1 : 0;
            s->compact = c.compact_schur != 0;
            c.go = s->go;
            HIP_TRY(launch_condense(m->ops, c, qs));
            s->spec_condensed = true;
        }
        return FR_OK;
    };
    // After each GMRES chunk the update of the Newton iterate and the next
    // checks are queued gated by the solve's `finished` flag, so the host's
    // wait for the solve also covers them and the device does not idle.
    const int* gate = &s->gs->finished;
    auto after_solve = [&]() -> fr_status {
        int tk = tbegin(s, HFR_T_RECOVER, qs);
        HIP_TRY(launch_recover_update(m->ops, m->efr, m->Nim, s->M, s->opts.precision,
                                      s->piv, s->yr, m->d_trace_map, s->duhat, s->du,
                                      m->Ne, m->d_imp, u, 4 * m->Ntp, uhat, qs, gate,
                                      s->compact));
        tend(s, tk, qs);
        return queue_checks(gate);          // it_next: the iteration after this solve's
    };
    // Graph form (hfr_opts.iteration_graph): the linearisation's elimination,
    // assembly and preconditioner, the start and first chunk of the trace
    // solve, and the chain are recorded once per first-chunk length K and
    // stage arguments, then replayed; the sequence numbers they publish come
    // from device counters, so a replay is indistinguishable from the eager
    // queue.  Later chunks of a solve that needs more than K steps are
    // queued eagerly by gmres().
    auto replay_iteration = [&](int K) -> fr_status {
        hfr_solver_s::IterGraph* gr = nullptr;
        for (auto& g : s->graphs)
            if (g.K == K && g.u == u && g.uhat == uhat && g.ustar == ustar &&
                g.aii_dt == aii_dt && g.R_out == R_out)
                gr = &g;
        if (!gr) {
            if (!s->cst) HIP_TRY(hipStreamCreateWithFlags(&s->cst, hipStreamNonBlocking));
            const long long sg = s->seq_gmres, sn = s->seq_norms;
            qs = s->cst;
            HIP_TRY(hipStreamBeginCapture(s->cst, hipStreamCaptureModeThreadLocal));
            fr_status e2 = condense_internal(s, u, uhat, aii_dt, s->cst, true, true);
            if (!e2) e2 = gmres_first_chunk(s, s->duhat, K, s->cst, after_solve);
            hipGraph_t g = nullptr;
            const hipError_t ce = hipStreamEndCapture(s->cst, &g);
            qs = st;
            s->seq_gmres = sg;                 // counted again at each replay
            s->seq_norms = sn;
            if (e2 || ce != hipSuccess || !g) {
                if (g) (void)hipGraphDestroy(g);
                return e2 ? e2 : fail(FR_E_DEVICE, std::string("recording the Newton "
                                                               "iteration: ") +
                                                       hipGetErrorString(ce));
            }
            hipGraphExec_t x = nullptr;
            const hipError_t ie = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                (void)hipGraphDestroy(g);
                return fail(FR_E_DEVICE, std::string("hipGraphInstantiate: ") +
                                             hipGetErrorString(ie));
            }
            if (s->graphs.size() >= 8) {       // keep a handful (K, stage pointers)
                (void)hipGraphExecDestroy(s->graphs.front().x);
                (void)hipGraphDestroy(s->graphs.front().g);
                s->graphs.erase(s->graphs.begin());
            }
            s->graphs.push_back({K, u, uhat, ustar, aii_dt, R_out, g, x});
            gr = &s->graphs.back();
        }
        HIP_TRY(hipGraphLaunch(gr->x, st));
        s->seq_gmres += 2;                     // the two restart kernels
        s->seq_norms += 1;                     // the chain's norms
        ++loc.graph_replays;
        return FR_OK;
    };
    // damped Newton: a step that leaves a non-finite residual is halved (at
    // most seven times) by moving the iterate back along du, duhat
    double theta = 1.0;
    int halvings = 0;
    bool queued = false;
    for (int it = 0;; ++it) {
        it_next = it;
        if (!queued && (e = queue_checks(nullptr, it == 0))) return e;
        queued = false;
        if ((e = wait_seq(s, s->hpin + kPinNormSeq, s->seq_norms, st))) return e;
        const double hmax = s->hpin[0], gmax = s->hpin[1];
        tol = s->hpin[2];
        const double res = std::max(hmax, gmax);
        if (s->verbose)
            fprintf(stderr, "[hfr] newton it %d |h| %.3e |g| %.3e tol %.3e\n", it,
                    hmax, gmax, tol);
        loc.residual = res;
        loc.newton_iters = it;
        if (!(hmax == hmax) || !(gmax == gmax) || std::isinf(res)) {
            if (s->opts.newton_damping && it > 0 && halvings < 7) {
                ++halvings;
                theta *= 0.5;
                HIP_TRY(launch_newton_update(m->Np, m->Nim, m->Ne, m->d_imp, s->du, u,
                                             4 * m->Ntp, s->duhat, uhat, st, nullptr, -theta));
                if ((e = queue_checks(nullptr))) return e;
                queued = true;
                --it;                              // the same Newton iteration
                continue;
            }
            if (stats) *stats = loc;
            return fail(FR_E_NONFINITE, "non-finite Newton residual");
        }
        theta = 1.0;
        halvings = 0;
        if (res <= tol) {
            s->newton_prev_iters = it;
            break;
        }
        if (it >= s->opts.newton_max_iters) {
            if (stats) *stats = loc;
            return fail(FR_E_NOT_CONVERGED, "Newton did not converge");
        }
        {
            const int prev = it < 8 ? s->newton_solve_iters[it] : 0;
            s->chunk_hint = std::max(2, std::min(s->restart,
                                                 (prev > 0 ? prev : s->last_gmres_iters) + 1));
        }
        const bool relin = lag <= 0 || !s->have_factors ||
                           (it == 0 && (s->stage_calls % lag) == 0);
        int pre = -1;
        if (relin) {
            // first Schur-only linearisation with the automatic choice: pick
            // the condensation kernel (the tableaux are filled again after)
            if (spec && s->ck < 0 && s->opts.condense_kernel == HFR_CK_AUTO &&
                (e = tune_condense(s, u, uhat, aii_dt, st)))
                return e;
            const int K = std::max(2, std::min(s->restart, s->chunk_hint));
            if (spec && s->opts.iteration_graph && !s->timing && s->N > 0 &&
                K < s->opts.gmres_max_iters) {
                if ((e = replay_iteration(K))) return e;
                pre = K;
            } else {
                // factors that are never reused need only the Schur part
                const bool queued_c = s->spec_condensed;
                s->spec_condensed = false;
                if (queued_c) ++loc.queued_linearisations;
                if ((e = condense_internal(s, u, uhat, aii_dt, st, spec, lag <= 0, queued_c)))
                    return e;
            }
            s->have_factors = lag > 0;
        } else {
            if ((e = recondense_rhs_internal(s, st))) return e;
        }
        hfr_solve_stats ks{};
        bool chained = false;
        int tk = tbegin(s, HFR_T_TRACE_SOLVE, st);
        // inside Newton a cycle whose residual estimate is on target ends the
        // solve (the FP64 residuals of the next iterate are checked anyway)
        it_next = it + 1;
        e = gmres(s, s->duhat, &ks, st, after_solve, &chained, false, pre);
        s->chunk_hint = 0;
        if (it < 8) s->newton_solve_iters[it] = ks.iterations;
        tend(s, tk, st);
        if (s->verbose)
            fprintf(stderr, "[hfr]   gmres its %d restarts %d relres %.3e status %d\n",
                    ks.iterations, ks.restarts, ks.rel_residual, int(e));
        loc.gmres_iters += ks.iterations;
        if (e && e != FR_E_NOT_CONVERGED) return e;
        if (chained) {
            queued = true;                     // checks of the new iterate queued
        } else {                               // no trace unknowns: no chain ran
            tk = tbegin(s, HFR_T_RECOVER, st);
            HIP_TRY(launch_recover(m->ops, m->efr, m->Nim, s->M, s->opts.precision, s->piv,
                                   s->yr, m->d_trace_map, s->duhat, s->du, st, nullptr,
                                   s->compact));
            HIP_TRY(launch_newton_update(m->Np, m->Nim, m->Ne, m->d_imp, s->du, u,
                                         4 * m->Ntp, s->duhat, uhat, st));
            tend(s, tk, st);
        }
    }
    s->stage_calls++;
    // failure flags as of the last check (published with its norms)
    int fl[2] = {0, 0};
    std::memcpy(fl, s->hpin + kPinFlags, sizeof(fl));
    if (fl[0] || fl[1]) {
        HIP_TRY(hipMemsetAsync(s->flags, 0, sizeof(fl), st));
        if (stats) *stats = loc;
        return fail(FR_E_NONFINITE, "zero pivot in an element or face block");
    }
    if (stats) *stats = loc;
    return FR_OK;
}

}  // namespace

extern "C" fr_status hfr_solver_create(fr_mesh_t mesh, const hfr_opts* o,
                                       size_t* ws, hfr_solver_t* out) {
    if (!mesh || !o || !out) return fail(FR_E_INVALID, "null argument");
    *out = nullptr;
    if (mesh->host_only) return fail(FR_E_INVALID, "host-only mesh");
    if (o->precision != HFR_PREC_FP64 && o->precision != HFR_PREC_FP32)
        return fail(FR_E_INVALID, "unknown precision");
    if (o->precond < HFR_PC_FP64 || o->precond > HFR_PC_BF16)
        return fail(FR_E_INVALID, "unknown preconditioner storage");
    if (o->gmres_restart < 1 || o->gmres_restart > kGmresMaxK - 1)
        return fail(FR_E_INVALID, "gmres_restart must be in 1..64");
    if (o->newton_max_iters < 0 || !(o->newton_tol > 0.0) || !(o->gmres_rtol > 0.0) ||
        o->jacobian_lag < 0 || o->gmres_cgs_passes < 0 || o->gmres_cgs_passes > 2 ||
        (o->caller_workspace != 0 && o->caller_workspace != 1) ||
        o->condense_kernel < HFR_CK_AUTO || o->condense_kernel > HFR_CK_BLOCKED_W8 ||
        (o->newton_damping != 0 && o->newton_damping != 1) ||
        (o->iteration_graph != 0 && o->iteration_graph != 1) ||
        !(o->gmres_forcing_max >= 0.0) ||
        (o->gmres_forcing_max > 0.0 &&
         !(o->gmres_forcing_max >= o->gmres_rtol && o->gmres_forcing_max < 1.0)))
        return fail(FR_E_INVALID, "bad tolerance or iteration cap");
    auto s = new hfr_solver_s();
    s->mesh = mesh;
    s->opts = *o;
    fr_mesh_s* m = mesh;
    const int P = m->P;
    s->n = 4 * m->Np;
    s->m = 16 * P;
    s->bs = m->efr ? 4 : 4 * P;
    s->nbr = m->efr ? m->Ntp : m->Ntf;
    s->N = 4 * m->Ntp;
    s->restart = o->gmres_restart;
    s->elem_M = size_t(s->n + s->m) * (s->n + s->m);
    // block-sparse structure of L.  HFR: one block row per trace face;
    // columns are the trace faces of the two elements sharing it.  EFR: one
    // 4x4 block row per trace node; columns are the nodes of the elements
    // around it, each block summing (element, slot row, slot column)
    // contributions of the transformed element Schur blocks.
    std::vector<int> rowptr(s->nbr + 1, 0), col, contrib, tside(4 * size_t(m->Ntf), -1),
        diag(s->nbr, -1), ecptr(1, 0), econtrib;
    if (m->efr) {
        std::vector<std::map<int, std::vector<int>>> rows(s->nbr);
        for (int k = 0; k < m->Nim; ++k)
            for (int sa = 0; sa < 4 * P; ++sa) {
                const int a = m->trace_map[size_t(k) * 4 * P + sa];
                if (a < 0) continue;
                for (int sb = 0; sb < 4 * P; ++sb) {
                    const int b = m->trace_map[size_t(k) * 4 * P + sb];
                    if (b < 0) continue;
                    auto& v = rows[a][b];
                    v.push_back(k);
                    v.push_back(sa);
                    v.push_back(sb);
                }
            }
        for (int a = 0; a < s->nbr; ++a) {
            for (auto& kv : rows[a]) {
                if (kv.first == a) diag[a] = int(col.size());
                col.push_back(kv.first);
                econtrib.insert(econtrib.end(), kv.second.begin(), kv.second.end());
                ecptr.push_back(int(econtrib.size() / 3));
            }
            rowptr[a + 1] = int(col.size());
        }
    } else
    for (int F = 0; F < m->Ntf; ++F) {
        const int f = m->trace_faces[F];
        std::map<int, std::vector<int>> cols;   // G -> contributions
        for (int sd = 0; sd < 2; ++sd) {
            const int e = m->face_e[2 * f + sd], lr = m->face_l[2 * f + sd];
            const int imp = m->elem_to_imp[e];
            tside[(size_t(F) * 2 + sd) * 2] = imp;
            tside[(size_t(F) * 2 + sd) * 2 + 1] = lr;
            for (int lc = 0; lc < 4; ++lc) {
                const int fc = m->elem_face[4 * e + lc];
                const int G = m->trace_of_face[fc];
                if (G < 0) continue;
                const int sc = m->elem_side[4 * e + lc];
                auto& v = cols[G];
                v.push_back(imp);
                v.push_back(lr * 2 + sd);
                v.push_back(lc * 2 + sc);
            }
        }
        for (auto& kv : cols) {
            if (kv.first == F) diag[F] = int(col.size());
            col.push_back(kv.first);
            for (int c = 0; c < 2; ++c)
                for (int z = 0; z < 3; ++z)
                    contrib.push_back(size_t(3 * c + z) < kv.second.size()
                                          ? kv.second[3 * c + z] : -1);
        }
        rowptr[F + 1] = int(col.size());
    }
    s->nblocks = int(col.size());
    // the same structure with every row padded to the longest one
    for (int a = 0; a < s->nbr; ++a) s->kmax = std::max(s->kmax, rowptr[a + 1] - rowptr[a]);
    std::vector<int> ell(2 * size_t(s->nbr) * std::max(1, s->kmax), -1);
    for (int a = 0; a < s->nbr; ++a)
        for (int p = rowptr[a]; p < rowptr[a + 1]; ++p) {
            const size_t i = size_t(a) * s->kmax + (p - rowptr[a]);
            ell[2 * i] = p;
            ell[2 * i + 1] = col[p];
        }
    // the blocks of each block column (HFR: the block pattern is that of
    // face adjacency, symmetric, so a column holds at most kmax blocks)
    std::vector<int> tcol;
    if (!m->efr) {
        tcol.assign(size_t(s->nbr) * std::max(1, s->kmax), -1);
        std::vector<int> cnt(s->nbr, 0);
        for (int a = 0; a < s->nbr && !tcol.empty(); ++a)
            for (int p = rowptr[a]; p < rowptr[a + 1]; ++p) {
                const int G = col[p];
                if (cnt[G] >= s->kmax) {
                    tcol.clear();
                    break;
                }
                tcol[size_t(G) * s->kmax + cnt[G]++] = p;
            }
    }
    size_t& tot = s->table_bytes;
    const size_t scal = o->precision == HFR_PREC_FP64 ? 8 : 4;
    const size_t nimp = size_t(m->Nim), np4 = 4 * size_t(m->Np);
    const size_t bb = size_t(s->bs) * s->bs;
    fr_status e;
    // read-only tables: library-owned
    if ((e = dalloc(&s->rowptr, rowptr.size(), tot)) ||
        (e = dalloc(&s->tcol, tcol.size(), tot)) ||
        (e = dalloc(&s->col, col.size(), tot)) ||
        (e = dalloc(&s->ell, ell.size(), tot)) ||
        (e = dalloc(&s->contrib, contrib.size(), tot)) ||
        (e = dalloc(&s->tside, tside.size(), tot)) ||
        (e = dalloc(&s->efr_cptr, m->efr ? ecptr.size() : 0, tot)) ||
        (e = dalloc(&s->efr_contrib, econtrib.size(), tot)) ||
        (e = dalloc(&s->diag_blk, diag.size(), tot)) ||
        (e = (hipHostMalloc(reinterpret_cast<void**>(&s->hpin), kPinDoubles * sizeof(double),
                            hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
                      hipHostGetDevicePointer(reinterpret_cast<void**>(&s->dpin), s->hpin, 0) ==
                          hipSuccess
                  ? FR_OK
                  : fail(FR_E_NOMEM, "pinned readback buffer: hipHostMalloc or "
                                     "hipHostGetDevicePointer failed")))) {
        free_solver(s);
        delete s;
        return e;
    }
    std::memset(s->hpin, 0, kPinDoubles * sizeof(double));
    // working buffers: one block, carved in this order
    plan(s, reinterpret_cast<char**>(&s->M), nimp * s->elem_M * scal);
    if (o->keep_blocks) plan(s, &s->blocks_copy, nimp * size_t(s->n + s->m) * (s->n + s->m));
    plan(s, &s->h, nimp * np4);
    plan(s, &s->gk, nimp * 16 * P);
    plan(s, &s->g, size_t(s->N));
    plan(s, &s->ustar, nimp * np4);
    plan(s, &s->du, nimp * np4);
    plan(s, &s->duhat, size_t(s->N));
    if (o->precision == HFR_PREC_FP64) {
        plan(s, &s->L64, size_t(s->nblocks) * bb);
        plan(s, &s->Lt64, size_t(s->nblocks) * bb);
    } else {
        plan(s, &s->L32, size_t(s->nblocks) * bb);
        plan(s, &s->Lt32, size_t(s->nblocks) * bb);
    }
    plan(s, &s->W, 2 * size_t(std::max(1, s->N)));
    plan(s, reinterpret_cast<char**>(&s->gs), sizeof(GmresState));
    plan(s, &s->part, size_t(std::max(256, s->nbr / std::max(1, 2048 / s->bs) + 1)) * kGmresMaxK);
    plan(s, &s->part2, size_t(std::max(256, s->nbr / std::max(1, 2048 / s->bs) + 1)) * kGmresMaxK);
    plan(s, &s->part3, size_t(std::max(1024, s->nbr + 1)) * kGmresMaxK);
    plan(s, &s->counters, 4);
    plan(s, &s->piv, nimp * size_t(s->n));
    plan(s, &s->lin, nimp * 2 * 4 * 16 * size_t(P));
    plan(s, &s->yr, nimp * size_t(s->n));
    plan(s, &s->zz, nimp * size_t(s->m));
    plan(s, &s->t, size_t(s->N));
    plan(s, reinterpret_cast<char**>(&s->Dinv),
         size_t(s->nbr) * bb * (o->precond == HFR_PC_FP64 ? 8 : o->precond == HFR_PC_FP32 ? 4 : 2));
    plan(s, &s->flags, 2);
    plan(s, &s->V, size_t(s->restart + 1) * std::max(1, s->N));
    plan(s, &s->scratch, size_t(4096) * 66);
    plan(s, &s->go, 1);
    plan(s, &s->dscale, 1);
    s->ws_bytes = 0;
    for (auto& it : s->ws_items) s->ws_bytes += ws_align(it.bytes);
    s->verbose = std::getenv("HFR_VERBOSE") != nullptr;
    s->fpb = 256 / s->bs;
    s->gblk = std::max(1, (s->nbr + s->fpb - 1) / s->fpb);
    // vector kernels: about 256 workgroups of 512 threads, each owning whole
    // faces, at most 2048 rows (4 per thread)
    s->fpb = std::min(std::max((s->nbr + 255) / 256, std::max(1, 512 / s->bs)),
                      2048 / s->bs);
    s->gblk = std::max(1, (s->nbr + s->fpb - 1) / s->fpb);
    // product kernel: up to 1024 workgroups, 64 rows per pass, 8 passes max
    s->fpbA = std::max(std::max(1, 64 / s->bs), (s->nbr + 1023) / 1024);
    s->fpbA = std::min(s->fpbA, std::max(1, 512 / s->bs));
    s->gblkA = std::max(1, (s->nbr + s->fpbA - 1) / s->fpbA);
    auto up = [&](int* d, const std::vector<int>& h) {
        return h.empty() ? hipSuccess
                         : hipMemcpy(d, h.data(), 4 * h.size(), hipMemcpyHostToDevice);
    };
    if (up(s->rowptr, rowptr) != hipSuccess || up(s->col, col) != hipSuccess ||
        up(s->tcol, tcol) != hipSuccess ||
        up(s->ell, ell) != hipSuccess ||
        up(s->contrib, contrib) != hipSuccess || up(s->tside, tside) != hipSuccess ||
        up(s->diag_blk, diag) != hipSuccess ||
        (m->efr && up(s->efr_cptr, ecptr) != hipSuccess) ||
        up(s->efr_contrib, econtrib) != hipSuccess ||
        false) {
        free_solver(s);
        delete s;
        return fail(FR_E_DEVICE, "upload of solver tables failed");
    }
    if (!o->caller_workspace) {
        if (hipMalloc(&s->ws_owned, std::max<size_t>(256, s->ws_bytes)) != hipSuccess) {
            s->ws_owned = nullptr;
            free_solver(s);
            delete s;
            return fail(FR_E_NOMEM, "hipMalloc of the solver workspace failed (" +
                                        std::to_string(s->ws_bytes) + " bytes)");
        }
        if ((e = bind_internal(s, static_cast<char*>(s->ws_owned)))) {
            free_solver(s);
            delete s;
            return e;
        }
    }
    if (ws) *ws = s->ws_bytes;
    *out = s;
    return FR_OK;
}

extern "C" fr_status hfr_solver_bind_workspace(hfr_solver_t s, void* dev_ptr,
                                               size_t bytes) {
    if (!s || !dev_ptr) return fail(FR_E_INVALID, "null argument");
    if (!s->opts.caller_workspace)
        return fail(FR_E_INVALID, "solver owns its workspace (caller_workspace = 0)");
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 256)
        return fail(FR_E_INVALID, "workspace must be 256-byte aligned");
    if (bytes < s->ws_bytes)
        return fail(FR_E_INVALID, "workspace too small: " + std::to_string(bytes) + " < " +
                                      std::to_string(s->ws_bytes) + " bytes");
    return bind_internal(s, static_cast<char*>(dev_ptr));
}

extern "C" void hfr_solver_destroy(hfr_solver_t s) {
    if (!s) return;
    free_solver(s);
    delete s;
}

extern "C" fr_status hfr_residual(hfr_solver_t s, const double* u,
                                  const double* uhat, const double* ustar,
                                  double aii_dt, double* h, double* g,
                                  double* R_im, void* stream) {
    if (!s || !u || (!uhat && s->mesh->Ntp) || !ustar)
        return fail(FR_E_INVALID, "null argument");
    if (fr_status ew = need_workspace(s)) return ew;
    hipStream_t st = hipStream_t(stream);
    fr_mesh_s* m = s->mesh;
    fr_status e = residual_internal(s, u, uhat, ustar, aii_dt, R_im, st);
    if (e) return e;
    if (h && m->Nim)
        HIP_TRY(hipMemcpyAsync(h, s->h, sizeof(double) * 4 * m->Nim * m->Np,
                               hipMemcpyDeviceToDevice, st));
    if (g && m->Ntp)
        HIP_TRY(hipMemcpyAsync(g, s->g, sizeof(double) * 4 * m->Ntp,
                               hipMemcpyDeviceToDevice, st));
    return FR_OK;
}

extern "C" fr_status hfr_assemble_condense(hfr_solver_t s, const double* u,
                                           const double* uhat,
                                           const double* ustar, double aii_dt,
                                           void* stream) {
    if (!s || !u || (!uhat && s->mesh->Ntp) || !ustar)
        return fail(FR_E_INVALID, "null argument");
    if (fr_status ew = need_workspace(s)) return ew;
    hipStream_t st = hipStream_t(stream);
    fr_status e = residual_internal(s, u, uhat, ustar, aii_dt, nullptr, st);
    if (e) return e;
    e = condense_internal(s, u, uhat, aii_dt, st);
    if (!e) s->have_factors = true;
    return e;
}

extern "C" fr_status hfr_trace_solve(hfr_solver_t s, double* duhat,
                                     hfr_solve_stats* stats, void* stream) {
    if (!s || (!duhat && s->N)) return fail(FR_E_INVALID, "null argument");
    if (fr_status ew = need_workspace(s)) return ew;
    return gmres(s, duhat, stats, hipStream_t(stream));
}

extern "C" fr_status hfr_recover(hfr_solver_t s, const double* duhat,
                                 double* du, void* stream) {
    if (!s || (!duhat && s->N) || (!du && s->mesh->Nim))
        return fail(FR_E_INVALID, "null argument");
    if (fr_status ew = need_workspace(s)) return ew;
    fr_mesh_s* m = s->mesh;
    HIP_TRY(launch_recover(m->ops, m->efr, m->Nim, s->M, s->opts.precision, s->piv, s->yr,
                           m->d_trace_map, duhat, du, hipStream_t(stream), nullptr,
                           s->compact));
    return FR_OK;
}

extern "C" fr_status hfr_trace_matvec(hfr_solver_t s, const double* x,
                                      double* y, void* stream) {
    if (!s || (s->N && (!x || !y))) return fail(FR_E_INVALID, "null argument");
    if (fr_status ew = need_workspace(s)) return ew;
    fr_mesh_s* m = s->mesh;
    if (fr_status el = form_L(s, hipStream_t(stream))) return el;
    HIP_TRY(launch_spmv(s->nbr, s->bs, s->rowptr, s->col, s->L64,
                        s->L64 ? nullptr : s->L32, x, y, 1.0, nullptr,
                        hipStream_t(stream)));
    return FR_OK;
}

extern "C" fr_status hfr_trace_product(hfr_solver_t s, const double* x, double* y,
                                       void* stream) {
    if (!s || (s->N && (!x || !y))) return fail(FR_E_INVALID, "null argument");
    if (fr_status ew = need_workspace(s)) return ew;
    if (s->N == 0) return FR_OK;
    HIP_TRY(launch_block_product(gmres_args(s), x, y, hipStream_t(stream)));
    return FR_OK;
}

extern "C" fr_status hfr_get_system(hfr_solver_t s, double* t, double* h,
                                    double* g, void* stream) {
    if (!s) return fail(FR_E_INVALID, "null solver");
    if (fr_status ew = need_workspace(s)) return ew;
    fr_mesh_s* m = s->mesh;
    hipStream_t st = hipStream_t(stream);
    if (t && s->N) HIP_TRY(hipMemcpyAsync(t, s->t, 8 * size_t(s->N), hipMemcpyDeviceToDevice, st));
    if (g && s->N) HIP_TRY(hipMemcpyAsync(g, s->g, 8 * size_t(s->N), hipMemcpyDeviceToDevice, st));
    if (h && m->Nim)
        HIP_TRY(hipMemcpyAsync(h, s->h, 8 * size_t(4) * m->Nim * m->Np,
                               hipMemcpyDeviceToDevice, st));
    return FR_OK;
}

extern "C" fr_status hfr_get_blocks(hfr_solver_t s, double* blocks,
                                    void* stream) {
    if (!s || !blocks) return fail(FR_E_INVALID, "null argument");
    if (fr_status ew = need_workspace(s)) return ew;
    if (!s->blocks_copy) return fail(FR_E_INVALID, "solver created without keep_blocks");
    fr_mesh_s* m = s->mesh;
    const size_t nb = size_t(m->Nim) * (s->n + s->m) * (s->n + s->m) * 8;
    HIP_TRY(hipMemcpyAsync(blocks, s->blocks_copy, nb, hipMemcpyDeviceToDevice,
                           hipStream_t(stream)));
    return FR_OK;
}

extern "C" fr_status hfr_get_factors(hfr_solver_t s, void* factors,
                                     int32_t* piv, void* stream) {
    if (!s || !factors) return fail(FR_E_INVALID, "null argument");
    if (fr_status ew = need_workspace(s)) return ew;
    fr_mesh_s* m = s->mesh;
    const size_t scal = s->opts.precision == HFR_PREC_FP64 ? 8 : 4;
    hipStream_t st = hipStream_t(stream);
    if (m->Nim) {
        HIP_TRY(hipMemcpyAsync(factors, s->M, size_t(m->Nim) * s->elem_M * scal,
                               hipMemcpyDeviceToDevice, st));
        if (piv)
            HIP_TRY(hipMemcpyAsync(piv, s->piv, size_t(m->Nim) * s->n * 4,
                                   hipMemcpyDeviceToDevice, st));
    }
    return FR_OK;
}

extern "C" fr_status hfr_get_preconditioner(hfr_solver_t s, void* dinv,
                                            void* stream) {
    if (!s || !dinv) return fail(FR_E_INVALID, "null argument");
    if (fr_status ew = need_workspace(s)) return ew;
    fr_mesh_s* m = s->mesh;
    const int pc = s->opts.precond;
    const size_t scal = pc == HFR_PC_FP64 ? 8 : pc == HFR_PC_FP32 ? 4 : 2;
    if (s->nbr)
        HIP_TRY(hipMemcpyAsync(dinv, s->Dinv, size_t(s->nbr) * s->bs * s->bs * scal,
                               hipMemcpyDeviceToDevice, hipStream_t(stream)));
    return FR_OK;
}

extern "C" fr_status imex_stage(fr_mesh_t mesh, hfr_solver_t s,
                                const imex_tableau* tab, int32_t stage,
                                double dt, const imex_state* stt,
                                hfr_newton_stats* stats, void* stream) {
    if (!mesh || !tab || !stt || !stt->u_n || !stt->u)
        return fail(FR_E_INVALID, "null argument");
    fr_mesh_s* m = mesh;
    const int S = tab->s;
    if (S < 1 || S > 4) return fail(FR_E_INVALID, "tableau stages must be 1..4");
    if (stage < 0 || stage > S + 1) return fail(FR_E_INVALID, "stage out of range");
    if ((m->Nex && !stt->R_ex) || (m->Nim && !stt->R_im) || (m->Ntp && !stt->uhat))
        return fail(FR_E_INVALID, "missing stage buffers");
    hipStream_t st = hipStream_t(stream);
    const size_t pex = 4 * size_t(m->Nex) * m->Np, pim = 4 * size_t(m->Nim) * m->Np;
    {
        // every stage reads u_n after u (and the stage buffers) were written
        const size_t nall = 4 * size_t(m->Ne) * m->Np;
        auto overlaps = [&](const double* b, size_t nb) {
            return b && nb && stt->u_n < b + nb && b < stt->u_n + nall;
        };
        if (overlaps(stt->u, nall) || overlaps(stt->uhat, 4 * size_t(m->Ntp)) ||
            overlaps(stt->R_im, size_t(S) * pim) || overlaps(stt->R_ex, size_t(S + 1) * pex))
            return fail(FR_E_INVALID, "u_n overlaps u, uhat, R_im or R_ex");
    }
    if (m->host_only) return fail(FR_E_INVALID, "host-only mesh");
    if (m->Nim && (!s || s->mesh != mesh))
        return fail(FR_E_INVALID, "a solver of this mesh is required");
    if (m->Nim)
        if (fr_status ew = need_workspace(s)) return ew;
    if (stats) *stats = hfr_newton_stats{};
    if (stage == 0) {
        HIP_TRY(hipMemcpyAsync(stt->u, stt->u_n, 8 * 4 * size_t(m->Ne) * m->Np,
                               hipMemcpyDeviceToDevice, st));
        int tk = tbegin(s, HFR_T_EXPLICIT, st);
        fr_status ex = fr_explicit_rhs(mesh, stt->u_n, stt->R_ex, stream);
        tend(s, tk, st);
        return ex;
    }
    if (stage == S + 1) {
        const double* terms[6];
        double coefs[6];
        for (int j = 0; j <= S; ++j) {
            terms[j] = stt->R_ex + j * pex;
            coefs[j] = dt * tab->bbar[j];
        }
        HIP_TRY(launch_combine(m->Nex, m->Np, m->Ne, m->d_exp, stt->u_n, S + 1,
                               terms, coefs, stt->u, 1, m->d_dtscale, st));
        for (int j = 0; j < S; ++j) {
            terms[j] = stt->R_im + j * pim;
            coefs[j] = dt * tab->b[j];
        }
        HIP_TRY(launch_combine(m->Nim, m->Np, m->Ne, m->d_imp, stt->u_n, S,
                               terms, coefs, stt->u, 1, m->d_dtscale, st));
        return FR_OK;
    }
    const int I = stage;   // 1-based implicit stage
    {
        const double* terms[6];
        double coefs[6];
        for (int j = 0; j < I; ++j) {
            terms[j] = stt->R_ex + j * pex;
            coefs[j] = dt * tab->Abar[I * (S + 1) + j];
        }
        HIP_TRY(launch_combine(m->Nex, m->Np, m->Ne, m->d_exp, stt->u_n, I,
                               terms, coefs, stt->u, 1, m->d_dtscale, st));
    }
    if (m->Nim) {
        // the implicit stage's wall time runs from here (queued work
        // drained) to R_i ready: u*, the initial trace, Newton and R_i
        fr_status e = sync_check(st);
        if (e) return e;
        const auto t0 = std::chrono::steady_clock::now();
        const double* terms[6];
        double coefs[6];
        for (int j = 0; j < I - 1; ++j) {
            terms[j] = stt->R_im + j * pim;
            coefs[j] = dt * tab->A[(I - 1) * S + j];
        }
        HIP_TRY(launch_combine(m->Nim, m->Np, m->Ne, m->d_imp, stt->u_n, I - 1,
                               terms, coefs, s->ustar, 0, m->d_dtscale, st));
        const double aii_dt = dt * tab->A[(I - 1) * S + (I - 1)];
        if (m->efr)
            HIP_TRY(launch_efr_trace_average(m->ops, m->Ntp, m->Ne, m->d_efr_inc_ptr,
                                             m->d_efr_inc, m->d_imp, stt->u,
                                             stt->uhat, st));
        else
            HIP_TRY(launch_trace_average_ops(m->ops, m->Ntp, m->Ne, m->d_tpside,
                                             m->d_imp, stt->u, stt->uhat, st));
        hfr_newton_stats ns{};
        // R_i of the converged iterate comes with Newton's last check
        e = newton(s, stt->u, stt->uhat, s->ustar, aii_dt, &ns, st,
                   stt->R_im + (I - 1) * pim);
        const fr_status e2 = sync_check(st);
        ns.implicit_ms = std::chrono::duration<double, std::milli>(
                             std::chrono::steady_clock::now() - t0).count();
        if (stats) *stats = ns;
        if (e) return e;
        if (e2) return e2;
    }
    int tk = tbegin(s, HFR_T_EXPLICIT, st);
    fr_status ex = fr_explicit_rhs(mesh, stt->u, stt->R_ex + I * pex, stream);
    tend(s, tk, st);
    if (s && s->pending.size() > 4096) tflush(s);
    return ex;
}

extern "C" fr_status imex_tableau_get(int32_t id, imex_tableau* out) {
    if (!out) return fail(FR_E_INVALID, "null tableau");
    if (id != IMEX_HIMEX2C && id != IMEX_ARS222)
        return fail(FR_E_INVALID, "unknown tableau id");
    *out = imex_tableau{};
    // implicit part: the SDIRK2 tableau of Section 3.1
    const double g = 1.0 - std::sqrt(0.5);
    out->s = 2;
    out->A[0] = g;
    out->A[2] = 1.0 - g;
    out->A[3] = g;
    out->b[0] = 1.0 - g;
    out->b[1] = g;
    // explicit partner in the padded form (c_bar = [0 c]), second order
    const double d = 1.0 - 1.0 / (2.0 * g);
    out->Abar[1 * 3 + 0] = g;
    out->Abar[2 * 3 + 0] = d;
    out->Abar[2 * 3 + 1] = 1.0 - d;
    if (id == IMEX_HIMEX2C) {
        out->bbar[1] = out->b[0];
        out->bbar[2] = out->b[1];
    } else {
        out->bbar[0] = d;
        out->bbar[1] = 1.0 - d;
    }
    return FR_OK;
}

extern "C" fr_status hfr_condense_choice(hfr_solver_t s, int32_t* kernel,
                                         double* candidate_ms) {
    if (!s || !kernel) return fail(FR_E_INVALID, "null argument");
    *kernel = s->ck > 0 ? s->ck : s->opts.condense_kernel;
    if (candidate_ms)
        for (int i = 0; i < 3; ++i) candidate_ms[i] = s->tune_ms[i];
    return FR_OK;
}

extern "C" fr_status hfr_timing(hfr_solver_t s, int32_t enable, double* ms,
                                int64_t* counts) {
    if (!s) return fail(FR_E_INVALID, "null solver");
    if (ms || counts) {
        tflush(s);
        for (int i = 0; i < HFR_NTIMERS; ++i) {
            if (ms) ms[i] = s->tms[i];
            if (counts) counts[i] = s->tcnt[i];
        }
    }
    if (enable == -1) {
        // leave the timers as they are
    } else if (enable == 1 || (enable > 0 && (enable & HFR_TIMING_SELECT))) {
        tflush(s);
        for (int i = 0; i < HFR_NTIMERS; ++i) {
            s->tms[i] = 0.0;
            s->tcnt[i] = 0;
        }
        s->timing = true;
        s->tmask = enable == 1 ? (1u << HFR_NTIMERS) - 1
                               : unsigned(enable) & ((1u << HFR_NTIMERS) - 1);
    } else if (enable == 0) {
        s->timing = false;
    } else {
        return fail(FR_E_INVALID, "hfr_timing: enable must be -1, 0, 1 or "
                                  "HFR_TIMING_SELECT | categories");
    }
    return FR_OK;
}
