/*
 * hfr_imex.h -- C ABI of the MI355X (gfx950) hot path of hybridized
 * implicit-explicit flux reconstruction (Pereira & Vermeire, "Hybridized
 * Implicit-Explicit Flux Reconstruction Methods", arXiv 2401.16632).
 *
 * Scope: two-dimensional Euler equations on bilinear quadrilaterals of one
 * polynomial degree p (1..5), Gauss-Legendre solution and flux points,
 * DG-recovering correction functions.  The explicit region uses standard FR
 * (Section 2.1), the implicit region hybridized FR (Section 2.2) advanced by
 * the padded SDIRK part of an additive IMEX Runge-Kutta pair (Sections 3.1
 * and 4), coupled through standard FR fluxes on the interface Upsilon
 * (eq:hfrimex).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All device pointers are HIP device memory owned by the caller unless
 *    stated otherwise.  Streams are hipStream_t passed as void* (NULL = the
 *    null stream).  Calls are asynchronous on that stream unless stated.
 *  - Element state layout ("SoA"): double u[4][N][Np], variable-major, then
 *    element, then solution point; Np = (p+1)^2 and point index j*(p+1)+i
 *    with i the xi index.  Variables: rho, rho*u, rho*v, E.  N is the number
 *    of elements of the set the array covers (all, implicit or explicit, in
 *    the order returned by fr_mesh_get_maps).
 *  - Trace layout: double uhat[Ntp][4] (point-major).  Trace point id =
 *    trace_face * (p+1) + (point index along the owner, counter-clockwise).
 *  - Canonical numbering: local face f of a quad joins local vertices f and
 *    f+1 (counter-clockwise; f=0: eta=-1, 1: xi=+1, 2: eta=+1, 3: xi=-1);
 *    faces are numbered on first encounter in (element, local face) order,
 *    the first element being the owner; trace faces (both sides implicit)
 *    are numbered densely in face order.
 *  - Every call returns an fr_status.  No call throws.  On a non-OK status
 *    fr_last_error() returns a message for the calling thread.  Asynchronous
 *    device faults surface as FR_E_DEVICE at the next call that
 *    synchronises.
 */
#ifndef HFR_IMEX_H
#define HFR_IMEX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FR_MAX_ORDER 5

typedef enum {
    FR_OK = 0,
    FR_E_INVALID = -1,       /* bad argument (null pointer, size, range)   */
    FR_E_MESH = -2,          /* inconsistent or clockwise mesh             */
    FR_E_NOMEM = -3,         /* device or host allocation failed           */
    FR_E_DEVICE = -4,        /* HIP runtime error                          */
    FR_E_NOT_CONVERGED = -5, /* Newton or Krylov iteration cap reached     */
    FR_E_NONFINITE = -6,     /* NaN/Inf met in a residual                  */
    FR_E_UNSUPPORTED = -7    /* option not built for this configuration    */
} fr_status;

enum { FR_BC_INTERIOR = 0, FR_BC_WALL = 1, FR_BC_FARFIELD = 2 };
enum { FR_FACE_EXPLICIT = 0, FR_FACE_UPSILON = 1, FR_FACE_TRACE = 2,
       FR_FACE_BOUNDARY = 3 };

typedef struct fr_mesh_s* fr_mesh_t;       /* opaque, library-owned */
typedef struct hfr_solver_s* hfr_solver_t; /* opaque, library-owned */

/*
 * Mesh description (host arrays, copied by fr_mesh_create).
 *   node_xy[2*n_nodes]          vertex coordinates (x0,y0,x1,y1,...)
 *   node_topo[n_nodes]          topological vertex id (periodic twins share
 *                               one id); NULL = identity
 *   elem_nodes[4*n_elems]       vertex ids, counter-clockwise
 *   elem_face_bc[4*n_elems]     FR_BC_* per local edge; NULL = all interior
 *   order                       polynomial degree p, 1..FR_MAX_ORDER
 *   implicit_mask[n_elems]      1 = implicit (hybridized) element; if NULL
 *                               an element is implicit iff its stiffness
 *                               indicator E_s = area/perimeter (Section 5)
 *                               is <= es_cutoff
 *   gamma, uinf[4]              ratio of specific heats; far-field state
 *                               (in the variables of the physics)
 *   physics                     FR_PHYS_EULER: two-dimensional Euler,
 *                               u = (rho, rho u, rho v, E);
 *                               FR_PHYS_EDAC: the EDAC equations of
 *                               Appendix A (inviscid part), u = (P, v_x,
 *                               v_y, v_z) on the two-dimensional mesh (fields
 *                               independent of z, v_z passive), hybridized
 *                               stabilisation s = 3/2 |vhat| + dhat,
 *                               dhat^2 = |vhat|^2/4 + Phat + theta
 *   theta                       EDAC: 1/M^2 (artificial Mach number M), > 0
 *   flags                       FR_MESH_HOST_ONLY: build the host tables
 *                               only (maps and counts; no device upload,
 *                               compute calls on it return FR_E_INVALID)
 */
#define FR_MESH_HOST_ONLY 1
/* FR_MESH_EFR: interior-embedded trace (Section 2.3, the EFR choice after
 * eq:hfrspaces): the trace of the implicit region is nodal at the
 * Gauss-Lobatto-Legendre points of each trace face and continuous, a node
 * at a vertex being shared by every trace face incident to it.  Nodes are
 * numbered over the trace faces in order: on each, along the owner's
 * counter-clockwise direction, the start vertex (if new), the p-1 interior
 * GLL nodes, the end vertex (if new).  Without it the trace is the
 * discontinuous HFR trace at the Gauss flux points. */
#define FR_MESH_EFR 2
enum { FR_PHYS_EULER = 0, FR_PHYS_EDAC = 1 };
typedef struct {
    int32_t n_nodes;
    const double* node_xy;
    const int32_t* node_topo;
    int32_t n_elems;
    const int32_t* elem_nodes;
    const int8_t* elem_face_bc;
    int32_t order;
    const uint8_t* implicit_mask;
    double es_cutoff;
    double gamma;
    double uinf[4];
    int32_t flags;
    int32_t physics;
    double theta;
    /* several independent meshes in one: with n_instances > 0, elem_instance
     * [n_elems] gives each element's instance (0..n_instances-1); no face may
     * join elements of two instances (FR_E_MESH).  NULL / 0: one instance */
    const int32_t* elem_instance;
    int32_t n_instances;
} fr_mesh_desc;

typedef struct {
    int32_t order, n_pts, n_elems, n_faces, n_implicit, n_explicit;
    int32_t n_trace_faces, n_trace_points, n_upsilon, n_boundary;
    int32_t n_loc;   /* element block size n = 4 (p+1)^2                  */
    int32_t m_loc;   /* element trace block size m = 16 (p+1) (all faces) */
    size_t device_table_bytes;
    int32_t efr;     /* 1 for the interior-embedded trace (FR_MESH_EFR);
                        n_trace_points then counts trace nodes             */
    int32_t n_instances;  /* independent instances (0: one mesh)           */
} fr_mesh_info;

/*
 * fr_mesh_create: builds the skeleton (Section 2), the IMEX partition and
 * Upsilon (Section 4), the flux-point-to-trace-point map of eq:assembly and
 * the device tables.  Host-synchronous.  FR_E_MESH for a clockwise or
 * folded element, an edge traversed twice, an unmatched edge without a
 * boundary tag, a boundary tag on a matched edge or an element that is its
 * own neighbour.
 */
fr_status fr_mesh_create(const fr_mesh_desc* desc, fr_mesh_t* out);
void fr_mesh_destroy(fr_mesh_t mesh);
/*
 * fr_mesh_set_instance_dt: per-instance time steps of a mesh with
 * n_instances > 0 (host array dt[n_instances], each > 0 and finite):
 * afterwards every time-step factor of imex_stage on an element is the
 * stage call's dt times its instance's dt[...] (call imex_stage with
 * dt = 1 to advance every instance by its own step).  The stage residual h
 * and the element blocks scale a_ii dt the same way.  Host-synchronous.
 * FR_E_INVALID for a mesh without instances, a null pointer or a
 * non-positive step.
 */
fr_status fr_mesh_set_instance_dt(fr_mesh_t mesh, const double* dt);
fr_status fr_mesh_get_info(fr_mesh_t mesh, fr_mesh_info* out);

/*
 * fr_mesh_get_maps: copies host tables into caller buffers (any may be
 * NULL): face_elem[2*Nf], face_local[2*Nf] (owner, neighbour; -1 for a
 * boundary face's neighbour), face_kind[Nf] (FR_FACE_*),
 * trace_map[Nim*4*(p+1)] (trace point of each flux point of each implicit
 * element in its own counter-clockwise order, -1 off the trace; with
 * FR_MESH_EFR, the trace node of each face GLL node instead),
 * implicit_elems[Nim], explicit_elems[Nex], es[Ne], sol_xy[Ne*Np*2]
 * (solution-point coordinates, element-major, point, then x/y).
 */
fr_status fr_mesh_get_maps(fr_mesh_t mesh, int32_t* face_elem,
                           int32_t* face_local, int32_t* face_kind,
                           int32_t* trace_map, int32_t* implicit_elems,
                           int32_t* explicit_elems, double* es,
                           double* sol_xy);

/*
 * fr_explicit_rhs: standard FR residual R = du/dt of eq:freq1 (Rusanov flux
 * of Section 2.1 on every interior face, the same flux against a ghost state
 * on boundary faces: the slip wall mirrors the normal momentum, the far field
 * is uinf) for every explicit element.  At Upsilon faces the implicit
 * neighbour's current state is used (eq:explicitimex).
 *   u     [4][Ne][Np]   full state (device, read)
 *   R_ex  [4][Nex][Np]  residual of the explicit elements (device, written)
 */
fr_status fr_explicit_rhs(fr_mesh_t mesh, const double* u, double* R_ex,
                          void* stream);

/*
 * Modal filter of Appendix B: F = V Lambda* V^-1 per element and variable,
 * V the Vandermonde matrix of the tensor-product orthonormal Legendre basis
 * psi_a(xi) psi_b(eta) at the solution points, Lambda diagonal with
 * sigma(a + b):
 *   1                                                    a + b <  eta_c
 *   exp(-alpha ((a + b - eta_c) / (eta_max - eta_c))^s)  otherwise,
 * eta_max = 2p the largest exponent sum of the basis.  The time-step
 * normalisation Lambda* is taken as Lambda^kappa (kappa = 1: the filter
 * as written; kappa = dt / dt_ref keeps the damping per unit time fixed).
 * The airfoil run of Section 5 uses alpha = 100, s = 1, eta_c = 3.
 */
typedef struct {
    double alpha;   /* damping, >= 0                      */
    double s;       /* strength (exponent), > 0           */
    double eta_c;   /* cut-off exponent sum               */
    double kappa;   /* time-step normalisation exponent, >= 0 */
} fr_filter_params;

/*
 * fr_modal_filter: u [4][Ne][Np] (device, read and written in place) is
 * replaced by its filtered values on every element, on `stream`.  The mean
 * mode is never damped.  FR_E_INVALID for a null argument, a host-only mesh
 * or a parameter outside the ranges above.
 */
fr_status fr_modal_filter(fr_mesh_t mesh, const fr_filter_params* prm,
                          double* u, void* stream);

/* ----------------------------------------------------------------------- */
/* Implicit (hybridized) stage                                             */
/* ----------------------------------------------------------------------- */

enum { HFR_PREC_FP64 = 0,   /* element tableaux eliminated in FP64         */
       HFR_PREC_FP32 = 1 }; /* element tableaux (A^-1 B, Schur complement)
                               formed and stored in FP32, by the kernel
                               hfr_opts.condense_kernel selects: the
                               vector-ALU Gauss-Jordan sweep, or panels of
                               16 exchanges whose updates of the rest of the
                               tableau run on FP32 matrix-core tiles; the
                               condensed right-hand side is accumulated in
                               FP64                                        */
enum { HFR_PC_FP64 = 0, HFR_PC_FP32 = 1, HFR_PC_BF16 = 2 };

typedef struct {
    int32_t precision;        /* HFR_PREC_*                                  */
    int32_t precond;          /* HFR_PC_*: storage of the block-Jacobi inverse */
    int32_t gmres_restart;    /* Krylov dimension before restart (<= 64)     */
    int32_t gmres_max_iters;  /* total inner iterations per trace solve      */
    double gmres_rtol;        /* relative residual target of a trace solve   */
    int32_t newton_max_iters; /* per stage                                   */
    double newton_tol;        /* stop when max(|h|inf,|g|inf) <=
                                 newton_tol * max(1, |u*|inf)                */
    int32_t keep_blocks;      /* 1: keep a copy of the element blocks
                                 [A B; C D] (FP64) for inspection            */
    int32_t jacobian_lag;     /* 0: re-linearise at every Newton iteration;
                                 K > 0: re-linearise (blocks, LU, Schur, L)
                                 only at the first iteration of every K-th
                                 stage solve and otherwise reuse the stored
                                 factors, re-condensing only the right-hand
                                 side (the paper updates its Jacobian every
                                 100 steps, Sec. 5.3)                        */
    int32_t gmres_cgs_passes; /* classical Gram-Schmidt passes per Arnoldi
                                 step: 1 (also when 0) or 2 (each new
                                 vector orthogonalised twice)                */
    int32_t caller_workspace; /* 0: hfr_solver_create allocates the working
                                 device memory itself; 1: the caller owns it
                                 and passes it to hfr_solver_bind_workspace
                                 before any other call on the solver         */
    int32_t condense_kernel;  /* element elimination inside Newton (the
                                 Schur-only condensation): HFR_CK_AUTO,
                                 HFR_CK_SWEEP or HFR_CK_BLOCKED              */
    int32_t newton_damping;   /* 1: a Newton update after which the
                                 residual is not finite is halved, up to
                                 seven times, before the iteration goes on
                                 (the paper's Newton takes full steps; this
                                 guards impulsive starts at high local CFL,
                                 where a full step can leave the admissible
                                 states); 0: full steps only                  */
    int32_t iteration_graph;  /* 1: inside Newton (Jacobian re-formed every
                                 iteration, timers off) the elimination,
                                 assembly, preconditioner set-up, the first
                                 chunk of the trace solve and the checks of
                                 the next iterate are recorded as a HIP graph
                                 once per chunk length and stage arguments
                                 and replayed on the caller's stream: the same
                                 kernels in the same order as the eager queue,
                                 hence the same results bit for bit; a solve
                                 that needs more steps goes on eagerly.
                                 The graphs name the stage buffers and the
                                 workspace; rebinding the workspace drops
                                 them.  0: eager launches only               */
    double gmres_forcing_max; /* 0: every trace solve inside Newton to
                                 gmres_rtol.  In [gmres_rtol, 1): inexact
                                 Newton; the k-th solve of a stage stops at
                                 the relative residual eta_k = 0.1 max(r_k
                                 (r_k/r_{k-1})^2, tol) / r_k clamped to
                                 [gmres_rtol, gmres_forcing_max], with r_k =
                                 max(|h|inf, |g|inf) of the current iterate
                                 and tol the Newton tolerance (the quadratic
                                 model of the next residual, so the linear
                                 error stays below it); eta_0 =
                                 gmres_forcing_max.  Formed on the device
                                 with the Newton norms.  The converged stage
                                 is the same to the Newton tolerance;
                                 hfr_trace_solve always uses gmres_rtol      */
} hfr_opts;
/* HFR_CK_SWEEP: register-resident Gauss-Jordan sweep on the vector ALUs, one
 * exchange per step; HFR_CK_BLOCKED: panels of 16 exchanges, the update of
 * the rest of the tableau a product on the 16x16x4 matrix-core tiles (4 or
 * more waves per element), the Schur complement formed in the same launch,
 * and in FP32 up to p = 4 the element linearisation as well (no separate
 * tableau fill); HFR_CK_BLOCKED_W8: the same with 8 waves per element;
 * HFR_CK_AUTO: the library's choice for the order and precision. */
enum { HFR_CK_AUTO = 0, HFR_CK_SWEEP = 1, HFR_CK_BLOCKED = 2, HFR_CK_BLOCKED_W8 = 3 };

typedef struct {
    int32_t iterations;       /* Krylov iterations of the last trace solve   */
    int32_t restarts;
    double rel_residual;      /* |t - L x| / |t| at exit (FP64)              */
} hfr_solve_stats;

typedef struct {
    int32_t newton_iters;
    int32_t gmres_iters;      /* summed over Newton iterations               */
    double residual;          /* final max(|h|inf, |g|inf)                   */
    double implicit_ms;       /* imex_stage: host wall time of the implicit
                                 stage, from its entry (queued work drained)
                                 to R_i ready: u*, initial trace, every
                                 Newton iteration, R_i                      */
    int32_t graph_replays;    /* Newton iterations run as a replayed graph
                                 (hfr_opts.iteration_graph)                 */
    int32_t queued_linearisations; /* Newton iterations whose condensation
                                 was queued behind the previous iterate's
                                 checks, before the host read them (blocked
                                 elimination kernel, no timers, graphs or
                                 damping; the device skips such a launch
                                 when the checks pass)                      */
} hfr_newton_stats;

/*
 * hfr_solver_create: builds the block structure of the condensed trace
 * system of Section 3.2 (one block row per trace face, or per trace node
 * with FR_MESH_EFR) and the element-to-block assembly lists of eq:assembly,
 * uploaded once as library-owned read-only device tables, and a small
 * pinned host buffer for the convergence readbacks.  The working device
 * memory (element tableaux, trace matrix and its preconditioned copy,
 * Krylov basis, residuals; one block) is *workspace_bytes long (reported
 * when non-NULL): with opts->caller_workspace = 0 the library allocates and
 * frees it, with 1 the caller provides it through
 * hfr_solver_bind_workspace.  Host-synchronous.
 */
fr_status hfr_solver_create(fr_mesh_t mesh, const hfr_opts* opts,
                            size_t* workspace_bytes, hfr_solver_t* out);
/*
 * hfr_solver_bind_workspace: hands the solver the caller-owned working
 * memory (device, >= the size hfr_solver_create reported, 256-byte
 * aligned; for example a PyTorch tensor).  It must outlive the solver's use
 * of it; the library never frees it.  Binding again (for example another
 * buffer) is allowed between calls; the solver's convergence state and any
 * stored factorisation are reset.  Host-synchronous (clears the Krylov
 * state).  FR_E_INVALID for a null pointer, a solver created with
 * caller_workspace = 0, a misaligned pointer or a short buffer.  Every
 * compute call on a solver without a bound workspace returns FR_E_INVALID.
 */
fr_status hfr_solver_bind_workspace(hfr_solver_t solver, void* dev_ptr,
                                    size_t bytes);
void hfr_solver_destroy(hfr_solver_t solver);

/*
 * hfr_residual: the stage residuals of eq:9oind / eq:23nffsd with the
 * hybridized operator (eq:hfr1, eq:hfr2, eq:hfrimex):
 *   h = u_im - ustar - aii_dt * R^im(u, uhat),  R = du/dt (sign reading of
 *   the paper's inconsistent printed forms), g = transmission residual
 *   collocated at the trace points (face mass diag(w_q J_f)).  On boundary
 *   faces the implicit elements take the hybridized flux against a boundary
 *   trace; reading the undefined boundary flux F^BC of eq:hfr2 as the jump
 *   of the hybridized flux against the ghost state, its transmission
 *   condition s(uhat)|S| (u + u_ghost - 2 uhat) = 0 gives that trace in
 *   closed form, uhat = (u + u_ghost)/2, so it never enters L or g.
 *   u [4][Ne][Np] full state (explicit part used on Upsilon), uhat [Ntp][4],
 *   ustar [4][Nim][Np]; outputs h [4][Nim][Np], g [Ntp][4], R_im
 *   [4][Nim][Np]; any output may be NULL.
 */
fr_status hfr_residual(hfr_solver_t s, const double* u, const double* uhat,
                       const double* ustar, double aii_dt, double* h,
                       double* g, double* R_im, void* stream);

/*
 * hfr_residual_noalloc: hfr_residual for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc); it takes the mesh instead of a solver and calls no
 * allocating routine.  h [4][Nim][Np] and g [Ntp][4] are required outputs,
 * R_im [4][Nim][Np] is optional; inputs as hfr_residual; same kernels, same
 * results.  Its one intermediate, the element shares of g (Nim * 16 (p+1)
 * doubles), lives in a static device array of 2^20 doubles (8 MiB) that
 * every GPU the library runs on holds until the process ends: a mesh whose
 * Nim * 16 (p+1) exceeds 2^20 is refused with FR_E_INVALID before any
 * launch.  All calls on one GPU share that array (every entry a call reads
 * it has written first): calls that overlap on one GPU, on different
 * streams or from different threads, race.
 */
fr_status hfr_residual_noalloc(fr_mesh_t mesh, const double* u,
                               const double* uhat, const double* ustar,
                               double aii_dt, double* h, double* g,
                               double* R_im, void* stream);

/*
 * hfr_assemble_condense: one Newton linearisation (Section 3.2): residuals,
 * element blocks A, B, C, D (eq:elemA, eq:elemsystemB, as exact derivatives
 * of h and g), per-element pivoted LU / Gauss-Jordan of A, X = A^-1 [B r],
 * L^k = D^k - C^k X_B, t^k = s^k - C^k X_r with r = -h, s = -g, and the
 * element-by-element assembly of eq:assembly into a block-sparse L and t
 * (kept inside the solver).  Inputs as hfr_residual.
 */
fr_status hfr_assemble_condense(hfr_solver_t s, const double* u,
                                const double* uhat, const double* ustar,
                                double aii_dt, void* stream);

/*
 * hfr_trace_solve: solves L duhat = t (the condensed trace system of
 * Section 3.2) by restarted GMRES with FP64 Arnoldi (one classical
 * Gram-Schmidt pass per step, two with hfr_opts.gmres_cgs_passes = 2), a
 * right block-Jacobi preconditioner (one diagonal face block per trace face)
 * and an FP64 true-residual recomputation at every restart.
 * Host-synchronous (reads the Krylov coefficients).
 *   duhat [Ntp][4] (device, written).  FR_E_NOT_CONVERGED when the
 *   iteration cap is hit (duhat holds the last iterate).
 */
fr_status hfr_trace_solve(hfr_solver_t s, double* duhat,
                          hfr_solve_stats* stats, void* stream);

/*
 * hfr_recover: local back-substitution eq:localproblems,
 * du_k = A_k^-1 (r_k - B_k duhat_k) = X_r - X_B duhat_k.
 *   duhat [Ntp][4] (device, read), du [4][Nim][Np] (device, written).
 */
fr_status hfr_recover(hfr_solver_t s, const double* duhat, double* du,
                      void* stream);

/* Inspection helpers (tests): y = L x with the assembled trace matrix (the
 * Newton path with the compact element layout forms only L Dinv, and its
 * restarts sum L x from the element sub-blocks; hfr_trace_matvec then forms
 * L first);
 * copies of t [Ntp][4], h [4][Nim][Np], g [Ntp][4] of the last
 * hfr_assemble_condense (device pointers, any may be NULL); element blocks
 * kept with keep_blocks=1, FP64 row-major (n+m) x (n+m) per implicit
 * element with the local ordering (point, variable) for u and
 * (face, point, variable) for the trace. */
fr_status hfr_trace_matvec(hfr_solver_t s, const double* x, double* y,
                           void* stream);
fr_status hfr_get_system(hfr_solver_t s, double* t, double* h, double* g,
                         void* stream);
/* y = L D^-1 x: the product the Krylov solver runs (the trace matrix of the
 * last linearisation times the inverse of its diagonal face blocks, the
 * right block-Jacobi preconditioner of Section 3.2's trace solve), by the
 * block-row code of the Arnoldi product kernel.  x, y [Ntp][4] (device). */
fr_status hfr_trace_product(hfr_solver_t s, const double* x, double* y,
                            void* stream);
fr_status hfr_get_blocks(hfr_solver_t s, double* blocks, void* stream);
/* Swept element tableaux of the last linearisation (static condensation,
 * Section 3.2), N x N per implicit element with N = n + m, COLUMN-major,
 * FP64 or FP32 as the solver's precision.  With p_k the pivot row of
 * exchange k (returned in piv, int32 [Nim][n], may be NULL):
 *   T[p_k][j]   = A^-1[k][p_j]          T[p_k][n+b] = -(A^-1 B)[k][b]
 *   T[n+i][j]   = (C A^-1)[i][p_j]      T[n+i][n+b] = (D - C A^-1 B)[i][b]
 * for j < n, b < m, i < m (element-local ordering as in hfr_get_blocks).
 * After hfr_assemble_condense all four blocks are stored.  The Newton
 * solver with jacobian_lag = 0 never reuses the factors and stores only the
 * columns n+b (A^-1 B and the Schur complement): the first n columns then
 * hold no meaningful values.  With the blocked elimination and face blocks
 * of 20 or 24 rows (p = 4, 5; not with FR_MESH_EFR) it stores the Schur
 * complement instead at the start of the slot as 4 x 4 contiguous face
 * sub-blocks (sub-block (lr, lc) column-major at (4 lc + lr) bs^2, bs =
 * 4(p+1)), followed by -A^-1 B (n x m, column-major, rows in the pivot
 * order above); nothing else in the slot is then meaningful. */
fr_status hfr_get_factors(hfr_solver_t s, void* factors, int32_t* piv,
                          void* stream);
/* Block-Jacobi preconditioner of the last linearisation (the trace solve of
 * Section 3.2 is preconditioned on the right by the inverses of the
 * diagonal face blocks of L): Ntf blocks of bs x bs, bs = 4(p+1), each
 * column-major (dinv[F][b][a] = (L_FF^-1)[a][b]), in the preconditioner
 * precision (FP64, FP32 or BF16 bit patterns). */
fr_status hfr_get_preconditioner(hfr_solver_t s, void* dinv, void* stream);

/*
 * hfr_timing: HIP-event timers around the solver's kernels, on the stream
 * each kernel is launched on (the phases timed in the paper's performance
 * tables: implicit residual t_R^im, Jacobian and condensation t_J, global
 * solve t_G, local solve t_L, explicit residual t_R^ex).  enable = 1 resets
 * and starts every category, HFR_TIMING_SELECT | (1 << HFR_T_x) | ... resets
 * and starts the listed ones only, 0 stops, -1 leaves the state as it is;
 * when ms / counts are non-NULL the accumulated totals (HFR_NTIMERS entries,
 * milliseconds and launch counts) are copied out after a device
 * synchronisation.  Every timed launch adds two event records to the
 * stream, which costs device time: time the phases in a separate pass from
 * the one whose wall time is measured.
 */
/*
 * hfr_condense_choice: the condensation kernel the solver uses inside Newton
 * (HFR_CK_*; HFR_CK_AUTO until the automatic choice has been made) and,
 * when candidate_ms is non-NULL, the times of the automatic choice's
 * candidates (sweep, blocked, blocked with 8 waves; milliseconds per launch
 * on the solver's first linearisation, -1 if not measured).  With
 * hfr_opts.condense_kernel = HFR_CK_AUTO the solver measures every candidate
 * once per (order, precision) and process, on its first Schur-only
 * linearisation (each candidate timed with the tableau fill it needs), and
 * keeps the fastest;
 * later solvers of the same order and precision reuse that choice.
 */
fr_status hfr_condense_choice(hfr_solver_t s, int32_t* kernel, double* candidate_ms);

#define HFR_TIMING_SELECT 0x10000
enum { HFR_T_RESIDUAL = 0,   /* hybridized residual kernel                 */
       HFR_T_CONDENSE = 1,   /* element elimination kernel (condensation;
                                with the linearisation where fused)       */
       HFR_T_ASSEMBLE = 2,   /* block-sparse assembly kernel (t only where
                                L is formed with L Dinv, p = 3..5 HFR)    */
       HFR_T_PCSETUP = 3,    /* block-Jacobi inversion and L Dinv kernels  */
       HFR_T_SPMV = 4,       /* Arnoldi product kernel (block-sparse
                                product + first projection)               */
       HFR_T_TRACE_SOLVE = 5,/* whole trace solve (all Krylov kernels)     */
       HFR_T_RECOVER = 6,    /* local recovery kernel                      */
       HFR_T_EXPLICIT = 7,   /* explicit residual kernel (via imex_stage)  */
       HFR_T_FILL = 8,       /* element linearisation + tableau fill kernel
                                (where not fused into the elimination)    */
       HFR_NTIMERS = 9 };
fr_status hfr_timing(hfr_solver_t s, int32_t enable, double* ms,
                     int64_t* counts);

/* ----------------------------------------------------------------------- */
/* IMEX step (alg:imex with the element partition of Section 4)            */
/* ----------------------------------------------------------------------- */

/*
 * Tableau of an additive pair: s implicit stages (unpadded SDIRK matrix A,
 * weights b) and sigma = s+1 explicit stages (A_bar, b_bar) with
 * c_bar = [0 c] (table:butcherimex).  Row-major, s <= 4.
 */
typedef struct {
    int32_t s;
    double A[16];
    double b[4];
    double Abar[25];
    double bbar[5];
} imex_tableau;

/*
 * imex_tableau_get: fills *out with one of the additive pairs built into the
 * library.  The implicit part of both is the two-stage, second-order SDIRK
 * tableau of Section 3.1 (gamma = 1 - sqrt(2)/2, A = [[gamma, 0],
 * [1 - gamma, gamma]], b = (1 - gamma, gamma)).  The paper's own explicit
 * partners are in a tableau appendix that its text does not contain; the
 * partner here satisfies the second-order conditions in the padded form of
 * table:butcherimex (c_bar = [0 c]): A_bar rows (0,0,0), (gamma,0,0),
 * (delta, 1-delta, 0) with delta = 1 - 1/(2 gamma), and
 *   IMEX_HIMEX2C: b_bar = (0, b), so the Upsilon fluxes cancel over a step
 *                 (exact conservation across the interface, Section 4);
 *   IMEX_ARS222:  b_bar = (delta, 1 - delta, 0).
 * FR_E_INVALID for a null pointer or an unknown id.
 */
enum { IMEX_HIMEX2C = 0, IMEX_ARS222 = 1 };
fr_status imex_tableau_get(int32_t id, imex_tableau* out);

/*
 * Device buffers of one step (all caller-owned):
 *   u_n  [4][Ne][Np]        state at t_n (read)
 *   u    [4][Ne][Np]        stage state; holds u_{n+1} after stage s+1
 *   uhat [Ntp][4]           trace (initial guess in, stage trace out)
 *   R_im [s][4][Nim][Np]    implicit stage residuals R_i
 *   R_ex [s+1][4][Nex][Np]  explicit stage residuals R_bar_j
 */
typedef struct {
    const double* u_n;
    double* u;
    double* uhat;
    double* R_im;
    double* R_ex;
} imex_state;

/*
 * imex_stage: stage = 0 starts a step (u = u_n, R_bar_1 = R^ex(u_n));
 * stage i = 1..s forms u_i^ex (eq:explicitimex) and u* = u_n + dt sum_{j<i}
 * a_ij R_j, solves the hybridized stage by Newton (trace initial guess: the
 * average of the two sides' interpolated states), stores
 * R_i = R^im(u_i, uhat_i) and R_bar_{i+1} = R^ex(u_i); stage s+1 forms
 * u_{n+1}.  Host-synchronous for i = 1..s (Newton convergence test).  On
 * FR_E_NOT_CONVERGED / FR_E_NONFINITE the implicit part of u holds the last
 * Newton iterate and u_n is untouched.  u_n must not overlap u, uhat, R_im
 * or R_ex (FR_E_INVALID): every stage reads it after u has been written.
 */
fr_status imex_stage(fr_mesh_t mesh, hfr_solver_t s, const imex_tableau* tab,
                     int32_t stage, double dt, const imex_state* st,
                     hfr_newton_stats* stats, void* stream);

const char* fr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HFR_IMEX_H */
