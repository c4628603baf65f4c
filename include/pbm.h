/*
 * pbm.h -- C ABI of the MI355X boundary-element Poisson-Boltzmann library.
 *
 * The library computes, for a closed triangulated molecular surface Gamma
 * with point charges inside, the interior surface potential gamma_D^- phi and
 * its normal derivative gamma_N^- phi (the unknowns of the paper's internal
 * direct formulation, Eq. bie:dirichlet:int, and Juffer formulation,
 * Eq. bie:juffer:int) and the polar solvation energy Delta G (Eq. dG) of the
 * linearised Poisson-Boltzmann interface problem (Eq. poissonboltzmann) of
 * Search, Cooper & van 't Wout, arXiv 2108.10481.
 *
 * Discretisation: continuous piecewise-linear (P1) Galerkin on flat
 * triangles (Numerical discretization), one degree of freedom per vertex per
 * trace; the Laplace ("int") and Yukawa ("ext", screening kappa) single-,
 * double-, adjoint double-layer and hypersingular operators (Eq.
 * layer_potentials); regular 6-point degree-4 quadrature on triangle pairs
 * sharing no vertex and Sauter-Schwab quadrature on pairs sharing a vertex;
 * block-diagonal preconditioner (Preconditioning, Algebraic preconditioners);
 * GMRES without restart (Results, tolerance 1e-5).
 *
 * Conventions for every entry point:
 *   - Units: angstrom, elementary charge, 1/angstrom; Delta G in kcal/mol.
 *   - Unless a name ends in _device or _noalloc, pointer arguments are HOST
 *     pointers.
 *     Inputs are read-only and copied during the call; the caller keeps
 *     ownership.  Output arrays are caller-allocated with the stated length.
 *   - Handles are owned by the library: every *_create has a *_destroy.
 *   - Return value: PB_OK (0); a positive value is a warning with a valid
 *     result; a negative value is an error with no result, and
 *     pb_last_error() returns a message for the calling thread.
 *   - No exceptions or callbacks cross the ABI.  Calls on one handle must not
 *     overlap in time; different handles may be used from different threads.
 *   - All device work of a handle runs on its own HIP stream (default
 *     priority).  The library allocates its own device memory.
 */
#ifndef PBM_H
#define PBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- status codes */
typedef int32_t pb_status;
#define PB_OK              0
#define PB_NOT_CONVERGED   1   /* max_iter reached; outputs filled, rel_residual > tol */
#define PB_E_INVALID_ARG  (-1) /* NULL pointer, bad size, NaN input, bad option value */
#define PB_E_MESH         (-2) /* open, non-manifold, inverted or degenerate mesh */
#define PB_E_CHARGES      (-3) /* a charge lies outside the surface */
#define PB_E_NOMEM        (-4) /* device memory or admission budget exceeded */
#define PB_E_DEVICE       (-5) /* HIP runtime error or no usable GPU */
#define PB_E_STATE        (-6) /* call not valid for this handle's configuration */

/* ------------------------------------------------------------------ options */
/* Formulations (e = e_in/e_out; L, Y = Laplace, Yukawa kernels; unknowns are the
 * interior traces (gamma_D^- phi, gamma_N^- phi) unless marked exterior, in which
 * case the solver converts the exterior traces to interior ones,
 * gamma_N^- = (e_out/e_in) gamma_N^+, before Delta G and before returning them). */
#define PB_DIRECT_INT   0  /* Eq. bie:dirichlet:int: [[M/2+K_L, -V_L], [M/2-K_Y, e V_Y]] */
#define PB_JUFFER       1  /* Eq. bie:juffer:int: second-kind, uses all four operators */
#define PB_DIRECT_EXT   2  /* Eq. bie:dirichlet:ext (exterior): [[M/2-K_Y, V_Y], [M/2+K_L, -V_L/e]] */
#define PB_DIRECT_INT_PERM 3  /* Eq. bie:dirichlet:int with its rows swapped */
#define PB_DIRECT_EXT_PERM 4  /* Eq. bie:dirichlet:ext with its rows swapped (exterior) */
#define PB_MULLER_INT   5  /* Eq. bie:muller:int: second-kind */
#define PB_MULLER_EXT   6  /* Eq. bie:muller:ext: second-kind (exterior) */
#define PB_LU           7  /* Eq. bie:lu:ext: second-kind (exterior) */
#define PB_PMCHWT_INT   8  /* Eq. bie:pmchwt:int: first-kind */
#define PB_PMCHWT_EXT   9  /* Eq. bie:pmchwt:ext: first-kind (exterior) */
/* Combined-field formulations with real constants alpha = cfie_alpha, beta =
 * cfie_beta (The combined field formulation):
 *   PB_CFIE_INT, Eq. bie:combined:int, interior unknowns:
 *     [[M/2+K_L, -V_L], [-D_L, M/2-T_L]] + diag(alpha, beta) [[M/2-K_Y, e V_Y], [D_Y/e, M/2+T_Y]],
 *     right-hand side [phi_D; phi_N];
 *   PB_CFIE_EXT, Eq. bie:combined:ext, exterior unknowns:
 *     [[M/2-K_Y, V_Y], [D_Y, M/2+T_Y]] + diag(alpha, beta) [[M/2+K_L, -V_L/e], [-e D_L, M/2-T_L]],
 *     right-hand side diag(alpha, beta) [phi_D; e phi_N].
 * alpha = beta = 1 gives Mueller, alpha = beta = -1 PMCHWT (Eq. bie:pmchwt:ext
 * as printed, Eq. bie:pmchwt:int with the opposite sign), (e_out/e_in,
 * e_in/e_out) Juffer, and the external form at (e, 1/e) is Lu before its
 * second row is scaled.  Any
 * real alpha, beta is accepted; alpha = beta = 0 leaves one side's trace
 * equations alone, which do not couple the interior and exterior problems:
 * such a handle applies its operator (pb_mesh_apply) but every solve entry
 * point refuses it with PB_E_STATE.  With a zero coefficient in the external form
 * a block has no Laplace term; every far-field mode (matrix-free, treecode,
 * assembled) takes such systems. */
#define PB_CFIE_INT    10
#define PB_CFIE_EXT    11

#define PB_PREC_NONE    0
#define PB_BLOCK_DIAG   1  /* per-vertex 2x2 inverse of the four blocks' diagonals */
#define PB_MASS         2  /* blockdiag(M, M)^-1, M the P1 mass matrix (Eq. prec:mass) */
#define PB_SCALED_MASS  3  /* blockdiag(aM, bM)^-1 with a = 1 + e_out/e_in, b = 1 + e_in/e_out
                              (Eq. prec:mass:scaled; Juffer formulation only) */
/* Calderon preconditioners, PMCHWT formulations only (Calderon preconditioning,
 * Eqs. prec:calderon:int and prec:calderon:ext).  The system A u = b is solved
 * as B A u = B b with B = blockdiag(aM, bM)^-1 P blockdiag(M, M)^-1: the
 * Galerkin form of the operator product P A, mass matrices inverted as for
 * PB_MASS.  P is assembled like A (same precision, operator mode, near field). */
#define PB_CALDERON     4  /* P = A itself (an operator of its own with calderon_fast);
                              a = b = 1 (Eqs. prec:calderon:int:full, ext:full) */
#define PB_CALDERON_INT 5  /* P = the Laplace ("interior") part of A; a = b = 1 */
#define PB_CALDERON_EXT 6  /* P = the Yukawa ("exterior") part of A; a = b = 1 */
#define PB_SCALED_CALDERON_INT 7  /* PB_CALDERON_INT with a, b = the two half accumulation
                                     points of Eq. precond:calderon:eigenval_semi, each on
                                     the block row whose eigenvalues gather there */
#define PB_SCALED_CALDERON_EXT 8  /* PB_CALDERON_EXT scaled the same way */

#define PB_FP64         0  /* every kernel evaluation and sum in FP64 */
#define PB_FP32         1  /* far-field kernel evaluations in FP32, tile sums FP32,
                              cross-tile sums, near field and Krylov in FP64 */
#define PB_MIXED_BF16   2  /* assembled far field stored BF16 (FP32 accumulate) for an
                              inner GMRES; FP64 iterative refinement on the FP32 operator */
#define PB_MIXED_FP16   3  /* as PB_MIXED_BF16 with FP16 storage and per-block scales */

#define PB_MATRIX_FREE  0  /* far field recomputed on every matvec */
#define PB_ASSEMBLED    1  /* far field assembled once as a dense 2V x 2V matrix */
#define PB_AUTO         2  /* assembled when it fits the device-memory budget */
#define PB_TREECODE     3  /* matrix-free with the far field approximated by a barycentric
                              Lagrange treecode (a hierarchical scheme in place of the paper's
                              FMM, Implementation): source clusters whose bounding spheres and
                              the target batch's are well separated (r_batch + r_cluster <
                              tree_theta * distance) act through (tree_degree + 1)^3 Chebyshev
                              proxy points; other pairs are summed directly as in
                              PB_MATRIX_FREE.  FP64 or FP32 evaluation as for PB_MATRIX_FREE. */

typedef struct {
    int32_t n_vertices;
    int32_t n_triangles;
    const double *xyz;    /* n_vertices x 3, row-major, angstrom */
    const int32_t *tri;   /* n_triangles x 3, 0-based vertex ids, counter-clockwise
                             seen from the solvent (outward normal) */
} pb_mesh;

typedef struct {
    int32_t n;
    const double *xyz;    /* n x 3, angstrom, strictly inside the surface */
    const double *q;      /* n, elementary charges */
} pb_charges;

typedef struct {
    double eps_in;            /* interior permittivity (paper: 4) */
    double eps_out;           /* exterior permittivity (paper: 80) */
    double kappa;             /* inverse Debye length, 1/angstrom (paper: 0.125) */
    int32_t formulation;      /* PB_DIRECT_INT ... PB_CFIE_EXT */
    int32_t preconditioner;   /* PB_PREC_NONE ... PB_SCALED_CALDERON_EXT */
    int32_t precision;        /* PB_FP64, PB_FP32, PB_MIXED_BF16, PB_MIXED_FP16 */
    int32_t operator_mode;    /* PB_MATRIX_FREE, PB_ASSEMBLED, PB_AUTO, PB_TREECODE */
    double tol;               /* relative preconditioned residual (paper: 1e-5) */
    int32_t max_iter;         /* GMRES iterations (no restart), default 1000 */
    int32_t singular_order;   /* Gauss points per dimension, Sauter-Schwab (default 4) */
    int32_t source_chunks;    /* far-field split of the source range; 0 = automatic */
    int32_t inner_max_iter;   /* mixed modes: inner GMRES cap (default 200) */
    double inner_tol;         /* mixed modes: inner relative tolerance (default 1e-3) */
    size_t memory_budget;     /* bytes the handle may hold on the device; 0 = 90% of free */
    int32_t use_graph;        /* 1 (default): GMRES iterations replayed from a captured HIP
                                 graph with device-side Givens rotations; 0: eager launches */
    int32_t calderon_fast;    /* Calderon preconditioners only.  0 (default): P integrated like A;
                                 1: fast Calderon (Discussion): P with relaxed quadrature, the
                                 one-point (centroid) rule on triangle pairs sharing no vertex,
                                 evaluated matrix-free in FP32 whatever the handle's precision
                                 and operator mode, and Sauter-Schwab with singular_order - 1
                                 Gauss points per dimension (at least 1) on pairs sharing one */
    int32_t tree_degree;      /* PB_TREECODE: interpolation degree per dimension, 2..7 (default 6) */
    double tree_theta;        /* PB_TREECODE: separation ratio, 0 < theta < 1 (default 0.7) */
    double cfie_alpha;        /* PB_CFIE_INT / PB_CFIE_EXT: alpha (default 1) */
    double cfie_beta;         /* PB_CFIE_INT / PB_CFIE_EXT: beta (default 1) */
    int32_t regular_order;    /* quadrature of the triangle pairs sharing no vertex (Numerical
                                 discretization; the paper's "quadrature order"): 4 (default, 0
                                 means the same): the symmetric 6-point degree-4 rule on each
                                 triangle; 1: the one-point (centroid) rule, matrix-free in FP64
                                 or FP32 only, not with the Calderon preconditioners.  The source
                                 projections and Delta G always use the 6-point rule. */
    int32_t far_symmetric;    /* FP32 matrix-free far field, screened or not (Numerical
                                 discretization; the kernels are symmetric in x, y): every
                                 unordered triangle pair evaluated once for both directions or
                                 every ordered pair.  0 (default): once per unordered pair on
                                 meshes of 3584 triangles and more, per ordered pair below (where
                                 one mesh leaves most of the device idle); 1: once per unordered
                                 pair at every size (faster for many small meshes solved together
                                 by pb_solve_batch); -1: per ordered pair.  Single and batched
                                 solves of a handle use the same choice, so their results stay
                                 bitwise equal; the two choices agree to FP32 rounding. */
} pb_options;

typedef struct {
    double *phi;              /* caller-allocated, n_vertices: gamma_D^- phi at the vertices */
    double *dphi;             /* caller-allocated, n_vertices: gamma_N^- phi at the vertices */
    double dG_kcal;           /* polar solvation energy, kcal/mol */
    int32_t iterations;       /* total GMRES iterations (inner iterations in mixed modes) */
    int32_t outer_iterations; /* iterative-refinement sweeps (1 outside mixed modes) */
    double rel_residual;      /* final |P^-1(b - A u)| / |P^-1 b|, recomputed */
    double t_setup;           /* seconds: geometry, near field, assembly ("LHS") */
    double t_rhs;             /* seconds: source projections ("RHS") */
    double t_prec;            /* seconds: preconditioner build and apply to b */
    double t_gmres;           /* seconds: Krylov solve */
    double t_dG;              /* seconds: reaction potential and Delta G */
    size_t device_bytes;      /* device memory held by the mesh handle */
} pb_result;

typedef struct pb_mesh_handle pb_mesh_handle;

typedef struct {
    int32_t n_vertices, n_triangles;
    int64_t n_near_pairs;     /* ordered triangle pairs sharing >= 1 vertex */
    int64_t near_nnz;         /* nonzeros of each near-field vertex block */
    int32_t source_chunks;    /* far-field source split in use */
    int32_t assembled;        /* 1 if the far field is held as a dense matrix */
    size_t device_bytes;
    int32_t far_symmetric;    /* 1 if matrix-free products evaluate every unordered
                                 triangle pair once (FP32, see pb_options.far_symmetric) */
} pb_mesh_info;

/* Fill *opt with the paper's settings: eps 4/80, kappa 0.125, direct
 * formulation, block-diagonal preconditioner, FP64, matrix-free, tol 1e-5,
 * max_iter 1000, singular order 4, regular order 4; cfie_alpha = cfie_beta = 1;
 * far_symmetric 0 (automatic). */
void pb_default_options(pb_options *opt);

/* Thread-local description of the last error on this thread ("" if none). */
const char *pb_last_error(void);

/* Number of visible GPUs (0 if none); does not initialise a context. */
int32_t pb_device_count(void);

/* ------------------------------------------------------------- whole solve */

/* One complete solve (setup, RHS, preconditioner, GMRES, Delta G).
 * result->phi / result->dphi must hold n_vertices doubles each, or be NULL. */
pb_status pb_solve(const pb_mesh *mesh, const pb_charges *charges,
                   const pb_options *opt, pb_result *result);

/* -------------------------------------------------------- resident meshes */

/* Validate the mesh, sort its triangles along a space-filling curve, compute
 * geometry, the Sauter-Schwab near field (FP64, Numerical discretization), the
 * mass matrix, the block-diagonal preconditioner and, in assembled modes, the
 * dense far field.  All of it stays on the device until pb_mesh_destroy.
 * The options fix formulation, precision and operator mode for the handle. */
pb_status pb_mesh_create(const pb_mesh *mesh, const pb_options *opt, pb_mesh_handle **out);
pb_status pb_mesh_destroy(pb_mesh_handle *h);
/* Fill *info (caller-owned) with the handle's sizes, the far-field layout in
 * use (source split, assembled or not, the symmetric FP32 kernel or not) and
 * the device bytes it holds.  PB_E_INVALID_ARG for NULL arguments. */
pb_status pb_mesh_get_info(const pb_mesh_handle *h, pb_mesh_info *info);

/* Redo every device-side setup stage of the handle from the resident mesh:
 * geometry, Sauter-Schwab near field, near-field blocks and preconditioner,
 * and the dense far field in assembled modes.  The host-side index plan
 * (validation, triangle order, sparsity) is kept.  Used to time complete
 * solves with inputs resident on the device. */
pb_status pb_mesh_refresh(pb_mesh_handle *h);

/* Solve for one charge set on a resident mesh (same outputs as pb_solve). */
pb_status pb_mesh_solve(pb_mesh_handle *h, const pb_charges *charges, pb_result *result);

/* Solve one charge set on each of n resident meshes of any, unequal, sizes
 * (1 <= n <= PB_MAX_BATCH_REQUESTS, distinct handles): their GMRES runs in
 * lockstep and every iteration computes the far fields of all requests still
 * iterating in one persistent kernel launch per kernel form, over a work queue
 * of (request, 64 target triangles, source chunk) items, heaviest first
 * (Numerical discretization: regular quadrature of the far pairs; the same
 * operators and GMRES as pb_mesh_solve).  Every request's arithmetic equals
 * that of pb_mesh_solve on its handle, so results[r] equals that solve's
 * result bit for bit, timings aside: t_rhs, t_prec are the request's own,
 * t_gmres the whole batch's.  charges[r] and results[r] belong to handles[r]
 * and follow the pb_mesh_solve contract; the call returns PB_NOT_CONVERGED if
 * any request did not converge (all results filled), and fails as a whole,
 * with no result, if any request's charges are invalid (the message names the
 * request).  The handles must share
 * the precision (PB_FP64 or PB_FP32) and be matrix-free (operator mode
 * PB_MATRIX_FREE, or PB_AUTO resolved to it; no treecode), with any
 * formulation and the block-diagonal or mass preconditioners; otherwise
 * PB_E_STATE.  All work runs on handles[0]'s stream; each handle's stream is
 * drained first.  Not thread-safe against other calls on the same handles.
 * With pb_mesh_profile bit 0 on handles[0], its operator profile records the
 * fused launches (work = kernel pairs of the requests in each launch) and
 * nothing else of the call. */
#define PB_MAX_BATCH_REQUESTS 1024
pb_status pb_solve_batch(int32_t n, pb_mesh_handle *const *handles, const pb_charges *charges,
                         pb_result *results);

/* Solve for n_sets charge sets on one resident mesh.  In assembled modes the
 * right-hand sides are advanced together and every operator application is
 * one batched dense product (MFMA for 16-bit storage; the first such product
 * adds to the handle a copy of the 16-bit matrix in the MFMA operand order,
 * 2 bytes per entry, rebuilt after each reassembly, or reads the row-major
 * copy when the budget leaves no room for it).  out[k] follows the pb_result
 * contract for set k.  PB_E_STATE for the Calderon preconditioners. */
pb_status pb_solve_multi(pb_mesh_handle *h, int32_t n_sets, const pb_charges *sets,
                         pb_result *out);

/* ------------------------------------------------- hot-path building blocks
 * Exposed for verification and measurement; each runs on the handle's stream
 * and returns after the result is on the host. */

/* y = A x (flags & PB_APPLY_PRECOND: y = P^-1 A x, or B A x for the Calderon
 * preconditioners) for the handle's formulation.  x and y are host arrays of 2 n_vertices doubles laid out as
 * [trace_D; trace_N].  PB_APPLY_FAR_ONLY / PB_APPLY_NEAR_ONLY restrict the sum
 * to triangle pairs sharing no vertex / sharing a vertex (plus the mass terms). */
#define PB_APPLY_PRECOND    1
#define PB_APPLY_FAR_ONLY   2
#define PB_APPLY_NEAR_ONLY  4
pb_status pb_mesh_apply(pb_mesh_handle *h, const double *x, double *y, int32_t flags);

/* Same as pb_mesh_apply on device vectors (2 n_vertices doubles each) and on
 * the caller's HIP stream (NULL = the handle's stream); returns without
 * synchronising. */
pb_status pb_mesh_apply_device(pb_mesh_handle *h, const double *x_device, double *y_device,
                               int32_t flags, void *hip_stream);

/* Galerkin-tested source projections of Eq. sources: b = [<phi_i, phi_D>;
 * <phi_i, phi_N>] (host array of 2 n_vertices doubles).  The second half is
 * computed for both formulations (the direct formulation does not use it). */
pb_status pb_mesh_rhs(pb_mesh_handle *h, const pb_charges *charges, double *b);

/* Reaction potential (Eq. phireac_bie) at npts points from P1 traces phi and
 * dphi (host, n_vertices each); out: npts doubles. */
pb_status pb_mesh_reaction_potential(pb_mesh_handle *h, const double *phi, const double *dphi,
                                     int32_t npts, const double *pts, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the reaction
 * potential of pb_mesh_reaction_potential on device arrays, allocating nothing.
 * traces_device: 2 n_vertices doubles [phi; dphi] (the P1 interior traces);
 * pts_device: npts x 3 doubles (row-major points); out_device: npts doubles.
 * All three are device pointers owned by the caller.  Runs on hip_stream
 * (NULL = the handle's stream) and returns without synchronising.
 * Per-point partial sums over the source chunks (min(1, ceil(T / 4096)) of
 * them) go to a static device array of 4 MiB (524288 doubles) that each GPU the
 * library runs on holds until the process ends: npts x chunks above 524288 is
 * rejected with PB_E_INVALID_ARG (at 81920 triangles, 20 chunks, up to 26214
 * points).  Every call on one GPU shares that array, so calls that overlap in
 * time on one GPU (any handles, any streams) race; every call writes all the
 * partial sums it reads, so nothing needs clearing between calls.  Results
 * equal pb_mesh_reaction_potential's bit for bit. */
pb_status pb_mesh_reaction_potential_noalloc(pb_mesh_handle *h, const double *traces_device, int32_t npts,
                                             const double *pts_device, double *out_device, void *hip_stream);

/* Sauter-Schwab local blocks of near pairs (original triangle ids t[k], s[k],
 * which must share a vertex): out[36 k + 9 op + 3 a + b] with op = 0 V_L,
 * 1 K_L, 2 V_Y, 3 K_Y, a the local vertex of t[k], b of s[k] (input order). */
pb_status pb_mesh_near_blocks(pb_mesh_handle *h, int32_t n, const int32_t *t, const int32_t *s,
                              double *out);

/* Per-vertex 2x2 preconditioner inverses, out: n_vertices x 4 (row-major). */
pb_status pb_mesh_preconditioner(pb_mesh_handle *h, double *out);

/* Kernel timing for measurement: `enable` is a bit mask of kinds whose kernels
 * are bracketed by HIP events on the stream they run on (bit 0: kind 0, bit 1:
 * kind 1; 0 turns timing off).  Timing kind 0 makes GMRES launch its iterations
 * eagerly instead of replaying a captured graph.  read returns, since the last
 * pb_mesh_profile call, the launches, summed milliseconds and summed
 * algorithmic work of one kind:
 *   kind 0: operator product -- matrix-free far-field kernel (work = kernel
 *           pairs, (6T)^2 per launch) or dense far-field GEMV (work = bytes of
 *           the stored 2V x 2V entries plus the vectors);
 *   kind 1: dense far-field assembly (work = point-pair evaluations).
 * total_work may be NULL. */
pb_status pb_mesh_profile(pb_mesh_handle *h, int32_t enable);
pb_status pb_mesh_profile_read(pb_mesh_handle *h, int32_t kind, int64_t *launches, double *total_ms,
                               double *total_work);

/* ------------------------------------------------------------------ serving
 * A solve server batches independent requests continuously: each submitted
 * request (mesh, charges, options; all copied at submission) waits in arrival
 * order until a slot is free and its estimated device footprint fits in the
 * budget beside the requests already running (first fit in arrival order);
 * then it runs on its own worker thread, HIP stream and memory, overlapping on
 * the device with the other running requests.  A request's result does not
 * depend on what runs beside it.  Device blocks of 64 MiB and more (the
 * assembled far field, the near-field blocks) that a finished request leaves
 * are kept by the server and handed to later requests of similar size
 * (best fit within 5/4, in 256 MiB steps); idle blocks go back to the device
 * while a new one would take the server past its budget, and all of them at
 * pb_server_destroy.  Times are seconds since pb_server_create. */
typedef struct pb_server pb_server;

typedef struct {
    double t_submit, t_start, t_end;
} pb_request_times;

typedef struct {
    int64_t submitted, completed, cancelled, failed;
    int32_t running, queued, peak_running;
    size_t inflight_bytes, peak_inflight_bytes, budget;
} pb_server_stats;

/* Device bytes a handle for this mesh and these options is expected to hold
 * (the admission footprint; the server caps each request's handle at it). */
pb_status pb_estimate_device_bytes(const pb_mesh *mesh, const pb_options *opt, size_t *bytes);

/* hbm_budget: device bytes shared by running requests (0 = 90% of free memory);
 * max_slots: concurrent requests, 1..64. */
pb_status pb_server_create(size_t hbm_budget, int32_t max_slots, pb_server **out);
/* Cancels queued requests, waits for running ones, frees everything. */
pb_status pb_server_destroy(pb_server *s);
/* Queue a request; *ticket identifies it.  PB_E_NOMEM if its footprint exceeds
 * the whole budget (it could never be admitted). */
pb_status pb_submit(pb_server *s, const pb_mesh *mesh, const pb_charges *charges, const pb_options *opt,
                    uint64_t *ticket);
/* *done = 1 once the request has finished (successfully or not). */
pb_status pb_poll(pb_server *s, uint64_t ticket, int32_t *done);
/* Remove a request that has not started; PB_E_STATE if it is running or done. */
pb_status pb_cancel(pb_server *s, uint64_t ticket);
/* Block until the request finishes, fill *out (phi / dphi: caller buffers of
 * n_vertices doubles or NULL) and *times (may be NULL), and release the
 * ticket.  Returns the solve's status (or the error that ended it). */
pb_status pb_wait(pb_server *s, uint64_t ticket, pb_result *out, pb_request_times *times);
pb_status pb_server_get_stats(pb_server *s, pb_server_stats *stats);

/* Block until all work of the handle is done. */
pb_status pb_mesh_synchronize(pb_mesh_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* PBM_H */
