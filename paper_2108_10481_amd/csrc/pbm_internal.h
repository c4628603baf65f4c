// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pbm.h"

namespace pbm {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
struct Error {
    pb_status code;
    std::string msg;
};
[[noreturn]] void fail(pb_status code, const std::string &msg);
void hip_check(hipError_t e, const char *what, const char *file, int line);
#define HIPCHECK(x) ::pbm::hip_check((x), #x, __FILE__, __LINE__)

// ------------------------------------------------------------- quadrature
// 6-point degree-4 symmetric triangle rule (Dunavant 1985, symmetric rule of
// degree 4): orbits (1-2a, a, a) with weight wa and (1-2b, b, b) with weight
// wb, weights relative to the triangle area (they sum to 1).
constexpr double kRuleA = 0.445948490915964886318329253883;
constexpr double kRuleB = 0.0915762135097707434595714634022;
constexpr double kRuleWA = 0.223381589678011465695007008433;
constexpr double kRuleWB = 0.1099517436553218676383263249;
// barycentric coordinate k of rule point p, and its weight
__host__ __device__ constexpr double rule_bary(int p, int k)
{
    return p < 3 ? (k == p ? 1.0 - 2.0 * kRuleA : kRuleA) : (k == p - 3 ? 1.0 - 2.0 * kRuleB : kRuleB);
}
__host__ __device__ constexpr double rule_w(int p) { return p < 3 ? kRuleWA : kRuleWB; }
constexpr double kPi = 3.14159265358979323846;
constexpr double kInv4Pi = 1.0 / (4.0 * kPi);
// Gauss-Legendre on [0,1] (Golub-Welsch: eigenvalues of the Jacobi matrix).
void gauss_legendre01(int n, double *x, double *w);

// ----------------------------------------------------------- host mesh prep
// Everything here is index work on the host: validation, a Morton ordering
// of triangles, vertex -> triangle incidence, the near-pair lists (ordered
// pairs of triangles sharing >= 1 vertex) and the sparsity of the near-field
// vertex blocks.
struct HostMesh {
    int V = 0, T = 0;
    std::vector<double> xyz;          // V x 3
    std::vector<int32_t> tri;         // T x 3, sorted triangle order, input local order
    std::vector<int32_t> perm;        // sorted position -> input triangle id
    std::vector<uint32_t> mkey;       // 30-bit Morton code of each sorted triangle's centroid (ascending)
    std::vector<int32_t> iperm;       // input triangle id -> sorted position
    std::vector<int32_t> inc_ptr;     // V + 1
    std::vector<int32_t> inc_tk;      // 4 t + k for each incidence (t sorted id)
    std::vector<int32_t> pair_ptr;    // T + 1 (sorted t)
    std::vector<int32_t> pair_s;      // sorted s, ascending within a row
    std::vector<int32_t> pair_rev;    // index of the reversed pair (s, t)
    std::vector<int32_t> row_ptr;     // V + 1, near vertex CSR
    std::vector<int32_t> col;         // columns, ascending within a row
    std::vector<int32_t> diag_slot;   // V: slot of (i, i)
    std::vector<int32_t> slot_ptr;    // nnz + 1
    std::vector<uint32_t> slot_code;  // p << 4 | k << 2 | l per contribution, in row visiting order
};
void build_host_mesh(const pb_mesh *m, HostMesh &hm);

// ------------------------------------------------------------ device state
// Source / target records of the far-field kernels, one per triangle:
//   static  (kStat reals): 6 quadrature points x 3, normal 3, y_q . n 6, area 1,
//                          surface curls of the three hat functions 9, centroid 3
//   dynamic (kDyn reals) : b1[6] = w_q|s| u1(y_q), b2[6] = w_q|s| u2(y_q), C[3] = |s| curl u1|_s
constexpr int kStat = 40;
constexpr int kDyn = 16;
// per-triangle FP64 geometry: pts 18, normal 3, area 1, curl 9 -> 31, padded
constexpr int kGeo = 32;

// Device-side control of a captured GMRES iteration: kernels offset their
// vector arguments by (*j) * stride and return at once when *skip is set.
// Default-constructed (eager launches): no offset, never skip.
struct DevCtl {
    const int *j = nullptr;
    const int *skip = nullptr;
    size_t stride = 0;
};
__device__ inline bool ctl_skip(const DevCtl &c) { return c.skip && *c.skip; }
__device__ inline size_t ctl_off(const DevCtl &c) { return c.j ? (size_t)(*c.j) * c.stride : 0; }

// Every FP64 dot product of the Krylov solvers (eager, captured, batched) has
// this one shape: kDotThreads threads stride over the vector, then a fixed
// LDS tree, so the three paths round identically.
constexpr int kDotThreads = 1024;
__device__ inline double dot_block_sum(double acc, double *sh)
{
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}
// The near-field product of one vertex row uses kRowLanes lanes (slots
// strided by kRowLanes, then a butterfly inside the lane group), in the
// single and the batched gather alike.
constexpr int kRowLanes = 4;

struct GraphGmres;   // captured GMRES iteration (runtime.hip)

// device state of a captured GMRES solve
struct GState {
    int j;          // iterations done (basis vectors 0..j exist)
    int done;       // stop flag: converged, breakdown, or m reached
    int m;          // capacity (max iterations)
    int pad;
    double tolb;    // tol * |pb|
    double res;     // current residual estimate |g_j|
    double nrm2;    // |w|^2 of the new vector
    double inv;     // 1 / |w|
};

// One solve of a lockstep batch, for the batched steps of a captured
// iteration: its mesh data (source weights, far-field finish, gather) and its
// Krylov state (basis, Hessenberg, rotations, CGS2 coefficients).
struct KrylovReq {
    int n, m;                  // 2V, basis capacity
    double *Vb;                // basis, column-major n x (m + 1)
    GState *st;
    double *H, *cs, *sn, *g, *h1, *h2;
};
struct TailReq {
    int T, V, S;               // triangles, vertices, source chunks of the regular split
    int rt, nr;                // symmetric split (nr = 0: regular)
    int family, swap, precond;
    const int32_t *tri;
    const double *geo;
    double *dyn64;
    float *dyn32;
    const void *part;          // far-field partial sums (float or double)
    double *triout;
    const int32_t *inc_ptr, *inc_tk, *row_ptr, *col;
    const double *N, *pinv;
    int64_t nnz;
    const double *x;           // the basis: input column V_j (offset by ctl)
    double *gout;              // gather output: V_{j+1} (offset by ctl), or a plain vector (mass mode)
    int gout_offset;           // 1: gout is offset by j n like the input
    DevCtl ctl;                // j, stop flag, stride n: the input column V_j
};

struct Params {
    double eps_in, eps_out, kappa;
    int formulation, preconditioner, precision, operator_mode;
};

// A formulation's Galerkin block system as combinations of the Laplace (L)
// and Yukawa (Y) operators.  Every formulation of the paper takes, for each
// output row, c_I times an interior trace equation plus c_E times an exterior
// one (Eqs. bie, bie:ext:int, bie:int:ext, with interior or exterior traces as
// unknowns): rows of kind 1 (Dirichlet trace equations) use K in column 1 and
// V in column 2, rows of kind 2 (Neumann trace equations) D and T.
//   family 0: both rows of kind 1 (direct formulations, permuted or not);
//   family 1: row 1 of kind 1, row 2 of kind 2 (Juffer, Mueller, Lu, PMCHWT).
// block (r, c) = mass[r][c] M + aL[r][c] Op_L + aY[r][c] Op_Y, and the
// right-hand side row r = rhsD[r] <phi_i, varphi_D> + rhsN[r] <phi_i, varphi_N>.
struct FormCoef {
    int family = 0;
    int exterior = 0;          // unknowns are the exterior traces
    double mass[2][2] = {}, aL[2][2] = {}, aY[2][2] = {};
    double rhsD[2] = {}, rhsN[2] = {};
};
FormCoef formulation_coef(int formulation, double eps_in, double eps_out, double alpha, double beta);
int laplace_row(const FormCoef &f);   // family 0: the row with only Laplace terms
// family 1 with no Laplace term in any block (the Yukawa part of a PMCHWT matrix)
bool yukawa_only(const FormCoef &f);
// Calderon preconditioners: the operator P (the PMCHWT matrix or one kernel's
// part of it) and the scales (a, b) of blockdiag(aM, bM)^-1 on the left
FormCoef calderon_coef(int formulation, int preconditioner, double eps_in, double eps_out);
void calderon_scales(int formulation, int preconditioner, double eps_in, double eps_out, double *a, double *b);

// HIP-event timing of the dominant kernels on the stream they run on.
// kind 0: far-field operator product (matrix-free kernel or dense GEMV),
// kind 1: dense far-field assembly.  work = algorithmic kernel pairs
// (matrix-free), bytes (dense product) or point-pair evaluations (assembly).
struct Profiler {
    int mask = 0;   // bit 0: kind 0 (operator product), bit 1: kind 1 (assembly)
    bool on(int kind) const { return (mask >> kind) & 1; }
    std::vector<hipEvent_t> ev[2];   // start/stop pairs
    std::vector<double> pend_work[2];
    int64_t launches[2] = {0, 0};
    double total_ms[2] = {0.0, 0.0};
    double work[2] = {0.0, 0.0};
    void record(int kind, hipEvent_t a, hipEvent_t b, double w)
    {
        ev[kind].push_back(a);
        ev[kind].push_back(b);
        pend_work[kind].push_back(w);
    }
};

struct Dense;       // assembled far field (k_dense.hip)
struct Tree;        // treecode far field (k_tree.hip)
constexpr int kTreeMaxDegree = 7;
struct BatchWork;   // multi right-hand side workspaces (k_batch.hip)

struct Krylov {
    double *basis = nullptr;   // cap x n Arnoldi vectors
    int cap = 0;
    double *kbuf = nullptr;    // dot-product results copied to the host each iteration
    double *y = nullptr;       // least-squares coefficients
};

// Device blocks of at least kCacheMin bytes that a server keeps after its
// requests finish and hands to later requests (runtime.hip): mapping and
// unmapping tens of GB per request took longer than the request's
// arithmetic and serialised concurrent requests.
constexpr size_t kCacheMin = (size_t)64 << 20;
struct BlockCache;
BlockCache *block_cache_create(size_t limit);
void block_cache_destroy(BlockCache *c);
size_t block_cache_bytes(const BlockCache *c);   // held, idle and in use
size_t cache_charge(size_t n);                    // bytes a cached block for n bytes can hold

struct DevMesh {
    HostMesh hm;
    Params prm;
    pb_options opt;
    int S = 1;                     // far-field source chunks
    // symmetric FP32 far field (k_far_sym.hip): tiles per range, ranges, work
    // list of range pairs (heaviest first), its counter, blocks per kernel form
    int sym_rt = 0, sym_nr = 0, sym_nitems = 0;
    int2 *sym_items = nullptr;
    int *sym_next = nullptr;
    int sym_blocks[3] = {1, 1, 1};
    hipStream_t stream = nullptr;
    size_t bytes = 0;
    std::vector<void *> allocs;
    BlockCache *cache = nullptr;   // server handles: large blocks come from and return to it
    std::vector<std::pair<void *, size_t>> cached;   // (block, its size) taken from the cache

    // geometry (sorted triangle order)
    double *xyz = nullptr;         // V x 3
    int32_t *tri = nullptr;        // T x 3
    double *geo = nullptr;         // T x kGeo
    double *stat64 = nullptr;      // T x kStat
    float *stat32 = nullptr;       // T x kStat
    int32_t *inc_ptr = nullptr, *inc_tk = nullptr;
    int32_t *pair_ptr = nullptr, *pair_s = nullptr, *pair_rev = nullptr, *pair_t = nullptr;
    int32_t *ss_idx = nullptr;     // near pairs grouped by case (identical, edge, vertex)
    int ss_count[4] = {0, 0, 0, 0};   // pairs sharing 0..3 vertices
    int32_t *row_ptr = nullptr, *col = nullptr, *diag_slot = nullptr;
    int32_t *slot_ptr = nullptr;
    uint32_t *slot_code = nullptr;
    double *pair_sums = nullptr;   // npair x 2: sum of the 3 x 3 V_L and V_Y entries
    double *pairblk = nullptr;     // npair x 36
    double *N = nullptr;           // 4 x nnz near blocks (N11, N12, N21, N22), mass included
    double *pinv = nullptr;        // V x 4
    // mass preconditioners: M over the near CSR slots, 1 / M_ii, Chebyshev
    // state and a product buffer (kMassBatch systems)
    double *Mval = nullptr, *Mdinv = nullptr, *cheb = nullptr, *mtmp = nullptr;
    // matvec workspaces
    double *dyn64 = nullptr;       // T x kDyn
    float *dyn32 = nullptr;        // T x kDyn
    void *part = nullptr;          // S x T x 16 reals
    double *triout = nullptr;      // T x 6
    double *xtmp = nullptr;        // 2V
    double *ytmp = nullptr;        // 2V
    double *ztmp = nullptr;        // 2V
    double *ytmp2 = nullptr;       // 2V (iterative refinement residual)
    double *ztmp2 = nullptr;       // 2V (iterative refinement correction)
    double *red1 = nullptr;        // small reduction scratch
    double *yfar = nullptr;        // 2V far-field product (assembled mode)
    double *u = nullptr;           // 2V solution
    Krylov kry;
    DevCtl ctl;                    // set while a GMRES iteration is being captured
    GraphGmres *gg[2] = {nullptr, nullptr};   // per operator level
    double t_setup = 0.0;
    bool want_dense = false;
    // charges workspace
    double *qbuf = nullptr;        // 7 x qcap: SoA x, y, z, q then AoS xyz
    int qcap = 0;
    double *fpts = nullptr;        // 2 x T x 6 (RHS point values)
    double *red = nullptr;         // reduction scratch
    int redcap = 0;
    Dense *dense = nullptr;
    const int32_t *dense_vpos = nullptr;   // vertex -> row of the dense far field
    Tree *tree = nullptr;                  // treecode plan (PB_TREECODE)
    BatchWork *bw = nullptr;

    Profiler prof;
    int64_t npair() const { return (int64_t)hm.pair_s.size(); }
    FormCoef fm;                    // the formulation's block coefficients
    // Calderon preconditioners: P's coefficients, near-field values (4 x nnz)
    // and assembled far field; NP and denseP stay null when P is A itself.
    // cal1, cal2: 2V work vectors of the product chain.
    FormCoef fmP;
    double *NP = nullptr;
    Dense *denseP = nullptr;
    double *cal1 = nullptr, *cal2 = nullptr;
    // far-field rule of the current operator: 0 = 6-point rule (the handle's
    // precision and mode), 1 = one-point rule, matrix-free FP32 (fast
    // Calderon's P), 2 = one-point rule, matrix-free in the handle's precision
    // (A with regular_order 1); swapped with far_ruleP like the fields above
    int far_rule = 0, far_ruleP = 0;
    // fast Calderon: P's Sauter-Schwab blocks and pair sums at the relaxed
    // order, and the centroid source weights (T x 2: |s| mean u1, |s| mean u2)
    double *pairblkP = nullptr, *pair_sumsP = nullptr;
    float *dync32 = nullptr;
    double *dync64 = nullptr;   // the same weights in FP64 (far_rule 2, FP64 precision)
    int64_t nnz() const { return (int64_t)hm.col.size(); }
    void *alloc(size_t n);
    ~DevMesh();
};

// kernels / launchers (k_*.hip)
void launch_geometry(DevMesh &d);
void launch_near_field(DevMesh &d);
void launch_near_assemble(DevMesh &d);
// near-field values of coefficients f from pair blocks blk and pair sums into N (4 x nnz);
// Mval (may be null): the mass matrix
void launch_near_values(DevMesh &d, const FormCoef &f, const double *blk, const double *sums, double *N,
                        double *Mval);
// fast Calderon's P: Sauter-Schwab blocks at the relaxed order and their pair sums
void launch_near_field_fast(DevMesh &d);
// one-point-rule far field (FP32) of the current operator fields into d.part
void launch_far_centroid(DevMesh &d, bool fp32);
void launch_source_prep(DevMesh &d, const double *x, bool fp32);
void launch_far(DevMesh &d, bool fp32);
void launch_far_finish(DevMesh &d, bool fp32);
// batched far field of several matrix-free handles (requests of uneven size):
// the work-queue plan of the requests still iterating, then one persistent
// launch per kernel form; each request's sources must be prepared first
// (launch_source_prep) and its k_far_finish follows as usual
struct FarBatch {
    hipStream_t stream = nullptr;
    void *reqs = nullptr;
    void *items = nullptr;
    int *next = nullptr;           // one queue counter per kernel form, then six for the symmetric queues
    size_t req_cap = 0, item_cap = 0;
    int first[4] = {0, 0, 0, 0}, nitems[4] = {0, 0, 0, 0}, nblocks[4] = {0, 0, 0, 0};
    // symmetric FP32 items {request, a, b} of the requests with a symmetric split:
    // queues for forms 0, 1, 3 (kappa > 0), then the same for kappa = 0
    void *sym_items = nullptr;
    size_t sym_cap = 0;
    int sym_first[6] = {}, sym_n[6] = {}, sym_nblocks[6] = {};
};
// skip (empty, or one per handle): device stop flags; a request whose flag is
// set contributes no work (captured iterations keep replaying after it stops)
void far_batch_plan(const std::vector<DevMesh *> &ds, const std::vector<int> &live, bool fp32, FarBatch &fb,
                    const std::vector<const int *> &skip = {});
void launch_far_batch(FarBatch &fb, bool fp32);
void far_batch_free(FarBatch &fb);
// use_far: 0 = near only, 1 = far from per-triangle outputs, 2 = far from d.yfar
// y_offset false: y is a plain vector even inside a captured iteration
void launch_gather(DevMesh &d, const double *x, double *y, int flags, int use_far, bool y_offset);
void apply_operator(DevMesh &d, const double *x, double *y, int flags, hipStream_t s);
void launch_rhs(DevMesh &d, int nq, const double *qbuf, double *b);
// launch_rhs combined into the formulation's right-hand side rows
void formulation_rhs(DevMesh &d, int nq, const double *qbuf, double *b);
void launch_reaction(DevMesh &d, int nq, const double *qpts, double *out);
void launch_inside_test(DevMesh &d, int nq, const double *qbuf, double *out);
void launch_pair_blocks_subset(DevMesh &d, int n, const int32_t *t_sorted, const int32_t *s_sorted,
                               const int32_t *idx, const int count[4], double *out);
void ss_group(const std::vector<int32_t> &tri, int n, const int32_t *t, const int32_t *s, std::vector<int32_t> &idx,
              int count[4]);
int choose_chunks(int T);
// symmetric FP32 far field (k_far_sym.hip)
bool sym_eligible(int T, double kappa, int mode);
void sym_plan(int T, int &rt, int &nr, std::vector<int2> &items);
int sym_blocks(int nitems, int form, bool k0);
void launch_far_sym(DevMesh &d);
void launch_far_sym_finish(DevMesh &d);
int sym_batch_blocks_for(int form, bool k0, int n);
void launch_far_sym_batch(int form, bool k0, const void *reqs, const int4 *items, int n, int nblocks, int *next,
                          hipStream_t s);
int reduction_chunks(int T);
pb_status solve_on_mesh(DevMesh &d, const pb_charges *ch, pb_result *res);
int gmres(DevMesh &d, const double *pb, double *x, double tol, int max_iter, double *est);
int gmres_solve(DevMesh &d, const double *pb, double *x, double tol, int max_iter, double *est);
void destroy_graphs(DevMesh &d);
void check_solvable(const DevMesh &d);   // PB_E_STATE for systems that are no formulation

// treecode far field (k_tree.hip): plan built on the host at creation; the
// product writes d.part in the layout of tree_splits() source chunks
Tree *tree_create(DevMesh &d);
int tree_splits(const Tree &t);
void tree_destroy(DevMesh &d);
void launch_tree_far(DevMesh &d, bool fp32);

// assembled far field and mixed precision (k_dense.hip)
bool dense_fits(const DevMesh &d, int copies = 1);
void build_dense(DevMesh &d);
void destroy_dense(DevMesh &d);
void dense_apply(DevMesh &d, const double *x, double *yfar);
int mixed_refinement_solve(DevMesh &d, const double *b, const double *pb, double *u, double *est, int *outer);
pb_status solve_multi(DevMesh &d, int n_sets, const pb_charges *sets, pb_result *out);
void destroy_batch(DevMesh &d);
void charges_to_device(DevMesh &d, const pb_charges *c);
void check_charges_inside(DevMesh &d, int nq);
// reaction potential with its partial sums in the library's static scratch
// (k_geometry.hip): no allocation; npts x reduction_chunks(T) must fit
constexpr size_t kNoAllocScratchDoubles = size_t(1) << 19;   // 4 MiB
void reaction_potential_noalloc(DevMesh &d, const double *traces, int npts, const double *pts, double *out,
                                hipStream_t stream);
pb_status finish_result(DevMesh &d, const pb_charges *ch, const double *pb, double *u, int its, int outer,
                        double t_rhs, double t_prec, double t_gmres, pb_result *res);

// Krylov kernels (k_krylov.hip)
void kr_dots(hipStream_t s, int n, int nvec, const double *V, size_t ldv, const double *w, double *out);
void kr_update(hipStream_t s, int n, int nvec, const double *V, size_t ldv, const double *h, double *w,
               double sign);
void kr_scale_copy(hipStream_t s, int n, const double *x, double a, double *y);
void kr_axpy(hipStream_t s, int n, double a, const double *x, double *y);
void kr_combine(hipStream_t s, int n, int nvec, const double *V, size_t ldv, const double *y, double *x);
void kr_precond(hipStream_t s, int V, const double *pinv, const double *x, double *y);
// mass preconditioners (k_near.hip)
constexpr int kMassBatch = 16;
inline bool mass_mode(const DevMesh &d)
{
    return d.prm.preconditioner == PB_MASS || d.prm.preconditioner == PB_SCALED_MASS;
}
inline bool is_calderon(int preconditioner)
{
    return preconditioner >= PB_CALDERON && preconditioner <= PB_SCALED_CALDERON_EXT;
}
inline bool calderon_mode(const DevMesh &d) { return is_calderon(d.prm.preconditioner); }
// P is an operator of its own (a kernel's part of A, or relaxed quadrature), not A itself
inline bool calderon_separate(const DevMesh &d)
{
    return calderon_mode(d) && (d.prm.preconditioner != PB_CALDERON || d.opt.calderon_fast);
}
// Sauter-Schwab order of fast Calderon's P
inline int calderon_fast_order(const pb_options &o) { return o.singular_order > 1 ? o.singular_order - 1 : 1; }
// blockdiag(M, M)^-1 scaled by (sa, sb) = (1/a, 1/b) per half: of the mass
// preconditioners (first form) or explicit
void mass_precond(DevMesh &d, int nvec, const double *in, double *out, const DevCtl &ctl);
void mass_precond(DevMesh &d, int nvec, const double *in, double *out, const DevCtl &ctl, double sa, double sb);
// Calderon chain on a plain vector: out (offset by ctl) = blockdiag(aM, bM)^-1 P blockdiag(M, M)^-1 in
void calderon_left(DevMesh &d, const double *in, double *out, const DevCtl &ctl);
int kr_batch_blocks(int n);
// boff: prefix of kr_batch_blocks(n_r) over the R solves (device); ndot: an
// upper bound of the dot-product items (sum of the capacities + 1)
void kr_batch_iteration_tail(hipStream_t s, int R, const KrylovReq *rq, const int *boff, int nblocks, int ndot);
// batched source weights, far-field finish (regular and symmetric splits) and
// gather of R solves; boff_* prefixes of the blocks each solve takes
int tail_blocks_source(const TailReq &q);
int tail_blocks_finish(const TailReq &q);
int tail_blocks_gather(const TailReq &q);
void launch_batch_source_prep(hipStream_t s, int R, const TailReq *rq, const int *boff, int nblocks);
void launch_batch_finish(hipStream_t s, bool fp32, int R, const TailReq *rq, const int *boff, int nblocks);
void launch_batch_gather(hipStream_t s, int R, const TailReq *rq, const int *boff, int nblocks);
void kr_graph_iteration_tail(hipStream_t s, int n, int m, double *Vb, GState *st, double *H, double *cs, double *sn,
                             double *g, double *h1, double *h2);

}  // namespace pbm
