// Host runtime and C ABI: mesh handles, operator application, GMRES
// (Preconditioning; tolerance 1e-5 without restart in the Results), right-hand
// side (Eq. sources), reaction potential and solvation energy (Eqs.
// phireac_bie, dG).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "dense.h"
#include "trace.h"

namespace pbm {

// e^2 / (4 pi eps0 angstrom) in kcal/mol; potentials here carry 1/(4 pi).
constexpr double kCoulombKcal = 332.0637;
constexpr double kEnergyC = 4.0 * kPi * kCoulombKcal;

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
void fail(pb_status code, const std::string &msg) { throw Error{code, msg}; }
void hip_check(hipError_t e, const char *what, const char *file, int line)
{
    if (e == hipSuccess) return;
    std::string m = std::string(what) + " failed: " + hipGetErrorString(e) + " (" + file + ":" + std::to_string(line) + ")";
    throw Error{e == hipErrorOutOfMemory ? PB_E_NOMEM : PB_E_DEVICE, m};
}

// ------------------------------------------------------ server block cache
struct BlockCache {
    std::mutex mu;
    std::multimap<size_t, void *> idle;   // by size
    size_t held = 0;                       // idle + in use
    size_t limit = 0;
};

BlockCache *block_cache_create(size_t limit)
{
    BlockCache *c = new BlockCache();
    c->limit = limit;
    return c;
}

void block_cache_destroy(BlockCache *c)
{
    if (!c) return;
    for (auto &e : c->idle) (void)hipFree(e.second);
    delete c;
}

size_t block_cache_bytes(const BlockCache *c) { return c ? c->held : 0; }

// A block of at least n bytes: an idle one of at most 5/4 of n rounded up to
// 256 MiB (best fit), else a new one, after idle blocks are given back to the
// device while the new one would pass the limit (or the device is full).
static void *cache_take(BlockCache &c, size_t n, size_t *got)
{
    const size_t gran = (size_t)256 << 20;
    const size_t want = (n + gran - 1) / gran * gran;
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.idle.lower_bound(want);
    if (it != c.idle.end() && it->first <= want + want / 4) {
        void *p = it->second;
        *got = it->first;
        c.idle.erase(it);
        return p;
    }
    while (!c.idle.empty() && c.held + want > c.limit) {
        auto big = std::prev(c.idle.end());
        (void)hipFree(big->second);
        c.held -= big->first;
        c.idle.erase(big);
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    while (e != hipSuccess && !c.idle.empty()) {
        (void)hipGetLastError();
        auto big = std::prev(c.idle.end());
        (void)hipFree(big->second);
        c.held -= big->first;
        c.idle.erase(big);
        e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(PB_E_NOMEM, "device memory exhausted");
    }
    c.held += want;
    *got = want;
    return p;
}

static void cache_give(BlockCache &c, void *p, size_t size)
{
    std::lock_guard<std::mutex> lk(c.mu);
    c.idle.insert({size, p});
}

// Give every idle block back to the device (a smaller allocation outside the
// cache failed); returns whether any was held.
static bool cache_trim(BlockCache &c)
{
    std::lock_guard<std::mutex> lk(c.mu);
    const bool any = !c.idle.empty();
    for (auto &e : c.idle) {
        (void)hipFree(e.second);
        c.held -= e.first;
    }
    c.idle.clear();
    return any;
}

// Bytes a block taken for a request of n bytes can hold: n rounded up to the
// cache's 256 MiB steps, plus the best-fit slack of a quarter.  Handles and
// admission estimates charge this much for every block of kCacheMin or more.
size_t cache_charge(size_t n)
{
    if (n < kCacheMin) return n;
    const size_t gran = (size_t)256 << 20;
    const size_t want = (n + gran - 1) / gran * gran;
    return want + want / 4;
}

void *DevMesh::alloc(size_t n)
{
    void *p = nullptr;
    n = std::max<size_t>(n, 256);
    if (opt.memory_budget && bytes + n > opt.memory_budget)
        fail(PB_E_NOMEM, "device memory budget of the handle exceeded");
    if (cache && n >= kCacheMin) {
        // charge the whole block the cache hands out (rounded up, best fit)
        size_t got = 0;
        if (opt.memory_budget && bytes + cache_charge(n) > opt.memory_budget)
            fail(PB_E_NOMEM, "device memory budget of the handle exceeded");
        p = cache_take(*cache, n, &got);
        cached.push_back({p, got});
        bytes += got;
        return p;
    }
    // stream-ordered allocation: frees of one handle never stall another handle's stream
    hipError_t e = hipMallocAsync(&p, n, stream);
    if (e == hipErrorOutOfMemory && cache) {
        // idle blocks of finished requests may hold the memory: give them back and retry
        (void)hipGetLastError();
        if (cache_trim(*cache)) e = hipMallocAsync(&p, n, stream);
    }
    HIPCHECK(e);
    allocs.push_back(p);
    bytes += n;
    return p;
}

DevMesh::~DevMesh()
{
    if (stream) (void)hipStreamSynchronize(stream);
    for (int k = 0; k < 2; ++k)
        for (hipEvent_t e : prof.ev[k]) (void)hipEventDestroy(e);
    destroy_graphs(*this);
    destroy_dense(*this);
    std::swap(dense, denseP);
    destroy_dense(*this);
    tree_destroy(*this);
    destroy_batch(*this);
    for (void *p : allocs) (void)hipFreeAsync(p, stream);
    if (stream) (void)hipStreamSynchronize(stream);
    // the stream is idle: the cached blocks may serve the next request
    for (auto &b : cached) cache_give(*cache, b.first, b.second);
    if (stream) (void)hipStreamDestroy(stream);
}

template <typename T>
static T *upload(DevMesh &d, const std::vector<T> &v)
{
    T *p = (T *)d.alloc(sizeof(T) * v.size());
    if (!v.empty()) HIPCHECK(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, d.stream));
    return p;
}

static double now()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static void check_options(const pb_options *o)
{
    if (!o) fail(PB_E_INVALID_ARG, "options must not be NULL");
    if (!(o->eps_in > 0) || !(o->eps_out > 0) || !(o->kappa >= 0) || !std::isfinite(o->kappa))
        fail(PB_E_INVALID_ARG, "eps_in, eps_out must be > 0 and kappa >= 0");
    if (o->formulation < PB_DIRECT_INT || o->formulation > PB_CFIE_EXT) fail(PB_E_INVALID_ARG, "unknown formulation");
    if ((o->formulation == PB_CFIE_INT || o->formulation == PB_CFIE_EXT) &&
        !(std::isfinite(o->cfie_alpha) && std::isfinite(o->cfie_beta)))
        fail(PB_E_INVALID_ARG, "cfie_alpha and cfie_beta must be finite");
    if (o->preconditioner < PB_PREC_NONE || o->preconditioner > PB_SCALED_CALDERON_EXT)
        fail(PB_E_INVALID_ARG, "unknown preconditioner");
    if (o->preconditioner == PB_SCALED_MASS && o->formulation != PB_JUFFER)
        fail(PB_E_INVALID_ARG, "the scaled mass preconditioner is defined for the Juffer formulation");
    if (is_calderon(o->preconditioner) && o->formulation != PB_PMCHWT_INT && o->formulation != PB_PMCHWT_EXT)
        fail(PB_E_INVALID_ARG, "Calderon preconditioners are defined for the PMCHWT formulations");
    if (o->calderon_fast != 0 && o->calderon_fast != 1) fail(PB_E_INVALID_ARG, "calderon_fast must be 0 or 1");
    if (o->calderon_fast && !is_calderon(o->preconditioner))
        fail(PB_E_INVALID_ARG, "calderon_fast needs a Calderon preconditioner");
    if (o->precision < PB_FP64 || o->precision > PB_MIXED_FP16) fail(PB_E_INVALID_ARG, "unknown precision");
    if (o->operator_mode < PB_MATRIX_FREE || o->operator_mode > PB_TREECODE)
        fail(PB_E_INVALID_ARG, "unknown operator mode");
    if (o->operator_mode == PB_TREECODE) {
        if (o->precision >= PB_MIXED_BF16)
            fail(PB_E_INVALID_ARG, "the treecode far field runs in FP64 or FP32 (mixed modes need the assembled field)");
        if (o->tree_degree < 2 || o->tree_degree > kTreeMaxDegree) fail(PB_E_INVALID_ARG, "tree_degree must be in [2, 7]");
        if (!(o->tree_theta > 0.0 && o->tree_theta < 1.0)) fail(PB_E_INVALID_ARG, "tree_theta must be in (0, 1)");
    }
    if (!(o->tol > 0) || o->max_iter < 1) fail(PB_E_INVALID_ARG, "tol must be > 0 and max_iter >= 1");
    if (o->singular_order < 1 || o->singular_order > 8) fail(PB_E_INVALID_ARG, "singular_order must be in [1, 8]");
    if (o->source_chunks < 0 || o->source_chunks > 1024) fail(PB_E_INVALID_ARG, "source_chunks must be in [0, 1024]");
    if (o->far_symmetric < -1 || o->far_symmetric > 1)
        fail(PB_E_INVALID_ARG, "far_symmetric must be 0 (automatic), 1 (always) or -1 (never)");
    if (o->regular_order != 0 && o->regular_order != 1 && o->regular_order != 4)
        fail(PB_E_INVALID_ARG, "regular_order must be 4 (the 6-point rule) or 1 (the one-point rule)");
    if (o->regular_order == 1) {
        if (o->operator_mode == PB_ASSEMBLED || o->operator_mode == PB_TREECODE || o->precision >= PB_MIXED_BF16)
            fail(PB_E_INVALID_ARG, "regular_order 1 (one-point rule) runs matrix-free in FP64 or FP32");
        if (is_calderon(o->preconditioner))
            fail(PB_E_INVALID_ARG, "regular_order 1 is not combined with the Calderon preconditioners "
                                   "(calderon_fast relaxes the preconditioner's quadrature)");
    }
}

// Coefficients of a formulation from the combination rule: output row r is
// c_I (interior equation of kind k) + c_E (exterior equation of kind k), in
// interior or exterior unknowns.  With e = eps_in / eps_out the four trace
// equations read, in interior unknowns (Eqs. bie:int:int, bie:ext:int):
//   kind 1, interior: [M/2 + K_L, -V_L]          = varphi_D
//   kind 1, exterior: [M/2 - K_Y, e V_Y]         = 0
//   kind 2, interior: [-D_L, M/2 - T_L]          = varphi_N
//   kind 2, exterior: [D_Y / e, M/2 + T_Y]       = 0
// and in exterior unknowns (Eqs. bie:ext:ext, bie:int:ext):
//   kind 1, interior: [M/2 + K_L, -V_L / e]      = varphi_D
//   kind 1, exterior: [M/2 - K_Y, V_Y]           = 0
//   kind 2, interior: [-e D_L, M/2 - T_L]        = e varphi_N
//   kind 2, exterior: [D_Y, M/2 + T_Y]           = 0
FormCoef formulation_coef(int formulation, double eps_in, double eps_out, double alpha, double beta)
{
    const double e = eps_in / eps_out;
    struct Row { int kind; double cI, cE; };
    Row r[2];
    int ext = 0;
    switch (formulation) {
    case PB_DIRECT_INT: r[0] = {1, 1, 0}; r[1] = {1, 0, 1}; break;                  // Eq. bie:dirichlet:int
    case PB_DIRECT_EXT: ext = 1; r[0] = {1, 0, 1}; r[1] = {1, 1, 0}; break;         // Eq. bie:dirichlet:ext
    case PB_DIRECT_INT_PERM: r[0] = {1, 0, 1}; r[1] = {1, 1, 0}; break;
    case PB_DIRECT_EXT_PERM: ext = 1; r[0] = {1, 1, 0}; r[1] = {1, 0, 1}; break;
    case PB_JUFFER: r[0] = {1, 1, 1 / e}; r[1] = {2, 1, e}; break;                  // alpha, beta = 1/e, e
    case PB_MULLER_INT: r[0] = {1, 1, 1}; r[1] = {2, 1, 1}; break;
    case PB_MULLER_EXT: ext = 1; r[0] = {1, 1, 1}; r[1] = {2, 1, 1}; break;
    case PB_LU: ext = 1; r[0] = {1, e, 1}; r[1] = {2, 1, e}; break;                 // alpha = e, beta = 1/e, row 2 times e
    case PB_PMCHWT_INT: r[0] = {1, -1, 1}; r[1] = {2, -1, 1}; break;                // the paper's sign: -(I) + (E)
    case PB_PMCHWT_EXT: ext = 1; r[0] = {1, -1, 1}; r[1] = {2, -1, 1}; break;
    case PB_CFIE_INT: r[0] = {1, 1, alpha}; r[1] = {2, 1, beta}; break;            // Eq. bie:combined:int
    case PB_CFIE_EXT: ext = 1; r[0] = {1, alpha, 1}; r[1] = {2, beta, 1}; break;    // Eq. bie:combined:ext
    default: fail(PB_E_INVALID_ARG, "unknown formulation");
    }
    FormCoef f;
    f.exterior = ext;
    f.family = r[1].kind == 2 ? 1 : 0;
    for (int i = 0; i < 2; ++i) {
        const double cI = r[i].cI, cE = r[i].cE, h = 0.5 * (cI + cE);
        if (r[i].kind == 1) {
            f.mass[i][0] = h;
            f.aL[i][0] = cI;                      // K_L
            f.aY[i][0] = -cE;                     // K_Y
            f.aL[i][1] = ext ? -cI / e : -cI;     // V_L
            f.aY[i][1] = ext ? cE : cE * e;       // V_Y
            f.rhsD[i] = cI;
        } else {
            f.aL[i][0] = ext ? -cI * e : -cI;     // D_L
            f.aY[i][0] = ext ? cE : cE / e;       // D_Y
            f.mass[i][1] = h;
            f.aL[i][1] = -cI;                     // T_L
            f.aY[i][1] = cE;                      // T_Y
            f.rhsN[i] = ext ? cI * e : cI;
        }
    }
    return f;
}

bool yukawa_only(const FormCoef &f)
{
    if (f.family != 1) return false;
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c)
            if (f.aL[r][c] != 0.0) return false;
    return true;
}

// Calderon preconditioning (Eqs. prec:calderon:int, prec:calderon:ext): P is
// the PMCHWT matrix itself or the part of it with one kernel.  The PMCHWT rows
// combine interior (Laplace) and exterior (Yukawa) trace equations with
// c_I = -1, c_E = 1 and no identity term; keeping only the interior or the
// exterior operators gives the printed halves, e.g. for the internal system
// [[-K_L, V_L], [D_L, T_L]] and [[-K_Y, e V_Y], [D_Y / e, T_Y]].
FormCoef calderon_coef(int formulation, int preconditioner, double eps_in, double eps_out)
{
    FormCoef f = formulation_coef(formulation, eps_in, eps_out, 1.0, 1.0);
    const bool keep_int = preconditioner == PB_CALDERON || preconditioner == PB_CALDERON_INT ||
                          preconditioner == PB_SCALED_CALDERON_INT;
    const bool keep_ext = preconditioner == PB_CALDERON || preconditioner == PB_CALDERON_EXT ||
                          preconditioner == PB_SCALED_CALDERON_EXT;
    for (int r = 0; r < 2; ++r) {
        for (int c = 0; c < 2; ++c) {
            f.mass[r][c] = 0.0;
            if (!keep_int) f.aL[r][c] = 0.0;
            if (!keep_ext) f.aY[r][c] = 0.0;
        }
        f.rhsD[r] = f.rhsN[r] = 0.0;
    }
    return f;
}

// (a, b) of blockdiag(aM, bM) for the scaled halves: the two half points
// h1 = 1/4 + eps_out/(4 eps_in), h2 = 1/4 + eps_in/(4 eps_out) (Eq.
// precond:calderon:eigenval_semi), each on the block row whose eigenvalues
// gather there.  At high frequency V D = D V -> 1/4 for both kernels while
// K K, K V and V T vanish, so P A tends to a triangular matrix with diagonal
// (gamma beta, delta alpha) / 4 for A = [[., alpha V], [beta D, .]] and
// P = [[., gamma V], [delta D, .]]: internal system alpha = 1 + e, beta = 1 + 1/e,
// external system alpha = 1 + 1/e, beta = 1 + e (e = eps_in / eps_out).
void calderon_scales(int formulation, int preconditioner, double eps_in, double eps_out, double *a, double *b)
{
    *a = *b = 1.0;
    if (preconditioner != PB_SCALED_CALDERON_INT && preconditioner != PB_SCALED_CALDERON_EXT) return;
    const double h1 = 0.25 + eps_out / (4.0 * eps_in), h2 = 0.25 + eps_in / (4.0 * eps_out);
    // internal system: interior part gamma = delta = 1 -> (h1, h2), exterior part
    // gamma = e, delta = 1/e -> (h2, h1); external system: interior part
    // gamma = 1/e, delta = e -> (h1, h2), exterior part -> (h2, h1)
    (void)formulation;
    const bool interior_part = preconditioner == PB_SCALED_CALDERON_INT;
    *a = interior_part ? h1 : h2;
    *b = interior_part ? h2 : h1;
}

// direct formulations: one row has only Laplace, the other only Yukawa terms;
// returns the Laplace row
int laplace_row(const FormCoef &f)
{
    if (f.aY[0][0] == 0.0 && f.aY[0][1] == 0.0 && f.aL[1][0] == 0.0 && f.aL[1][1] == 0.0) return 0;
    if (f.aL[0][0] == 0.0 && f.aL[0][1] == 0.0 && f.aY[1][0] == 0.0 && f.aY[1][1] == 0.0) return 1;
    fail(PB_E_STATE, "direct formulation with mixed kernels in one row");
}

// Scope in which the handle's operator fields (coefficients, near-field
// values, assembled far field) are those of the Calderon preconditioner's
// operator P, so the formulation's launchers build or apply P instead of A.
// Launches recorded inside the scope (eager or captured) keep P's buffers.
struct PrecondOperator {
    DevMesh &d;
    const int32_t *vpos;
    explicit PrecondOperator(DevMesh &dm) : d(dm), vpos(dm.dense_vpos)
    {
        if (d.dense && d.denseP) d.denseP->level = d.dense->level;   // same storage level as A
        swap();
        if (d.dense) d.dense_vpos = d.dense->vpos;
    }
    PrecondOperator(const PrecondOperator &) = delete;
    PrecondOperator &operator=(const PrecondOperator &) = delete;
    ~PrecondOperator()
    {
        swap();
        d.dense_vpos = vpos;
    }
    void swap()
    {
        std::swap(d.fm, d.fmP);
        std::swap(d.N, d.NP);
        std::swap(d.dense, d.denseP);
        std::swap(d.far_rule, d.far_ruleP);
    }
};

// every device-side setup stage: geometry, near field, near blocks +
// preconditioner, dense far field (assembled modes)
static void device_setup(DevMesh &d)
{
    launch_geometry(d);
    launch_near_field(d);
    if (d.pairblkP) launch_near_field_fast(d);
    launch_near_assemble(d);
    if (d.want_dense) {
        build_dense(d);
        if (calderon_separate(d) && d.far_ruleP == 0) {
            PrecondOperator use(d);
            build_dense(d);
        }
    }
}

// the setup phase (geometry, near field, assembly) run to completion
static void setup_and_wait(DevMesh &d)
{
    TraceRange range("pb.setup");
    device_setup(d);
    HIPCHECK(hipStreamSynchronize(d.stream));
}

static DevMesh *create_mesh(const pb_mesh *mesh, const pb_options *opt, BlockCache *cache = nullptr)
{
    check_options(opt);
    const double t0 = now();
    std::unique_ptr<DevMesh> d(new DevMesh());
    d->cache = cache;
    d->opt = *opt;
    d->prm = {opt->eps_in, opt->eps_out, opt->kappa, opt->formulation, opt->preconditioner, opt->precision,
              opt->operator_mode};
    d->fm = formulation_coef(opt->formulation, opt->eps_in, opt->eps_out, opt->cfie_alpha, opt->cfie_beta);
    if (is_calderon(opt->preconditioner))
        d->fmP = calderon_coef(opt->formulation, opt->preconditioner, opt->eps_in, opt->eps_out);
    build_host_mesh(mesh, d->hm);   // validation happens before any device call
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) fail(PB_E_DEVICE, "no HIP device available");
    HIPCHECK(hipSetDevice(0));
    HIPCHECK(hipStreamCreateWithFlags(&d->stream, hipStreamNonBlocking));
    const HostMesh &hm = d->hm;
    const int V = hm.V, T = hm.T;
    d->S = opt->source_chunks > 0 ? std::min(opt->source_chunks, T) : choose_chunks(T);
    if (opt->operator_mode == PB_TREECODE) {
        d->tree = tree_create(*d);
        d->S = tree_splits(*d->tree);
    }

    d->xyz = upload(*d, hm.xyz);
    d->tri = upload(*d, hm.tri);
    d->inc_ptr = upload(*d, hm.inc_ptr);
    d->inc_tk = upload(*d, hm.inc_tk);
    d->pair_ptr = upload(*d, hm.pair_ptr);
    d->pair_s = upload(*d, hm.pair_s);
    d->pair_rev = upload(*d, hm.pair_rev);
    {
        std::vector<int32_t> pt(hm.pair_s.size());
        for (int t = 0; t < T; ++t)
            for (int p = hm.pair_ptr[t]; p < hm.pair_ptr[t + 1]; ++p) pt[p] = t;
        d->pair_t = upload(*d, pt);
        std::vector<int32_t> gi;
        ss_group(hm.tri, (int)pt.size(), pt.data(), hm.pair_s.data(), gi, d->ss_count);
        d->ss_idx = upload(*d, gi);
    }
    d->row_ptr = upload(*d, hm.row_ptr);
    d->col = upload(*d, hm.col);
    d->diag_slot = upload(*d, hm.diag_slot);
    d->slot_ptr = upload(*d, hm.slot_ptr);
    d->slot_code = upload(*d, hm.slot_code);
    d->pair_sums = (double *)d->alloc(sizeof(double) * 2 * std::max<int64_t>(d->npair(), 1));
    d->geo = (double *)d->alloc(sizeof(double) * kGeo * T);
    d->stat64 = (double *)d->alloc(sizeof(double) * kStat * T);
    d->stat32 = (float *)d->alloc(sizeof(float) * kStat * T);
    d->pairblk = (double *)d->alloc(sizeof(double) * 36 * d->npair());
    d->N = (double *)d->alloc(sizeof(double) * 4 * d->nnz());
    d->pinv = (double *)d->alloc(sizeof(double) * 4 * V);
    if (mass_mode(*d) || calderon_mode(*d)) {
        d->Mval = (double *)d->alloc(sizeof(double) * std::max<int64_t>(d->nnz(), 1));
        d->Mdinv = (double *)d->alloc(sizeof(double) * V);
        // Chebyshev state (x, r, d, d') and the unpreconditioned products, for
        // up to kMassBatch systems
        d->cheb = (double *)d->alloc(sizeof(double) * 4 * kMassBatch * 2 * (size_t)V);
        d->mtmp = (double *)d->alloc(sizeof(double) * kMassBatch * 2 * (size_t)V);
    }
    if (calderon_mode(*d)) {
        d->cal1 = (double *)d->alloc(sizeof(double) * 2 * (size_t)V);
        d->cal2 = (double *)d->alloc(sizeof(double) * 2 * (size_t)V);
        if (calderon_separate(*d)) d->NP = (double *)d->alloc(sizeof(double) * 4 * d->nnz());
        if (opt->calderon_fast) {
            d->far_ruleP = 1;
            d->pairblkP = (double *)d->alloc(sizeof(double) * 36 * std::max<int64_t>(d->npair(), 1));
            d->pair_sumsP = (double *)d->alloc(sizeof(double) * 2 * std::max<int64_t>(d->npair(), 1));
            d->dync32 = (float *)d->alloc(sizeof(float) * 2 * (size_t)T);
        }
    }
    if (opt->regular_order == 1) {
        d->far_rule = 2;
        d->dync32 = (float *)d->alloc(sizeof(float) * 2 * (size_t)T);
        d->dync64 = (double *)d->alloc(sizeof(double) * 2 * (size_t)T);
    }
    d->dyn64 = (double *)d->alloc(sizeof(double) * kDyn * T);
    d->dyn32 = (float *)d->alloc(sizeof(float) * kDyn * T);
    size_t part_bytes = sizeof(double) * 16 * (size_t)d->S * T;
    if (opt->precision == PB_FP32 && opt->operator_mode != PB_TREECODE && d->far_rule == 0 &&
        sym_eligible(T, opt->kappa, opt->far_symmetric)) {
        // symmetric FP32 far field: 2 nr slots of 16 values per triangle
        std::vector<int2> items;
        sym_plan(T, d->sym_rt, d->sym_nr, items);
        d->sym_items = upload(*d, items);
        d->sym_nitems = (int)items.size();
        d->sym_next = (int *)d->alloc(sizeof(int));
        const bool k0 = !(opt->kappa > 0.0);
        d->sym_blocks[0] = sym_blocks(d->sym_nitems, 0, k0);
        d->sym_blocks[1] = sym_blocks(d->sym_nitems, 1, k0);
        d->sym_blocks[2] = sym_blocks(d->sym_nitems, 3, k0);
        part_bytes = std::max(part_bytes, sizeof(float) * 16 * 2 * (size_t)d->sym_nr * T);
    }
    d->part = d->alloc(part_bytes);
    d->triout = (double *)d->alloc(sizeof(double) * 6 * T);
    d->fpts = (double *)d->alloc(sizeof(double) * 12 * T);
    d->xtmp = (double *)d->alloc(sizeof(double) * 2 * V);
    d->ytmp = (double *)d->alloc(sizeof(double) * 2 * V);
    d->ztmp = (double *)d->alloc(sizeof(double) * 2 * V);
    d->ytmp2 = (double *)d->alloc(sizeof(double) * 2 * V);
    d->ztmp2 = (double *)d->alloc(sizeof(double) * 2 * V);
    d->red1 = (double *)d->alloc(sizeof(double) * 8);
    d->yfar = (double *)d->alloc(sizeof(double) * 2 * V);

    d->want_dense = opt->operator_mode == PB_ASSEMBLED || opt->precision >= PB_MIXED_BF16 ||
                    (opt->operator_mode == PB_AUTO && d->far_rule == 0 &&
                     dense_fits(*d, calderon_separate(*d) && !opt->calderon_fast ? 2 : 1));
    setup_and_wait(*d);
    d->t_setup = now() - t0;
    return d.release();
}

DevMesh *create_mesh_checked(const pb_mesh *mesh, const pb_options *opt, BlockCache *cache)
{
    return create_mesh(mesh, opt, cache);
}

// Device bytes a handle is expected to hold for V vertices, T triangles:
// geometry and source/target records, far-field partial sums, near pairs and
// near blocks (about 14 T pairs and 20 V nonzeros per block on molecular
// surfaces, with margin), work vectors, the Arnoldi basis, and the dense far
// field in assembled modes.
size_t estimate_device_bytes(int V, int T, const pb_options *o)
{
    const double v = V, t = T, n = 2.0 * V;
    // a buffer of kCacheMin bytes or more may come from a server's block cache,
    // which hands out whole blocks: charge what such a block can hold
    auto buf = [](double bytes) { return (double)cache_charge((size_t)bytes); };
    const int S = o->source_chunks > 0 ? std::min(o->source_chunks, T) : choose_chunks(T);
    double b = t * (kGeo * 8 + kStat * 12 + kDyn * 12 + 6 * 8 + 12 * 8 + 3 * 4 * 2);
    double part = (double)S * t * 16 * 8;
    if (o->precision == PB_FP32 && o->operator_mode != PB_TREECODE && o->regular_order != 1 &&
        sym_eligible(T, o->kappa, o->far_symmetric)) {
        const double ntile = std::ceil(t / 64.0), rt = std::ceil(ntile / 320.0);
        part = std::max(part, 2.0 * std::ceil(ntile / rt) * t * 16 * 4);   // the symmetric far field's slots
    }
    b += buf(part);
    b += buf(16.0 * t * (36 * 8 + 3 * 4));
    b += 24.0 * v * (4 * 8 + 4) + v * (4 * 8 + 4 * 4);
    b += 12.0 * n * 8;
    const bool mixed = o->precision >= PB_MIXED_BF16;
    const double m = std::min<double>(mixed ? std::min(o->inner_max_iter, o->max_iter) : o->max_iter, n) + 2;
    b += buf(m * n * 8);
    const double Vp = std::ceil(v / 64.0) * 64.0;
    // FP64 matrix, or FP32 matrix plus the 16-bit copy (mixed) or the assembly's
    // side matrix (FP32) of half its size
    const double dense = o->precision == PB_FP64 ? buf(n * 2.0 * Vp * 8.0)
                                                 : buf(n * 2.0 * Vp * 4.0) + buf(n * 2.0 * Vp * 2.0);
    const bool cal = is_calderon(o->preconditioner);
    const bool cal_sep = cal && (o->preconditioner != PB_CALDERON || o->calderon_fast);
    if (o->operator_mode == PB_ASSEMBLED || mixed) b += dense * (cal_sep && !o->calderon_fast ? 2.0 : 1.0);
    if (o->preconditioner == PB_MASS || o->preconditioner == PB_SCALED_MASS || cal)
        b += 5.0 * kMassBatch * n * 8 + 20.0 * v * 8 + v * 8;   // Chebyshev state, products, M, 1 / M_ii
    if (cal) b += 2.0 * n * 8 + (cal_sep ? 4.0 * 20.0 * v * 8 : 0.0);   // work vectors, P's near field
    if (cal && o->calderon_fast) b += buf(16.0 * t * (38 * 8)) + t * 8;   // P's pair blocks and sums, centroid weights
    if (o->operator_mode == PB_TREECODE) {
        const double np = std::pow(o->tree_degree + 1.0, 3.0);
        b += t / 16.0 * np * (12 * 8 + 8 * 8) + 64.0 * t;   // proxies and charges of about T/16 nodes, lists
        b += buf(16.0 * std::min(64.0, 4.0 * std::ceil(65536.0 / std::ceil(t / 64.0))) * t * 8);   // pieces' partial sums
    }
    b += 64.0 * 1024 * 1024;   // small buffers, charges, allocator rounding
    return (size_t)(b * 1.1);
}

// far-field product of the current operator fields into d.yfar (dense) or
// the per-triangle outputs (matrix-free); returns launch_gather's use_far
static int far_product(DevMesh &d, const double *x, int flags)
{
    if (flags & PB_APPLY_NEAR_ONLY) return 0;
    if (d.far_rule != 0) {
        // one-point rule: FP32 for fast Calderon's P, else the handle's precision
        const bool fp32c = d.far_rule == 1 || d.prm.precision == PB_FP32;
        launch_source_prep(d, x, fp32c);
        launch_far_centroid(d, fp32c);
        launch_far_finish(d, fp32c);
        return 1;
    }
    if (d.dense) {
        dense_apply(d, x, d.yfar);
        return 2;
    }
    const bool fp32 = d.prm.precision == PB_FP32;
    if (d.tree) {
        launch_source_prep(d, x, fp32);
        launch_tree_far(d, fp32);
        launch_far_finish(d, fp32);
        return 1;
    }
    launch_source_prep(d, x, fp32);
    launch_far(d, fp32);
    launch_far_finish(d, fp32);
    return 1;
}

// out = blockdiag(aM, bM)^-1 P blockdiag(M, M)^-1 in, in a plain vector, out
// offset like a captured iteration's output (ctl).  The inner steps honour the
// stop flag but take no offsets.
void calderon_left(DevMesh &d, const double *in, double *out, const DevCtl &ctl)
{
    const DevCtl inner{nullptr, ctl.skip, 0};
    mass_precond(d, 1, in, d.cal1, inner, 1.0, 1.0);
    {
        const DevCtl keep = d.ctl;
        d.ctl = inner;
        std::unique_ptr<PrecondOperator> use(calderon_separate(d) ? new PrecondOperator(d) : nullptr);
        const int use_far = far_product(d, d.cal1, 0);
        launch_gather(d, d.cal1, d.cal2, 0, use_far, true);
        use.reset();
        d.ctl = keep;
    }
    double a = 1.0, b = 1.0;
    calderon_scales(d.prm.formulation, d.prm.preconditioner, d.prm.eps_in, d.prm.eps_out, &a, &b);
    mass_precond(d, 1, d.cal2, out, ctl, 1.0 / a, 1.0 / b);
}

// the rest of the product once the far field is in (use_far as launch_gather)
static void apply_after_far(DevMesh &d, const double *x, double *y, int flags, int use_far)
{
    if ((flags & PB_APPLY_PRECOND) && mass_mode(d)) {
        launch_gather(d, x, d.mtmp, flags & ~PB_APPLY_PRECOND, use_far, false);
        mass_precond(d, 1, d.mtmp, y, d.ctl);
    } else if ((flags & PB_APPLY_PRECOND) && calderon_mode(d)) {
        launch_gather(d, x, d.mtmp, flags & ~PB_APPLY_PRECOND, use_far, false);
        calderon_left(d, d.mtmp, y, d.ctl);
    } else {
        launch_gather(d, x, y, flags, use_far, true);
    }
}

// y = A x (or P^-1 A x, or B A x for the Calderon preconditioners) on device
// vectors, on stream s of the handle.
void apply_operator(DevMesh &d, const double *x, double *y, int flags, hipStream_t s)
{
    hipStream_t keep = d.stream;
    if (s) d.stream = s;
    apply_after_far(d, x, y, flags, far_product(d, x, flags));
    d.stream = keep;
}

// ------------------------------------------------------------------- GMRES

static void ensure_krylov(DevMesh &d, int m)
{
    const int n = 2 * d.hm.V;
    if (d.kry.cap >= m + 1) return;
    d.kry.basis = (double *)d.alloc(sizeof(double) * (size_t)n * (m + 1));
    d.kry.kbuf = (double *)d.alloc(sizeof(double) * (2 * (m + 2) + 2));
    d.kry.y = (double *)d.alloc(sizeof(double) * (m + 1));
    d.kry.cap = m + 1;
}

// Host side of one unrestarted GMRES: Hessenberg columns from the device's
// CGS2 coefficients, Givens rotations, and the final triangular solve.  The
// single-handle and the batched solvers share it, so they round identically.
struct HostArnoldi {
    int m = 0, k = 0;
    double beta = 0.0, res = 0.0;
    std::vector<double> H, cs, sn, g, hb;
    void init(int m_, double beta_)
    {
        m = m_;
        beta = beta_;
        res = beta_;
        k = 0;
        H.assign((size_t)(m + 1) * m, 0.0);
        cs.assign(m, 0.0);
        sn.assign(m, 0.0);
        g.assign(m + 1, 0.0);
        hb.assign(2 * (m + 1) + 1, 0.0);
        g[0] = beta;
    }
    // hb holds the two CGS passes' coefficients and |w|^2 of step j; returns the
    // norm that w must be divided by (0: breakdown, leave w)
    double column(int j)
    {
        double *col = &H[(size_t)j * (m + 1)];
        for (int i = 0; i <= j; ++i) col[i] = hb[i] + hb[j + 1 + i];
        col[j + 1] = std::sqrt(std::max(hb[2 * (j + 1)], 0.0));
        return col[j + 1];
    }
    // rotations of step j; true when converged or broken down
    bool rotate(int j, double tol)
    {
        double *col = &H[(size_t)j * (m + 1)];
        for (int i = 0; i < j; ++i) {   // explicit FMAs: same arithmetic as the device Givens kernel
            const double a = std::fma(cs[i], col[i], sn[i] * col[i + 1]);
            col[i + 1] = std::fma(-sn[i], col[i], cs[i] * col[i + 1]);
            col[i] = a;
        }
        const double den = std::sqrt(std::fma(col[j], col[j], col[j + 1] * col[j + 1]));
        cs[j] = col[j] / den;
        sn[j] = col[j + 1] / den;
        col[j] = den;
        col[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        k = j + 1;
        res = std::fabs(g[j + 1]);
        return res <= tol * beta || !(den > 0.0);
    }
    std::vector<double> solution() const
    {
        std::vector<double> y(k);
        for (int i = k - 1; i >= 0; --i) {
            double a = g[i];
            for (int l = i + 1; l < k; ++l) a -= H[(size_t)l * (m + 1) + i] * y[l];
            y[i] = a / H[(size_t)i * (m + 1) + i];
        }
        return y;
    }
};

// device part of Arnoldi step j: w <- w - V h twice (CGS2), |w|^2; the
// coefficients land in kb
static void arnoldi_device(hipStream_t s, int n, int j, const double *Vb, double *w, double *kb)
{
    double *h1 = kb, *h2 = kb + (j + 1), *nr = kb + 2 * (j + 1);
    kr_dots(s, n, j + 1, Vb, n, w, h1);
    kr_update(s, n, j + 1, Vb, n, h1, w, -1.0);
    kr_dots(s, n, j + 1, Vb, n, w, h2);
    kr_update(s, n, j + 1, Vb, n, h2, w, -1.0);
    kr_dots(s, n, 1, w, n, w, nr);
}

// Unrestarted GMRES from x0 = 0 on P^-1 A u = pb (pb already preconditioned):
// classical Gram-Schmidt applied twice (CGS2) for the Arnoldi step, Givens
// rotations on the host.  Returns the number of iterations; *est receives the
// final residual estimate relative to |pb|.
int gmres(DevMesh &d, const double *pb, double *x, double tol, int max_iter, double *est)
{
    const int n = 2 * d.hm.V;
    const int m = std::min(max_iter, n);
    ensure_krylov(d, m);
    double *Vb = d.kry.basis, *kb = d.kry.kbuf;
    hipStream_t s = d.stream;
    kr_dots(s, n, 1, pb, n, pb, kb);
    double beta2 = 0.0;
    HIPCHECK(hipMemcpyAsync(&beta2, kb, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const double beta = std::sqrt(beta2);
    if (!(beta > 0.0)) {
        HIPCHECK(hipMemsetAsync(x, 0, sizeof(double) * n, s));
        *est = 0.0;
        return 0;
    }
    kr_scale_copy(s, n, pb, 1.0 / beta, Vb);
    HostArnoldi ha;
    ha.init(m, beta);
    for (int j = 0; j < m; ++j) {
        double *w = Vb + (size_t)(j + 1) * n;
        apply_operator(d, Vb + (size_t)j * n, w, PB_APPLY_PRECOND, nullptr);
        arnoldi_device(s, n, j, Vb, w, kb);
        HIPCHECK(hipMemcpyAsync(ha.hb.data(), kb, sizeof(double) * (2 * (j + 1) + 1), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        const double h = ha.column(j);
        if (h > 0.0) kr_scale_copy(s, n, w, 1.0 / h, w);
        if (ha.rotate(j, tol)) break;
    }
    const std::vector<double> y = ha.solution();
    HIPCHECK(hipMemcpyAsync(d.kry.y, y.data(), sizeof(double) * ha.k, hipMemcpyHostToDevice, s));
    kr_combine(s, n, ha.k, Vb, n, d.kry.y, x);
    *est = ha.res / beta;
    HIPCHECK(hipStreamSynchronize(s));   // y is a host vector
    return ha.k;
}

// ------------------------------------------------------ captured GMRES
// One Arnoldi step (operator product, CGS2, norm, device Givens, normalise)
// is captured once per handle and operator level as a HIP graph whose kernels
// read the iteration index and stop flag from device memory; the host replays
// it kReplay times between convergence checks, so iterations run back to back
// without a host round trip.  Same arithmetic as the eager loop except that the
// Givens rotations run on the device.
struct GraphGmres {
    int m = 0, n = 0;
    const double *basis = nullptr;
    GState *st = nullptr;
    double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *h1 = nullptr, *h2 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~GraphGmres()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

constexpr int kReplay = 8;

// device state of one handle's captured GMRES (Hessenberg, rotations, stop
// flag); shared by its own captured iteration and by batched solves
static GraphGmres *graph_state(DevMesh &d, int m)
{
    const int n = 2 * d.hm.V;
    std::unique_ptr<GraphGmres> G(new GraphGmres());
    G->m = m;
    G->n = n;
    G->basis = d.kry.basis;
    G->st = (GState *)d.alloc(sizeof(GState));
    G->H = (double *)d.alloc(sizeof(double) * (size_t)(m + 1) * m);
    G->cs = (double *)d.alloc(sizeof(double) * m);
    G->sn = (double *)d.alloc(sizeof(double) * m);
    G->g = (double *)d.alloc(sizeof(double) * (m + 1));
    G->h1 = (double *)d.alloc(sizeof(double) * (m + 1));
    G->h2 = (double *)d.alloc(sizeof(double) * (m + 1));
    return G.release();
}

// the handle's Arnoldi step after its far field (as apply_operator without
// far_product) and the device Givens step, for capture under d.ctl
static void iteration_tail(DevMesh &d, GraphGmres &G, int use_far)
{
    double *Vb = d.kry.basis;
    apply_after_far(d, Vb, Vb + G.n, PB_APPLY_PRECOND, use_far);
    kr_graph_iteration_tail(d.stream, G.n, G.m, Vb, G.st, G.H, G.cs, G.sn, G.g, G.h1, G.h2);
}

static void capture_into(DevMesh &d, GraphGmres &G)
{
    const int n = G.n;
    // one eager product first: settles autotuned launch shapes outside the capture
    apply_operator(d, d.kry.basis, d.ztmp, PB_APPLY_PRECOND, nullptr);
    HIPCHECK(hipStreamSynchronize(d.stream));
    double *Vb = d.kry.basis;
    d.ctl = DevCtl{&G.st->j, &G.st->done, (size_t)n};
    HIPCHECK(hipStreamBeginCapture(d.stream, hipStreamCaptureModeThreadLocal));
    try {
        iteration_tail(d, G, far_product(d, Vb, 0));
        HIPCHECK(hipGetLastError());
    } catch (...) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(d.stream, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        d.ctl = DevCtl();
        throw;
    }
    d.ctl = DevCtl();
    HIPCHECK(hipStreamEndCapture(d.stream, &G.graph));
    HIPCHECK(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
}

void destroy_graphs(DevMesh &d)
{
    for (auto &g : d.gg) {
        delete g;
        g = nullptr;
    }
}

// x = V y after k captured iterations: the triangular solve on the device's
// Hessenberg matrix and rotated right-hand side, on the host
static void graph_solution(DevMesh &d, GraphGmres &G, int k, double *x)
{
    const int n = G.n, m = G.m;
    hipStream_t s = d.stream;
    std::vector<double> H((size_t)(m + 1) * k), g(k + 1), y(k);
    HIPCHECK(hipMemcpyAsync(H.data(), G.H, sizeof(double) * H.size(), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(g.data(), G.g, sizeof(double) * (k + 1), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    for (int i = k - 1; i >= 0; --i) {
        double a = g[i];
        for (int l = i + 1; l < k; ++l) a -= H[(size_t)l * (m + 1) + i] * y[l];
        y[i] = a / H[(size_t)i * (m + 1) + i];
    }
    HIPCHECK(hipMemcpyAsync(d.kry.y, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    kr_combine(s, n, k, d.kry.basis, n, d.kry.y, x);
    HIPCHECK(hipStreamSynchronize(s));   // y is a host vector
}

static int gmres_graph(DevMesh &d, const double *pb, double *x, double tol, int max_iter, double *est)
{
    const int n = 2 * d.hm.V;
    const int m = std::min(max_iter, n);
    ensure_krylov(d, m);
    const int level = d.dense ? d.dense->level : 1;
    GraphGmres *&G = d.gg[level];
    if (G && (G->m != m || G->basis != d.kry.basis)) {
        delete G;
        G = nullptr;
    }
    hipStream_t s = d.stream;
    kr_dots(s, n, 1, pb, n, pb, d.red1);
    double beta2 = 0.0;
    HIPCHECK(hipMemcpyAsync(&beta2, d.red1, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const double beta = std::sqrt(beta2);
    if (!(beta > 0.0)) {
        HIPCHECK(hipMemsetAsync(x, 0, sizeof(double) * n, s));
        *est = 0.0;
        return 0;
    }
    kr_scale_copy(s, n, pb, 1.0 / beta, d.kry.basis);
    if (!G) G = graph_state(d, m);
    if (!G->exec) capture_into(d, *G);
    GState h0{};
    h0.j = 0;
    h0.done = 0;
    h0.m = m;
    h0.tolb = tol * beta;
    h0.res = beta;
    std::vector<double> g0(m + 1, 0.0);
    g0[0] = beta;
    HIPCHECK(hipMemcpyAsync(G->st, &h0, sizeof(GState), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(G->g, g0.data(), sizeof(double) * (m + 1), hipMemcpyHostToDevice, s));
    GState hs{};
    for (;;) {
        for (int r = 0; r < kReplay; ++r) HIPCHECK(hipGraphLaunch(G->exec, s));
        HIPCHECK(hipMemcpyAsync(&hs, G->st, sizeof(GState), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        if (hs.done || hs.j >= m) break;
    }
    graph_solution(d, *G, hs.j, x);
    *est = hs.res / beta;
    return hs.j;
}

// captured iterations unless profiling the operator kernels (their events
// are recorded eagerly) or the handle asks for eager launches
int gmres_solve(DevMesh &d, const double *pb, double *x, double tol, int max_iter, double *est)
{
    if (d.prof.on(0) || d.opt.use_graph == 0) return gmres(d, pb, x, tol, max_iter, est);
    return gmres_graph(d, pb, x, tol, max_iter, est);
}

// ------------------------------------------- batched solves of uneven requests
// GMRES of several matrix-free handles in lockstep on one stream: per
// iteration the far fields of every request still iterating run as one
// persistent launch per kernel form (k_far_batch, a work queue over all of
// them), the rest of each product and each request's Arnoldi step as in
// gmres(), and one host synchronisation serves every request.  Every
// request's arithmetic is that of gmres(), so its iterates are bitwise those
// of its own solve.
static void gmres_batch(const std::vector<DevMesh *> &ds, hipStream_t s, bool fp32, std::vector<int> &its,
                        std::vector<double> &est)
{
    const int R = (int)ds.size();
    std::vector<HostArnoldi> ha(R);
    std::vector<int> n(R), live;
    std::vector<double> beta2(R, 0.0);
    its.assign(R, 0);
    est.assign(R, 0.0);
    for (int r = 0; r < R; ++r) {
        DevMesh &d = *ds[r];
        n[r] = 2 * d.hm.V;
        ensure_krylov(d, std::min(d.opt.max_iter, n[r]));
        kr_dots(s, n[r], 1, d.ytmp, n[r], d.ytmp, d.kry.kbuf);
        HIPCHECK(hipMemcpyAsync(&beta2[r], d.kry.kbuf, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIPCHECK(hipStreamSynchronize(s));
    for (int r = 0; r < R; ++r) {
        DevMesh &d = *ds[r];
        const double beta = std::sqrt(beta2[r]);
        ha[r].init(std::min(d.opt.max_iter, n[r]), beta);
        if (!(beta > 0.0)) {
            HIPCHECK(hipMemsetAsync(d.u, 0, sizeof(double) * n[r], s));
            continue;
        }
        kr_scale_copy(s, n[r], d.ytmp, 1.0 / beta, d.kry.basis);
        live.push_back(r);
    }
    FarBatch fb;
    fb.stream = s;
    struct Free {
        FarBatch &fb;
        ~Free() { far_batch_free(fb); }
    } free_fb{fb};
    std::vector<int> planned;
    for (int j = 0; !live.empty(); ++j) {
        if (live != planned) {
            far_batch_plan(ds, live, fp32, fb);
            planned = live;
        }
        for (int r : live) launch_source_prep(*ds[r], ds[r]->kry.basis + (size_t)j * n[r], fp32);
        // the first handle's profiler (operator kind) times the fused launches
        Profiler &pf = ds[0]->prof;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (pf.on(0)) {
            HIPCHECK(hipEventCreate(&e0));
            HIPCHECK(hipEventCreate(&e1));
            HIPCHECK(hipEventRecord(e0, s));
        }
        launch_far_batch(fb, fp32);
        if (pf.on(0)) {
            HIPCHECK(hipEventRecord(e1, s));
            double pairs = 0.0;   // kernel pairs, near-masked pairs included
            for (int r : live) pairs += 36.0 * (double)ds[r]->hm.T * (double)ds[r]->hm.T;
            pf.record(0, e0, e1, pairs);
        }
        for (int r : live) {
            DevMesh &d = *ds[r];
            double *Vb = d.kry.basis, *w = Vb + (size_t)(j + 1) * n[r];
            launch_far_finish(d, fp32);
            apply_after_far(d, Vb + (size_t)j * n[r], w, PB_APPLY_PRECOND, 1);
            arnoldi_device(s, n[r], j, Vb, w, d.kry.kbuf);
            HIPCHECK(hipMemcpyAsync(ha[r].hb.data(), d.kry.kbuf, sizeof(double) * (2 * (j + 1) + 1),
                                    hipMemcpyDeviceToHost, s));
        }
        HIPCHECK(hipStreamSynchronize(s));
        std::vector<int> next;
        for (int r : live) {
            DevMesh &d = *ds[r];
            double *w = d.kry.basis + (size_t)(j + 1) * n[r];
            const double h = ha[r].column(j);
            if (h > 0.0) kr_scale_copy(s, n[r], w, 1.0 / h, w);
            if (!ha[r].rotate(j, d.opt.tol) && j + 1 < ha[r].m) next.push_back(r);
        }
        live.swap(next);
    }
    for (int r = 0; r < R; ++r) {
        if (!(ha[r].beta > 0.0)) continue;
        DevMesh &d = *ds[r];
        const std::vector<double> y = ha[r].solution();
        HIPCHECK(hipMemcpyAsync(d.kry.y, y.data(), sizeof(double) * ha[r].k, hipMemcpyHostToDevice, s));
        kr_combine(s, n[r], ha[r].k, d.kry.basis, n[r], d.kry.y, d.u);
        HIPCHECK(hipStreamSynchronize(s));   // y is a host vector
        its[r] = ha[r].k;
        est[r] = ha[r].res / ha[r].beta;
    }
}

// The same lockstep with the whole iteration of every request captured into
// one HIP graph of batched launches: the source weights of every request, the
// fused far-field launches, every request's far-field finish, gather (near
// field, preconditioner) and each CGS2 / norm / Givens / normalisation step
// run as one launch for all requests (KrylovReq / TailReq tables; each block
// runs the single kernel's code for its request), replayed kReplay times
// between checks.  A request's arithmetic is that of its own captured
// iteration (gmres_graph), so its results are bitwise those of its single
// solve; once its stop flag is set its blocks and far-field items do nothing,
// and at the next check the requests still iterating continue on a graph of
// their own, so stopped requests leave the work queues.  Graphs, tables and
// far-field work lists are kept per set of requests for later calls (key: the
// bytes of everything a graph refers to), so repeated calls with the same
// resident handles plan and capture nothing.
struct LockstepGraph {
    std::vector<char> key;
    unsigned long long used = 0;
    FarBatch fb;
    void *tables = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void release()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (tables) (void)hipFree(tables);
        far_batch_free(fb);
        exec = nullptr;
        graph = nullptr;
        tables = nullptr;
        key.clear();
    }
};
// per device, the kLockstepCache most recently used graphs, kept until the
// process ends (never destroyed from a static destructor, which may run after
// the HIP runtime's)
constexpr int kLockstepCache = 16;
static std::mutex g_lockstep_mu;
static std::map<int, std::vector<LockstepGraph *>> g_lockstep;
static unsigned long long g_lockstep_clock = 0;

template <typename T>
static void key_append(std::vector<char> &k, const T &v)
{
    const char *p = reinterpret_cast<const char *>(&v);
    k.insert(k.end(), p, p + sizeof(T));
}

// The captured iteration of the requests `live` (indices into ds), from the
// cache or captured now; caller holds g_lockstep_mu.
static LockstepGraph &lockstep_graph(const std::vector<DevMesh *> &ds, const std::vector<int> &live,
                                     const std::vector<GraphGmres *> &G, const std::vector<int> &n,
                                     const std::vector<int> &m, bool fp32, hipStream_t s)
{
    const int L = (int)live.size();
    std::vector<TailReq> tq(L);
    std::vector<KrylovReq> kq(L);
    std::vector<int> bsrc(L + 1, 0), bfin(L + 1, 0), bgat(L + 1, 0), bkry(L + 1, 0);
    int ndot = 0;
    std::vector<char> key;
    key_append(key, fp32);
    for (int k = 0; k < L; ++k) {
        const int r = live[k];
        DevMesh &d = *ds[r];
        GraphGmres &g = *G[r];
        const bool mass = mass_mode(d);
        const bool sym = fp32 && d.sym_nitems > 0;
        TailReq &t = tq[k];
        t = TailReq{};
        t.T = d.hm.T;
        t.V = d.hm.V;
        t.S = d.S;
        t.rt = sym ? d.sym_rt : 0;
        t.nr = sym ? d.sym_nr : 0;
        t.family = d.fm.family;
        t.swap = d.fm.family == 0 && laplace_row(d.fm) == 1;
        t.precond = mass ? 0 : 1;
        t.tri = d.tri;
        t.geo = d.geo;
        t.dyn64 = d.dyn64;
        t.dyn32 = d.dyn32;
        t.part = d.part;
        t.triout = d.triout;
        t.inc_ptr = d.inc_ptr;
        t.inc_tk = d.inc_tk;
        t.row_ptr = d.row_ptr;
        t.col = d.col;
        t.N = d.N;
        t.pinv = d.pinv;
        t.nnz = d.nnz();
        t.x = d.kry.basis;
        t.gout = mass ? d.mtmp : d.kry.basis + n[r];
        t.gout_offset = mass ? 0 : 1;
        t.ctl = DevCtl{&g.st->j, &g.st->done, (size_t)n[r]};
        KrylovReq &q = kq[k];
        q = KrylovReq{n[r], m[r], d.kry.basis, g.st, g.H, g.cs, g.sn, g.g, g.h1, g.h2};
        bsrc[k + 1] = bsrc[k] + tail_blocks_source(t);
        bfin[k + 1] = bfin[k] + tail_blocks_finish(t);
        bgat[k + 1] = bgat[k] + tail_blocks_gather(t);
        bkry[k + 1] = bkry[k] + kr_batch_blocks(n[r]);
        ndot += m[r] + 1;
        key_append(key, t);
        key_append(key, q);
        key_append(key, d.fm);   // the far-field coefficients follow from fm and kappa
        key_append(key, d.prm.kappa);
        key_append(key, sym);
        key_append(key, d.stat32);
        key_append(key, d.stat64);
        if (mass) {   // the mass preconditioner's launches: buffers and scales
            key_append(key, d.prm.preconditioner);
            key_append(key, d.prm.eps_in);
            key_append(key, d.prm.eps_out);
            key_append(key, d.cheb);
            key_append(key, d.Mdinv);
            key_append(key, d.Mval);
        }
    }
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    std::vector<LockstepGraph *> &cache = g_lockstep[dev];
    for (LockstepGraph *e : cache)
        if (e->exec && e->key == key) {
            e->used = ++g_lockstep_clock;
            return *e;
        }
    LockstepGraph *slot = nullptr;
    if ((int)cache.size() < kLockstepCache) {
        cache.push_back(new LockstepGraph());
        slot = cache.back();
    } else {
        slot = *std::min_element(cache.begin(), cache.end(),
                                 [](const LockstepGraph *x, const LockstepGraph *y) { return x->used < y->used; });
    }
    LockstepGraph &lg = *slot;
    lg.release();
    lg.fb.stream = s;
    std::vector<const int *> skip(ds.size(), nullptr);
    for (int r : live) skip[r] = &G[r]->st->done;
    far_batch_plan(ds, live, fp32, lg.fb, skip);
    const size_t bt = sizeof(TailReq) * L, bk = sizeof(KrylovReq) * L, bi = sizeof(int) * (L + 1);
    HIPCHECK(hipMalloc(&lg.tables, bt + bk + 4 * bi));
    char *base = (char *)lg.tables;
    HIPCHECK(hipMemcpyAsync(base, tq.data(), bt, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(base + bt, kq.data(), bk, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(base + bt + bk, bsrc.data(), bi, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(base + bt + bk + bi, bfin.data(), bi, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(base + bt + bk + 2 * bi, bgat.data(), bi, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(base + bt + bk + 3 * bi, bkry.data(), bi, hipMemcpyHostToDevice, s));
    HIPCHECK(hipStreamSynchronize(s));   // host tables go out of scope
    const TailReq *dt = (const TailReq *)base;
    const KrylovReq *dk = (const KrylovReq *)(base + bt);
    const int *dsrc = (const int *)(base + bt + bk), *dfin = dsrc + (L + 1), *dgat = dfin + (L + 1),
              *dkry = dgat + (L + 1);
    for (int r : live) ds[r]->ctl = DevCtl{&G[r]->st->j, &G[r]->st->done, (size_t)n[r]};
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
        launch_batch_source_prep(s, L, dt, dsrc, bsrc[L]);
        launch_far_batch(lg.fb, fp32);
        launch_batch_finish(s, fp32, L, dt, dfin, bfin[L]);
        launch_batch_gather(s, L, dt, dgat, bgat[L]);
        for (int r : live)   // apply_after_far's mass-preconditioner step, per request
            if (mass_mode(*ds[r])) mass_precond(*ds[r], 1, ds[r]->mtmp, ds[r]->kry.basis + n[r], ds[r]->ctl);
        kr_batch_iteration_tail(s, L, dk, dkry, bkry[L], ndot);
        HIPCHECK(hipGetLastError());
    } catch (...) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(s, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        for (int r : live) ds[r]->ctl = DevCtl();
        lg.release();
        throw;
    }
    for (int r : live) ds[r]->ctl = DevCtl();
    try {
        HIPCHECK(hipStreamEndCapture(s, &lg.graph));
        HIPCHECK(hipGraphInstantiate(&lg.exec, lg.graph, nullptr, nullptr, 0));
    } catch (...) {
        lg.release();
        throw;
    }
    lg.key = key;
    lg.used = ++g_lockstep_clock;
    return lg;
}

static void gmres_batch_graph(const std::vector<DevMesh *> &ds, hipStream_t s, bool fp32, std::vector<int> &its,
                              std::vector<double> &est)
{
    const int R = (int)ds.size();
    std::vector<int> n(R), m(R), live;
    std::vector<double> beta2(R, 0.0), beta(R, 0.0);
    std::vector<GraphGmres *> G(R, nullptr);
    its.assign(R, 0);
    est.assign(R, 0.0);
    for (int r = 0; r < R; ++r) {
        DevMesh &d = *ds[r];
        n[r] = 2 * d.hm.V;
        m[r] = std::min(d.opt.max_iter, n[r]);
        ensure_krylov(d, m[r]);
        kr_dots(s, n[r], 1, d.ytmp, n[r], d.ytmp, d.red1);
        HIPCHECK(hipMemcpyAsync(&beta2[r], d.red1, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIPCHECK(hipStreamSynchronize(s));
    std::vector<GState> h0(R);
    std::vector<std::vector<double>> g0(R);
    for (int r = 0; r < R; ++r) {
        DevMesh &d = *ds[r];
        beta[r] = std::sqrt(beta2[r]);
        if (!(beta[r] > 0.0)) {
            HIPCHECK(hipMemsetAsync(d.u, 0, sizeof(double) * n[r], s));
            continue;
        }
        kr_scale_copy(s, n[r], d.ytmp, 1.0 / beta[r], d.kry.basis);
        GraphGmres *&g = d.gg[d.dense ? d.dense->level : 1];
        if (g && (g->m != m[r] || g->basis != d.kry.basis)) {
            delete g;
            g = nullptr;
        }
        if (!g) g = graph_state(d, m[r]);
        G[r] = g;
        h0[r] = GState{};
        h0[r].m = m[r];
        h0[r].tolb = d.opt.tol * beta[r];
        h0[r].res = beta[r];
        g0[r].assign(m[r] + 1, 0.0);
        g0[r][0] = beta[r];
        HIPCHECK(hipMemcpyAsync(g->st, &h0[r], sizeof(GState), hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(g->g, g0[r].data(), sizeof(double) * (m[r] + 1), hipMemcpyHostToDevice, s));
        live.push_back(r);
    }
    HIPCHECK(hipStreamSynchronize(s));   // h0, g0 are host vectors
    if (live.empty()) return;
    std::vector<GState> hs(R);
    std::vector<int> running = live;
    {
        std::lock_guard<std::mutex> lk(g_lockstep_mu);
        while (!running.empty()) {
            LockstepGraph &lg = lockstep_graph(ds, running, G, n, m, fp32, s);
            for (int k = 0; k < kReplay; ++k) HIPCHECK(hipGraphLaunch(lg.exec, s));
            for (int r : running)
                HIPCHECK(hipMemcpyAsync(&hs[r], G[r]->st, sizeof(GState), hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            std::vector<int> next;
            for (int r : running)
                if (!(hs[r].done || hs[r].j >= m[r])) next.push_back(r);
            running.swap(next);
        }
    }
    for (int r : live) {
        graph_solution(*ds[r], *G[r], hs[r].j, ds[r]->u);
        its[r] = hs[r].j;
        est[r] = hs[r].res / beta[r];
    }
}

// Solves one charge set per handle with the far-field products of all of
// them fused (gmres_batch), everything on the first handle's stream; the
// handles' own streams are drained first and restored afterwards.
static pb_status solve_batch(const std::vector<DevMesh *> &ds, const pb_charges *ch, pb_result *res)
{
    for (const DevMesh *d : ds) check_solvable(*d);
    TraceRange batch_range("pb.batch");
    const int R = (int)ds.size();
    hipStream_t s = ds[0]->stream;
    std::vector<hipStream_t> keep(R);
    for (int r = 0; r < R; ++r) {
        keep[r] = ds[r]->stream;
        HIPCHECK(hipStreamSynchronize(keep[r]));
    }
    struct Restore {
        const std::vector<DevMesh *> &ds;
        const std::vector<hipStream_t> &keep;
        ~Restore()
        {
            for (size_t r = 0; r < ds.size(); ++r) ds[r]->stream = keep[r];
        }
    } restore{ds, keep};
    for (DevMesh *d : ds) d->stream = s;
    std::vector<double> t_rhs(R), t_prec(R);
    for (int r = 0; r < R; ++r) {
        TraceRange range("pb.rhs+precond");
        DevMesh &d = *ds[r];
        const double t0 = now();
        try {
            charges_to_device(d, &ch[r]);
            check_charges_inside(d, ch[r].n);
        } catch (const Error &e) {
            fail(e.code, "request " + std::to_string(r) + ": " + e.msg);
        }
        formulation_rhs(d, ch[r].n, d.qbuf, d.xtmp);
        HIPCHECK(hipStreamSynchronize(s));
        const double t1 = now();
        if (mass_mode(d)) mass_precond(d, 1, d.xtmp, d.ytmp, DevCtl());
        else kr_precond(s, d.hm.V, d.pinv, d.xtmp, d.ytmp);
        if (!d.u) d.u = (double *)d.alloc(sizeof(double) * 2 * (size_t)d.hm.V);
        HIPCHECK(hipStreamSynchronize(s));
        t_rhs[r] = t1 - t0;
        t_prec[r] = now() - t1;
    }
    const double t2 = now();
    std::vector<int> its;
    std::vector<double> est;
    const bool fp32 = ds[0]->prm.precision == PB_FP32;
    {
        TraceRange range("pb.gmres");
        // captured iterations unless timing the fused launches or eager launches are asked for
        if (ds[0]->opt.use_graph && !ds[0]->prof.on(0)) gmres_batch_graph(ds, s, fp32, its, est);
        else gmres_batch(ds, s, fp32, its, est);
    }
    const double t_gmres = now() - t2;
    pb_status worst = PB_OK;
    for (int r = 0; r < R; ++r) {
        // the profile keeps the fused launches only, not the residual check's product
        const int mask = ds[r]->prof.mask;
        ds[r]->prof.mask = 0;
        const pb_status st = finish_result(*ds[r], &ch[r], ds[r]->ytmp, ds[r]->u, its[r], 1, t_rhs[r], t_prec[r],
                                           t_gmres, &res[r]);
        ds[r]->prof.mask = mask;
        if (st != PB_OK) worst = st;
    }
    return worst;
}

// ------------------------------------------------------------ charges, dG
void charges_to_device(DevMesh &d, const pb_charges *c)
{
    if (!c || c->n < 1 || !c->xyz || !c->q) fail(PB_E_INVALID_ARG, "charges must hold n >= 1 points");
    const int nq = c->n;
    for (int i = 0; i < 3 * nq; ++i)
        if (!std::isfinite(c->xyz[i])) fail(PB_E_INVALID_ARG, "charge positions must be finite");
    for (int i = 0; i < nq; ++i)
        if (!std::isfinite(c->q[i])) fail(PB_E_INVALID_ARG, "charge values must be finite");
    if (nq > d.qcap) {
        d.qbuf = (double *)d.alloc(sizeof(double) * 7 * (size_t)nq);
        d.qcap = nq;
    }
    std::vector<double> h(7 * (size_t)nq);
    for (int i = 0; i < nq; ++i) {
        for (int c3 = 0; c3 < 3; ++c3) {
            h[(size_t)c3 * nq + i] = c->xyz[3 * i + c3];
            h[(size_t)4 * nq + 3 * i + c3] = c->xyz[3 * i + c3];
        }
        h[(size_t)3 * nq + i] = c->q[i];
    }
    HIPCHECK(hipMemcpyAsync(d.qbuf, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, d.stream));
}

static double *reduction_buffer(DevMesh &d, int npts)
{
    const int need = npts * reduction_chunks(d.hm.T);
    if (need > d.redcap) {
        d.red = (double *)d.alloc(sizeof(double) * need);
        d.redcap = need;
    }
    return d.red;
}

void check_charges_inside(DevMesh &d, int nq)
{
    const int C = reduction_chunks(d.hm.T);
    double *part = reduction_buffer(d, nq);
    launch_inside_test(d, nq, d.qbuf + 4 * (size_t)nq, part);
    std::vector<double> h((size_t)nq * C);
    HIPCHECK(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, d.stream));
    HIPCHECK(hipStreamSynchronize(d.stream));
    for (int k = 0; k < nq; ++k) {
        double s = 0.0;
        for (int c = 0; c < C; ++c) s += h[(size_t)k * C + c];
        if (!(s > 2.0 * kPi)) fail(PB_E_CHARGES, "charge " + std::to_string(k) + " lies outside the surface");
    }
}

// phi_reac at npts device points (AoS) from the device traces u (2V)
static void reaction_potential(DevMesh &d, const double *u, int npts, const double *pts_dev, double *out_host)
{
    const int C = reduction_chunks(d.hm.T);
    launch_source_prep(d, u, false);
    double *part = reduction_buffer(d, npts);
    launch_reaction(d, npts, pts_dev, part);
    std::vector<double> h((size_t)npts * C);
    HIPCHECK(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, d.stream));
    HIPCHECK(hipStreamSynchronize(d.stream));
    for (int k = 0; k < npts; ++k) {
        double s = 0.0;
        for (int c = 0; c < C; ++c) s += h[(size_t)k * C + c];
        out_host[k] = s * kInv4Pi;
    }
}

static void rhs_device(DevMesh &d, int nq, double *b)
{
    launch_rhs(d, nq, d.qbuf, b);
}

// Accurate preconditioned residual, reaction potential and Delta G for the
// solution u of one charge set; fills *res.
pb_status finish_result(DevMesh &d, const pb_charges *ch, const double *pb, double *u, int its, int outer,
                        double t_rhs, double t_prec, double t_gmres, pb_result *res)
{
    TraceRange range("pb.dG");
    const int V = d.hm.V, n = 2 * V;
    const double t3 = now();
        apply_operator(d, u, d.ztmp, PB_APPLY_PRECOND, nullptr);
    kr_axpy(d.stream, n, -1.0, pb, d.ztmp);
    kr_dots(d.stream, n, 1, d.ztmp, n, d.ztmp, d.red1);
    kr_dots(d.stream, n, 1, pb, n, pb, d.red1 + 1);
    double rr[2];
    HIPCHECK(hipMemcpyAsync(rr, d.red1, sizeof(rr), hipMemcpyDeviceToHost, d.stream));
    // exterior unknowns -> interior traces (interface conditions)
    if (d.fm.exterior) kr_scale_copy(d.stream, V, u + V, d.prm.eps_out / d.prm.eps_in, u + V);
    charges_to_device(d, ch);
    const int nq = ch->n;
    std::vector<double> pr(nq);
    reaction_potential(d, u, nq, d.qbuf + 4 * (size_t)nq, pr.data());
    double e = 0.0;
    for (int k = 0; k < nq; ++k) e += ch->q[k] * pr[k];
    res->dG_kcal = 0.5 * kEnergyC * e;
    if (res->phi) HIPCHECK(hipMemcpyAsync(res->phi, u, sizeof(double) * V, hipMemcpyDeviceToHost, d.stream));
    if (res->dphi) HIPCHECK(hipMemcpyAsync(res->dphi, u + V, sizeof(double) * V, hipMemcpyDeviceToHost, d.stream));
    HIPCHECK(hipStreamSynchronize(d.stream));
    res->iterations = its;
    res->outer_iterations = outer;
    res->rel_residual = rr[1] > 0 ? std::sqrt(std::max(rr[0], 0.0) / rr[1]) : 0.0;
    res->t_setup = d.t_setup;
    res->t_rhs = t_rhs;
    res->t_prec = t_prec;
    res->t_gmres = t_gmres;
    res->t_dG = now() - t3;
    res->device_bytes = d.bytes;
    return res->rel_residual <= d.opt.tol * 1.0000001 ? PB_OK : PB_NOT_CONVERGED;
}

// The combined field with alpha = beta = 0 is one side's trace equations
// alone: a well-defined operator (pb_mesh_apply), but no formulation of the
// interface problem, so the solvers refuse it.
void check_solvable(const DevMesh &d)
{
    if ((d.prm.formulation == PB_CFIE_INT || d.prm.formulation == PB_CFIE_EXT) && d.opt.cfie_alpha == 0.0 &&
        d.opt.cfie_beta == 0.0)
        fail(PB_E_STATE, "cfie_alpha = cfie_beta = 0 keeps one side's trace equations only, which do not couple "
                         "the two problems: the operator can be applied, not solved");
}

pb_status solve_on_mesh(DevMesh &d, const pb_charges *ch, pb_result *res)
{
    check_solvable(d);
    if (!res) fail(PB_E_INVALID_ARG, "result must not be NULL");
    const int V = d.hm.V, n = 2 * V;
    TraceRange solve_range("pb.solve");
    double t0 = now();
    double *b = d.xtmp, *pb = d.ytmp;
    {
        TraceRange range("pb.rhs");
        charges_to_device(d, ch);
        const int nq = ch->n;
        check_charges_inside(d, nq);
        formulation_rhs(d, nq, d.qbuf, b);
        HIPCHECK(hipStreamSynchronize(d.stream));
    }
    double t1 = now();
    {
        TraceRange range("pb.precond");
        if (mass_mode(d)) mass_precond(d, 1, b, pb, DevCtl());
        else if (calderon_mode(d)) calderon_left(d, b, pb, DevCtl());
        else kr_precond(d.stream, V, d.pinv, b, pb);
        HIPCHECK(hipStreamSynchronize(d.stream));
    }
    double t2 = now();
    if (!d.u) d.u = (double *)d.alloc(sizeof(double) * n);
    double est = 0.0;
    int outer = 1, its;
    {
        TraceRange range("pb.gmres");
        if (d.prm.precision >= PB_MIXED_BF16)
            its = mixed_refinement_solve(d, b, pb, d.u, &est, &outer);
        else
            its = gmres_solve(d, pb, d.u, d.opt.tol, d.opt.max_iter, &est);
        HIPCHECK(hipStreamSynchronize(d.stream));
    }
    double t3 = now();
    return finish_result(d, ch, pb, d.u, its, outer, t1 - t0, t2 - t1, t3 - t2, res);
}

}  // namespace pbm

// =================================================================== C ABI
using namespace pbm;

struct pb_mesh_handle {
    DevMesh *d;
};

#define PB_TRY try {
#define PB_CATCH                                                         \
    }                                                                    \
    catch (const Error &e) {                                             \
        set_error(e.msg);                                                \
        return e.code;                                                   \
    }                                                                    \
    catch (const std::bad_alloc &) {                                     \
        set_error("host out of memory");                                 \
        return PB_E_NOMEM;                                               \
    }                                                                    \
    catch (...) {                                                        \
        set_error("unexpected internal error");                          \
        return PB_E_DEVICE;                                              \
    }

extern "C" {

void pb_default_options(pb_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->eps_in = 4.0;
    o->eps_out = 80.0;
    o->kappa = 0.125;
    o->formulation = PB_DIRECT_INT;
    o->preconditioner = PB_BLOCK_DIAG;
    o->precision = PB_FP64;
    o->operator_mode = PB_MATRIX_FREE;
    o->tol = 1e-5;
    o->max_iter = 1000;
    o->singular_order = 4;
    o->source_chunks = 0;
    o->inner_max_iter = 200;
    o->inner_tol = 1e-3;
    o->memory_budget = 0;
    o->use_graph = 1;
    o->tree_degree = 6;
    o->tree_theta = 0.7;
    o->cfie_alpha = 1.0;
    o->cfie_beta = 1.0;
    o->regular_order = 4;
    o->far_symmetric = 0;
}

const char *pb_last_error(void) { return g_err.c_str(); }

int32_t pb_device_count(void)
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    return n;
}

pb_status pb_mesh_create(const pb_mesh *mesh, const pb_options *opt, pb_mesh_handle **out)
{
    PB_TRY
    if (!out) fail(PB_E_INVALID_ARG, "out must not be NULL");
    *out = nullptr;
    DevMesh *d = create_mesh(mesh, opt);
    *out = new pb_mesh_handle{d};
    set_error("");
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_destroy(pb_mesh_handle *h)
{
    PB_TRY
    if (!h) return PB_OK;
    delete h->d;
    delete h;
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_get_info(const pb_mesh_handle *h, pb_mesh_info *info)
{
    PB_TRY
    if (!h || !info) fail(PB_E_INVALID_ARG, "NULL argument");
    const DevMesh &d = *h->d;
    info->n_vertices = d.hm.V;
    info->n_triangles = d.hm.T;
    info->n_near_pairs = d.npair();
    info->near_nnz = d.nnz();
    info->source_chunks = d.S;
    info->assembled = d.dense ? 1 : 0;
    info->device_bytes = d.bytes;
    info->far_symmetric = (d.sym_nitems > 0 && !d.dense && !d.tree) ? 1 : 0;
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_refresh(pb_mesh_handle *h)
{
    PB_TRY
    if (!h) fail(PB_E_INVALID_ARG, "NULL handle");
    DevMesh &d = *h->d;
    const double t0 = now();
    setup_and_wait(d);
    d.t_setup = now() - t0;
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_solve(pb_mesh_handle *h, const pb_charges *charges, pb_result *result)
{
    PB_TRY
    if (!h) fail(PB_E_INVALID_ARG, "NULL handle");
    return solve_on_mesh(*h->d, charges, result);
    PB_CATCH
}

pb_status pb_solve(const pb_mesh *mesh, const pb_charges *charges, const pb_options *opt, pb_result *result)
{
    PB_TRY
    std::unique_ptr<DevMesh> d(create_mesh(mesh, opt));
    return solve_on_mesh(*d, charges, result);
    PB_CATCH
}

pb_status pb_solve_multi(pb_mesh_handle *h, int32_t n_sets, const pb_charges *sets, pb_result *out)
{
    PB_TRY
    if (!h || n_sets < 1 || !sets || !out) fail(PB_E_INVALID_ARG, "bad pb_solve_multi arguments");
    if (calderon_mode(*h->d)) fail(PB_E_STATE, "batched solves do not support the Calderon preconditioners");
    return solve_multi(*h->d, n_sets, sets, out);
    PB_CATCH
}

pb_status pb_solve_batch(int32_t n, pb_mesh_handle *const *handles, const pb_charges *charges,
                         pb_result *results)
{
    PB_TRY
    if (n < 1 || n > PB_MAX_BATCH_REQUESTS || !handles || !charges || !results)
        fail(PB_E_INVALID_ARG, "bad pb_solve_batch arguments");
    std::vector<DevMesh *> ds(n);
    for (int r = 0; r < n; ++r) {
        if (!handles[r]) fail(PB_E_INVALID_ARG, "NULL handle in pb_solve_batch");
        ds[r] = handles[r]->d;
        for (int q = 0; q < r; ++q)
            if (ds[q] == ds[r]) fail(PB_E_INVALID_ARG, "a handle appears twice in pb_solve_batch");
    }
    const int prec = ds[0]->prm.precision;
    for (DevMesh *d : ds) {
        if (d->prm.precision != prec || (prec != PB_FP32 && prec != PB_FP64))
            fail(PB_E_STATE, "pb_solve_batch needs handles of one precision, PB_FP64 or PB_FP32");
        if (d->dense || d->tree || d->far_rule != 0)
            fail(PB_E_STATE, "pb_solve_batch needs matrix-free handles (no assembled far field, no treecode)");
        if (calderon_mode(*d)) fail(PB_E_STATE, "pb_solve_batch does not support the Calderon preconditioners");
    }
    return solve_batch(ds, charges, results);
    PB_CATCH
}

pb_status pb_mesh_apply(pb_mesh_handle *h, const double *x, double *y, int32_t flags)
{
    PB_TRY
    if (!h || !x || !y) fail(PB_E_INVALID_ARG, "NULL argument");
    DevMesh &d = *h->d;
    const int n = 2 * d.hm.V;
    HIPCHECK(hipMemcpyAsync(d.xtmp, x, sizeof(double) * n, hipMemcpyHostToDevice, d.stream));
    apply_operator(d, d.xtmp, d.ytmp, flags, nullptr);
    HIPCHECK(hipMemcpyAsync(y, d.ytmp, sizeof(double) * n, hipMemcpyDeviceToHost, d.stream));
    HIPCHECK(hipStreamSynchronize(d.stream));
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_apply_device(pb_mesh_handle *h, const double *x, double *y, int32_t flags, void *stream)
{
    PB_TRY
    if (!h || !x || !y) fail(PB_E_INVALID_ARG, "NULL argument");
    apply_operator(*h->d, x, y, flags, (hipStream_t)stream);
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_rhs(pb_mesh_handle *h, const pb_charges *charges, double *b)
{
    PB_TRY
    if (!h || !b) fail(PB_E_INVALID_ARG, "NULL argument");
    DevMesh &d = *h->d;
    charges_to_device(d, charges);
    rhs_device(d, charges->n, d.xtmp);
    HIPCHECK(hipMemcpyAsync(b, d.xtmp, sizeof(double) * 2 * d.hm.V, hipMemcpyDeviceToHost, d.stream));
    HIPCHECK(hipStreamSynchronize(d.stream));
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_reaction_potential(pb_mesh_handle *h, const double *phi, const double *dphi, int32_t npts,
                                     const double *pts, double *out)
{
    PB_TRY
    if (!h || !phi || !dphi || !pts || !out || npts < 1) fail(PB_E_INVALID_ARG, "bad arguments");
    DevMesh &d = *h->d;
    const int V = d.hm.V;
    HIPCHECK(hipMemcpyAsync(d.xtmp, phi, sizeof(double) * V, hipMemcpyHostToDevice, d.stream));
    HIPCHECK(hipMemcpyAsync(d.xtmp + V, dphi, sizeof(double) * V, hipMemcpyHostToDevice, d.stream));
    std::vector<double> q(npts, 0.0);
    pb_charges c{npts, pts, q.data()};
    charges_to_device(d, &c);
    reaction_potential(d, d.xtmp, npts, d.qbuf + 4 * (size_t)npts, out);
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_reaction_potential_noalloc(pb_mesh_handle *h, const double *traces_device, int32_t npts,
                                             const double *pts_device, double *out_device, void *hip_stream)
{
    PB_TRY
    if (!h || !traces_device || !pts_device || !out_device || npts < 1) fail(PB_E_INVALID_ARG, "bad arguments");
    reaction_potential_noalloc(*h->d, traces_device, npts, pts_device, out_device, (hipStream_t)hip_stream);
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_near_blocks(pb_mesh_handle *h, int32_t n, const int32_t *t, const int32_t *s, double *out)
{
    PB_TRY
    if (!h || !t || !s || !out || n < 1) fail(PB_E_INVALID_ARG, "bad arguments");
    DevMesh &d = *h->d;
    const HostMesh &hm = d.hm;
    std::vector<int32_t> ts(n), ss(n);
    for (int k = 0; k < n; ++k) {
        if (t[k] < 0 || t[k] >= hm.T || s[k] < 0 || s[k] >= hm.T) fail(PB_E_INVALID_ARG, "triangle id out of range");
        ts[k] = hm.iperm[t[k]];
        ss[k] = hm.iperm[s[k]];
        int shared = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) shared += hm.tri[3 * ts[k] + a] == hm.tri[3 * ss[k] + b];
        if (shared == 0) fail(PB_E_INVALID_ARG, "pair does not share a vertex");
    }
    std::vector<int32_t> gi;
    int count[4];
    ss_group(hm.tri, n, ts.data(), ss.data(), gi, count);
    int32_t *dt = (int32_t *)d.alloc(sizeof(int32_t) * n), *ds = (int32_t *)d.alloc(sizeof(int32_t) * n);
    int32_t *di = (int32_t *)d.alloc(sizeof(int32_t) * n);
    double *o = (double *)d.alloc(sizeof(double) * 36 * n);
    HIPCHECK(hipMemcpyAsync(dt, ts.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, d.stream));
    HIPCHECK(hipMemcpyAsync(ds, ss.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, d.stream));
    HIPCHECK(hipMemcpyAsync(di, gi.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, d.stream));
    launch_pair_blocks_subset(d, n, dt, ds, di, count, o);
    HIPCHECK(hipMemcpyAsync(out, o, sizeof(double) * 36 * n, hipMemcpyDeviceToHost, d.stream));
    HIPCHECK(hipStreamSynchronize(d.stream));
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_preconditioner(pb_mesh_handle *h, double *out)
{
    PB_TRY
    if (!h || !out) fail(PB_E_INVALID_ARG, "NULL argument");
    DevMesh &d = *h->d;
    HIPCHECK(hipMemcpyAsync(out, d.pinv, sizeof(double) * 4 * d.hm.V, hipMemcpyDeviceToHost, d.stream));
    HIPCHECK(hipStreamSynchronize(d.stream));
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_profile(pb_mesh_handle *h, int32_t enable)
{
    PB_TRY
    if (!h) fail(PB_E_INVALID_ARG, "NULL handle");
    Profiler &p = h->d->prof;
    HIPCHECK(hipStreamSynchronize(h->d->stream));
    for (int k = 0; k < 2; ++k) {
        for (hipEvent_t e : p.ev[k]) (void)hipEventDestroy(e);
        p.ev[k].clear();
        p.pend_work[k].clear();
        p.launches[k] = 0;
        p.total_ms[k] = 0.0;
        p.work[k] = 0.0;
    }
    p.mask = enable & 3;
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_profile_read(pb_mesh_handle *h, int32_t kind, int64_t *launches, double *total_ms,
                               double *total_work)
{
    PB_TRY
    if (!h || !launches || !total_ms || kind < 0 || kind > 1) fail(PB_E_INVALID_ARG, "bad arguments");
    Profiler &p = h->d->prof;
    HIPCHECK(hipStreamSynchronize(h->d->stream));
    for (size_t i = 0; i + 1 < p.ev[kind].size(); i += 2) {
        float ms = 0.0f;
        HIPCHECK(hipEventElapsedTime(&ms, p.ev[kind][i], p.ev[kind][i + 1]));
        p.total_ms[kind] += ms;
        p.launches[kind] += 1;
        p.work[kind] += p.pend_work[kind][i / 2];
        (void)hipEventDestroy(p.ev[kind][i]);
        (void)hipEventDestroy(p.ev[kind][i + 1]);
    }
    p.ev[kind].clear();
    p.pend_work[kind].clear();
    *launches = p.launches[kind];
    *total_ms = p.total_ms[kind];
    if (total_work) *total_work = p.work[kind];
    return PB_OK;
    PB_CATCH
}

pb_status pb_mesh_synchronize(pb_mesh_handle *h)
{
    PB_TRY
    if (!h) fail(PB_E_INVALID_ARG, "NULL handle");
    HIPCHECK(hipStreamSynchronize(h->d->stream));
    return PB_OK;
    PB_CATCH
}

}  // extern "C"
