// Far field, matrix-free: regular 6 x 6 point quadrature over every ordered
// triangle pair that shares no vertex (Numerical discretization), fused over
// the operators of one formulation (Eqs. bie:dirichlet:int, bie:juffer:int).
//
// Work split:
//   k_source_prep : x (2V) -> per-triangle source weights b1 = w|s| u1(y_q),
//                   b2 = w|s| u2(y_q), C = |s| curl u1|_s.
//   k_far         : one lane per target triangle (6 target points held in
//                   registers), grid.y splits the source triangles into chunks;
//                   the source loop is wavefront-uniform, so source records
//                   come through scalar loads and feed the VALU as scalar
//                   operands.  Pairs sharing a vertex are skipped (they are in
//                   the near field).  Per-chunk partial sums are written out.
//   k_far_finish  : FP64 sum over chunks, P1 test projection on the target
//                   triangle -> 3 values per block row.
//   k_gather      : per vertex, fixed-order sum of triangle contributions,
//                   near-field CSR product, optional 2x2 preconditioner.
#include <algorithm>

#include <type_traits>

#include "far.h"

namespace pbm {

// Source weights of triangle s from the vector x (2V): b1 = w |s| u1(y_q),
// b2 = w |s| u2(y_q), C = |s| curl u1; dync, dync64 (either may be null): the
// one-point rule's source weights |s| mean(u1), |s| mean(u2) in FP32 / FP64.
__device__ __forceinline__ void source_prep_tri(int s, int V, const int32_t *__restrict__ tri,
                                                const double *__restrict__ geo, const double *__restrict__ x,
                                                double *__restrict__ dyn64, float *__restrict__ dyn32,
                                                float *__restrict__ dync, double *__restrict__ dync64)
{
    const double *g = geo + (size_t)s * kGeo;
    const double area = g[21];
    double u1[3], u2[3];
    for (int k = 0; k < 3; ++k) {
        int v = tri[3 * s + k];
        u1[k] = x[v];
        u2[k] = x[V + v];
    }
    double *d64 = dyn64 + (size_t)s * kDyn;
    float *d32 = dyn32 + (size_t)s * kDyn;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        double a = rule_bary(q, 0) * u1[0] + rule_bary(q, 1) * u1[1] + rule_bary(q, 2) * u1[2];
        double b = rule_bary(q, 0) * u2[0] + rule_bary(q, 1) * u2[1] + rule_bary(q, 2) * u2[2];
        double w = rule_w(q) * area;
        d64[q] = w * a;
        d64[6 + q] = w * b;
        d32[q] = (float)(w * a);
        d32[6 + q] = (float)(w * b);
    }
    for (int c = 0; c < 3; ++c) {
        double cu = area * (u1[0] * g[22 + c] + u1[1] * g[25 + c] + u1[2] * g[28 + c]);
        d64[12 + c] = cu;
        d32[12 + c] = (float)cu;
    }
    d64[15] = 0.0;
    d32[15] = 0.0f;
    if (dync) {
        dync[2 * (size_t)s] = (float)(area * (u1[0] + u1[1] + u1[2]) / 3.0);
        dync[2 * (size_t)s + 1] = (float)(area * (u2[0] + u2[1] + u2[2]) / 3.0);
    }
    if (dync64) {
        dync64[2 * (size_t)s] = area * (u1[0] + u1[1] + u1[2]) / 3.0;
        dync64[2 * (size_t)s + 1] = area * (u2[0] + u2[1] + u2[2]) / 3.0;
    }
}

__global__ void k_source_prep(int T, int V, const int32_t *__restrict__ tri, const double *__restrict__ geo,
                              const double *__restrict__ x, double *__restrict__ dyn64, float *__restrict__ dyn32,
                              float *__restrict__ dync, double *__restrict__ dync64, DevCtl ctl)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= T || ctl_skip(ctl)) return;
    source_prep_tri(s, V, tri, geo, x + ctl_off(ctl), dyn64, dyn32, dync, dync64);
}

void launch_source_prep(DevMesh &d, const double *x, bool)
{
    int T = d.hm.T;
    hipLaunchKernelGGL(k_source_prep, dim3((T + 255) / 256), dim3(256), 0, d.stream, T, d.hm.V, d.tri, d.geo, x,
                       d.dyn64, d.dyn32, d.far_rule != 0 ? d.dync32 : nullptr, d.far_rule == 2 ? d.dync64 : nullptr,
                       d.ctl);
    HIPCHECK(hipGetLastError());
}

constexpr int kFarBlock = 256;

// FORM 0: direct formulations (one row Laplace, the other Yukawa).  Per target
// point p accumulates (no 1/4pi)
//   a1 += kL F_L (d.n_s) b1 + vL G_L b2                (Laplace row)
//   a2 += kY F_Y (d.n_s) b1 + vY G_Y b2                (Yukawa row)
// FORM 1: second-kind, PMCHWT and combined-field formulations.
//   a1 += (cKL F_L + cKY F_Y)(d.n_s) b1 + (cVL G_L + cVY G_Y) b2
//   a2 += (cTL F_L + cTY F_Y)(d.n_t) b2 + cDY kappa^2 (n_t.n_s) G_Y b1   (cT = -a of T)
//   and the hypersingular curl part, per source triangle:
//   W  += [sum_pq w_p w_q (cDL G_L + cDY G_Y)] C_s
// FORM 3: no Laplace term (the Yukawa part of a PMCHWT matrix, a Calderon
//   preconditioner's operator): the FORM 1 sums without F_L, G_L.
// with d = x_p - y_q, G = e/r, F = e (1 + kappa r)/r^3 (e = 1 for Laplace).
// The sums of target triangle t over the sources s0..s1-1 (pairs sharing a
// vertex skipped) into o[0..15]: one lane's work, shared by k_far and the
// batched k_far_batch so that both round identically.
template <typename R, int FORM, typename IP, typename SP, typename OP>
__device__ __forceinline__ void far_lane(const FarCoef<R> &cf, IP __restrict__ tri, SP __restrict__ stat,
                                         SP __restrict__ dyn, int t, int s0, int s1, OP __restrict__ o)
{
    const SP ts = stat + (size_t)t * kStat;
    R tx[6], ty[6], tz[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) { tx[p] = ts[3 * p]; ty[p] = ts[3 * p + 1]; tz[p] = ts[3 * p + 2]; }
    const R ntx = ts[18], nty = ts[19], ntz = ts[20], ot = ts[21];
    const int v0 = tri[3 * t], v1 = tri[3 * t + 1], v2 = tri[3 * t + 2];
    R a1[6], a2[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) { a1[p] = 0; a2[p] = 0; }
    R W0 = 0, W1 = 0, W2 = 0;

    for (int s = s0; s < s1; ++s) {
        const int j0 = tri[3 * s], j1 = tri[3 * s + 1], j2 = tri[3 * s + 2];
        const bool adj = (j0 == v0) | (j0 == v1) | (j0 == v2) | (j1 == v0) | (j1 == v1) | (j1 == v2) |
                         (j2 == v0) | (j2 == v1) | (j2 == v2);
        if (adj) continue;
        far_source<R, FORM>(cf, stat + (size_t)s * kStat, dyn + (size_t)s * kDyn, tx, ty, tz, ot, ntx, nty, ntz,
                            a1, a2, W0, W1, W2);
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) { o[p] = a1[p]; o[6 + p] = a2[p]; }
    o[12] = W0; o[13] = W1; o[14] = W2; o[15] = 0;
}

template <typename R, int FORM>
__global__ __launch_bounds__(kFarBlock) void k_far(int T, int chunk, FarCoef<R> cf, const int32_t *__restrict__ tri,
                                                    const R *__restrict__ stat, const R *__restrict__ dyn,
                                                    R *__restrict__ part, DevCtl ctl)
{
    const int t = blockIdx.x * kFarBlock + threadIdx.x;
    const int s0 = blockIdx.y * chunk;
    const int s1 = min(T, s0 + chunk);
    if (t >= T || ctl_skip(ctl)) return;
    far_lane<R, FORM>(cf, tri, stat, dyn, t, s0, s1, part + ((size_t)blockIdx.y * T + t) * 16);
}

// Persistent far field over several meshes at once (requests of uneven
// size): a work queue of items {request, first target of a wavefront, source
// chunk}, heaviest first.  Each wavefront takes the next item from a device
// counter until the queue is empty (every wavefront reaches that exit), and
// computes its 64 targets over the chunk exactly as k_far does, into the
// request's own partial-sum buffer in k_far's layout.
template <typename R, int FORM>
__global__ __launch_bounds__(kFarBlock) void k_far_batch(const FarReq<R> *__restrict__ reqs,
                                                          const int4 *__restrict__ items, int nitems,
                                                          int *__restrict__ next)
{
    const int lane = threadIdx.x & 63;
    for (;;) {
        int i = 0;
        if (lane == 0) i = atomicAdd(next, 1);
        i = __builtin_amdgcn_readfirstlane(__shfl(i, 0));
        if (i >= nitems) return;
        const int4 it = items[i];
        const FarReq<R> rq = reqs[it.x];
        if (rq.skip && *rq.skip) continue;
        const int t = it.y + lane;
        const int s0 = it.z * rq.chunk;
        const int s1 = min(rq.T, s0 + rq.chunk);
        // the mesh data are not written during the launch: read through the
        // constant address space so that wavefront-uniform records come
        // through scalar loads (as in k_far) although the loop stores results
        using CI = const __attribute__((address_space(4))) int32_t *;
        using CR = const __attribute__((address_space(4))) R *;
        using GR = __attribute__((address_space(1))) R *;
        if (t < rq.T)
            far_lane<R, FORM>(rq.cf, (CI)rq.tri, (CR)rq.stat, (CR)rq.dyn, t, s0, s1,
                              (GR)(rq.part + ((size_t)it.z * rq.T + t) * 16));
    }
}

__global__ void k_set_int(int *p, int v) { *p = v; }

// One-point (centroid) rule on every triangle pair sharing no vertex, FP32:
// the relaxed far field of fast Calderon's preconditioner.  Same sums as
// k_far with the centroids c_t, c_s as the only points, source weights
// b1 = |s| mean(u1), b2 = |s| mean(u2) and unit pair weight for the curl sum;
// the per-point outputs repeat the centroid value, so k_far_finish's test
// projection with the 6-point rule yields exactly |t| / 3 per hat (the rule
// integrates the hats exactly).  One evaluation per source is too little work
// to hide per-source scalar loads, so each block stages kFarBlock source
// records (centroid, normal, weights, curl weights, vertex ids) in LDS with
// coalesced loads and every lane reads them as broadcasts.  Terms are summed in
// FP32 over runs of kCenRun sources and the runs in FP64: long FP32 sums would
// put a rounding noise of about 1e-6 into every product, the order of the
// preconditioned residual GMRES stops at.
constexpr int kCenRun = 16;
template <typename R>
struct Rec4 {
    R x, y, z, w;
};
template <typename R, int FORM>
__global__ __launch_bounds__(kFarBlock) void k_far_centroid(int T, int chunk, FarCoef<R> cf,
                                                             const int32_t *__restrict__ tri,
                                                             const R *__restrict__ stat,
                                                             const R *__restrict__ dyn,
                                                             const R *__restrict__ dync, R *__restrict__ part,
                                                             DevCtl ctl)
{
    __shared__ Rec4<R> rec[3][kFarBlock];   // (c, b1), (n, b2), (C, -)
    __shared__ int4 vid[kFarBlock];
    const int t = blockIdx.x * kFarBlock + threadIdx.x;
    const int s0 = blockIdx.y * chunk;
    const int s1 = min(T, s0 + chunk);
    if (ctl_skip(ctl)) return;   // uniform: the whole block leaves
    const int tc = t < T ? t : T - 1;   // lanes past the end compute, never store
    const R *ts = stat + (size_t)tc * kStat;
    const R cx = ts[37], cy = ts[38], cz = ts[39];
    const R ntx = ts[18], nty = ts[19], ntz = ts[20];
    const int v0 = tri[3 * tc], v1 = tri[3 * tc + 1], v2 = tri[3 * tc + 2];
    double A1 = 0, A2 = 0, X0 = 0, X1 = 0, X2 = 0;
    for (int sb = s0; sb < s1; sb += kFarBlock) {
        const int ns = min(kFarBlock, s1 - sb);
        __syncthreads();   // the previous tile is consumed
        if ((int)threadIdx.x < ns) {
            const int s = sb + threadIdx.x;
            const R *st = stat + (size_t)s * kStat;
            const R *sd = dyn + (size_t)s * kDyn;
            rec[0][threadIdx.x] = Rec4<R>{st[37], st[38], st[39], dync[2 * (size_t)s]};
            rec[1][threadIdx.x] = Rec4<R>{st[18], st[19], st[20], dync[2 * (size_t)s + 1]};
            rec[2][threadIdx.x] = Rec4<R>{sd[12], sd[13], sd[14], R(0)};
            vid[threadIdx.x] = make_int4(tri[3 * s], tri[3 * s + 1], tri[3 * s + 2], 0);
        }
        __syncthreads();
        for (int r0 = 0; r0 < ns; r0 += kCenRun) {
            R a1 = 0, a2 = 0, W0 = 0, W1 = 0, W2 = 0;
            for (int k = r0; k < min(ns, r0 + kCenRun); ++k) {
                const int4 j = vid[k];
                const bool adj = (j.x == v0) | (j.x == v1) | (j.x == v2) | (j.y == v0) | (j.y == v1) |
                                 (j.y == v2) | (j.z == v0) | (j.z == v1) | (j.z == v2);
                if (adj) continue;
                const Rec4<R> c = rec[0][k], n = rec[1][k];
                const R b1 = c.w, b2 = n.w;
                const R dx = cx - c.x, dy = cy - c.y, dz = cz - c.z;
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R ri = rsqrt_r(r2);
                const R r = r2 * ri;
                const R e = expneg(cf.kexp, r);
                const R ri3 = ri * ri * ri;
                const R dns = dx * n.x + dy * n.y + dz * n.z;
                const R tt = cf.kappa * r + R(1);
                if (FORM == 0) {
                    a1 += ri3 * dns * cf.kL * b1 + ri * cf.vL * b2;
                    a2 += e * (ri3 * tt * dns * cf.kY * b1 + ri * cf.vY * b2);
                } else {
                    const R fy = e * tt * ri3, gy = e * ri;
                    const R dnt = dx * ntx + dy * nty + dz * ntz;
                    const R k2nn = cf.cDY * cf.k2 * (ntx * n.x + nty * n.y + ntz * n.z);
                    const R fk = FORM == 3 ? cf.cKY * fy : cf.cKL * ri3 + cf.cKY * fy;
                    const R fv = FORM == 3 ? cf.cVY * gy : cf.cVL * ri + cf.cVY * gy;
                    const R ft = FORM == 3 ? cf.cTY * fy : cf.cTL * ri3 + cf.cTY * fy;
                    a1 += fk * dns * b1 + fv * b2;
                    a2 += ft * dnt * b2 + k2nn * gy * b1;
                    const R g = FORM == 3 ? cf.cDY * gy : cf.cDL * ri + cf.cDY * gy;
                    const Rec4<R> C = rec[2][k];
                    W0 += g * C.x;
                    W1 += g * C.y;
                    W2 += g * C.z;
                }
            }
            A1 += a1;
            A2 += a2;
            X0 += W0;
            X1 += W1;
            X2 += W2;
        }
    }
    if (t >= T) return;
    R *o = part + ((size_t)blockIdx.y * T + t) * 16;
#pragma unroll
    for (int p = 0; p < 6; ++p) { o[p] = (R)A1; o[6 + p] = (R)A2; }
    o[12] = (R)X0; o[13] = (R)X1; o[14] = (R)X2; o[15] = 0;
}

template <typename R>
__global__ __launch_bounds__(256) void k_far_finish(int T, int S, int family, int swap,
                                                    const double *__restrict__ geo, const R *__restrict__ part,
                                                    double *__restrict__ triout, DevCtl ctl)
{
    if (ctl_skip(ctl)) return;
    const int t = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kFinishLanes);
    const int l = threadIdx.x % kFinishLanes;
    finish_group<R>(t, l, t < T, T, S, family, swap, geo, part, triout);   // the whole lane group agrees on t < T
}

// Row i of the product, lane c of its kRowLanes group (every lane of the group
// calls it): near-field CSR product, the far field (1: per-triangle outputs
// through the vertex's incidence list, 2: a dense product's rows in dense
// vertex order), optional 2x2 preconditioner; x, y already offset.
__device__ __forceinline__ void gather_row(int i, int c, int V, int use_far, int use_near, int precond,
                                           const int32_t *__restrict__ inc_ptr, const int32_t *__restrict__ inc_tk,
                                           const double *__restrict__ triout, const double *__restrict__ yfar,
                                           const int32_t *__restrict__ vpos, const int32_t *__restrict__ row_ptr,
                                           const int32_t *__restrict__ col, const double *__restrict__ N,
                                           int64_t nnz, const double *__restrict__ pinv,
                                           const double *__restrict__ x, double *__restrict__ y)
{
    double n1 = 0.0, n2 = 0.0;
    if (use_near) {
        for (int sl = row_ptr[i] + c; sl < row_ptr[i + 1]; sl += kRowLanes) {
            const int j = col[sl];
            const double x1 = x[j], x2 = x[V + j];
            n1 += N[sl] * x1 + N[nnz + sl] * x2;
            n2 += N[2 * nnz + sl] * x1 + N[3 * nnz + sl] * x2;
        }
#pragma unroll
        for (int off = 1; off < kRowLanes; off <<= 1) {
            n1 += __shfl_xor(n1, off);
            n2 += __shfl_xor(n2, off);
        }
    }
    if (c != 0) return;
    double y1 = 0.0, y2 = 0.0;
    if (use_far == 2) {   // dense far product, rows in dense vertex order
        const int r = vpos[i];
        y1 = yfar[r];
        y2 = yfar[V + r];
    } else if (use_far == 1) {
        for (int e = inc_ptr[i]; e < inc_ptr[i + 1]; ++e) {
            const int tk = inc_tk[e];
            const int t = tk >> 2, k = tk & 3;
            y1 += triout[6 * (size_t)t + k];
            y2 += triout[6 * (size_t)t + 3 + k];
        }
    }
    if (use_near) {
        y1 += n1;
        y2 += n2;
    }
    if (precond) {
        const double *P = pinv + 4 * (size_t)i;
        const double z1 = P[0] * y1 + P[1] * y2, z2 = P[2] * y1 + P[3] * y2;
        y1 = z1;
        y2 = z2;
    }
    y[i] = y1;
    y[V + i] = y2;
}

// flags: PB_APPLY_PRECOND, PB_APPLY_NEAR_ONLY, PB_APPLY_FAR_ONLY (near part skipped)
__global__ void k_gather(int V, int use_far, int use_near, int precond, const int32_t *__restrict__ inc_ptr,
                         const int32_t *__restrict__ inc_tk, const double *__restrict__ triout,
                         const double *__restrict__ yfar, const int32_t *__restrict__ vpos,
                         const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                         const double *__restrict__ N, int64_t nnz, const double *__restrict__ pinv,
                         const double *__restrict__ x, double *__restrict__ y, DevCtl ctl, DevCtl ctly)
{
    // kRowLanes lanes per row; the lane group sits inside one wavefront, so a
    // whole group is either active or retired together
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes;
    const int c = threadIdx.x % kRowLanes;
    if (i >= V || ctl_skip(ctl)) return;
    gather_row(i, c, V, use_far, use_near, precond, inc_ptr, inc_tk, triout, yfar, vpos, row_ptr, col, N, nnz,
               pinv, x + ctl_off(ctl), y + ctl_off(ctly));
}

// ------------------------- batched steps of a captured lockstep iteration
// One launch per step for every solve of the batch (TailReq per solve, block
// ranges boff per solve as in the batched Krylov steps); each block runs the
// single kernel's code for its solve, so the results are bitwise the same.
__device__ __forceinline__ int tail_owner(const int *__restrict__ boff, int R, int b)
{
    int lo = 0, hi = R - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_bsource_prep(int R, const TailReq *__restrict__ rq, const int *__restrict__ boff)
{
    const int r = tail_owner(boff, R, blockIdx.x);
    const TailReq &q = rq[r];
    const int s = (blockIdx.x - boff[r]) * blockDim.x + threadIdx.x;
    if (s >= q.T || ctl_skip(q.ctl)) return;
    source_prep_tri(s, q.V, q.tri, q.geo, q.x + ctl_off(q.ctl), q.dyn64, q.dyn32, nullptr, nullptr);
}

template <typename R>
__global__ __launch_bounds__(256) void k_bfinish(int NR, const TailReq *__restrict__ rq, const int *__restrict__ boff)
{
    const int r = tail_owner(boff, NR, blockIdx.x);
    const TailReq &q = rq[r];
    if (ctl_skip(q.ctl)) return;   // uniform: the block belongs to one solve
    const int t = (int)(((blockIdx.x - boff[r]) * (size_t)blockDim.x + threadIdx.x) / kFinishLanes);
    const int l = threadIdx.x % kFinishLanes;
    if (sizeof(R) == 4 && q.nr > 0)
        sym_finish_group(t, l, t < q.T, q.T, q.rt, q.nr, q.family, q.swap, q.geo, (const float *)q.part, q.triout);
    else
        finish_group<R>(t, l, t < q.T, q.T, q.S, q.family, q.swap, q.geo, (const R *)q.part, q.triout);
}

__global__ void k_bgather(int R, const TailReq *__restrict__ rq, const int *__restrict__ boff)
{
    const int r = tail_owner(boff, R, blockIdx.x);
    const TailReq &q = rq[r];
    const int i = ((blockIdx.x - boff[r]) * blockDim.x + threadIdx.x) / kRowLanes;
    const int c = threadIdx.x % kRowLanes;
    if (i >= q.V || ctl_skip(q.ctl)) return;
    const size_t off = ctl_off(q.ctl);
    gather_row(i, c, q.V, 1, 1, q.precond, q.inc_ptr, q.inc_tk, q.triout, nullptr, nullptr, q.row_ptr, q.col, q.N,
               q.nnz, q.pinv, q.x + off, q.gout + (q.gout_offset ? off : 0));
}

int tail_blocks_source(const TailReq &q) { return (q.T + 255) / 256; }
int tail_blocks_finish(const TailReq &q) { return (int)(((size_t)q.T * kFinishLanes + 255) / 256); }
int tail_blocks_gather(const TailReq &q) { return (q.V + 256 / kRowLanes - 1) / (256 / kRowLanes); }

void launch_batch_source_prep(hipStream_t s, int R, const TailReq *rq, const int *boff, int nblocks)
{
    if (nblocks < 1) return;
    hipLaunchKernelGGL(k_bsource_prep, dim3(nblocks), dim3(256), 0, s, R, rq, boff);
    HIPCHECK(hipGetLastError());
}

void launch_batch_finish(hipStream_t s, bool fp32, int R, const TailReq *rq, const int *boff, int nblocks)
{
    if (nblocks < 1) return;
    if (fp32) hipLaunchKernelGGL(k_bfinish<float>, dim3(nblocks), dim3(256), 0, s, R, rq, boff);
    else hipLaunchKernelGGL(k_bfinish<double>, dim3(nblocks), dim3(256), 0, s, R, rq, boff);
    HIPCHECK(hipGetLastError());
}

void launch_batch_gather(hipStream_t s, int R, const TailReq *rq, const int *boff, int nblocks)
{
    if (nblocks < 1) return;
    hipLaunchKernelGGL(k_bgather, dim3(nblocks), dim3(256), 0, s, R, rq, boff);
    HIPCHECK(hipGetLastError());
}

int choose_chunks(int T)
{
    // about 64 wavefronts per SIMD on 256 CUs x 4 SIMDs, at most 128 chunks of
    // at least 32 triangles: with 4 per SIMD (13 chunks at 20480 triangles) the
    // kernel kept 2.2 wavefronts resident and the VALU 79% busy; 104 chunks
    // took 20% less time there, 52 chunks 5% less at 81920 triangles
    const int waves = (T + 63) / 64;
    int S = (65536 + waves - 1) / waves;
    S = std::max(1, std::min(S, 128));
    while (S > 1 && (T + S - 1) / S < 32) --S;
    return S;
}

template <typename R>
static void far_launch(DevMesh &d, const R *stat, const R *dyn)
{
    if (sizeof(R) == 4 && d.sym_nitems > 0) {
        launch_far_sym(d);   // FP32, every unordered pair once (k_far_sym.hip)
        return;
    }
    const int T = d.hm.T, S = d.S;
    const int chunk = (T + S - 1) / S;
    FarCoef<R> cf;
    const int form = far_coef(d, cf);
    dim3 grid((T + kFarBlock - 1) / kFarBlock, S), block(kFarBlock);
    R *part = (R *)d.part;
    if (form == 0)
        hipLaunchKernelGGL((k_far<R, 0>), grid, block, 0, d.stream, T, chunk, cf, d.tri, stat, dyn, part, d.ctl);
    else if (form == 1)
        hipLaunchKernelGGL((k_far<R, 1>), grid, block, 0, d.stream, T, chunk, cf, d.tri, stat, dyn, part, d.ctl);
    else
        hipLaunchKernelGGL((k_far<R, 3>), grid, block, 0, d.stream, T, chunk, cf, d.tri, stat, dyn, part, d.ctl);
    HIPCHECK(hipGetLastError());
}

void launch_far(DevMesh &d, bool fp32)
{
    Profiler &pf = d.prof;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (pf.on(0)) {
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        HIPCHECK(hipEventRecord(e0, d.stream));
    }
    if (fp32) far_launch<float>(d, d.stat32, d.dyn32);
    else far_launch<double>(d, d.stat64, d.dyn64);
    if (pf.on(0)) {
        HIPCHECK(hipEventRecord(e1, d.stream));
        const double P = 6.0 * d.hm.T;
        pf.record(0, e0, e1, P * P);   // kernel pairs, near-masked pairs included
    }
}

// One queue per kernel form over the requests in `live` (indices into ds);
// items of a request follow its own source split (d.S chunks), so
// k_far_finish applies unchanged.
template <typename R, int FORM>
static int batch_blocks(int n)
{
    int dev = 0, ncu = 0, per_cu = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(&k_far_batch<R, FORM>), kFarBlock, 0));
    const int waves = kFarBlock / 64;
    return (int)std::max(1LL, std::min((long long)(n + waves - 1) / waves,
                                       (long long)std::max(ncu, 1) * std::max(per_cu, 1)));
}

template <typename R>
static void batch_plan(const std::vector<DevMesh *> &ds, const std::vector<int> &live,
                       const std::vector<const int *> &skip, FarBatch &fb)
{
    for (int f = 0; f < 4; ++f) fb.nitems[f] = 0;
    std::vector<FarReq<R>> reqs(ds.size());
    std::vector<std::vector<std::pair<int, int4>>> q(4);   // (cost, item) per form
    // symmetric items per form 0, 1, 3 (kappa > 0), then per form with kappa = 0
    std::vector<std::vector<std::pair<int, int4>>> sq(6);
    for (int r : live) {
        DevMesh &d = *ds[r];
        FarReq<R> &rq = reqs[r];
        const int form = far_coef(d, rq.cf);
        const int T = d.hm.T, S = d.S, chunk = (T + S - 1) / S;
        rq.tri = d.tri;
        rq.stat = sizeof(R) == 4 ? (const R *)d.stat32 : (const R *)d.stat64;
        rq.dyn = sizeof(R) == 4 ? (const R *)d.dyn32 : (const R *)d.dyn64;
        rq.part = (R *)d.part;
        rq.skip = skip.empty() ? nullptr : skip[r];
        rq.T = T;
        rq.chunk = chunk;
        rq.rt = rq.nr = 0;
        if (sizeof(R) == 4 && d.sym_nitems > 0) {
            // symmetric split: the request's range pairs, in its own (heaviest first)
            // order, with the split's scaled coefficients
            if constexpr (std::is_same<R, float>::value) far_coef_sym(d, rq.cf);
            rq.rt = d.sym_rt;
            rq.nr = d.sym_nr;
            std::vector<int2> its;
            int rt = 0, nr = 0;
            sym_plan(T, rt, nr, its);
            const int sf = (form == 0 ? 0 : form == 1 ? 1 : 2) + (d.prm.kappa > 0.0 ? 0 : 3);
            for (const int2 &e : its) {
                const int na = std::min((T + 63) / 64, (e.x + 1) * rt) - e.x * rt;
                const int nb = std::min((T + 63) / 64, (e.y + 1) * rt) - e.y * rt;
                sq[sf].push_back({e.x == e.y ? na * (na + 1) / 2 : na * nb, make_int4(r, e.x, e.y, 0)});
            }
            continue;
        }
        // every chunk, empty ones too: k_far_finish sums all S of them
        for (int c = 0; c < S; ++c) {
            const int len = std::max(0, std::min(T, (c + 1) * chunk) - c * chunk);
            for (int t0 = 0; t0 < T; t0 += 64) q[form].push_back({len, make_int4(r, t0, c, 0)});
        }
    }
    std::vector<int4> items, sitems;
    for (int f = 0; f < 4; ++f) {
        std::stable_sort(q[f].begin(), q[f].end(),
                         [](const std::pair<int, int4> &a, const std::pair<int, int4> &b) { return a.first > b.first; });
        fb.first[f] = (int)items.size();
        for (auto &e : q[f]) items.push_back(e.second);
        fb.nitems[f] = (int)q[f].size();
    }
    for (int f = 0; f < 6; ++f) {
        std::stable_sort(sq[f].begin(), sq[f].end(),
                         [](const std::pair<int, int4> &a, const std::pair<int, int4> &b) { return a.first > b.first; });
        fb.sym_first[f] = (int)sitems.size();
        for (auto &e : sq[f]) sitems.push_back(e.second);
        fb.sym_n[f] = (int)sq[f].size();
        const int kf = f % 3 == 0 ? 0 : f % 3 == 1 ? 1 : 3;
        fb.sym_nblocks[f] = fb.sym_n[f] ? sym_batch_blocks_for(kf, f >= 3, fb.sym_n[f]) : 0;
    }
    const size_t sb = sizeof(int4) * std::max<size_t>(sitems.size(), 1);
    if (sb > fb.sym_cap) {
        if (fb.sym_items) HIPCHECK(hipFree(fb.sym_items));
        HIPCHECK(hipMalloc(&fb.sym_items, sb));
        fb.sym_cap = sb;
    }
    if (!sitems.empty())
        HIPCHECK(hipMemcpyAsync(fb.sym_items, sitems.data(), sizeof(int4) * sitems.size(), hipMemcpyHostToDevice,
                                fb.stream));
    fb.nblocks[0] = fb.nitems[0] ? batch_blocks<R, 0>(fb.nitems[0]) : 0;
    fb.nblocks[1] = fb.nitems[1] ? batch_blocks<R, 1>(fb.nitems[1]) : 0;
    fb.nblocks[2] = 0;   // kernel forms 0, 1 and 3 only
    fb.nblocks[3] = fb.nitems[3] ? batch_blocks<R, 3>(fb.nitems[3]) : 0;
    const size_t rb = sizeof(FarReq<R>) * reqs.size(), ib = sizeof(int4) * std::max<size_t>(items.size(), 1);
    if (rb > fb.req_cap) {
        if (fb.reqs) HIPCHECK(hipFree(fb.reqs));
        HIPCHECK(hipMalloc(&fb.reqs, rb));
        fb.req_cap = rb;
    }
    if (ib > fb.item_cap) {
        if (fb.items) HIPCHECK(hipFree(fb.items));
        HIPCHECK(hipMalloc(&fb.items, ib));
        fb.item_cap = ib;
    }
    if (!fb.next) HIPCHECK(hipMalloc(&fb.next, 10 * sizeof(int)));
    HIPCHECK(hipMemcpyAsync(fb.reqs, reqs.data(), rb, hipMemcpyHostToDevice, fb.stream));
    if (!items.empty())
        HIPCHECK(hipMemcpyAsync(fb.items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice,
                                fb.stream));
    HIPCHECK(hipStreamSynchronize(fb.stream));   // host vectors go out of scope
}

// launch only (no host query or synchronisation), so it can be captured
template <typename R, int FORM>
static void batch_launch(FarBatch &fb)
{
    const int n = fb.nitems[FORM];
    if (n == 0) return;
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, fb.stream, fb.next + FORM, 0);
    hipLaunchKernelGGL((k_far_batch<R, FORM>), dim3((unsigned)fb.nblocks[FORM]), dim3(kFarBlock), 0, fb.stream,
                       (const FarReq<R> *)fb.reqs, (const int4 *)fb.items + fb.first[FORM], n, fb.next + FORM);
    HIPCHECK(hipGetLastError());
}

void far_batch_plan(const std::vector<DevMesh *> &ds, const std::vector<int> &live, bool fp32, FarBatch &fb,
                    const std::vector<const int *> &skip)
{
    if (fp32) batch_plan<float>(ds, live, skip, fb);
    else batch_plan<double>(ds, live, skip, fb);
}

void launch_far_batch(FarBatch &fb, bool fp32)
{
    if (fp32) {
        batch_launch<float, 0>(fb); batch_launch<float, 1>(fb); batch_launch<float, 3>(fb);
        const int forms[3] = {0, 1, 3};
        for (int f = 0; f < 6; ++f)
            launch_far_sym_batch(forms[f % 3], f >= 3, fb.reqs, (const int4 *)fb.sym_items + fb.sym_first[f],
                                 fb.sym_n[f], fb.sym_nblocks[f], fb.next + 4 + f, fb.stream);
    } else {
        batch_launch<double, 0>(fb); batch_launch<double, 1>(fb); batch_launch<double, 3>(fb);
    }
}

void far_batch_free(FarBatch &fb)
{
    if (fb.reqs) (void)hipFree(fb.reqs);
    if (fb.items) (void)hipFree(fb.items);
    if (fb.sym_items) (void)hipFree(fb.sym_items);
    if (fb.next) (void)hipFree(fb.next);
    fb.reqs = nullptr;
    fb.items = nullptr;
    fb.sym_items = nullptr;
    fb.next = nullptr;
    fb.req_cap = fb.item_cap = fb.sym_cap = 0;
}

template <typename R>
static void centroid_launch(DevMesh &d, const R *stat, const R *dyn, const R *dync)
{
    const int T = d.hm.T, S = d.S;
    const int chunk = (T + S - 1) / S;
    FarCoef<R> cf;
    const int form = far_coef(d, cf);
    const dim3 grid((T + kFarBlock - 1) / kFarBlock, S), block(kFarBlock);
    R *part = (R *)d.part;
#define FAR_C(F)                                                                                                \
    hipLaunchKernelGGL((k_far_centroid<R, F>), grid, block, 0, d.stream, T, chunk, cf, d.tri, stat, dyn, dync, \
                       part, d.ctl)
    if (form == 0) FAR_C(0);
    else if (form == 1) FAR_C(1);
    else FAR_C(3);
#undef FAR_C
    HIPCHECK(hipGetLastError());
}

void launch_far_centroid(DevMesh &d, bool fp32)
{
    if (fp32) centroid_launch<float>(d, d.stat32, d.dyn32, d.dync32);
    else centroid_launch<double>(d, d.stat64, d.dyn64, d.dync64);
}

void launch_far_finish(DevMesh &d, bool fp32)
{
    if (fp32 && d.sym_nitems > 0 && d.far_rule == 0 && !d.tree) {
        launch_far_sym_finish(d);   // the symmetric far field's slots
        return;
    }
    const int T = d.hm.T;
    dim3 grid((unsigned)(((size_t)T * kFinishLanes + 255) / 256)), block(256);
    const FormCoef &f = d.fm;
    const int swap = f.family == 0 && laplace_row(f) == 1;
    if (fp32)
        hipLaunchKernelGGL(k_far_finish<float>, grid, block, 0, d.stream, T, d.S, f.family, swap, d.geo,
                           (const float *)d.part, d.triout, d.ctl);
    else
        hipLaunchKernelGGL(k_far_finish<double>, grid, block, 0, d.stream, T, d.S, f.family, swap, d.geo,
                           (const double *)d.part, d.triout, d.ctl);
    HIPCHECK(hipGetLastError());
}

void launch_gather(DevMesh &d, const double *x, double *y, int flags, int use_far, bool y_offset)
{
    const int V = d.hm.V;
    const int use_near = (flags & PB_APPLY_FAR_ONLY) ? 0 : 1;
    DevCtl ctly = d.ctl;
    if (!y_offset) ctly.stride = 0;
    hipLaunchKernelGGL(k_gather, dim3((V + 256 / kRowLanes - 1) / (256 / kRowLanes)), dim3(256), 0, d.stream, V,
                       use_far, use_near,
                       (flags & PB_APPLY_PRECOND) ? 1 : 0, d.inc_ptr, d.inc_tk, d.triout, d.yfar, d.dense_vpos, d.row_ptr, d.col, d.N,
                       d.nnz(), d.pinv, x, y, d.ctl, ctly);
    HIPCHECK(hipGetLastError());
}

}  // namespace pbm
