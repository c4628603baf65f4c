// Far field, matrix-free, FP32, with every unordered triangle pair evaluated
// once (the kernel values G(x, y) = G(y, x) and the kernel factors of the
// four operators serve both (target t <- source s) and (s <- t); Numerical
// discretization: regular quadrature of the pairs sharing no vertex).
//
// Work: tiles of 64 Morton-consecutive triangles, tile ranges of `rt` tiles;
// an item (a, b), a <= b, is the pairs of triangles of range a x range b
// (I <= J when a == b) and is done by one wavefront.  For a tile pair (I, J)
// lane l holds target t = 64 I + l; in step k = 0..63 it meets source
// s = 64 J + ((l + k) mod 64) (on a diagonal tile I == J only the steps and
// lanes that meet each unordered pair once: 1 <= k <= 31, and k = 32 on the
// lower half of the lanes).  Its target's sums (a1, a2, W) stay in the lane;
// the sums of the source side -- the transposed pair -- are held by the lane
// that meets that source and move one lane down after every step, so after
// 64 steps each source's sums are back in lane (s mod 64): no cross-lane
// reduction is needed.  Tile J's source records are staged once per wavefront
// in LDS (one array per field, so the lanes' rotated reads hit distinct
// banks).
//
// Coordinates (points and the plane offsets) are used scaled by s = kappa
// log2(e), with the coefficients of far_coef_sym: then exp(-kappa r) =
// exp2(-r') with r' = r2' / sqrt(r2') and no multiply for the argument.
// Unscreened meshes (kappa = 0, K0) keep their coordinates and skip the
// exponential: e = 1, so the Yukawa kernels are the Laplace ones.
//
// The quadrature points of a flat triangle lie in its plane, so the normal
// components of d = x_p - y_q factor: d . n_s = x_p . n_s - o_s depends on the
// target point only and d . n_t = o_t - y_q . n_t on the source point only
// (o = the triangle's plane offset, y . n for any of its points).  Both are
// formed once per triangle pair, not per point pair.
//
// Output: per triangle, one 16-value partial (6 + 6 point sums, 3 curl sums)
// per target-side item (slot b, the source range) and one per source-side
// item (slot nr + a, the target range): every slot is written by exactly one
// item, so no atomics and a fixed summation order.  k_far_sym_finish adds a
// triangle's nr + 1 slots in FP64 and projects them as k_far_finish does.
#include <algorithm>

#include "far.h"

namespace pbm {

constexpr int kSymWaves = 2;   // independent wavefronts (items) per block
// staged source record, one LDS array per field: 0..17 points, 18..20 normal,
// 21 plane offset o_s, then per source point
//   FORM 0: 22..27 kL b1, 28..33 vL b2, 34..39 kY b1, 40..45 vY b2 (the
//           source-point constants of the direct form's target-side sums);
//   else:   22..27 b1, 28..33 b2, 34..36 C.
template <int FORM> struct SymLds {
    static constexpr int NF = FORM == 0 ? 46 : 37;
    float f[NF][64];
    int id[3][64];
};

// one step: the 36 point pairs of target t (lane registers) and source j
// (LDS column j); adds t's sums to a1, a2, W and the source's sums to acc
template <int FORM, bool K0>
__device__ __forceinline__ void sym_pair(const FarCoef<float> &cf, const SymLds<FORM> &L, int j, const float (&tx)[6],
                                         const float (&ty)[6], const float (&tz)[6], float ot, float ntx,
                                         float nty, float ntz, const float (&cs)[9][6], const float (&Ct)[3],
                                         float (&a1)[6], float (&a2)[6], float (&W)[3], float (&acc)[15])
{
    const float nsx = L.f[18][j], nsy = L.f[19][j], nsz = L.f[20][j], os = L.f[21][j];
    // dns[p] = (x_p - y) . n_s, dnt[q] = (x - y_q) . n_t
    float dns[6], dnt[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) dns[p] = fmaf(tx[p], nsx, fmaf(ty[p], nsy, fmaf(tz[p], nsz, -os)));
#pragma unroll
    for (int q = 0; q < 6; ++q)
        dnt[q] = fmaf(-L.f[3 * q][j], ntx, fmaf(-L.f[3 * q + 1][j], nty, fmaf(-L.f[3 * q + 2][j], ntz, ot)));
    float gL = 0.0f, gY = 0.0f, nn = 0.0f;
    float P[6];   // FORM 1, 3: target p's row-1 double-layer sum before its factor dns[p]
#pragma unroll
    for (int p = 0; p < 6; ++p) P[p] = 0.0f;
    if (FORM >= 1) nn = cf.cDY * cf.k2 * (ntx * nsx + nty * nsy + ntz * nsz);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const float yx = L.f[3 * q][j], yy = L.f[3 * q + 1][j], yz = L.f[3 * q + 2][j];
        if (FORM == 0) {
            // target side: Laplace row kL K_L + vL V_L, Yukawa row kY K_Y + vY V_Y, the
            // source point's constants c1..c4 staged (kYk = kappa kY); source side (K at
            // the target's normal: -F d.n_t): cs = -kL b1_t, vL b2_t, -kY b1_t, vY b2_t,
            // -kY kappa b1_t per target point
            const float c1 = L.f[22 + q][j], c2 = L.f[28 + q][j], c3 = L.f[34 + q][j], c4 = L.f[40 + q][j];
            const float c3k = cf.kappa * c3;   // kYk = kappa kY (unused when K0)
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const float dx = tx[p] - yx, dy = ty[p] - yy, dz = tz[p] - yz;
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float ri = rsqrt_r(r2);
                const float ri2 = ri * ri;
                const float g = dns[p] * ri2, h = dnt[q] * ri2;
                a1[p] = fmaf(ri, fmaf(c1, g, c2), a1[p]);
                acc[q] = fmaf(ri, fmaf(cs[0][p], h, cs[1][p]), acc[q]);
                if constexpr (K0) {
                    a2[p] = fmaf(ri, fmaf(c3, g, c4), a2[p]);
                    acc[6 + q] = fmaf(ri, fmaf(cs[2][p], h, cs[3][p]), acc[6 + q]);
                } else {
                    const float e = __builtin_amdgcn_exp2f(-(r2 * ri));
                    a2[p] = fmaf(e, fmaf(ri, fmaf(c3, g, c4), c3k * g), a2[p]);
                    acc[6 + q] = fmaf(e, fmaf(ri, fmaf(cs[2][p], h, cs[3][p]), cs[4][p] * h), acc[6 + q]);
                }
            }
        } else {
            // target side as far_source; source side: row 1 with -h (K at n_t), row 2
            // with -g (T at n_s): cs = -cKL b1_t, -cKY b1_t, (unused), cVL b2_t,
            // cVY b2_t, -cTL b2_t, -cTY b2_t, (unused), b1_t.  The Yukawa double-layer
            // kernel e (1 + kappa r) / r^3 d.n is E d.n with E = e (r^-3 + kappa r^-2).
            const float b1 = L.f[22 + q][j], b2 = L.f[28 + q][j];
            const float c1L = cf.cKL * b1, c1Y = cf.cKY * b1, c2L = cf.cVL * b2, c2Y = cf.cVY * b2;
            const float c3L = cf.cTL * b2, c3Y = cf.cTY * b2, kb1 = nn * b1;
            float S = 0.0f;   // source q's row-1 double-layer sum before its factor dnt[q]
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const float dx = tx[p] - yx, dy = ty[p] - yy, dz = tz[p] - yz;
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float ri = rsqrt_r(r2);
                const float ri2 = ri * ri;
                const float e = K0 ? 1.0f : __builtin_amdgcn_exp2f(-(r2 * ri));
                const float gy = K0 ? ri : e * ri;
                // F_L d.n = R3 (d.n), F_Y d.n = E (d.n) with R3 = r^-3 and E = e (1/r + kappa)
                // r^-2 = e (R3 + kappa r^-2); the factors dns[p] of target p's row 1 and
                // dnt[q] of source q's row 1 are applied once per triangle pair (P, S)
                const float R3 = ri * ri2;
                const float E = K0 ? R3 : e * fmaf(cf.kappa, ri2, R3);
                if (FORM == 3) {
                    P[p] = fmaf(c1Y, E, P[p]);
                    a1[p] = fmaf(gy, c2Y, a1[p]);
                    a2[p] = fmaf(dnt[q] * c3Y, E, fmaf(gy, kb1, a2[p]));
                    S = fmaf(cs[1][p], E, S);
                    acc[q] = fmaf(gy, cs[4][p], acc[q]);
                    acc[6 + q] = fmaf(dns[p] * cs[6][p], E, fmaf(gy, nn * cs[8][p], acc[6 + q]));
                } else {
                    P[p] = fmaf(c1Y, E, fmaf(c1L, R3, P[p]));
                    a1[p] = fmaf(ri, c2L, fmaf(gy, c2Y, a1[p]));
                    a2[p] = fmaf(dnt[q], fmaf(c3Y, E, c3L * R3), fmaf(gy, kb1, a2[p]));
                    S = fmaf(cs[1][p], E, fmaf(cs[0][p], R3, S));
                    acc[q] = fmaf(ri, cs[3][p], fmaf(gy, cs[4][p], acc[q]));
                    acc[6 + q] = fmaf(dns[p], fmaf(cs[6][p], E, cs[5][p] * R3), fmaf(gy, nn * cs[8][p], acc[6 + q]));
                    gL = fmaf(float(rule_w(p) * rule_w(q)), ri, gL);
                }
                gY = fmaf(float(rule_w(p) * rule_w(q)), gy, gY);
            }
            acc[q] = fmaf(dnt[q], S, acc[q]);
        }
    }
    if (FORM >= 1) {
#pragma unroll
        for (int p = 0; p < 6; ++p) a1[p] = fmaf(dns[p], P[p], a1[p]);
    }
    if (FORM >= 1) {
        const float gc = FORM == 3 ? cf.cDY * gY : cf.cDL * gL + cf.cDY * gY;
        W[0] = fmaf(gc, L.f[34][j], W[0]);
        W[1] = fmaf(gc, L.f[35][j], W[1]);
        W[2] = fmaf(gc, L.f[36][j], W[2]);
        acc[12] = fmaf(gc, Ct[0], acc[12]);
        acc[13] = fmaf(gc, Ct[1], acc[13]);
        acc[14] = fmaf(gc, Ct[2], acc[14]);
    }
}

// Item (a, b) of one mesh by one wavefront; part holds the 2 nr slots
template <int FORM, bool K0, typename IP, typename RP>
__device__ __forceinline__ void sym_item(const FarCoef<float> &cf, IP __restrict__ tri, RP __restrict__ stat,
                                         RP __restrict__ dyn, int T, int rt, int nr, int a, int b,
                                         float *__restrict__ part, SymLds<FORM> &L, int lane)
{
    const int ntile = (T + 63) / 64;
    const int I0 = a * rt, I1 = min(ntile, I0 + rt);
    const int J0 = b * rt, J1 = min(ntile, J0 + rt);
    constexpr int NA = FORM == 0 ? 12 : 15;
    for (int J = J0; J < J1; ++J) {
        // stage tile J's sources (past the end: vertex ids -1, never met)
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        {
            const int s = 64 * J + lane;
            if (s < T) {
                const auto st = stat + (size_t)s * kStat;
                const auto sd = dyn + (size_t)s * kDyn;
                // points and the plane offset (its first point's y . n) scaled by s,
                // the normal as it is
#pragma unroll
                for (int c = 0; c < 22; ++c) L.f[c][lane] = (c < 18 || c == 21) ? st[c] * cf.kexp : st[c];
                if (FORM == 0) {
#pragma unroll
                    for (int q = 0; q < 6; ++q) {
                        L.f[22 + q][lane] = cf.kL * sd[q];
                        L.f[28 + q][lane] = cf.vL * sd[6 + q];
                        L.f[34 + q][lane] = cf.kY * sd[q];
                        L.f[40 + q][lane] = cf.vY * sd[6 + q];
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 15; ++c) L.f[22 + c][lane] = sd[c];
                }
                L.id[0][lane] = tri[3 * s];
                L.id[1][lane] = tri[3 * s + 1];
                L.id[2][lane] = tri[3 * s + 2];
            } else {
#pragma unroll
                for (int c = 0; c < SymLds<FORM>::NF; ++c) L.f[c][lane] = 0.0f;
                L.id[0][lane] = L.id[1][lane] = L.id[2][lane] = -1;
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        float acc[15];
#pragma unroll
        for (int v = 0; v < 15; ++v) acc[v] = 0.0f;
        const int Iend = (a == b) ? J + 1 : I1;
        for (int I = I0; I < Iend; ++I) {
            const int t = 64 * I + lane;
            const bool tv = t < T;
            const int tc = tv ? t : T - 1;
            const auto ts = stat + (size_t)tc * kStat;
            const auto td = dyn + (size_t)tc * kDyn;
            float tx[6], ty[6], tz[6];
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                tx[p] = ts[3 * p] * cf.kexp; ty[p] = ts[3 * p + 1] * cf.kexp; tz[p] = ts[3 * p + 2] * cf.kexp;
            }
            const float ot = ts[21] * cf.kexp;   // the target's plane offset
            const float ntx = ts[18], nty = ts[19], ntz = ts[20];
            const int v0 = tri[3 * tc], v1 = tri[3 * tc + 1], v2 = tri[3 * tc + 2];
            float cs[9][6], Ct[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const float b1 = td[p], b2 = td[6 + p];
                if (FORM == 0) {
                    cs[0][p] = -cf.kL * b1; cs[1][p] = cf.vL * b2; cs[2][p] = -cf.kY * b1;
                    cs[3][p] = cf.vY * b2; cs[4][p] = -cf.kYk * b1;
                } else {
                    cs[0][p] = -cf.cKL * b1; cs[1][p] = -cf.cKY * b1; cs[2][p] = 0.0f;
                    cs[3][p] = cf.cVL * b2; cs[4][p] = cf.cVY * b2;
                    cs[5][p] = -cf.cTL * b2; cs[6][p] = -cf.cTY * b2; cs[7][p] = 0.0f;
                    cs[8][p] = b1;
                }
            }
            if (FORM >= 1) { Ct[0] = td[12]; Ct[1] = td[13]; Ct[2] = td[14]; }
            float a1[6], a2[6], W[3];
            float *fo = part + ((size_t)b * T + tc) * 16;
            const bool first = (a == b) ? (J == I) : (J == J0);
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                a1[p] = first ? 0.0f : fo[p];
                a2[p] = first ? 0.0f : fo[6 + p];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) W[c] = first ? 0.0f : fo[12 + c];
            for (int k = 0; k < 64; ++k) {
                const int j = (lane + k) & 63;
                bool act = tv && (I != J || (k >= 1 && (k < 32 || (k == 32 && lane < 32))));
                const int j0 = L.id[0][j], j1 = L.id[1][j], j2 = L.id[2][j];
                act = act && j0 >= 0 &&
                      !((j0 == v0) | (j0 == v1) | (j0 == v2) | (j1 == v0) | (j1 == v1) | (j1 == v2) |
                        (j2 == v0) | (j2 == v1) | (j2 == v2));
                if (act) sym_pair<FORM, K0>(cf, L, j, tx, ty, tz, ot, ntx, nty, ntz, cs, Ct, a1, a2, W, acc);
                // the source sums move one lane down: lane l next meets source (l + k + 1) mod 64
#pragma unroll
                for (int v = 0; v < NA; ++v) acc[v] = __shfl(acc[v], (lane + 1) & 63);
            }
            if (tv) {
#pragma unroll
                for (int p = 0; p < 6; ++p) { fo[p] = a1[p]; fo[6 + p] = a2[p]; }
                fo[12] = W[0]; fo[13] = W[1]; fo[14] = W[2]; fo[15] = 0.0f;
            }
        }
        // back home after 64 rotations: lane l holds source 64 J + l
        const int s = 64 * J + lane;
        if (s < T) {
            float *so = part + ((size_t)(nr + a) * T + s) * 16;
#pragma unroll
            for (int v = 0; v < 12; ++v) so[v] = acc[v];
            so[12] = FORM == 0 ? 0.0f : acc[12];
            so[13] = FORM == 0 ? 0.0f : acc[13];
            so[14] = FORM == 0 ? 0.0f : acc[14];
            so[15] = 0.0f;
        }
    }
}

// One mesh: each wavefront takes items (heaviest first) from a device counter
// until the list is done.
template <int FORM, bool K0>
__global__ __launch_bounds__(64 * kSymWaves) void k_far_sym(int T, int rt, int nr, FarCoef<float> cf,
                                                              const int32_t *__restrict__ tri,
                                                              const float *__restrict__ stat,
                                                              const float *__restrict__ dyn,
                                                              const int2 *__restrict__ items, int nitems,
                                                              int *__restrict__ next, float *__restrict__ part,
                                                              DevCtl ctl)
{
    __shared__ SymLds<FORM> lds[kSymWaves];
    if (ctl_skip(ctl)) return;   // uniform: every wavefront leaves
    const int w = threadIdx.x / 64, lane = threadIdx.x & 63;
    for (;;) {
        int i = 0;
        if (lane == 0) i = atomicAdd(next, 1);
        i = __builtin_amdgcn_readfirstlane(__shfl(i, 0));
        if (i >= nitems) return;
        const int2 it = items[i];
        sym_item<FORM, K0>(cf, tri, stat, dyn, T, rt, nr, it.x, it.y, part, lds[w], lane);
    }
}

// Several meshes (batched requests): items {request, a, b}; a request whose
// stop flag is set contributes nothing.
template <int FORM, bool K0>
__global__ __launch_bounds__(64 * kSymWaves) void k_far_sym_batch(const FarReq<float> *__restrict__ reqs,
                                                                    const int4 *__restrict__ items, int nitems,
                                                                    int *__restrict__ next)
{
    __shared__ SymLds<FORM> lds[kSymWaves];
    const int w = threadIdx.x / 64, lane = threadIdx.x & 63;
    for (;;) {
        int i = 0;
        if (lane == 0) i = atomicAdd(next, 1);
        i = __builtin_amdgcn_readfirstlane(__shfl(i, 0));
        if (i >= nitems) return;
        const int4 it = items[i];
        const FarReq<float> rq = reqs[it.x];
        if (rq.skip && *rq.skip) continue;
        sym_item<FORM, K0>(rq.cf, rq.tri, rq.stat, rq.dyn, rq.T, rq.rt, rq.nr, it.y, it.z, rq.part, lds[w], lane);
    }
}

// kFinishLanes lanes per triangle over its nr + 1 slots, then the test
// projection of k_far_finish (sym_finish_group, far.h)
__global__ __launch_bounds__(256) void k_far_sym_finish(int T, int rt, int nr, int family, int swap,
                                                          const double *__restrict__ geo,
                                                          const float *__restrict__ part,
                                                          double *__restrict__ triout, DevCtl ctl)
{
    if (ctl_skip(ctl)) return;
    const int t = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kFinishLanes);
    const int l = threadIdx.x % kFinishLanes;
    sym_finish_group(t, l, t < T, T, rt, nr, family, swap, geo, part, triout);   // the group agrees on t < T
}

__global__ void k_sym_set(int *p, int v) { *p = v; }

// ------------------------------------------------------------------ host

// The symmetric split applies to FP32 matrix-free meshes.  Automatic (mode 0):
// 56 tiles (3584 triangles) and more -- on one smaller mesh too few tile pairs
// fill the device (measured: at 2880 triangles both kernels take about 0.25 ms
// per product, at 3920 the split is 7% / 33% faster, direct / Juffer, at 8000
// 35% / 40%), while many small meshes batched together fill it either way;
// mode 1 always, mode -1 never.
bool sym_eligible(int T, double kappa, int mode)
{
    (void)kappa;   // kappa = 0 takes the unscreened variant
    if (mode < 0) return false;
    return mode > 0 || T >= 3584;
}

// Ranges of rt tiles: about 320 ranges (51000 items) so that the heaviest-first
// work list ends with items of a few milliseconds at most.
void sym_plan(int T, int &rt, int &nr, std::vector<int2> &items)
{
    const int ntile = (T + 63) / 64;
    rt = std::max(1, (ntile + 319) / 320);
    nr = (ntile + rt - 1) / rt;
    std::vector<std::pair<int, int2>> w;
    for (int a = 0; a < nr; ++a)
        for (int b = a; b < nr; ++b) {
            const int na = std::min(ntile, (a + 1) * rt) - a * rt, nb = std::min(ntile, (b + 1) * rt) - b * rt;
            const int pairs = a == b ? na * (na + 1) / 2 : na * nb;
            w.push_back({pairs, make_int2(a, b)});
        }
    std::stable_sort(w.begin(), w.end(), [](const std::pair<int, int2> &x, const std::pair<int, int2> &y) {
        return x.first > y.first;
    });
    items.clear();
    for (auto &e : w) items.push_back(e.second);
}

// the kernel of a form (0, 1, 3) and screening (k0: kappa = 0)
static const void *sym_kernel(int form, bool k0)
{
    if (k0)
        return form == 0 ? reinterpret_cast<const void *>(&k_far_sym<0, true>)
               : form == 1 ? reinterpret_cast<const void *>(&k_far_sym<1, true>)
                           : reinterpret_cast<const void *>(&k_far_sym<3, true>);
    return form == 0 ? reinterpret_cast<const void *>(&k_far_sym<0, false>)
           : form == 1 ? reinterpret_cast<const void *>(&k_far_sym<1, false>)
                       : reinterpret_cast<const void *>(&k_far_sym<3, false>);
}

static const void *sym_batch_kernel(int form, bool k0)
{
    if (k0)
        return form == 0 ? reinterpret_cast<const void *>(&k_far_sym_batch<0, true>)
               : form == 1 ? reinterpret_cast<const void *>(&k_far_sym_batch<1, true>)
                           : reinterpret_cast<const void *>(&k_far_sym_batch<3, true>);
    return form == 0 ? reinterpret_cast<const void *>(&k_far_sym_batch<0, false>)
           : form == 1 ? reinterpret_cast<const void *>(&k_far_sym_batch<1, false>)
                       : reinterpret_cast<const void *>(&k_far_sym_batch<3, false>);
}

int sym_blocks(int nitems, int form, bool k0)
{
    int dev = 0, ncu = 0, per_cu = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const void *k = sym_kernel(form, k0);
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64 * kSymWaves, 0));
    const long long cap = (long long)std::max(ncu, 1) * std::max(per_cu, 1);
    return (int)std::max(1LL, std::min(cap, (long long)(nitems + kSymWaves - 1) / kSymWaves));
}

void launch_far_sym(DevMesh &d)
{
    FarCoef<float> cf;
    const int form = far_coef_sym(d, cf);
    const bool k0 = !(d.prm.kappa > 0.0);
    const int nb = d.sym_blocks[form == 0 ? 0 : form == 1 ? 1 : 2];
    hipLaunchKernelGGL(k_sym_set, dim3(1), dim3(1), 0, d.stream, d.sym_next, 0);
#define SYM(F, Z)                                                                                                 \
    hipLaunchKernelGGL((k_far_sym<F, Z>), dim3(nb), dim3(64 * kSymWaves), 0, d.stream, d.hm.T, d.sym_rt, d.sym_nr, \
                       cf, d.tri, d.stat32, d.dyn32, d.sym_items, d.sym_nitems, d.sym_next, (float *)d.part, d.ctl)
    if (k0) {
        if (form == 0) SYM(0, true);
        else if (form == 1) SYM(1, true);
        else SYM(3, true);
    } else {
        if (form == 0) SYM(0, false);
        else if (form == 1) SYM(1, false);
        else SYM(3, false);
    }
#undef SYM
    HIPCHECK(hipGetLastError());
}

void launch_far_sym_finish(DevMesh &d)
{
    const int T = d.hm.T;
    const FormCoef &f = d.fm;
    const int swap = f.family == 0 && laplace_row(f) == 1;
    hipLaunchKernelGGL(k_far_sym_finish, dim3((unsigned)(((size_t)T * kFinishLanes + 255) / 256)), dim3(256), 0,
                       d.stream, T, d.sym_rt, d.sym_nr, f.family, swap, d.geo, (const float *)d.part, d.triout,
                       d.ctl);
    HIPCHECK(hipGetLastError());
}

// batched requests: one queue per kernel form and screening of {request, a, b} items
int sym_batch_blocks_for(int form, bool k0, int n)
{
    int dev = 0, ncu = 0, per_cu = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sym_batch_kernel(form, k0), 64 * kSymWaves, 0));
    const long long cap = (long long)std::max(ncu, 1) * std::max(per_cu, 1);
    return (int)std::max(1LL, std::min(cap, (long long)(n + kSymWaves - 1) / kSymWaves));
}

void launch_far_sym_batch(int form, bool k0, const void *reqs, const int4 *items, int n, int nblocks, int *next,
                          hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_sym_set, dim3(1), dim3(1), 0, s, next, 0);
#define SYMB(F, Z)                                                                                 \
    hipLaunchKernelGGL((k_far_sym_batch<F, Z>), dim3(nblocks), dim3(64 * kSymWaves), 0, s,          \
                       (const FarReq<float> *)reqs, items, n, next)
    if (k0) {
        if (form == 0) SYMB(0, true);
        else if (form == 1) SYMB(1, true);
        else SYMB(3, true);
    } else {
        if (form == 0) SYMB(0, false);
        else if (form == 1) SYMB(1, false);
        else SYMB(3, false);
    }
#undef SYMB
    HIPCHECK(hipGetLastError());
}

}  // namespace pbm
