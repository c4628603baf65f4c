// Assembled far field and mixed-precision solves.
//
// The far-field part of the 2V x 2V system (all triangle pairs sharing no
// vertex, regular 6 x 6 point quadrature: the same sums the matrix-free
// kernels evaluate) is assembled once into a dense row-major matrix in the
// vertex basis, already combined into the formulation's four blocks.  The
// near field (FP64 CSR) and mass terms stay separate.
//
// Storage by precision mode:
//   PB_FP64        : FP64 entries, FP64 evaluation
//   PB_FP32        : FP32 entries, FP32 evaluation
//   PB_MIXED_BF16  : FP32 entries (outer residual) + BF16 copy (inner solves)
//   PB_MIXED_FP16  : FP32 entries (outer residual) + FP16 copy with one
//                    power-of-two scale per block (inner solves)
// Products are HBM-streaming GEMVs (one wavefront per row, 16-byte loads);
// several right-hand sides use the MFMA GEMM (k_gemm_mfma).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "dense.h"
#include "far.h"

namespace pbm {


// ------------------------------------------------------------ colouring
// Greedy colouring of the triangles: two triangles sharing a vertex never get
// the same colour, so all triangles of one colour update disjoint matrix rows.
static void color_triangles(const HostMesh &hm, std::vector<int32_t> &ptr, std::vector<int32_t> &list)
{
    const int T = hm.T;
    std::vector<int> col(T, -1);
    int ncol = 0;
    std::vector<char> used;
    for (int t = 0; t < T; ++t) {
        used.assign(ncol + 1, 0);
        for (int p = hm.pair_ptr[t]; p < hm.pair_ptr[t + 1]; ++p) {
            int c = col[hm.pair_s[p]];
            if (c >= 0) used[c] = 1;
        }
        int c = 0;
        while (c < ncol && used[c]) ++c;
        col[t] = c;
        ncol = std::max(ncol, c + 1);
    }
    ptr.assign(ncol + 1, 0);
    for (int t = 0; t < T; ++t) ptr[col[t] + 1]++;
    for (int c = 0; c < ncol; ++c) ptr[c + 1] += ptr[c];
    list.resize(T);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int t = 0; t < T; ++t) list[fill[col[t]]++] = t;
}

// ------------------------------------------------------------- assembly
template <typename R>
struct AsmCoef {
    R kappa, kexp, k2;
    // block (r, c) = aL[r][c] Op_L + aY[r][c] Op_Y (far field: no mass term)
    R aL[2][2], aY[2][2];
    // FORM 1: ratios aY / aL of the K, V, D and T blocks (aL != 0 there)
    R rK, rV, rD, rT;
};

// Orbit form of the 6-point rule (Numerical integration): its points form two
// orbits of three with barycentric coordinates (1-2a, a, a) and (1-2b, b, b).
// For any values v_p, sum_p w_p lambda_k(x_p) v_p equals
//   cA (v_k + rho v_{k+3} + al (v_0+v_1+v_2) + be (v_3+v_4+v_5))
// with cA = wA(1-3a), rho = wB(1-3b)/cA, al = wA a/cA, be = wB b/cA, which is
// 12 instead of 18 operations per value and weight pass.
struct RuleOrbit {
    static constexpr double cA = kRuleWA * (1.0 - 3.0 * kRuleA);
    static constexpr double rho = kRuleWB * (1.0 - 3.0 * kRuleB) / cA;
    static constexpr double al = kRuleWA * kRuleA / cA;
    static constexpr double be = kRuleWB * kRuleB / cA;
};

template <typename R> struct alignas(4 * sizeof(R)) Quad {
    R v[4];
};

// Block = (group of targets of the current colour, tile of TILE Morton-ordered
// source triangles of the current tile colour).  The source data and the
// tile's vertex lists are loaded once per block and reused for every target of
// the group, which is processed one after the other:
// Phase 1: lane s computes the whole local 3 x 3 block of the pair (t, s) for
//   the four combined operator values into LDS (zero if s shares a vertex with
//   t).  Per point pair (FORM 0, direct) F_L d.n_s, -G_L, -F_Y d.n_s, eps G_Y,
//   or (FORM 1, Juffer) (F_L - alpha F_Y) d.n_s, G_Y - G_L, G_Y,
//   (F_L - beta F_Y) d.n_t, with the hypersingular curl part added from
//   sum (G_Y - G_L) per pair.  Signs and constant factors are applied once per
//   block, not per point pair.
// Phase 2: lane v sums, for one vertex touched by the tile, the block columns
//   of its incident tile triangles, and adds the 3 x 4 values to rows t_0..t_2.
//   SYM reads the lane's matrix entries at the start of phase 2, where the
//   LDS sums cover part of their latency: held through phase 1, those 18
//   registers made the compiler spill.  The FP64 kernel, with fewer values
//   per pair, reads them before phase 1.
// SYM (one evaluation per unordered pair): only pairs with s > t are
// evaluated.  The symmetric values (V-type, and D in the Juffer system) are
// added in the (t, s) orientation only; the two non-symmetric ones (K-type,
// and K or T in the second block row) of the swapped pair (s, t) are computed
// from the same point-pair kernels and added, in the same (t, s) layout, to
// the side matrix C.  k_sym_finish then adds the transposes.
// Target colours keep rows disjoint and tile colours keep columns disjoint
// between concurrently running blocks, so there is no atomic and the result
// is deterministic.
template <typename R, typename S, int FORM, int TILE, bool SYM, int LROW>
__global__ __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(SYM ? 2 : 1))) void k_assemble_tile(
    int T, int V, AsmCoef<R> cf, const int32_t *__restrict__ targets, int ntarget, int group,
    const int32_t *__restrict__ tiles, const int4 *__restrict__ sym_blocks, const int32_t *__restrict__ tri,
    const R *__restrict__ stat, const int32_t *__restrict__ vpos,
    const int32_t *__restrict__ tv_ptr, const int32_t *__restrict__ tv_col, const int32_t *__restrict__ tv_eptr,
    const int32_t *__restrict__ te, S *__restrict__ A, size_t ld, size_t Vp, S *__restrict__ C, size_t ldc)
{
    constexpr int NV = SYM ? 6 : 4;
    __shared__ Quad<R> lds[9 * TILE];
    __shared__ R lds2[SYM ? 18 * TILE : 1];
    int tile, gbeg, gend;
    if (SYM) {
        const int4 bk = sym_blocks[blockIdx.x];
        tile = bk.x; gbeg = bk.y; gend = bk.z;
    } else {
        tile = tiles[blockIdx.x];
        gbeg = blockIdx.y * group;
        gend = min(gbeg + group, ntarget);
    }
    const int tid = threadIdx.x;
    const int s = tile * TILE + tid;
    // lanes past the last triangle evaluate the last one and are zeroed below
    const int sl = s < T ? s : T - 1;
    const int j0 = tri[3 * sl], j1 = tri[3 * sl + 1], j2 = tri[3 * sl + 2];
    const R *ss = stat + (size_t)sl * kStat;
    // os: the source plane's offset y . n_s (the same for its six points)
    const R nsx = ss[18], nsy = ss[19], nsz = ss[20], os = ss[21], sarea = ss[27];
    R sy[6][3];
#pragma unroll
    for (int q = 0; q < 6; ++q) { sy[q][0] = ss[3 * q]; sy[q][1] = ss[3 * q + 1]; sy[q][2] = ss[3 * q + 2]; }
    // the lane's vertex column of the tile (a lane without one re-reads the
    // tile's first and never stores it) and its first kPre incidences
    // (tile slot << 2 | local vertex)
    const int eb = tv_ptr[tile], ee = tv_ptr[tile + 1];
    const int e0 = eb + tid < ee ? eb + tid : eb;
    const size_t c0 = (size_t)tv_col[e0];
    const int fb0 = tv_eptr[e0], fe0 = tv_eptr[e0 + 1];
    // codes are below 4 TILE, so two share a register
    constexpr int kPre = 8;
    uint32_t ter[kPre / 2];
#pragma unroll
    for (int i = 0; i < kPre; i += 2)
        ter[i / 2] = (uint32_t)te[min(fb0 + i, fe0 - 1)] | ((uint32_t)te[min(fb0 + i + 1, fe0 - 1)] << 16);

    for (int g = gbeg; g < gend; ++g) {
        const int t = targets[g];
        const int v0 = tri[3 * t], v1 = tri[3 * t + 1], v2 = tri[3 * t + 2];
        const bool live = (s < T) & (!SYM | (s > t)) &
                          !((j0 == v0) | (j0 == v1) | (j0 == v2) | (j1 == v0) | (j1 == v1) | (j1 == v2) |
                            (j2 == v0) | (j2 == v1) | (j2 == v2));
        const R *ts = stat + (size_t)t * kStat;   // uniform: scalar loads
        const size_t rk[3] = {(size_t)vpos[v0], (size_t)vpos[v1], (size_t)vpos[v2]};
        S old[3][NV];
        auto load_old = [&](size_t c) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const S *r1 = A + rk[k] * ld, *r2 = A + ((size_t)V + rk[k]) * ld;
                old[k][0] = r1[c];
                old[k][1] = r1[Vp + c];
                old[k][2] = r2[c];
                old[k][3] = r2[Vp + c];
                if (SYM) {
                    old[k][4] = C[rk[k] * ldc + c];
                    old[k][5] = C[((size_t)V + rk[k]) * ldc + c];
                }
            }
        };
        if constexpr (!SYM) load_old(c0);

        const R ntx = ts[18], nty = ts[19], ntz = ts[20], ot = ts[21];
        const R rho = (R)RuleOrbit::rho, al = (R)RuleOrbit::al, be = (R)RuleOrbit::be;
        // Flat triangles: with d = x_p - y_q, d . n_s = x_p . n_s - os depends on
        // the target point only and d . n_t = ot - y_q . n_t on the source point only
        R dns[6];
#pragma unroll
        for (int p = 0; p < 6; ++p) dns[p] = ts[3 * p] * nsx + ts[3 * p + 1] * nsy + ts[3 * p + 2] * nsz - os;
        R blk[3][3][NV], Cq[3][NV];   // [l][k][o]; Cq: rank-two part of the target-side weights
        R Ssum = 0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const R dnt = (FORM == 1 || SYM) ? ot - (sy[q][0] * ntx + sy[q][1] * nty + sy[q][2] * ntz) : R(0);
            R X[3][NV], SA[NV], SB[NV];
            R sLA = 0, sLB = 0;   // orbit sums of G_L over the target points (FORM 1, LROW 2)
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const R tx = ts[3 * p], ty = ts[3 * p + 1], tz = ts[3 * p + 2];
                const R dx = tx - sy[q][0], dy = ty - sy[q][1], dz = tz - sy[q][2];
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R ri = rsqrt_r(r2);
                const R r = r2 * ri;
                const R ek = expneg(cf.kexp, r);
                const R ri3 = ri * ri * ri;
                const R ekk = ek * (cf.kappa * r + R(1));
                R v[NV];
                if (FORM == 0) {
                    // direct formulations: one row has Laplace (F_L d.n_s, G_L), the other
                    // Yukawa kernels (F_Y d.n_s, G_Y); the swapped pair's K of the first
                    // column with d.n_t.  Values ordered by block; LROW = the Laplace row.
                    const R kl = ri3 * dns[p], ky = ekk * kl;
                    v[LROW == 0 ? 0 : 2] = kl;
                    v[LROW == 0 ? 1 : 3] = ri;
                    v[LROW == 0 ? 2 : 0] = ky;
                    v[LROW == 0 ? 3 : 1] = ek * ri;
                    if (SYM) {
                        const R klt = ri3 * dnt;
                        v[LROW == 0 ? 4 : 5] = klt;
                        v[LROW == 0 ? 5 : 4] = ekk * klt;
                    }
                } else {
                    // (F_L + rK F_Y) d.n_s, G_L + rV G_Y, G_Y, (F_L + rT F_Y) d.n_t, without the
                    // factors aL; swapped pair: K with d.n_t, T with d.n_s.  LROW = 1: no
                    // Laplace term in any block, F_Y and G_Y alone with the factors aY.
                    // LROW = 2 (some block without a Laplace term, another with one):
                    // both coefficients of each block inside the values, no factor.
                    const R fy = ekk * ri3;
                    const R gy = ek * ri;
                    R a1, a2;
                    if (LROW == 0) { a1 = ri3 + cf.rK * fy; a2 = ri3 + cf.rT * fy; }
                    else if (LROW == 1) { a1 = fy; a2 = fy; }
                    else { a1 = cf.aL[0][0] * ri3 + cf.aY[0][0] * fy; a2 = cf.aL[1][1] * ri3 + cf.aY[1][1] * fy; }
                    v[0] = a1 * dns[p];
                    v[1] = LROW == 0 ? ri + cf.rV * gy : LROW == 1 ? gy : cf.aL[0][1] * ri + cf.aY[0][1] * gy;
                    v[2] = gy;
                    v[3] = a2 * dnt;
                    if (SYM) {
                        v[4] = a1 * dnt;
                        v[5] = a2 * dns[p];
                    }
                    // D's curl part integrates aL[1][0] G_L + aY[1][0] G_Y; the G_L part
                    // by its own orbit sums (LROW = 2)
                    if (LROW == 2) {
                        if (p < 3) sLA = p == 0 ? ri : sLA + ri;
                        else sLB = p == 3 ? ri : sLB + ri;
                    }
                }
#pragma unroll
                for (int o = 0; o < NV; ++o) {
                    if (p < 3) {
                        X[p][o] = v[o];
                        SA[o] = p == 0 ? v[o] : SA[o] + v[o];
                    } else {
                        X[p - 3][o] += rho * v[o];
                        SB[o] = p == 3 ? v[o] : SB[o] + v[o];
                    }
                }
            }
#pragma unroll
            for (int o = 0; o < NV; ++o) {
                const R cc = al * SA[o] + be * SB[o];
#pragma unroll
                for (int k = 0; k < 3; ++k) X[k][o] += cc;
            }
            // D's curl part integrates G_L + rD G_Y = v1 + (rD - rV) v2 (LROW 0, 1), or
            // aL[1][0] G_L + aY[1][0] G_Y (LROW 2)
            if (FORM == 1 && LROW != 2)
                Ssum += R(rule_w(q)) * ((R(kRuleWA) * SA[1] + R(kRuleWB) * SB[1]) +
                                        (cf.rD - cf.rV) * (R(kRuleWA) * SA[2] + R(kRuleWB) * SB[2]));
            if (FORM == 1 && LROW == 2)
                Ssum += R(rule_w(q)) * (cf.aL[1][0] * (R(kRuleWA) * sLA + R(kRuleWB) * sLB) +
                                        cf.aY[1][0] * (R(kRuleWA) * SA[2] + R(kRuleWB) * SB[2]));
            const R wc = q < 3 ? al : be;
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int o = 0; o < NV; ++o) {
                    if (q < 3) blk[q][k][o] = X[k][o];
                    else blk[q - 3][k][o] += rho * X[k][o];
                    Cq[k][o] = q == 0 ? wc * X[k][o] : Cq[k][o] + wc * X[k][o];
                }
        }
        const R sc = ts[27] * sarea * (R)kInv4Pi;
        const R sw = sc * (R)(RuleOrbit::cA * RuleOrbit::cA);
        // Per-value factors.  The double-layer kernel is +F d.n_y, the adjoint one
        // -F d.n_x, with d the test point minus the trial point; for the swapped
        // pair d changes sign.  FORM 0: each value has one block's coefficient
        // (Laplace row LROW, Yukawa row 1 - LROW).
        R f[NV];
        if (FORM == 0) {
            const R c00 = LROW == 0 ? cf.aL[0][0] : cf.aY[0][0], c01 = LROW == 0 ? cf.aL[0][1] : cf.aY[0][1];
            const R c10 = LROW == 0 ? cf.aY[1][0] : cf.aL[1][0], c11 = LROW == 0 ? cf.aY[1][1] : cf.aL[1][1];
            f[0] = sw * c00; f[1] = sw * c01; f[2] = sw * c10; f[3] = sw * c11;
            if (SYM) { f[4] = -sw * c00; f[5] = -sw * c10; }
        } else {
            // leading factors: aL (ratios aY / aL inside the values), aY (LROW = 1), or
            // none (LROW = 2: the coefficients are inside the values)
            const R l00 = LROW == 0 ? cf.aL[0][0] : LROW == 1 ? cf.aY[0][0] : R(1);
            const R l01 = LROW == 0 ? cf.aL[0][1] : LROW == 1 ? cf.aY[0][1] : R(1);
            const R l11 = LROW == 0 ? cf.aL[1][1] : LROW == 1 ? cf.aY[1][1] : R(1);
            f[0] = sw * l00;
            f[1] = sw * l01;
            f[2] = sw * cf.aY[1][0] * cf.k2 * (ntx * nsx + nty * nsy + ntz * nsz);
            f[3] = -sw * l11;
            if (SYM) { f[4] = -sw * l00; f[5] = sw * l11; }
        }
        // the rank-two target-side part, scaled once: value = f (blk + Cq)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int o = 0; o < NV; ++o) Cq[k][o] *= f[o];
        if (g > gbeg) __syncthreads();   // the previous target's phase 2 is done with lds
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                R val[NV];
#pragma unroll
                for (int o = 0; o < NV; ++o) val[o] = blk[l][k][o] * f[o] + Cq[k][o];
                if (FORM == 1) {
                    // hypersingular: curl_k(t) . curl_l(s) int int (G_Y - G_L) + kappa^2 (n_t . n_s) V_Y
                    const R cc = ts[28 + 3 * k] * ss[28 + 3 * l] + ts[29 + 3 * k] * ss[29 + 3 * l] +
                                 ts[30 + 3 * k] * ss[30 + 3 * l];
                    val[2] += sc * (LROW == 0 ? cf.aL[1][0] : LROW == 1 ? cf.aY[1][0] : R(1)) * cc * Ssum;
                }
                // a pair sharing a vertex may have produced inf or NaN: select, not scale
                Quad<R> qd;
#pragma unroll
                for (int o = 0; o < 4; ++o) qd.v[o] = live ? val[o] : R(0);
                lds[(3 * l + k) * TILE + tid] = qd;
                if (SYM) {
                    lds2[(2 * (3 * l + k)) * TILE + tid] = live ? val[4] : R(0);
                    lds2[(2 * (3 * l + k) + 1) * TILE + tid] = live ? val[5] : R(0);
                }
            }
        __syncthreads();

        for (int e = eb + tid; e < ee; e += TILE) {
            size_t c = c0;
            int fb = fb0, fe = fe0;
            if (e != eb + tid) {   // a tile with more vertices than lanes
                c = (size_t)tv_col[e];
                fb = tv_eptr[e];
                fe = tv_eptr[e + 1];
                if constexpr (!SYM) load_old(c);
            }
            if constexpr (SYM) load_old(c);
            R acc[3][NV];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int o = 0; o < NV; ++o) acc[k][o] = 0;
            auto add = [&](int code) {
                const int slot = code >> 2, l = code & 3;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const Quad<R> qd = lds[(3 * l + k) * TILE + slot];
#pragma unroll
                    for (int o = 0; o < 4; ++o) acc[k][o] += qd.v[o];
                    if (SYM) {
                        acc[k][4] += lds2[(2 * (3 * l + k)) * TILE + slot];
                        acc[k][5] += lds2[(2 * (3 * l + k) + 1) * TILE + slot];
                    }
                }
            };
            if (e == eb + tid) {
#pragma unroll
                for (int i = 0; i < kPre; ++i)
                    if (fb + i < fe) add((int)((ter[i / 2] >> (16 * (i & 1))) & 0xffffu));
                for (int f = fb + kPre; f < fe; ++f) add(te[f]);
            } else {
                for (int f = fb; f < fe; ++f) add(te[f]);
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                S *r1 = A + rk[k] * ld, *r2 = A + ((size_t)V + rk[k]) * ld;
                r1[c] = old[k][0] + (S)acc[k][0];
                r1[Vp + c] = old[k][1] + (S)acc[k][1];
                r2[c] = old[k][2] + (S)acc[k][2];
                r2[Vp + c] = old[k][3] + (S)acc[k][3];
                if (SYM) {
                    C[rk[k] * ldc + c] = old[k][4] + (S)acc[k][4];
                    C[((size_t)V + rk[k]) * ldc + c] = old[k][5] + (S)acc[k][5];
                }
            }
        }
    }
}

// Completion of the one-evaluation-per-pair assembly on one V x V block of A
// (rows r0.., columns c0..), in 64 x 64 tiles through LDS with 16-byte global
// accesses (A's row stride and both column offsets are multiples of 64):
//   MODE 0 (symmetric operator): A <- A + A^T;
//   MODE 1: A <- A + C_b^T, C_b = rows cr0.. of the side matrix C.
// Rows at or beyond V are neither read nor written; columns beyond V (zero
// padding) are read but never written.
template <int MODE>
__global__ __launch_bounds__(256) void k_sym_finish(int V, float *__restrict__ A, size_t ld, size_t r0, size_t c0,
                                                    const float *__restrict__ C, size_t ldc, size_t cr0)
{
    __shared__ float ta[64][65], tb[64][65];
    const int I = blockIdx.y, J = blockIdx.x;   // tile row, tile column of the block
    if (MODE == 0 && I > J) return;
    const int cx = (threadIdx.x & 15) * 4, ry = threadIdx.x >> 4;
    auto arow = [&](int i) { return A + (r0 + (size_t)i) * ld + c0; };
    auto put = [&](float (*t)[65], int r, float4 v) {
        t[r][cx] = v.x; t[r][cx + 1] = v.y; t[r][cx + 2] = v.z; t[r][cx + 3] = v.w;
    };
    // tb <- the mirrored tile (rows of J, columns of I) of A or of C; ta <- tile (I, J)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = ry + 16 * i, gi = J * 64 + r, gj = I * 64 + cx;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gi < V) v = MODE == 0 ? *(const float4 *)(arow(gi) + gj) : *(const float4 *)(C + (cr0 + gi) * ldc + gj);
        put(tb, r, v);
    }
    float4 base[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gi = I * 64 + ry + 16 * i, gj = J * 64 + cx;
        base[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gi < V && !(MODE == 0 && I == J)) base[i] = *(const float4 *)(arow(gi) + gj);
        if (MODE == 0 && I != J) put(ta, ry + 16 * i, base[i]);
    }
    __syncthreads();
    auto store = [&](int gi, int gj, float4 v) {
        if (gi >= V) return;
        float *p = arow(gi) + gj;
        if (gj + 3 < V) {
            *(float4 *)p = v;
        } else {
            const float e[4] = {v.x, v.y, v.z, v.w};
            for (int k = 0; k < 4 && gj + k < V; ++k) p[k] = e[k];
        }
    };
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = ry + 16 * i;
        float4 v = MODE == 0 && I == J ? make_float4(tb[r][cx], tb[r][cx + 1], tb[r][cx + 2], tb[r][cx + 3]) : base[i];
        v.x += tb[cx][r]; v.y += tb[cx + 1][r]; v.z += tb[cx + 2][r]; v.w += tb[cx + 3][r];
        store(I * 64 + r, J * 64 + cx, v);
    }
    if (MODE == 0 && I != J)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = ry + 16 * i;
            float4 v = make_float4(tb[r][cx], tb[r][cx + 1], tb[r][cx + 2], tb[r][cx + 3]);
            v.x += ta[cx][r]; v.y += ta[cx + 1][r]; v.z += ta[cx + 2][r]; v.w += ta[cx + 3][r];
            store(J * 64 + r, I * 64 + cx, v);
        }
}

template <typename S>
__global__ void k_fill(size_t n, S *__restrict__ a)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) a[i] = S(0);
}

// FP32 -> BF16 (round to nearest even) or FP16 with a per-block scale
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ void k_to16(int n, int V, size_t Vp, size_t ld, int kind, float s0, float s1, float s2, float s3,
                       const float *__restrict__ A, uint16_t *__restrict__ B)
{
    const size_t total = (size_t)n * ld;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < total; i += stride) {
        const float a = A[i];
        if (kind == 1) {
            B[i] = to_bf16(a);
        } else {
            const size_t r = i / ld, c = i - r * ld;
            const int blk = (r >= (size_t)V ? 2 : 0) + (c >= Vp ? 1 : 0);
            const float sc = blk == 0 ? s0 : blk == 1 ? s1 : blk == 2 ? s2 : s3;
            _Float16 h = (_Float16)(a * sc);
            B[i] = __builtin_bit_cast(uint16_t, h);
        }
    }
}

// per-block max |entry| (for the FP16 scales); one partial per block of threads
__global__ __launch_bounds__(256) void k_blockmax(int n, int V, size_t Vp, size_t ld, const float *__restrict__ A,
                                                  float *__restrict__ out)
{
    __shared__ float sh[4][256];
    float m[4] = {0, 0, 0, 0};
    const size_t total = (size_t)n * ld;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
        const size_t r = i / ld, c = i - r * ld;
        const int blk = (r >= (size_t)V ? 2 : 0) + (c >= Vp ? 1 : 0);
        m[blk] = fmaxf(m[blk], fabsf(A[i]));
    }
    for (int b = 0; b < 4; ++b) sh[b][threadIdx.x] = m[b];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int b = 0; b < 4; ++b) sh[b][threadIdx.x] = fmaxf(sh[b][threadIdx.x], sh[b][threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int b = 0; b < 4; ++b) out[4 * blockIdx.x + b] = sh[b][0];
}

// ----------------------------------------------------------------- GEMV
// y[r] = sum_c A[r][c] x[c], one wavefront per row, each lane streams 16-byte
// chunks; x is padded with zeros to ld.  ACC = accumulation type.
__device__ __forceinline__ void load16(const double *p, double *v) { const double2 a = *(const double2 *)p; v[0] = a.x; v[1] = a.y; }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename S> struct Vec;
template <> struct Vec<double> { static constexpr int W = 2; };
template <> struct Vec<float> { static constexpr int W = 4; };
template <> struct Vec<uint16_t> { static constexpr int W = 8; };

__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ float fp16_to_f(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

template <typename S, typename ACC, int KIND>
__global__ __launch_bounds__(256) void k_gemv(int n, int V, size_t Vp, size_t ld, const S *__restrict__ A,
                                              const ACC *__restrict__ x, float inv0, float inv1, float inv2, float inv3,
                                              double *__restrict__ y, DevCtl ctl)
{
    if (ctl_skip(ctl)) return;
    constexpr int W = Vec<S>::W;
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6;
    const int nwave = (gridDim.x * 256) >> 6;
    for (int r = wave; r < n; r += nwave) {
        const S *row = A + (size_t)r * ld;
        ACC s0 = 0, s1 = 0;   // columns < V and >= V (separate block scales for FP16)
        // four independent 16-byte streaming loads in flight per lane; the
        // matrix is read once, so loads are non-temporal and x stays in L2
        constexpr size_t step = 64 * W;
        auto consume = [&](size_t c, const u32x4 &u) {
            S v[W];
            __builtin_memcpy(v, &u, 16);
            ACC part = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                ACC a;
                if constexpr (KIND == 0) a = (ACC)v[w];
                else if constexpr (KIND == 1) a = (ACC)bf16_to_f((uint16_t)v[w]);
                else a = (ACC)fp16_to_f((uint16_t)v[w]);
                part += a * x[c + w];
            }
            if (c < Vp) s0 += part; else s1 += part;   // chunks never straddle Vp (multiple of 64)
        };
        size_t c = (size_t)lane * W;
        for (; c + 3 * step < ld; c += 4 * step) {
            const u32x4 u0 = __builtin_nontemporal_load((const u32x4 *)(row + c));
            const u32x4 u1 = __builtin_nontemporal_load((const u32x4 *)(row + c + step));
            const u32x4 u2 = __builtin_nontemporal_load((const u32x4 *)(row + c + 2 * step));
            const u32x4 u3 = __builtin_nontemporal_load((const u32x4 *)(row + c + 3 * step));
            consume(c, u0);
            consume(c + step, u1);
            consume(c + 2 * step, u2);
            consume(c + 3 * step, u3);
        }
        for (; c < ld; c += step) consume(c, __builtin_nontemporal_load((const u32x4 *)(row + c)));
        for (int off = 32; off > 0; off >>= 1) {
            s0 += __shfl_xor(s0, off);
            s1 += __shfl_xor(s1, off);
        }
        if (lane == 0) {
            double out;
            if (KIND == 2) {
                const bool top = r < V;
                out = (double)s0 * (top ? inv0 : inv2) + (double)s1 * (top ? inv1 : inv3);
            } else {
                out = (double)s0 + (double)s1;
            }
            y[r] = out;
        }
    }
}

// Row-tile GEMV: one wavefront per tile of 16 consecutive rows.  Each lane
// walks its column chunks once, loads the x chunk once and applies it to the
// 16 rows (16 independent 16-byte streaming loads in flight), keeping the
// x traffic at 1/16 of the matrix traffic.  Per-row lane partials are reduced
// across the wavefront at the end (fixed butterfly, deterministic).
template <typename S, typename ACC, int KIND, int R>
__global__ __launch_bounds__(256) void k_gemv_tile(int n, int V, size_t Vp, size_t ld, const S *__restrict__ A,
                                                   const ACC *__restrict__ x, float inv0, float inv1, float inv2,
                                                   float inv3, double *__restrict__ y, DevCtl ctl)
{
    if (ctl_skip(ctl)) return;
    constexpr int W = Vec<S>::W;
    constexpr size_t step = 64 * W;
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6;
    const int nwave = (gridDim.x * 256) >> 6;
    const int ntile = (n + R - 1) / R;
    for (int tile = wave; tile < ntile; tile += nwave) {
        const int r0 = tile * R;
        const S *rows[R];
#pragma unroll
        for (int i = 0; i < R; ++i) rows[i] = A + (size_t)min(r0 + i, n - 1) * ld;
        ACC s0[R], s1[R];
#pragma unroll
        for (int i = 0; i < R; ++i) { s0[i] = 0; s1[i] = 0; }
        for (size_t c = (size_t)lane * W; c < ld; c += step) {
            ACC xv[W];
#pragma unroll
            for (int w = 0; w < W; ++w) xv[w] = x[c + w];
            u32x4 u[R];
#pragma unroll
            for (int i = 0; i < R; ++i) u[i] = __builtin_nontemporal_load((const u32x4 *)(rows[i] + c));
            const bool first = c < Vp;   // chunks never straddle Vp (multiple of 64)
#pragma unroll
            for (int i = 0; i < R; ++i) {
                S v[W];
                __builtin_memcpy(v, &u[i], 16);
                ACC part = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    ACC a;
                    if constexpr (KIND == 0) a = (ACC)v[w];
                    else if constexpr (KIND == 1) a = (ACC)bf16_to_f((uint16_t)v[w]);
                    else a = (ACC)fp16_to_f((uint16_t)v[w]);
                    part += a * xv[w];
                }
                if (first) s0[i] += part; else s1[i] += part;
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i)
            for (int off = 32; off > 0; off >>= 1) {
                s0[i] += __shfl_xor(s0[i], off);
                s1[i] += __shfl_xor(s1[i], off);
            }
        if (lane < R && r0 + lane < n) {
            ACC a0 = 0, a1 = 0;
#pragma unroll
            for (int i = 0; i < R; ++i)
                if (i == lane) { a0 = s0[i]; a1 = s1[i]; }
            const int r = r0 + lane;
            double out;
            if (KIND == 2) {
                const bool top = r < V;
                out = (double)a0 * (top ? inv0 : inv2) + (double)a1 * (top ? inv1 : inv3);
            } else {
                out = (double)a0 + (double)a1;
            }
            y[r] = out;
        }
    }
}

// Split row-tile GEMV: the work unit is (tile of R rows, one of the two column
// blocks), so there are twice as many units as tiles and the wavefronts spread
// more evenly over the SIMDs; each unit writes its R partial sums, and
// k_gemv_join adds the two blocks' partials of a row in a fixed order.
template <typename S, typename ACC, int KIND, int R>
__global__ __launch_bounds__(256) void k_gemv_split(int n, size_t Vp, size_t ld, const S *__restrict__ A,
                                                    const ACC *__restrict__ x, ACC *__restrict__ part, DevCtl ctl)
{
    if (ctl_skip(ctl)) return;
    constexpr int W = Vec<S>::W;
    constexpr size_t step = 64 * W;
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6;
    const int nwave = (gridDim.x * 256) >> 6;
    const int nunit = 2 * ((n + R - 1) / R);
    for (int u = wave; u < nunit; u += nwave) {
        const int r0 = (u >> 1) * R;
        const size_t c0 = (u & 1) * Vp;   // column block; chunks never straddle Vp (multiple of 64)
        const S *rows[R];
#pragma unroll
        for (int i = 0; i < R; ++i) rows[i] = A + (size_t)min(r0 + i, n - 1) * ld + c0;
        ACC sacc[R];
#pragma unroll
        for (int i = 0; i < R; ++i) sacc[i] = 0;
        for (size_t c = (size_t)lane * W; c < Vp; c += step) {
            ACC xv[W];
#pragma unroll
            for (int w = 0; w < W; ++w) xv[w] = x[c0 + c + w];
            u32x4 uu[R];
#pragma unroll
            for (int i = 0; i < R; ++i) uu[i] = __builtin_nontemporal_load((const u32x4 *)(rows[i] + c));
#pragma unroll
            for (int i = 0; i < R; ++i) {
                S v[W];
                __builtin_memcpy(v, &uu[i], 16);
                ACC pp = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    ACC a;
                    if constexpr (KIND == 0) a = (ACC)v[w];
                    else if constexpr (KIND == 1) a = (ACC)bf16_to_f((uint16_t)v[w]);
                    else a = (ACC)fp16_to_f((uint16_t)v[w]);
                    pp += a * xv[w];
                }
                sacc[i] += pp;
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i)
            for (int off = 32; off > 0; off >>= 1) sacc[i] += __shfl_xor(sacc[i], off);
        if (lane < R && r0 + lane < n) {
            ACC a = 0;
#pragma unroll
            for (int i = 0; i < R; ++i)
                if (i == lane) a = sacc[i];
            part[(size_t)(u & 1) * n + r0 + lane] = a;
        }
    }
}

template <typename ACC, int KIND>
__global__ void k_gemv_join(int n, int V, float inv0, float inv1, float inv2, float inv3,
                            const ACC *__restrict__ part, double *__restrict__ y, DevCtl ctl)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n || ctl_skip(ctl)) return;
    const ACC a0 = part[r], a1 = part[(size_t)n + r];
    double out;
    if (KIND == 2) {
        const bool top = r < V;
        out = (double)a0 * (top ? inv0 : inv2) + (double)a1 * (top ? inv1 : inv3);
    } else {
        out = (double)a0 + (double)a1;
    }
    y[r] = out;
}

// copy x (2V doubles, two halves) into the padded layout: [x1 | x2 | 0...]
// x (2V doubles, vertex order) into the padded dense column order
// [x1 (dense index order) | 0 | x2 | 0]
template <typename ACC>
__global__ void k_pad_x(int V, size_t Vp, size_t ld, const int32_t *__restrict__ vperm, const double *__restrict__ x,
                        ACC *__restrict__ xp, DevCtl ctl)
{
    size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ld || ctl_skip(ctl)) return;
    x += ctl_off(ctl);
    ACC v = ACC(0);
    if (c < (size_t)V) v = (ACC)x[vperm[c]];
    else if (c >= Vp && c < Vp + (size_t)V) v = (ACC)x[V + vperm[c - Vp]];
    xp[c] = v;
}

// ------------------------------------------------------------- host side
// columns laid out as [x1 (V) | 0 | x2 (V) | 0] with each block padded to a
// multiple of 64 entries, so a 16-byte chunk never straddles the two blocks
static size_t dense_vp(int V) { return ((size_t)V + 63) / 64 * 64; }
static size_t dense_ld(int V) { return 2 * dense_vp(V); }

static size_t dense_bytes(const DevMesh &d)
{
    const size_t n = 2 * (size_t)d.hm.V, ld = dense_ld(d.hm.V);
    size_t per = d.prm.precision == PB_FP64 ? 8 : 4;
    // 16-bit copy; in FP32 mode the side matrix C of the same size
    if (d.prm.precision != PB_FP64) per += 2;
    return n * ld * per;
}

bool dense_fits(const DevMesh &d, int copies)
{
    size_t need = dense_bytes(d) * (size_t)copies;
    if (d.opt.memory_budget && d.bytes + need > d.opt.memory_budget) return false;
    // a server's handle: admission reserved its footprint, and the free memory
    // the device reports leaves out the blocks the server keeps for reuse
    if (d.cache) return true;
    size_t freeb = 0, total = 0;
    if (hipMemGetInfo(&freeb, &total) != hipSuccess) return false;
    return need < 0.8 * (double)freeb;
}

// Source tiles of `tile` consecutive Morton-ordered triangles; dense vertex
// numbering by first touch in tile order; per tile the touched vertices (in
// dense order) with their (slot, local vertex) incidences; tile colouring so
// that tiles of one colour share no vertex.
static void build_tiles(const HostMesh &hm, DevMesh &d, Dense &D, const std::vector<int32_t> &tcol_list)
{
    const int T = hm.T, V = hm.V, TL = D.tile;
    D.ntile = (T + TL - 1) / TL;
    std::vector<int32_t> vpos(V, -1), vperm(V);
    int next = 0;
    for (int s = 0; s < T; ++s)
        for (int k = 0; k < 3; ++k) {
            const int v = hm.tri[3 * s + k];
            if (vpos[v] < 0) { vpos[v] = next; vperm[next] = v; ++next; }
        }
    std::vector<int32_t> tv_ptr(D.ntile + 1, 0), tv_col, tv_eptr(1, 0), te;
    std::vector<std::pair<int32_t, int32_t>> buf;
    std::vector<std::vector<int32_t>> vtiles(V);
    for (int tl = 0; tl < D.ntile; ++tl) {
        buf.clear();
        for (int s = tl * TL; s < std::min(T, (tl + 1) * TL); ++s)
            for (int l = 0; l < 3; ++l) buf.push_back({vpos[hm.tri[3 * s + l]], ((s - tl * TL) << 2) | l});
        std::sort(buf.begin(), buf.end());
        for (size_t a = 0; a < buf.size();) {
            size_t b = a;
            while (b < buf.size() && buf[b].first == buf[a].first) te.push_back(buf[b++].second);
            tv_col.push_back(buf[a].first);
            tv_eptr.push_back((int32_t)te.size());
            vtiles[vperm[buf[a].first]].push_back(tl);
            a = b;
        }
        tv_ptr[tl + 1] = (int32_t)tv_col.size();
    }
    // colour tiles: neighbours = tiles sharing a vertex
    std::vector<int> col(D.ntile, -1);
    int ncol = 0;
    std::vector<char> used;
    for (int tl = 0; tl < D.ntile; ++tl) {
        used.assign(ncol + 1, 0);
        for (int e = tv_ptr[tl]; e < tv_ptr[tl + 1]; ++e)
            for (int o : vtiles[vperm[tv_col[e]]])
                if (col[o] >= 0) used[col[o]] = 1;
        int c = 0;
        while (c < ncol && used[c]) ++c;
        col[tl] = c;
        ncol = std::max(ncol, c + 1);
    }
    D.ntcolor = ncol;
    D.tcolor_ptr.assign(ncol + 1, 0);
    for (int tl = 0; tl < D.ntile; ++tl) D.tcolor_ptr[col[tl] + 1]++;
    for (int c = 0; c < ncol; ++c) D.tcolor_ptr[c + 1] += D.tcolor_ptr[c];
    std::vector<int32_t> lst(D.ntile), fill(D.tcolor_ptr.begin(), D.tcolor_ptr.end() - 1);
    for (int tl = 0; tl < D.ntile; ++tl) lst[fill[col[tl]]++] = tl;
    auto up = [&](const std::vector<int32_t> &v) {
        int32_t *p = (int32_t *)d.alloc(sizeof(int32_t) * std::max<size_t>(v.size(), 1));
        if (!v.empty()) HIPCHECK(hipMemcpyAsync(p, v.data(), sizeof(int32_t) * v.size(), hipMemcpyHostToDevice, d.stream));
        return p;
    };
    D.tcolor_tile = up(lst);
    if (D.sym) {
        // colour lists ascend in t, so the targets with t < (k + 1) * TL are a prefix
        std::vector<int4> blocks;
        D.sym_ptr.assign(1, 0);
        for (int kc = 0; kc < D.ntcolor; ++kc)
            for (int c = 0; c < D.ncolor; ++c) {
                const int32_t *cl = tcol_list.data() + D.color_ptr[c];
                const int n = D.color_ptr[c + 1] - D.color_ptr[c];
                for (int i = D.tcolor_ptr[kc]; i < D.tcolor_ptr[kc + 1]; ++i) {
                    const int k = lst[i];
                    const int nk = (int)(std::lower_bound(cl, cl + n, (k + 1) * TL) - cl);
                    for (int g = 0; g < nk; g += D.asm_group)
                        blocks.push_back(make_int4(k, D.color_ptr[c] + g, D.color_ptr[c] + std::min(g + D.asm_group, nk), 0));
                }
                D.sym_ptr.push_back(blocks.size());
            }
        D.sym_blocks = (int4 *)d.alloc(sizeof(int4) * std::max<size_t>(blocks.size(), 1));
        if (!blocks.empty())
            HIPCHECK(hipMemcpyAsync(D.sym_blocks, blocks.data(), sizeof(int4) * blocks.size(), hipMemcpyHostToDevice,
                                    d.stream));
        HIPCHECK(hipStreamSynchronize(d.stream));
    }
    D.tv_ptr = up(tv_ptr);
    D.tv_col = up(tv_col);
    D.tv_eptr = up(tv_eptr);
    D.te = up(te);
    D.vpos = up(vpos);
    D.vperm = up(vperm);
    HIPCHECK(hipStreamSynchronize(d.stream));   // host vectors go out of scope
}

template <typename R, typename S, int TILE>
static void assemble(DevMesh &d, S *A)
{
    Dense &D = *d.dense;
    const int V = d.hm.V, T = d.hm.T;
    AsmCoef<R> cf;
    const double kap = d.prm.kappa;
    cf.kappa = (R)kap;
    cf.kexp = sizeof(R) == 4 ? (R)(kap * 1.4426950408889634) : (R)kap;
    cf.k2 = (R)(kap * kap);
    const FormCoef &fm = d.fm;
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) { cf.aL[r][c] = (R)fm.aL[r][c]; cf.aY[r][c] = (R)fm.aY[r][c]; }
    const bool direct = fm.family == 0;   // FORM 0: K and V rows; FORM 1: K, V / D, T
    // FORM 0: the Laplace row.  FORM 1: 0 if every block has a Laplace term
    // (ratio form), 1 if none has (a Calderon preconditioner's part), 2 if
    // only some have (a combined field with one zero constant)
    bool all_laplace = true;
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) all_laplace &= fm.aL[r][c] != 0.0;
    const int lrow = direct ? laplace_row(fm) : yukawa_only(fm) ? 1 : all_laplace ? 0 : 2;
    if (!direct && lrow != 0) {
        cf.rK = cf.rV = cf.rD = cf.rT = R(0);
    } else if (!direct) {
        cf.rK = (R)(fm.aY[0][0] / fm.aL[0][0]);
        cf.rV = (R)(fm.aY[0][1] / fm.aL[0][1]);
        cf.rD = (R)(fm.aY[1][0] / fm.aL[1][0]);
        cf.rT = (R)(fm.aY[1][1] / fm.aL[1][1]);
    } else {
        cf.rK = cf.rV = cf.rD = cf.rT = R(0);
    }
    const R *stat = sizeof(R) == 4 ? (const R *)d.stat32 : (const R *)d.stat64;
    const size_t total = (size_t)D.n * D.ld;
    hipLaunchKernelGGL(k_fill<S>, dim3(4096), dim3(256), 0, d.stream, total, A);
    if constexpr (sizeof(R) == 4) {
        // one evaluation per unordered pair, then the transposes
        hipLaunchKernelGGL(k_fill<float>, dim3(4096), dim3(256), 0, d.stream, (size_t)D.n * D.Vp, D.C32);
        int li = 0;
        for (int kc = 0; kc < D.ntcolor; ++kc)
            for (int c = 0; c < D.ncolor; ++c, ++li) {
                const size_t b0 = D.sym_ptr[li], nb = D.sym_ptr[li + 1] - b0;
                if (nb == 0) continue;
#define ASM_SYM(F, L)                                                                                              \
    hipLaunchKernelGGL((k_assemble_tile<R, S, F, TILE, true, L>), dim3(nb), dim3(TILE), 0, d.stream, T, V, cf,      \
                       D.color_tri, 0, 0, nullptr, D.sym_blocks + b0, d.tri, stat, D.vpos, D.tv_ptr, D.tv_col,       \
                       D.tv_eptr, D.te, A, D.ld, D.Vp, D.C32, D.Vp)
                if (!direct && lrow == 0) ASM_SYM(1, 0);
                else if (!direct && lrow == 1) ASM_SYM(1, 1);
                else if (!direct) ASM_SYM(1, 2);
                else if (lrow == 0) ASM_SYM(0, 0);
                else ASM_SYM(0, 1);
#undef ASM_SYM
            }
        // V x V blocks of A (row block, column block): symmetric operators take
        // their own transpose, the others the transpose of C's rows.  Direct:
        // K_L, -V_L / -K_Y, eps V_Y.  Juffer: K, V / D, T.
        const int nt = (V + 63) / 64;
        const dim3 fg(nt, nt), fb(256);
        const size_t z = 0, Vs = (size_t)V;
        hipLaunchKernelGGL(k_sym_finish<1>, fg, fb, 0, d.stream, V, A, D.ld, z, z, D.C32, D.Vp, z);
        hipLaunchKernelGGL(k_sym_finish<0>, fg, fb, 0, d.stream, V, A, D.ld, z, D.Vp, D.C32, D.Vp, z);
        if (direct) {
            hipLaunchKernelGGL(k_sym_finish<1>, fg, fb, 0, d.stream, V, A, D.ld, Vs, z, D.C32, D.Vp, Vs);
            hipLaunchKernelGGL(k_sym_finish<0>, fg, fb, 0, d.stream, V, A, D.ld, Vs, D.Vp, D.C32, D.Vp, z);
        } else {
            hipLaunchKernelGGL(k_sym_finish<0>, fg, fb, 0, d.stream, V, A, D.ld, Vs, z, D.C32, D.Vp, z);
            hipLaunchKernelGGL(k_sym_finish<1>, fg, fb, 0, d.stream, V, A, D.ld, Vs, D.Vp, D.C32, D.Vp, Vs);
        }
    } else {
        // every ordered pair once, target colour x tile colour launches
        for (int kc = 0; kc < D.ntcolor; ++kc) {
            const int nk = D.tcolor_ptr[kc + 1] - D.tcolor_ptr[kc];
            if (nk == 0) continue;
            const int32_t *tl = D.tcolor_tile + D.tcolor_ptr[kc];
            for (int c = 0; c < D.ncolor; ++c) {
                const int nt = D.color_ptr[c + 1] - D.color_ptr[c];
                if (nt == 0) continue;
                const int32_t *tg = D.color_tri + D.color_ptr[c];
                const int grp = D.asm_group;
                dim3 grid(nk, (nt + grp - 1) / grp), block(TILE);
#define ASM_ALL(F, L)                                                                                              \
    hipLaunchKernelGGL((k_assemble_tile<R, S, F, TILE, false, L>), grid, block, 0, d.stream, T, V, cf, tg, nt, grp, \
                       tl, nullptr, d.tri, stat, D.vpos, D.tv_ptr, D.tv_col, D.tv_eptr, D.te, A, D.ld, D.Vp,       \
                       nullptr, (size_t)0)
                if (!direct && lrow == 0) ASM_ALL(1, 0);
                else if (!direct && lrow == 1) ASM_ALL(1, 1);
                else if (!direct) ASM_ALL(1, 2);
                else if (lrow == 0) ASM_ALL(0, 0);
                else ASM_ALL(0, 1);
#undef ASM_ALL
            }
        }
    }
    HIPCHECK(hipGetLastError());
}

void build_dense(DevMesh &d)
{
    const int V = d.hm.V;
    if (!d.dense) {
        if (!dense_fits(d)) fail(PB_E_NOMEM, "assembled far field does not fit the device memory budget");
        Dense *D = new Dense();
        d.dense = D;
        D->V = V;
        D->n = 2 * V;
        D->Vp = dense_vp(V);
        D->ld = dense_ld(V);
        std::vector<int32_t> lst;
        color_triangles(d.hm, D->color_ptr, lst);
        D->ncolor = (int)D->color_ptr.size() - 1;
        D->color_tri = (int32_t *)d.alloc(sizeof(int32_t) * lst.size());
        HIPCHECK(hipMemcpyAsync(D->color_tri, lst.data(), sizeof(int32_t) * lst.size(), hipMemcpyHostToDevice,
                                d.stream));
        const size_t total = (size_t)D->n * D->ld;
        if (d.prm.precision == PB_FP64) D->A64 = (double *)d.alloc(sizeof(double) * total);
        else D->A32 = (float *)d.alloc(sizeof(float) * total);
        if (d.prm.precision >= PB_MIXED_BF16) {
            D->A16 = (uint16_t *)d.alloc(sizeof(uint16_t) * total);
            D->kind16 = d.prm.precision == PB_MIXED_BF16 ? 1 : 2;
        }
        D->x32 = (float *)d.alloc(sizeof(float) * D->ld);
        D->x64 = (double *)d.alloc(sizeof(double) * D->ld);
        D->gpart = (double *)d.alloc(sizeof(double) * 2 * (size_t)D->n);
        D->tile = d.prm.precision == PB_FP64 ? 128 : 256;
        D->sym = d.prm.precision != PB_FP64;
        if (D->sym) {
            // n x Vp floats: the same bytes as the n x ld 16-bit copy, which is
            // written only after the assembly
            D->C32 = D->A16 ? (float *)D->A16 : (float *)d.alloc(sizeof(float) * (size_t)D->n * D->Vp);
        }
        build_tiles(d.hm, d, *D, lst);
        d.dense_vpos = D->vpos;
    }
    Dense &D = *d.dense;
    Profiler &pf = d.prof;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (pf.on(1)) {
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        HIPCHECK(hipEventRecord(e0, d.stream));
    }
    if (D.A64) assemble<double, double, 128>(d, D.A64);
    else assemble<float, float, 256>(d, D.A32);
    if (pf.on(1)) {
        HIPCHECK(hipEventRecord(e1, d.stream));
        // assembly work: 36 point pairs per ordered triangle pair, each evaluated once
        pf.record(1, e0, e1, 36.0 * (double)d.hm.T * (double)d.hm.T);
    }
    if (D.A16) {
        const size_t total = (size_t)D.n * D.ld;
        if (D.kind16 == 2) {
            const int nb = 1024;
            float *part = (float *)d.ztmp;   // 4 * nb floats fit in 2V doubles for V >= 2048; else temp
            float *tmp = nullptr;
            if ((size_t)4 * nb * sizeof(float) > sizeof(double) * 2 * (size_t)V) {
                tmp = (float *)d.alloc(sizeof(float) * 4 * nb);
                part = tmp;
            }
            hipLaunchKernelGGL(k_blockmax, dim3(nb), dim3(256), 0, d.stream, D.n, V, D.Vp, D.ld, D.A32, part);
            std::vector<float> h(4 * nb);
            HIPCHECK(hipMemcpyAsync(h.data(), part, sizeof(float) * h.size(), hipMemcpyDeviceToHost, d.stream));
            HIPCHECK(hipStreamSynchronize(d.stream));
            for (int b = 0; b < 4; ++b) {
                float m = 0.0f;
                for (int k = 0; k < nb; ++k) m = std::max(m, h[4 * k + b]);
                // largest |entry| scaled to about 2^14 (FP16 max 65504)
                int e = 0;
                if (m > 0.0f) { std::frexp(m, &e); e = 14 - e; }
                D.scale16[b] = std::ldexp(1.0f, e);
            }
        }
        hipLaunchKernelGGL(k_to16, dim3(8192), dim3(256), 0, d.stream, D.n, V, D.Vp, D.ld, D.kind16, D.scale16[0],
                           D.scale16[1], D.scale16[2], D.scale16[3], D.A32, D.A16);
        ++D.a16_version;   // a tiled copy for the batched GEMM is now stale
        (void)total;
    }
    HIPCHECK(hipGetLastError());
}

void destroy_dense(DevMesh &d)
{
    delete d.dense;   // device memory belongs to the handle's allocation list
    d.dense = nullptr;
}

// GEMV variants: 0 = one wavefront per row (four loads in flight per lane),
// 1 = 8-row tiles, 2 = 16-row tiles, 3-5 = split 4-, 8-, 16-row tiles.  The fastest for a given storage type and
// matrix is picked by timing them once on the real matrix (autotune cache).
template <typename S, typename ACC, int KIND>
static void gemv_launch(int variant, hipStream_t st, int n, int V, size_t Vp, size_t ld, const S *A, const ACC *x,
                        const float *inv, double *y, const DevCtl &ctl, double *part)
{
    if (variant >= 3) {
        // split variants: R = 4, 8, 16 rows per tile, two column blocks per tile
        const int R = variant == 3 ? 4 : variant == 4 ? 8 : 16;
        const int nunit = 2 * ((n + R - 1) / R);
        const int nwg = std::min((nunit + 3) / 4, 8192);
        ACC *pp = (ACC *)part;
        if (R == 4)
            hipLaunchKernelGGL((k_gemv_split<S, ACC, KIND, 4>), dim3(nwg), dim3(256), 0, st, n, Vp, ld, A, x, pp, ctl);
        else if (R == 8)
            hipLaunchKernelGGL((k_gemv_split<S, ACC, KIND, 8>), dim3(nwg), dim3(256), 0, st, n, Vp, ld, A, x, pp, ctl);
        else
            hipLaunchKernelGGL((k_gemv_split<S, ACC, KIND, 16>), dim3(nwg), dim3(256), 0, st, n, Vp, ld, A, x, pp,
                               ctl);
        hipLaunchKernelGGL((k_gemv_join<ACC, KIND>), dim3((n + 255) / 256), dim3(256), 0, st, n, V, inv[0], inv[1],
                           inv[2], inv[3], pp, y, ctl);
    } else if (variant == 0) {
        const int nwg = std::min(n / 4 + 1, 8192);
        hipLaunchKernelGGL((k_gemv<S, ACC, KIND>), dim3(nwg), dim3(256), 0, st, n, V, Vp, ld, A, x, inv[0], inv[1],
                           inv[2], inv[3], y, ctl);
    } else if (variant == 1) {
        const int nwg = std::min((n + 31) / 32, 8192);
        hipLaunchKernelGGL((k_gemv_tile<S, ACC, KIND, 8>), dim3(nwg), dim3(256), 0, st, n, V, Vp, ld, A, x, inv[0],
                           inv[1], inv[2], inv[3], y, ctl);
    } else {
        const int nwg = std::min((n + 63) / 64, 8192);
        hipLaunchKernelGGL((k_gemv_tile<S, ACC, KIND, 16>), dim3(nwg), dim3(256), 0, st, n, V, Vp, ld, A, x, inv[0],
                           inv[1], inv[2], inv[3], y, ctl);
    }
}

static void gemv_dispatch(Dense &D, int variant, hipStream_t st, bool lo, double *yfar, const DevCtl &ctl = DevCtl())
{
    const int V = D.V;
    float one[4] = {1.f, 1.f, 1.f, 1.f}, inv[4];
    for (int b = 0; b < 4; ++b) inv[b] = 1.f / D.scale16[b];
    if (D.A64) gemv_launch<double, double, 0>(variant, st, D.n, V, D.Vp, D.ld, D.A64, D.x64, one, yfar, ctl, D.gpart);
    else if (!lo) gemv_launch<float, double, 0>(variant, st, D.n, V, D.Vp, D.ld, D.A32, D.x64, one, yfar, ctl, D.gpart);
    else if (D.kind16 == 1)
        gemv_launch<uint16_t, float, 1>(variant, st, D.n, V, D.Vp, D.ld, D.A16, D.x32, one, yfar, ctl, D.gpart);
    else gemv_launch<uint16_t, float, 2>(variant, st, D.n, V, D.Vp, D.ld, D.A16, D.x32, inv, yfar, ctl, D.gpart);
}

int autotune_pick(const std::string &key, int nvariants, const std::function<void(int)> &run, hipStream_t st);
std::string size_class(long long n);

static int gemv_variant(DevMesh &d, bool lo)
{
    Dense &D = *d.dense;
    int &slot = lo ? D.gemv_lo : D.gemv_hi;
    if (slot >= 0) return slot;
    const char *kind = D.A64 ? "f64" : !lo ? "f32" : D.kind16 == 1 ? "bf16" : "fp16";
    const std::string key = std::string("gemv/") + kind + "/" + size_class(D.n);
    slot = autotune_pick(key, 6, [&](int v) { gemv_dispatch(D, v, d.stream, lo, d.yfar); }, d.stream);
    return slot;
}

// yfar (2V doubles, dense row order) = A_far x at the current operator level
void dense_apply(DevMesh &d, const double *x, double *yfar)
{
    Dense &D = *d.dense;
    const int V = d.hm.V;
    Profiler &pf = d.prof;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const dim3 gpad((unsigned)((D.ld + 255) / 256)), b256(256);
    const bool lo = D.level == 0 && D.A16;
    if (!lo) hipLaunchKernelGGL(k_pad_x<double>, gpad, b256, 0, d.stream, V, D.Vp, D.ld, D.vperm, x, D.x64, d.ctl);
    else hipLaunchKernelGGL(k_pad_x<float>, gpad, b256, 0, d.stream, V, D.Vp, D.ld, D.vperm, x, D.x32, d.ctl);
    const int variant = gemv_variant(d, lo);
    if (pf.on(0)) {
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        HIPCHECK(hipEventRecord(e0, d.stream));
    }
    gemv_dispatch(D, variant, d.stream, lo, yfar, d.ctl);
    if (pf.on(0)) {
        HIPCHECK(hipEventRecord(e1, d.stream));
        // algorithmic bytes: the stored 2V x 2V entries (padding excluded) + x and y
        const double ent = (double)D.n * (double)D.n;
        const double esz = D.A64 ? 8.0 : lo ? 2.0 : 4.0;
        pf.record(0, e0, e1, ent * esz + (double)D.n * (lo ? 4.0 : 8.0) + (double)D.n * 8.0);
    }
    HIPCHECK(hipGetLastError());
}

// Iterative refinement (north of the paper's plain solve): the outer residual
// uses the accurate operator (FP32-stored far field + FP64 near field, FP64
// vectors), each correction is solved by GMRES on the 16-bit far field.
int mixed_refinement_solve(DevMesh &d, const double *b, const double *pb, double *u, double *est, int *outer)
{
    (void)b;
    Dense &D = *d.dense;
    const int n = 2 * d.hm.V;
    hipStream_t s = d.stream;
    double *r = d.ytmp2, *c = d.ztmp2;
    double *kb = d.kry.kbuf;
    HIPCHECK(hipMemsetAsync(u, 0, sizeof(double) * n, s));
    kr_scale_copy(s, n, pb, 1.0, r);
    kr_dots(s, n, 1, pb, n, pb, d.red1);
    double nb2 = 0.0;
    HIPCHECK(hipMemcpyAsync(&nb2, d.red1, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const double nb = std::sqrt(nb2);
    int its = 0, k = 0;
    double rel = 1.0;
    const int max_outer = 30;
    for (k = 1; k <= max_outer; ++k) {
        double e_in = 0.0;
        D.level = 0;
        its += gmres_solve(d, r, c, std::max(d.opt.inner_tol, 0.5 * d.opt.tol * nb / std::max(rel * nb, 1e-300)),
                     std::min(d.opt.inner_max_iter, d.opt.max_iter), &e_in);
        D.level = 1;
        kr_axpy(s, n, 1.0, c, u);
        // r = pb - P^-1 A_hi u
        apply_operator(d, u, r, PB_APPLY_PRECOND, nullptr);
        kr_scale_copy(s, n, r, -1.0, r);
        kr_axpy(s, n, 1.0, pb, r);
        kr_dots(s, n, 1, r, n, r, d.red1);
        double r2 = 0.0;
        HIPCHECK(hipMemcpyAsync(&r2, d.red1, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        rel = nb > 0 ? std::sqrt(r2) / nb : 0.0;
        if (rel <= d.opt.tol || its >= d.opt.max_iter) break;
    }
    (void)kb;
    D.level = 1;
    *est = rel;
    *outer = std::min(k, max_outer);
    return its;
}

}  // namespace pbm
