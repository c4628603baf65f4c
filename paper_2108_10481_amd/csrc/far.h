// Far-field kernel pieces shared by the direct (k_far.hip) and the treecode
// (k_tree.hip) products: coefficients, math helpers, one source triangle's
// regular-rule sums against a target triangle.
#pragma once
#include "pbm_internal.h"

namespace pbm {

// ----------------------------------------------------------- math helpers
__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x)
{
    // hardware estimate refined by two Newton steps: y <- y (3 - x y^2) / 2
    double y = __builtin_amdgcn_rsq(x);
    double h = x * y;
    y = fma(0.5 * y, fma(-h, y, 1.0), y);
    h = x * y;
    y = fma(0.5 * y, fma(-h, y, 1.0), y);
    return y;
}
// exp(-kappa r) given kl = kappa * log2(e) (FP32) or kappa (FP64)
__device__ __forceinline__ float expneg(float kl, float r) { return __builtin_amdgcn_exp2f(-kl * r); }
__device__ __forceinline__ double expneg(double k, double r) { return exp(-k * r); }

template <typename R>
struct FarCoef {
    R kappa;   // screening
    R kexp;    // argument scale for expneg
    R k2;      // kappa^2
    // FORM 0 (direct formulations): coefficients of the Laplace row
    // (kL K_L + vL V_L) and of the Yukawa row (kY K_Y + vY V_Y); kYk = kY kappa
    R kL, vL, kY, vY, kYk;
    // FORM 1 (every other formulation) and FORM 3 (no Laplace term at all):
    // row 1 = cKL K_L + cKY K_Y + cVL V_L + cVY V_Y, row 2 = cTL (F_L d.n_t)
    // + cTY (F_Y d.n_t) + cDL D_L + cDY D_Y; the adjoint double layer's kernel
    // is -F d.n_t, so cTL, cTY carry that sign.  No coefficient divides
    // another: any of them may be zero.
    R cKL, cKY, cVL, cVY, cTL, cTY, cDL, cDY;
};

// one request of the batched far field: its mesh data, partial-sum buffer and
// coefficients
template <typename R>
struct FarReq {
    const int32_t *tri;
    const R *stat;
    const R *dyn;
    R *part;
    const int *skip;   // when set and nonzero (the request's GMRES stopped), its items do nothing
    FarCoef<R> cf;
    int T, chunk;
    int rt, nr;        // symmetric split (k_far_sym.hip): tiles per range, ranges; 0 if unused
};

// One source triangle against the six points of a target triangle: the
// regular-rule sums of k_far (the caller has excluded pairs sharing a vertex).
// st: the source's static record (entries 0..21 are read), sd: its dynamic
// record (entries 0..14); ot: the target's plane offset x . n_t (any of its
// points).  The points of a flat triangle lie in its plane, so with d =
// x_p - y_q the normal components d . n_s = x_p . n_s - o_s and d . n_t = o_t -
// y_q . n_t depend on one of the two points only and are formed once per
// point, not per point pair.
// SP: pointer type of the source records (a generic pointer, or one into the
// constant address space where the caller needs scalar loads)
// With d = x_p - y_q, r = |d|, e = exp(-kappa r), G_L = 1/r, G_Y = e/r,
// F_L = 1/r^3, F_Y = e (1 + kappa r)/r^3 = e (r^-3 + kappa r^-2): the direct
// form takes F d.n_s as g/r and e (g/r + kappa g) with g = (d.n_s)/r^2; the
// second-kind forms sum R3 = r^-3 and E = e (R3 + kappa r^-2) and apply the
// point's d.n once, so each row is a few fused multiply-adds on 1/r, e/r, R3
// and E with the source weights folded into per-point constants.
template <typename R, int FORM, typename SP = const R *>
__device__ __forceinline__ void far_source(const FarCoef<R> &cf, SP __restrict__ st,
                                           SP __restrict__ sd, const R (&tx)[6], const R (&ty)[6],
                                           const R (&tz)[6], R ot, R ntx, R nty, R ntz, R (&a1)[6],
                                           R (&a2)[6], R &W0, R &W1, R &W2)
{
    const R nsx = st[18], nsy = st[19], nsz = st[20], os = st[21];
    R dns[6];   // (x_p - y) . n_s
#pragma unroll
    for (int p = 0; p < 6; ++p) dns[p] = fma(tx[p], nsx, fma(ty[p], nsy, fma(tz[p], nsz, -os)));
    R gL = 0, gY = 0, k2nn = 0;
    R P[6];   // FORM 1, 3: row-1 double-layer sums of the target points before their factor dns[p]
#pragma unroll
    for (int p = 0; p < 6; ++p) P[p] = 0;
    if (FORM >= 1) k2nn = cf.cDY * cf.k2 * (ntx * nsx + nty * nsy + ntz * nsz);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const R yx = st[3 * q], yy = st[3 * q + 1], yz = st[3 * q + 2];
        const R b1 = sd[q], b2 = sd[6 + q];
        if (FORM == 0) {
            const R c1 = cf.kL * b1, c2 = cf.vL * b2, c3 = cf.kY * b1, c4 = cf.vY * b2, c3k = cf.kYk * b1;
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const R dx = tx[p] - yx, dy = ty[p] - yy, dz = tz[p] - yz;
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R ri = rsqrt_r(r2);
                const R g = dns[p] * (ri * ri);
                a1[p] = fma(ri, fma(c1, g, c2), a1[p]);
                const R e = expneg(cf.kexp, r2 * ri);
                a2[p] = fma(e, fma(ri, fma(c3, g, c4), c3k * g), a2[p]);
            }
        } else {
            const R dnt = fma(-yx, ntx, fma(-yy, nty, fma(-yz, ntz, ot)));   // (x - y_q) . n_t
            const R c1L = cf.cKL * b1, c1Y = cf.cKY * b1, c2L = cf.cVL * b2, c2Y = cf.cVY * b2;
            const R c3L = cf.cTL * b2, c3Y = cf.cTY * b2, kb1 = k2nn * b1;
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const R dx = tx[p] - yx, dy = ty[p] - yy, dz = tz[p] - yz;
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R ri = rsqrt_r(r2);
                const R ri2 = ri * ri;
                const R e = expneg(cf.kexp, r2 * ri);
                const R gy = e * ri;
                // F_L d.n = R3 (d.n), F_Y d.n = E (d.n) with R3 = r^-3 and E = e (1/r +
                // kappa) r^-2 = e (R3 + kappa r^-2); row 1's factor dns[p] is applied to its
                // sum P[p] once per source triangle
                const R R3 = ri * ri2;
                const R E = e * fma(cf.kappa, ri2, R3);
                if (FORM == 3) {
                    P[p] = fma(c1Y, E, P[p]);
                    a1[p] = fma(gy, c2Y, a1[p]);
                    a2[p] = fma(dnt * c3Y, E, fma(gy, kb1, a2[p]));
                } else {
                    P[p] = fma(c1Y, E, fma(c1L, R3, P[p]));
                    a1[p] = fma(ri, c2L, fma(gy, c2Y, a1[p]));
                    a2[p] = fma(dnt, fma(c3Y, E, c3L * R3), fma(gy, kb1, a2[p]));
                    gL = fma(R(rule_w(p) * rule_w(q)), ri, gL);
                }
                gY = fma(R(rule_w(p) * rule_w(q)), gy, gY);
            }
        }
    }
    if (FORM >= 1) {
#pragma unroll
        for (int p = 0; p < 6; ++p) a1[p] = fma(dns[p], P[p], a1[p]);
    }
    if (FORM >= 1) {
        const R gc = FORM == 3 ? cf.cDY * gY : cf.cDL * gL + cf.cDY * gY;
        W0 += gc * sd[12];
        W1 += gc * sd[13];
        W2 += gc * sd[14];
    }
}

// ------------------------------------------------- far-field finish pieces
// P1 test projection of one target triangle's 15 point sums (6 + 6 point
// sums, 3 curl sums) into its 6 outputs (3 hats x 2 rows, 1/4pi and |t|
// applied).  family 0: rows (Laplace, Yukawa), swapped when the Laplace row
// is row 2; family 1: row 2 gets D's curl part (its coefficients applied by
// the producers).
__device__ __forceinline__ void far_project(int t, int family, int swap, const double *__restrict__ geo,
                                            const double (&pot)[15], double *__restrict__ triout)
{
    const double *g = geo + (size_t)t * kGeo;
    const double sc = g[21] * kInv4Pi;
    for (int k = 0; k < 3; ++k) {
        double y1 = 0.0, y2 = 0.0;
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const double w = rule_w(p) * rule_bary(p, k);
            y1 += w * pot[p];
            y2 += w * pot[6 + p];
        }
        if (family == 1) y2 += g[22 + 3 * k] * pot[12] + g[23 + 3 * k] * pot[13] + g[24 + 3 * k] * pot[14];
        if (swap) { const double tmp = y1; y1 = y2; y2 = tmp; }
        triout[6 * (size_t)t + k] = sc * y1;
        triout[6 * (size_t)t + 3 + k] = sc * y2;
    }
}

// kFinishLanes lanes per target sum every kFinishLanes-th partial, then a
// fixed butterfly inside the lane group (one wavefront holds whole groups)
constexpr int kFinishLanes = 16;

// regular split: lane l of target t's group over the S chunk partials; every
// lane of the group calls it (ok: t < T, the same for the whole group)
template <typename R>
__device__ __forceinline__ void finish_group(int t, int l, bool ok, int T, int S, int family, int swap,
                                             const double *__restrict__ geo, const R *__restrict__ part,
                                             double *__restrict__ triout)
{
    double pot[15];
#pragma unroll
    for (int v = 0; v < 15; ++v) pot[v] = 0.0;
    if (ok)
        for (int c = l; c < S; c += kFinishLanes) {
            const R *o = part + ((size_t)c * T + t) * 16;
#pragma unroll
            for (int v = 0; v < 15; ++v) pot[v] += (double)o[v];
        }
#pragma unroll
    for (int v = 0; v < 15; ++v)
#pragma unroll
        for (int off = kFinishLanes / 2; off > 0; off >>= 1) pot[v] += __shfl_xor(pot[v], off);
    if (!ok || l != 0) return;
    far_project(t, family, swap, geo, pot, triout);
}

// symmetric split (ranges of rt tiles of 64 triangles, nr ranges): target t's
// nr + 1 slots, the target-side slots of the source ranges b >= c and the
// source-side slots of the target ranges a <= c (c its own range)
__device__ __forceinline__ void sym_finish_group(int t, int l, bool ok, int T, int rt, int nr, int family, int swap,
                                                 const double *__restrict__ geo, const float *__restrict__ part,
                                                 double *__restrict__ triout)
{
    double pot[15];
#pragma unroll
    for (int v = 0; v < 15; ++v) pot[v] = 0.0;
    if (ok) {
        const int c = (t / 64) / rt;
        const int nslot = (nr - c) + (c + 1);
        for (int k = l; k < nslot; k += kFinishLanes) {
            const int slot = k < nr - c ? c + k : nr + (k - (nr - c));
            const float *o = part + ((size_t)slot * T + t) * 16;
#pragma unroll
            for (int v = 0; v < 15; ++v) pot[v] += (double)o[v];
        }
    }
#pragma unroll
    for (int v = 0; v < 15; ++v)
#pragma unroll
        for (int off = kFinishLanes / 2; off > 0; off >>= 1) pot[v] += __shfl_xor(pot[v], off);
    if (!ok || l != 0) return;
    far_project(t, family, swap, geo, pot, triout);
}

// coefficients of the current operator fields; returns the kernel FORM
template <typename R>
inline int far_coef(const DevMesh &d, FarCoef<R> &cf)
{
    const double kap = d.prm.kappa;
    cf = FarCoef<R>{};
    cf.kappa = (R)kap;
    cf.kexp = (sizeof(R) == 4) ? (R)(kap * 1.4426950408889634) : (R)kap;
    cf.k2 = (R)(kap * kap);
    const FormCoef &f = d.fm;
    if (f.family == 0) {
        const int lr = laplace_row(f);
        cf.kL = (R)f.aL[lr][0]; cf.vL = (R)f.aL[lr][1];
        cf.kY = (R)f.aY[1 - lr][0]; cf.vY = (R)f.aY[1 - lr][1];
        cf.kYk = (R)(f.aY[1 - lr][0] * kap);
        return 0;
    }
    cf.cKL = (R)f.aL[0][0]; cf.cKY = (R)f.aY[0][0];
    cf.cVL = (R)f.aL[0][1]; cf.cVY = (R)f.aY[0][1];
    cf.cTL = (R)(-f.aL[1][1]); cf.cTY = (R)(-f.aY[1][1]);
    cf.cDL = (R)f.aL[1][0]; cf.cDY = (R)f.aY[1][0];
    return yukawa_only(f) ? 3 : 1;
}

// Coefficients of the symmetric kernel (k_far_sym.hip), whose coordinates are
// scaled by s = kappa log2(e) (kappa > 0): with x' = s x, 1/r = s / r', the
// normal-derivative factors (d.n)/r^2 = s (d'.n)/r'^2 and exp(-kappa r) =
// exp2(-r'), so the K- and T-type coefficients take s^2, the V-type ones, the
// kappa-weighted FORM 0 one and D's s, and kappa becomes kappa / s; kexp
// carries s.  For kappa = 0, s = 1 (coordinates and coefficients as they are,
// kappa 0).  Returns the kernel FORM.
inline int far_coef_sym(const DevMesh &d, FarCoef<float> &cf)
{
    FarCoef<double> c;
    const int form = far_coef(d, c);
    // unscreened meshes keep their coordinates (the kernel skips the exponential)
    const double s = d.prm.kappa > 0.0 ? d.prm.kappa * 1.4426950408889634 : 1.0, s2 = s * s;
    cf = FarCoef<float>{};
    cf.kappa = (float)(d.prm.kappa / s);
    cf.kexp = (float)s;
    cf.k2 = (float)c.k2;
    cf.kL = (float)(c.kL * s2); cf.vL = (float)(c.vL * s);
    cf.kY = (float)(c.kY * s2); cf.vY = (float)(c.vY * s); cf.kYk = (float)(c.kYk * s);
    cf.cKL = (float)(c.cKL * s2); cf.cKY = (float)(c.cKY * s2);
    cf.cVL = (float)(c.cVL * s); cf.cVY = (float)(c.cVY * s);
    cf.cTL = (float)(c.cTL * s2); cf.cTY = (float)(c.cTY * s2);
    cf.cDL = (float)(c.cDL * s); cf.cDY = (float)(c.cDY * s);
    return form;
}

}  // namespace pbm
