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
    // FORM 0: coefficients of the Laplace row (kL K_L + vL V_L) and of the
    // Yukawa row (kY K_Y + vY V_Y)
    R kL, vL, kY, vY;
    // FORM 1, 2: factors aL of the K and V blocks, -aL of the T block, aY of D's
    // kappa^2 term; ratios aY / aL of the K, V, D, T blocks
    R aK, aV, aT, aDY, rK, rV, rD, rT;
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
};

// One source triangle against the six points of a target triangle: the
// regular-rule sums of k_far (the caller has excluded pairs sharing a vertex).
// st: the source's static record (entries 0..26 are read), sd: its dynamic
// record (entries 0..14).
// SP: pointer type of the source records (a generic pointer, or one into the
// constant address space where the caller needs scalar loads)
template <typename R, int FORM, typename SP = const R *>
__device__ __forceinline__ void far_source(const FarCoef<R> &cf, SP __restrict__ st,
                                           SP __restrict__ sd, const R (&tx)[6], const R (&ty)[6],
                                           const R (&tz)[6], const R (&xnt)[6], R ntx, R nty, R ntz, R (&a1)[6],
                                           R (&a2)[6], R &W0, R &W1, R &W2)
{
    const R nsx = st[18], nsy = st[19], nsz = st[20];
    R xns[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) xns[p] = tx[p] * nsx + ty[p] * nsy + tz[p] * nsz;
    R g = 0, k2nn = 0;
    if (FORM >= 1) k2nn = cf.aDY * cf.k2 * (ntx * nsx + nty * nsy + ntz * nsz);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const R yx = st[3 * q], yy = st[3 * q + 1], yz = st[3 * q + 2];
        const R yns = st[21 + q];
        const R b1 = sd[q], b2 = sd[6 + q];
        R ynt = 0, kb1 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0;
        if (FORM == 0) { c1 = cf.kL * b1; c2 = cf.vL * b2; c3 = cf.kY * b1; c4 = cf.vY * b2; }
        else { ynt = yx * ntx + yy * nty + yz * ntz; kb1 = k2nn * b1; c1 = cf.aK * b1; c2 = cf.aV * b2; c3 = cf.aT * b2; }
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const R dx = tx[p] - yx, dy = ty[p] - yy, dz = tz[p] - yz;
            const R r2 = dx * dx + dy * dy + dz * dz;
            const R ri = rsqrt_r(r2);
            const R r = r2 * ri;
            const R e = expneg(cf.kexp, r);
            const R ri3 = ri * ri * ri;
            const R dns = xns[p] - yns;
            const R tt = cf.kappa * r + R(1);
            if (FORM == 0) {
                const R fl = dns * ri3;
                a1[p] += fl * c1 + ri * c2;
                a2[p] += e * (fl * tt * c3 + ri * c4);
            } else if (FORM == 3) {
                const R fy = e * tt * ri3;
                const R gy = e * ri;
                a1[p] += fy * dns * c1 + gy * c2;
                a2[p] += fy * (xnt[p] - ynt) * c3 + kb1 * gy;
                g += R(rule_w(p) * rule_w(q)) * gy;
            } else {
                const R fy = e * tt * ri3;
                const R gy = e * ri;
                const R gv = ri + cf.rV * gy;
                const R dnt = xnt[p] - ynt;
                a1[p] += (ri3 + cf.rK * fy) * dns * c1 + gv * c2;
                a2[p] += (ri3 + cf.rT * fy) * dnt * c3 + kb1 * gy;
                g += R(rule_w(p) * rule_w(q)) * (FORM == 1 ? gv : ri + cf.rD * gy);
            }
        }
    }
    if (FORM >= 1) {
        W0 += g * sd[12];
        W1 += g * sd[13];
        W2 += g * sd[14];
    }
}

// coefficients of the current operator fields; returns the kernel FORM
template <typename R>
inline int far_coef(const DevMesh &d, FarCoef<R> &cf)
{
    const double kap = d.prm.kappa;
    cf.kappa = (R)kap;
    cf.kexp = (sizeof(R) == 4) ? (R)(kap * 1.4426950408889634) : (R)kap;
    cf.k2 = (R)(kap * kap);
    const FormCoef &f = d.fm;
    int form = 0;
    if (f.family == 0) {
        const int lr = laplace_row(f);
        cf.kL = (R)f.aL[lr][0]; cf.vL = (R)f.aL[lr][1];
        cf.kY = (R)f.aY[1 - lr][0]; cf.vY = (R)f.aY[1 - lr][1];
    } else if (yukawa_only(f)) {
        cf.aK = (R)f.aY[0][0]; cf.aV = (R)f.aY[0][1]; cf.aT = (R)(-f.aY[1][1]); cf.aDY = (R)f.aY[1][0];
        cf.rK = cf.rV = cf.rD = cf.rT = R(0);
        form = 3;
    } else {
        // the adjoint double layer's kernel is -F d.n_t: its factor carries the sign
        cf.aK = (R)f.aL[0][0]; cf.aV = (R)f.aL[0][1]; cf.aT = (R)(-f.aL[1][1]); cf.aDY = (R)f.aY[1][0];
        const double rV = f.aY[0][1] / f.aL[0][1], rD = f.aY[1][0] / f.aL[1][0];
        cf.rK = (R)(f.aY[0][0] / f.aL[0][0]);
        cf.rV = (R)rV;
        cf.rD = (R)rD;
        cf.rT = (R)(f.aY[1][1] / f.aL[1][1]);
        form = rD == rV ? 1 : 2;
    }
    return form;
}

}  // namespace pbm
