// Near field: Sauter-Schwab quadrature of every ordered triangle pair that
// shares a vertex (Numerical discretization; S. Sauter and C. Schwab, Boundary
// Element Methods, Springer 2011, sec. 5.2), assembly of the four near-field
// vertex blocks of the chosen formulation (mass terms included), and the
// block-diagonal preconditioner (Preconditioning, Algebraic preconditioners).
// Everything here is FP64 in every precision mode.
#include <mutex>

#include "pbm_internal.h"

namespace pbm {

constexpr int kMaxGL = 16;
__constant__ double c_gl_x[kMaxGL + 1][kMaxGL];
__constant__ double c_gl_w[kMaxGL + 1][kMaxGL];

void upload_gauss_tables()
{
    static std::once_flag once;
    std::call_once(once, [] {
        static double hx[kMaxGL + 1][kMaxGL] = {}, hw[kMaxGL + 1][kMaxGL] = {};
        for (int n = 1; n <= kMaxGL; ++n) gauss_legendre01(n, hx[n], hw[n]);
        HIPCHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_x), hx, sizeof(hx)));
        HIPCHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_w), hw, sizeof(hw)));
    });
}

// Reference triangle {0 <= u2 <= u1 <= 1}, chi(u) = P0 + u1 (P1 - P0) + u2 (P2 - P1),
// barycentrics (1 - u1, u1 - u2, u2), surface element 2|T| du.  The unit
// hypercube (xi, a, b, c) is split into regions mapped onto the pair of
// reference triangles with Jacobians that cancel the 1/r singularity.
struct SSPoint { double u1, u2, v1, v2, jac; };

__device__ inline SSPoint ss_map(int cas, int r, double xi, double a, double b, double c)
{
    SSPoint m;
    if (cas == 3) {          // identical triangles: 6 regions
        m.jac = xi * xi * xi * a * a * b;
        switch (r) {
        case 0: m.u1 = xi; m.u2 = xi * (1 - a + a * b); m.v1 = xi * (1 - a * b * c); m.v2 = xi * (1 - a); break;
        case 1: m.u1 = xi * (1 - a * b * c); m.u2 = xi * (1 - a); m.v1 = xi; m.v2 = xi * (1 - a + a * b); break;
        case 2: m.u1 = xi; m.u2 = xi * a * (1 - b + b * c); m.v1 = xi * (1 - a * b); m.v2 = xi * a * (1 - b); break;
        case 3: m.u1 = xi * (1 - a * b); m.u2 = xi * a * (1 - b); m.v1 = xi; m.v2 = xi * a * (1 - b + b * c); break;
        case 4: m.u1 = xi * (1 - a * b * c); m.u2 = xi * a * (1 - b * c); m.v1 = xi; m.v2 = xi * a * (1 - b); break;
        default: m.u1 = xi; m.u2 = xi * a * (1 - b); m.v1 = xi * (1 - a * b * c); m.v2 = xi * a * (1 - b * c); break;
        }
    } else if (cas == 2) {   // common edge P0-P1 (u2 = 0 on both): 5 regions
        m.jac = xi * xi * xi * a * a * (r == 0 ? 1.0 : b);
        switch (r) {
        case 0: m.u1 = xi; m.u2 = xi * a * c; m.v1 = xi * (1 - a * b); m.v2 = xi * a * (1 - b); break;
        case 1: m.u1 = xi; m.u2 = xi * a; m.v1 = xi * (1 - a * b * c); m.v2 = xi * a * b * (1 - c); break;
        case 2: m.u1 = xi * (1 - a * b); m.u2 = xi * a * (1 - b); m.v1 = xi; m.v2 = xi * a * b * c; break;
        case 3: m.u1 = xi * (1 - a * b * c); m.u2 = xi * a * b * (1 - c); m.v1 = xi; m.v2 = xi * a; break;
        default: m.u1 = xi * (1 - a * b * c); m.u2 = xi * a * (1 - b * c); m.v1 = xi; m.v2 = xi * a * b; break;
        }
    } else {                 // common vertex P0: 2 regions
        m.jac = xi * xi * xi * b;
        if (r == 0) { m.u1 = xi; m.u2 = xi * a; m.v1 = xi * b; m.v2 = xi * b * c; }
        else { m.u1 = xi * b; m.u2 = xi * b * c; m.v1 = xi; m.v2 = xi * a; }
    }
    return m;
}

// Local vertex order: shared vertices first.  Identical: stored order.  Edge:
// the test triangle is rotated so the shared edge is (0,1) in its own cyclic
// order; the trial triangle lists the same two vertices in the same order
// then its free vertex.  Vertex: both rotated so the shared vertex is first.
// The stored (outward) normals are kept whatever the local order.
__device__ inline int ss_order(int t, int s, const int *tv, const int *sv, int *pt, int *ps)
{
    pt[0] = ps[0] = 0; pt[1] = ps[1] = 1; pt[2] = ps[2] = 2;
    if (t == s) return 3;
    int ns = 0, kt[3] = {0, 0, 0}, ks[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l)
            if (tv[k] == sv[l]) { kt[ns] = k; ks[ns] = l; ++ns; }
    if (ns == 2) {
        int k0 = kt[0], k1 = kt[1];
        if ((k0 + 1) % 3 != k1) { int tmp = k0; k0 = k1; k1 = tmp; }
        pt[0] = k0; pt[1] = k1; pt[2] = 3 - k0 - k1;
        for (int l = 0; l < 3; ++l) {
            if (sv[l] == tv[k0]) ps[0] = l;
            if (sv[l] == tv[k1]) ps[1] = l;
        }
        ps[2] = 3 - ps[0] - ps[1];
    } else if (ns == 1) {
        for (int m = 0; m < 3; ++m) { pt[m] = (kt[0] + m) % 3; ps[m] = (ks[0] + m) % 3; }
    }
    return ns;
}

// 1/sqrt(x) in FP64: hardware estimate and two Newton steps
__device__ inline double rsq64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double h = x * y;
    y = fma(0.5 * y, fma(-h, y, 1.0), y);
    h = x * y;
    y = fma(0.5 * y, fma(-h, y, 1.0), y);
    return y;
}

// LANES lanes per ordered pair (t, s), 64 / LANES pairs per wavefront, all of
// one case (CASE shared vertices, so the region of a Gauss point is uniform
// across the wavefront).  Lanes stride over the regions x N^4 Gauss points;
// each lane accumulates the 4 x 3 x 3 products in FP64, then a butterfly
// reduction inside the lane group.  out[36 p + 9 op + 3 a + b], op = V_L, K_L,
// V_Y, K_Y; a, b local vertex ids of t and s in stored order; p = idx[item].
template <int N, int CASE, int LANES>
__global__ __launch_bounds__(256) void k_near_ss(int count, const int32_t *__restrict__ idx,
                                                 const int32_t *__restrict__ pair_t, const int32_t *__restrict__ pair_s,
                                                 const int32_t *__restrict__ tri, const double *__restrict__ xyz,
                                                 const double *__restrict__ geo, double kappa, double *__restrict__ out)
{
    constexpr int G = 64 / LANES;
    const int lane = threadIdx.x & 63, sub = lane % LANES;
    const int first = (blockIdx.x * 4 + (threadIdx.x >> 6)) * G;
    if (first >= count) return;   // whole wavefront idle
    const int item = first + lane / LANES;
    const bool active = item < count;   // idle groups repeat the last pair and do not store
    const int p = idx[active ? item : count - 1];
    const int t = pair_t[p], s = pair_s[p];
    int tv[3], sv[3];
    for (int k = 0; k < 3; ++k) { tv[k] = tri[3 * t + k]; sv[k] = tri[3 * s + k]; }
    int pt[3], ps[3];
    (void)ss_order(t, s, tv, sv, pt, ps);
    double P[3][3], Q[3][3];
    for (int m = 0; m < 3; ++m)
        for (int c = 0; c < 3; ++c) {
            P[m][c] = xyz[3 * tv[pt[m]] + c];
            Q[m][c] = xyz[3 * sv[ps[m]] + c];
        }
    const double *gs = geo + (size_t)s * kGeo;
    const double nsx = gs[18], nsy = gs[19], nsz = gs[20];
    const double at = geo[(size_t)t * kGeo + 21], as = gs[21];
    double e1[3], e2[3], f1[3], f2[3];
    for (int c = 0; c < 3; ++c) {
        e1[c] = P[1][c] - P[0][c]; e2[c] = P[2][c] - P[1][c];
        f1[c] = Q[1][c] - Q[0][c]; f2[c] = Q[2][c] - Q[1][c];
    }
    constexpr int N4 = N * N * N * N;
    constexpr int nreg = CASE == 3 ? 6 : CASE == 2 ? 5 : 2;
    constexpr int npts = nreg * N4;
    double acc[36];
#pragma unroll
    for (int v = 0; v < 36; ++v) acc[v] = 0.0;
    for (int ix = sub; ix < npts; ix += LANES) {
        const int r = ix / N4;
        int rem = ix - r * N4;
        const int i0 = rem / (N * N * N); rem -= i0 * N * N * N;
        const int i1 = rem / (N * N); rem -= i1 * N * N;
        const int i2 = rem / N;
        const int i3 = rem - i2 * N;
        const SSPoint m = ss_map(CASE, r, c_gl_x[N][i0], c_gl_x[N][i1], c_gl_x[N][i2], c_gl_x[N][i3]);
        const double W = c_gl_w[N][i0] * c_gl_w[N][i1] * c_gl_w[N][i2] * c_gl_w[N][i3] * m.jac;
        const double dx = (P[0][0] + m.u1 * e1[0] + m.u2 * e2[0]) - (Q[0][0] + m.v1 * f1[0] + m.v2 * f2[0]);
        const double dy = (P[0][1] + m.u1 * e1[1] + m.u2 * e2[1]) - (Q[0][1] + m.v1 * f1[1] + m.v2 * f2[1]);
        const double dz = (P[0][2] + m.u1 * e1[2] + m.u2 * e2[2]) - (Q[0][2] + m.v1 * f1[2] + m.v2 * f2[2]);
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double ri = rsq64(r2);
        const double rr = r2 * ri;
        const double ek = exp(-kappa * rr);
        const double dn = dx * nsx + dy * nsy + dz * nsz;
        const double ri3 = ri * ri * ri;
        const double gL = ri, fL = dn * ri3, gY = ek * ri, fY = ek * (1.0 + kappa * rr) * dn * ri3;
        const double lx[3] = {1.0 - m.u1, m.u1 - m.u2, m.u2};
        const double ly[3] = {1.0 - m.v1, m.v1 - m.v2, m.v2};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double wk = W * lx[k];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const double bb = wk * ly[l];
                acc[3 * k + l] += bb * gL;
                acc[9 + 3 * k + l] += bb * fL;
                acc[18 + 3 * k + l] += bb * gY;
                acc[27 + 3 * k + l] += bb * fY;
            }
        }
    }
#pragma unroll
    for (int v = 0; v < 36; ++v) {
        double x = acc[v];
#pragma unroll
        for (int off = LANES / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
        acc[v] = x;
    }
    if (active && sub == 0) {
        const double scale = at * as / kPi;   // (2|t|)(2|s|) / (4 pi)
        double *o = out + (size_t)p * 36;
#pragma unroll
        for (int op = 0; op < 4; ++op)
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int l = 0; l < 3; ++l) o[9 * op + 3 * pt[k] + ps[l]] = acc[9 * op + 3 * k + l] * scale;
    }
}

// Pair indices 0..n-1 grouped by the number of shared vertices: identical,
// then edge, then vertex pairs; count[c] pairs share c vertices.
void ss_group(const std::vector<int32_t> &tri, int n, const int32_t *t, const int32_t *s, std::vector<int32_t> &idx,
              int count[4])
{
    std::vector<int32_t> by[4];
    for (int i = 0; i < n; ++i) {
        int c = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) c += tri[3 * t[i] + a] == tri[3 * s[i] + b];
        if (t[i] == s[i]) c = 3;
        by[std::min(c, 3)].push_back(i);
    }
    idx.clear();
    for (int c = 3; c >= 1; --c) idx.insert(idx.end(), by[c].begin(), by[c].end());
    for (int c = 0; c < 4; ++c) count[c] = (int)by[c].size();
    if (count[0]) fail(PB_E_INVALID_ARG, "pair does not share a vertex");
}

template <int N>
static void launch_ss_n(hipStream_t st, const int count[4], const int32_t *idx, const int32_t *pt, const int32_t *ps,
                        const DevMesh &d, double kap, double *out)
{
    const int n3 = count[3], n2 = count[2], n1 = count[1];
    // wavefronts of 64 / LANES pairs, 4 wavefronts per block
    auto grid = [](int n, int lanes) { const int per = 4 * (64 / lanes); return dim3((n + per - 1) / per); };
    if (n3)
        hipLaunchKernelGGL((k_near_ss<N, 3, 64>), grid(n3, 64), dim3(256), 0, st, n3, idx, pt, ps, d.tri, d.xyz, d.geo,
                           kap, out);
    if (n2)
        hipLaunchKernelGGL((k_near_ss<N, 2, 32>), grid(n2, 32), dim3(256), 0, st, n2, idx + n3, pt, ps, d.tri, d.xyz,
                           d.geo, kap, out);
    if (n1)
        hipLaunchKernelGGL((k_near_ss<N, 1, 16>), grid(n1, 16), dim3(256), 0, st, n1, idx + n3 + n2, pt, ps, d.tri,
                           d.xyz, d.geo, kap, out);
}

static void launch_ss(DevMesh &d, const int count[4], const int32_t *idx, const int32_t *pt, const int32_t *ps,
                      double *out, int order)
{
    if (count[1] + count[2] + count[3] == 0) return;
    upload_gauss_tables();
    const double kap = d.prm.kappa;
    switch (order) {
#define SS_CASE(n) \
    case n: launch_ss_n<n>(d.stream, count, idx, pt, ps, d, kap, out); break;
        SS_CASE(1) SS_CASE(2) SS_CASE(3) SS_CASE(4) SS_CASE(5) SS_CASE(6) SS_CASE(7) SS_CASE(8)
#undef SS_CASE
    default: fail(PB_E_INVALID_ARG, "singular_order must be in [1, 8]");
    }
    HIPCHECK(hipGetLastError());
}

void launch_near_field(DevMesh &d)
{
    launch_ss(d, d.ss_count, d.ss_idx, d.pair_t, d.pair_s, d.pairblk, d.opt.singular_order);
}

void launch_pair_blocks_subset(DevMesh &d, int n, const int32_t *t_sorted, const int32_t *s_sorted,
                               const int32_t *idx, const int count[4], double *out)
{
    (void)n;
    launch_ss(d, count, idx, t_sorted, s_sorted, out, d.opt.singular_order);
}

// Near-field vertex blocks (mass terms included) of the chosen formulation.
// One thread per nonzero slot (i, j) sums, in the fixed order row i visits
// them, the contributions of the near pairs (t containing i as local vertex k,
// s containing j as local vertex l); the slot is owned by one thread, so there
// is no atomic and the result is deterministic.
struct NearCoef {
    double kappa;
    FormCoef f;                // the formulation's block coefficients
};

// per pair: sum of its 3 x 3 V_L and V_Y entries (the hypersingular curl part)
__global__ void k_pair_sums(int64_t npair, const double *__restrict__ blk, double *__restrict__ sums)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npair) return;
    const double *B = blk + p * 36;
    double SL = 0.0, SY = 0.0;
    for (int a = 0; a < 9; ++a) { SL += B[a]; SY += B[18 + a]; }
    sums[2 * p] = SL;
    sums[2 * p + 1] = SY;
}

__global__ void k_near_slots(int64_t nnz, NearCoef cf, const int32_t *__restrict__ slot_ptr,
                             const uint32_t *__restrict__ slot_code, const int32_t *__restrict__ pair_t,
                             const int32_t *__restrict__ pair_s, const int32_t *__restrict__ pair_rev,
                             const double *__restrict__ geo, const double *__restrict__ blk,
                             const double *__restrict__ sums, double *__restrict__ N, double *__restrict__ Mval)
{
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= nnz) return;
    double n11 = 0.0, n12 = 0.0, n21 = 0.0, n22 = 0.0, mass = 0.0;
    for (int c = slot_ptr[slot]; c < slot_ptr[slot + 1]; ++c) {
        const uint32_t code = slot_code[c];
        const int p = (int)(code >> 4), k = (code >> 2) & 3, l = code & 3;
        const int t = pair_t[p], s = pair_s[p];
        const double *B = blk + (size_t)p * 36;
        const double *gt = geo + (size_t)t * kGeo;
        const double vL = B[3 * k + l], kL = B[9 + 3 * k + l];
        const double vY = B[18 + 3 * k + l], kY = B[27 + 3 * k + l];
        const double mss = (s == t) ? gt[21] / 12.0 * (k == l ? 2.0 : 1.0) : 0.0;
        mass += mss;
        const FormCoef &f = cf.f;
        // row 1: K and V (Dirichlet trace equations)
        n11 += f.mass[0][0] * mss + f.aL[0][0] * kL + f.aY[0][0] * kY;
        n12 += f.mass[0][1] * mss + f.aL[0][1] * vL + f.aY[0][1] * vY;
        if (f.family == 0) {
            n21 += f.mass[1][0] * mss + f.aL[1][0] * kL + f.aY[1][0] * kY;
            n22 += f.mass[1][1] * mss + f.aL[1][1] * vL + f.aY[1][1] * vY;
        } else {                                  // row 2: D and T (Neumann trace equations)
            const double *gs = geo + (size_t)s * kGeo;
            const double *R = blk + (size_t)pair_rev[p] * 36;
            const double nn = gt[18] * gs[18] + gt[19] * gs[19] + gt[20] * gs[20];
            const double cc = gt[22 + 3 * k] * gs[22 + 3 * l] + gt[23 + 3 * k] * gs[23 + 3 * l] +
                              gt[24 + 3 * k] * gs[24 + 3 * l];
            // D: curl_k . curl_l V + kappa^2 (n_t . n_s) V, by parts; T = K^T
            const double dL = cc * sums[2 * (size_t)p];
            const double dY = cc * sums[2 * (size_t)p + 1] + cf.kappa * cf.kappa * nn * vY;
            const double tL = R[9 + 3 * l + k], tY = R[27 + 3 * l + k];
            n21 += f.mass[1][0] * mss + f.aL[1][0] * dL + f.aY[1][0] * dY;
            n22 += f.mass[1][1] * mss + f.aL[1][1] * tL + f.aY[1][1] * tY;
        }
    }
    N[slot] = n11;
    N[nnz + slot] = n12;
    N[2 * nnz + slot] = n21;
    N[3 * nnz + slot] = n22;
    if (Mval) Mval[slot] = mass;
}

// per-vertex analytic inverse of [[A11_ii, A12_ii], [A21_ii, A22_ii]]; every
// diagonal entry comes from pairs sharing vertex i, i.e. from the near field.
__global__ void k_block_diag(int V, int enabled, const int32_t *__restrict__ diag, const double *__restrict__ N,
                             int64_t nnz, double *__restrict__ pinv)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    double *o = pinv + 4 * (size_t)i;
    if (!enabled) { o[0] = 1.0; o[1] = 0.0; o[2] = 0.0; o[3] = 1.0; return; }
    const int sl = diag[i];
    const double a = N[sl], b = N[nnz + sl], c = N[2 * nnz + sl], e = N[3 * nnz + sl];
    const double det = a * e - b * c;
    o[0] = e / det; o[1] = -b / det; o[2] = -c / det; o[3] = a / det;
}

// ------------------------------------------------ mass preconditioners
// blockdiag(aM, bM)^-1 (Eqs. prec:mass, prec:mass:scaled), M the P1 mass
// matrix.  M^-1 is applied as a fixed-degree Chebyshev iteration on the
// Jacobi-scaled mass matrix D^-1 M (Y. Saad, Iterative Methods for Sparse
// Linear Systems, 2nd ed., sec. 12.3): for P1 triangles every element's
// generalised eigenvalues against its diagonal are 2, 1/2, 1/2, so the
// spectrum of D^-1 M lies in [1/2, 2] on any mesh (element-by-element bound)
// and each step reduces the error by 1/3 at least.  kChebSteps steps give a
// fixed linear operator within 2 (1/3)^20 = 6e-10 of M^-1; no reductions, so
// it is capturable like every other part of an iteration.
constexpr int kChebSteps = 20;
constexpr double kChebTheta = 1.25, kChebDelta = 0.75;   // centre and half-width of [1/2, 2]

__global__ void k_mass_diag(int V, const int32_t *__restrict__ diag, const double *__restrict__ Mval,
                            double *__restrict__ Mdinv)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < V) Mdinv[i] = 1.0 / Mval[diag[i]];
}

// systems s < nvec of 2V entries (both halves use M); x = 0, r = in, d = D^-1 r / theta
__global__ void k_cheb_init(int V, const double *__restrict__ Mdinv, const double *__restrict__ in,
                            double *__restrict__ x, double *__restrict__ r, double *__restrict__ dv, DevCtl ctl)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * V || ctl_skip(ctl)) return;
    const size_t o = (size_t)blockIdx.y * 2 * V + e;
    const int i = e < V ? e : e - V;
    const double v = in[o];
    x[o] = 0.0;
    r[o] = v;
    dv[o] = v * Mdinv[i] * (1.0 / kChebTheta);
}

// x += d; r -= M d; d' = c1 d + c2 D^-1 r
__global__ void k_cheb_step(int V, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                            const double *__restrict__ Mval, const double *__restrict__ Mdinv, double c1, double c2,
                            double *__restrict__ x, double *__restrict__ r, const double *__restrict__ dv,
                            double *__restrict__ dn, DevCtl ctl)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * V || ctl_skip(ctl)) return;
    const size_t base = (size_t)blockIdx.y * 2 * V + (e < V ? 0 : V);
    const int i = e < V ? e : e - V;
    const size_t o = base + i;
    double md = 0.0;
    for (int sl = row_ptr[i]; sl < row_ptr[i + 1]; ++sl) md += Mval[sl] * dv[base + col[sl]];
    const double rv = r[o] - md;
    x[o] += dv[o];
    r[o] = rv;
    dn[o] = c1 * dv[o] + c2 * Mdinv[i] * rv;
}

// out = (x + d) scaled by 1/a (first half) and 1/b (second half)
__global__ void k_cheb_final(int V, double sa, double sb, const double *__restrict__ x, const double *__restrict__ dv,
                             double *__restrict__ out, DevCtl ctl)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * V || ctl_skip(ctl)) return;
    const size_t o = (size_t)blockIdx.y * 2 * V + e;
    out[o + ctl_off(ctl)] = (x[o] + dv[o]) * (e < V ? sa : sb);
}

void mass_precond(DevMesh &d, int nvec, const double *in, double *out, const DevCtl &ctl)
{
    double sa = 1.0, sb = 1.0;
    if (d.prm.preconditioner == PB_SCALED_MASS) {
        sa = 1.0 / (1.0 + d.prm.eps_out / d.prm.eps_in);
        sb = 1.0 / (1.0 + d.prm.eps_in / d.prm.eps_out);
    }
    mass_precond(d, nvec, in, out, ctl, sa, sb);
}

void mass_precond(DevMesh &d, int nvec, const double *in, double *out, const DevCtl &ctl, double sa, double sb)
{
    const int V = d.hm.V;
    if (nvec < 1 || nvec > kMassBatch) fail(PB_E_INVALID_ARG, "mass preconditioner batch size");
    const size_t n = 2 * (size_t)V * kMassBatch;
    double *x = d.cheb, *r = d.cheb + n, *dv[2] = {d.cheb + 2 * n, d.cheb + 3 * n};
    const dim3 g((unsigned)((2 * V + 255) / 256), (unsigned)nvec), b(256);
    hipLaunchKernelGGL(k_cheb_init, g, b, 0, d.stream, V, d.Mdinv, in, x, r, dv[0], ctl);
    const double s1 = kChebTheta / kChebDelta;
    double rho = 1.0 / s1;
    int cur = 0;
    for (int k = 1; k < kChebSteps; ++k, cur ^= 1) {
        const double rn = 1.0 / (2.0 * s1 - rho);
        hipLaunchKernelGGL(k_cheb_step, g, b, 0, d.stream, V, d.row_ptr, d.col, d.Mval, d.Mdinv, rn * rho,
                           2.0 * rn / kChebDelta, x, r, dv[cur], dv[cur ^ 1], ctl);
        rho = rn;
    }
    hipLaunchKernelGGL(k_cheb_final, g, b, 0, d.stream, V, sa, sb, x, dv[cur], out, ctl);
    HIPCHECK(hipGetLastError());
}

void launch_near_values(DevMesh &d, const FormCoef &f, const double *blk, const double *sums, double *N,
                        double *Mval)
{
    NearCoef cf;
    cf.kappa = d.prm.kappa;
    cf.f = f;
    const int64_t nnz = d.nnz();
    hipLaunchKernelGGL(k_near_slots, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, d.stream, nnz, cf,
                       d.slot_ptr, d.slot_code, d.pair_t, d.pair_s, d.pair_rev, d.geo, blk, sums, N, Mval);
    HIPCHECK(hipGetLastError());
}

void launch_near_field_fast(DevMesh &d)
{
    launch_ss(d, d.ss_count, d.ss_idx, d.pair_t, d.pair_s, d.pairblkP, calderon_fast_order(d.opt));
    const int64_t np = d.npair();
    hipLaunchKernelGGL(k_pair_sums, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, d.stream, np, d.pairblkP,
                       d.pair_sumsP);
    HIPCHECK(hipGetLastError());
}

// near-field values of the formulation (and of a Calderon preconditioner's
// operator P when it is not A), mass matrix, block-diagonal preconditioner
void launch_near_assemble(DevMesh &d)
{
    const int V = d.hm.V;
    const int64_t np = d.npair();
    if (d.fm.family == 1)
        hipLaunchKernelGGL(k_pair_sums, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, d.stream, np, d.pairblk,
                           d.pair_sums);
    launch_near_values(d, d.fm, d.pairblk, d.pair_sums, d.N, d.Mval);
    if (d.NP) {
        if (d.pairblkP) launch_near_values(d, d.fmP, d.pairblkP, d.pair_sumsP, d.NP, nullptr);
        else launch_near_values(d, d.fmP, d.pairblk, d.pair_sums, d.NP, nullptr);
    }
    if (d.Mval)
        hipLaunchKernelGGL(k_mass_diag, dim3((V + 255) / 256), dim3(256), 0, d.stream, V, d.diag_slot, d.Mval,
                           d.Mdinv);
    hipLaunchKernelGGL(k_block_diag, dim3((V + 255) / 256), dim3(256), 0, d.stream, V,
                       d.prm.preconditioner == PB_BLOCK_DIAG ? 1 : 0, d.diag_slot, d.N, d.nnz(), d.pinv);
    HIPCHECK(hipGetLastError());
}

}  // namespace pbm
