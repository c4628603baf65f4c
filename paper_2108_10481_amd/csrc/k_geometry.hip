// Geometry, charge-to-surface projections (Eq. sources), reaction potential
// (Eq. phireac_bie) and the charge-inside-surface check.
#include <mutex>

#include "pbm_internal.h"

namespace pbm {

// One thread per (Morton-sorted) triangle: area, outward unit normal, surface
// curls of the three P1 hats, the six regular quadrature points, and the
// FP64 / FP32 source-target records used by the far-field kernels.
__global__ void k_geometry(int T, const double *__restrict__ xyz, const int32_t *__restrict__ tri,
                           double *__restrict__ geo, double *__restrict__ stat64, float *__restrict__ stat32)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double P[3][3];
    for (int k = 0; k < 3; ++k) {
        int v = tri[3 * t + k];
        for (int c = 0; c < 3; ++c) P[k][c] = xyz[3 * v + c];
    }
    double e1[3], e2[3];
    for (int c = 0; c < 3; ++c) { e1[c] = P[1][c] - P[0][c]; e2[c] = P[2][c] - P[0][c]; }
    double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    double area = 0.5 * len;
    double n[3] = {cr[0] / len, cr[1] / len, cr[2] / len};
    double *g = geo + (size_t)t * kGeo;
    double *s64 = stat64 + (size_t)t * kStat;
    float *s32 = stat32 + (size_t)t * kStat;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        double x[3];
        for (int c = 0; c < 3; ++c)
            x[c] = rule_bary(p, 0) * P[0][c] + rule_bary(p, 1) * P[1][c] + rule_bary(p, 2) * P[2][c];
        double yn = x[0] * n[0] + x[1] * n[1] + x[2] * n[2];
        for (int c = 0; c < 3; ++c) {
            g[3 * p + c] = x[c];
            s64[3 * p + c] = x[c];
            s32[3 * p + c] = (float)x[c];
        }
        s64[21 + p] = yn;
        s32[21 + p] = (float)yn;
    }
    for (int c = 0; c < 3; ++c) {
        g[18 + c] = n[c];
        s64[18 + c] = n[c];
        s32[18 + c] = (float)n[c];
    }
    g[21] = area;
    // curl of hat k: n x grad(lambda_k) = -(P_{k+2} - P_{k+1}) / (2 |t|)
    for (int k = 0; k < 3; ++k) {
        int a = (k + 1) % 3, b = (k + 2) % 3;
        for (int c = 0; c < 3; ++c) g[22 + 3 * k + c] = -(P[b][c] - P[a][c]) / (2.0 * area);
    }
    g[31] = 0.0;
    s64[27] = area;
    s32[27] = (float)area;
    for (int i = 0; i < 9; ++i) {
        s64[28 + i] = g[22 + i];
        s32[28 + i] = (float)g[22 + i];
    }
    // centroid (the one-point rule of fast Calderon's preconditioner)
    for (int c = 0; c < 3; ++c) {
        const double m = (P[0][c] + P[1][c] + P[2][c]) / 3.0;
        s64[37 + c] = m;
        s32[37 + c] = (float)m;
    }
}

void launch_geometry(DevMesh &d)
{
    int T = d.hm.T;
    hipLaunchKernelGGL(k_geometry, dim3((T + 255) / 256), dim3(256), 0, d.stream, T, d.xyz, d.tri, d.geo,
                       d.stat64, d.stat32);
    HIPCHECK(hipGetLastError());
}

// ------------------------------------------------------------------ sources
// One thread per quadrature point: phi_D and phi_N of Eq. sources without the
// 1/(4 pi eps_in) factor.  Charges are read with uniform (scalar) loads.
__global__ void k_source_field(int T, int nq, const double *__restrict__ geo, const double *__restrict__ qb,
                               double *__restrict__ f)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 6 * T) return;
    int t = i / 6, p = i - 6 * t;
    const double *g = geo + (size_t)t * kGeo;
    double x = g[3 * p], y = g[3 * p + 1], z = g[3 * p + 2];
    double nx = g[18], ny = g[19], nz = g[20];
    const double *qx = qb, *qy = qb + nq, *qz = qb + 2 * nq, *qq = qb + 3 * nq;
    double sD = 0.0, sN = 0.0;
    for (int j = 0; j < nq; ++j) {
        double dx = x - qx[j], dy = y - qy[j], dz = z - qz[j];
        double r2 = dx * dx + dy * dy + dz * dz;
        double ri = 1.0 / sqrt(r2);
        sD += qq[j] * ri;
        sN -= qq[j] * (dx * nx + dy * ny + dz * nz) * ri * ri * ri;
    }
    f[i] = sD;
    f[(size_t)6 * T + i] = sN;
}

// per-triangle P1 test projection of point values: out[t][k] = |t| sum_p w_p lambda_k(p) f[t][p] * scale
__global__ void k_project2(int T, const double *__restrict__ geo, const double *__restrict__ f, double scale,
                           double *__restrict__ triout)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double area = geo[(size_t)t * kGeo + 21];
    for (int h = 0; h < 2; ++h) {
        const double *fp = f + (size_t)h * 6 * T + 6 * (size_t)t;
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
#pragma unroll
            for (int p = 0; p < 6; ++p) s += rule_w(p) * rule_bary(p, k) * fp[p];
            triout[6 * (size_t)t + 3 * h + k] = s * area * scale;
        }
    }
}

// per-vertex gather of triangle contributions in fixed incidence order
__global__ void k_gather_tri(int V, const int32_t *__restrict__ inc_ptr, const int32_t *__restrict__ inc_tk,
                             const double *__restrict__ triout, double *__restrict__ y)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    double a = 0.0, b = 0.0;
    for (int e = inc_ptr[i]; e < inc_ptr[i + 1]; ++e) {
        int tk = inc_tk[e];
        int t = tk >> 2, k = tk & 3;
        a += triout[6 * (size_t)t + k];
        b += triout[6 * (size_t)t + 3 + k];
    }
    y[i] = a;
    y[V + i] = b;
}

void launch_rhs(DevMesh &d, int nq, const double *qbuf, double *b)
{
    int T = d.hm.T, V = d.hm.V;
    hipLaunchKernelGGL(k_source_field, dim3((6 * T + 255) / 256), dim3(256), 0, d.stream, T, nq, d.geo, qbuf,
                       d.fpts);
    hipLaunchKernelGGL(k_project2, dim3((T + 255) / 256), dim3(256), 0, d.stream, T, d.geo, d.fpts,
                       kInv4Pi / d.prm.eps_in, d.triout);
    hipLaunchKernelGGL(k_gather_tri, dim3((V + 255) / 256), dim3(256), 0, d.stream, V, d.inc_ptr, d.inc_tk,
                       d.triout, b);
    HIPCHECK(hipGetLastError());
}

// right-hand side of the formulation from [<phi_i, varphi_D>; <phi_i, varphi_N>], in place
__global__ void k_rhs_combine(int V, double d1, double n1, double d2, double n2, double *__restrict__ b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    const double bD = b[i], bN = b[V + i];
    b[i] = d1 * bD + n1 * bN;
    b[V + i] = d2 * bD + n2 * bN;
}

void formulation_rhs(DevMesh &d, int nq, const double *qbuf, double *b)
{
    launch_rhs(d, nq, qbuf, b);
    const FormCoef &f = d.fm;
    const int V = d.hm.V;
    hipLaunchKernelGGL(k_rhs_combine, dim3((V + 255) / 256), dim3(256), 0, d.stream, V, f.rhsD[0], f.rhsN[0],
                       f.rhsD[1], f.rhsN[1], b);
    HIPCHECK(hipGetLastError());
}

// --------------------------------------------------------- reaction potential
// grid (point k, source chunk c); each block sums, over its chunk of source
// triangles, G(x_k, y) b2 - dG/dn_y(x_k, y) b1 with the Laplace kernel (no 4 pi),
// where b1 = w|s| phi(y), b2 = w|s| dphi(y) are the FP64 dynamic records of
// the traces.  Fixed-shape tree reduction -> deterministic partials.
constexpr int kRedBlock = 256;

__device__ inline double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kRedBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kRedBlock) void k_reaction(int T, int chunk, const double *__restrict__ pts,
                                                        const double *__restrict__ stat,
                                                        const double *__restrict__ dyn, double *__restrict__ part)
{
    __shared__ double sh[kRedBlock];
    int k = blockIdx.x, c = blockIdx.y;
    double x = pts[3 * k], y = pts[3 * k + 1], z = pts[3 * k + 2];
    int s0 = c * chunk, s1 = min(T, s0 + chunk);
    double acc = 0.0;
    for (int i = s0 * 6 + threadIdx.x; i < s1 * 6; i += kRedBlock) {
        int s = i / 6, q = i - 6 * s;
        const double *st = stat + (size_t)s * kStat;
        const double *dy = dyn + (size_t)s * kDyn;
        double dx = x - st[3 * q], dyy = y - st[3 * q + 1], dz = z - st[3 * q + 2];
        double r2 = dx * dx + dyy * dyy + dz * dz;
        double ri = 1.0 / sqrt(r2);
        double dn = dx * st[18] + dyy * st[19] + dz * st[20];
        acc += ri * dy[6 + q] - dn * ri * ri * ri * dy[q];
    }
    double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(size_t)k * gridDim.y + c] = tot;
}

// Solid angle subtended by each triangle at point k (Van Oosterom-Strackee);
// the sum is 4 pi for points inside a closed outward-oriented surface.
__global__ __launch_bounds__(kRedBlock) void k_solid_angle(int T, int chunk, const double *__restrict__ pts,
                                                           const double *__restrict__ xyz,
                                                           const int32_t *__restrict__ tri, double *__restrict__ part)
{
    __shared__ double sh[kRedBlock];
    int k = blockIdx.x, c = blockIdx.y;
    double x = pts[3 * k], y = pts[3 * k + 1], z = pts[3 * k + 2];
    int s0 = c * chunk, s1 = min(T, s0 + chunk);
    double acc = 0.0;
    for (int s = s0 + threadIdx.x; s < s1; s += kRedBlock) {
        double a[3], b[3], e[3];
        for (int m = 0; m < 3; ++m) {
            a[m] = xyz[3 * tri[3 * s] + m] - (m == 0 ? x : m == 1 ? y : z);
            b[m] = xyz[3 * tri[3 * s + 1] + m] - (m == 0 ? x : m == 1 ? y : z);
            e[m] = xyz[3 * tri[3 * s + 2] + m] - (m == 0 ? x : m == 1 ? y : z);
        }
        double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        double le = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        double det = a[0] * (b[1] * e[2] - b[2] * e[1]) - a[1] * (b[0] * e[2] - b[2] * e[0]) +
                     a[2] * (b[0] * e[1] - b[1] * e[0]);
        double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
        double ae = a[0] * e[0] + a[1] * e[1] + a[2] * e[2];
        double be = b[0] * e[0] + b[1] * e[1] + b[2] * e[2];
        acc += 2.0 * atan2(det, la * lb * le + ab * le + ae * lb + be * la);
    }
    double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(size_t)k * gridDim.y + c] = tot;
}

static int red_chunks(int T) { return T < 4096 ? 1 : (T + 4095) / 4096; }

void launch_reaction(DevMesh &d, int nq, const double *qpts, double *out_part)
{
    int T = d.hm.T, C = red_chunks(T);
    int chunk = (T + C - 1) / C;
    hipLaunchKernelGGL(k_reaction, dim3(nq, C), dim3(kRedBlock), 0, d.stream, T, chunk, qpts, d.stat64, d.dyn64,
                       out_part);
    HIPCHECK(hipGetLastError());
}

void launch_inside_test(DevMesh &d, int nq, const double *qpts, double *out_part)
{
    int T = d.hm.T, C = red_chunks(T);
    int chunk = (T + C - 1) / C;
    hipLaunchKernelGGL(k_solid_angle, dim3(nq, C), dim3(kRedBlock), 0, d.stream, T, chunk, qpts, d.xyz, d.tri,
                       out_part);
    HIPCHECK(hipGetLastError());
}

int reduction_chunks(int T) { return red_chunks(T); }

// ------------------------------------------- reaction potential, no allocation
// Partial sums (point x source chunk) of pb_mesh_reaction_potential_noalloc
// live in this file-scope array: one copy per device, held until the process
// ends.  Host code never uses the array's name as an address; it uses the
// device address resolved once per device by noalloc_scratch().
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

static double *noalloc_scratch()
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int dev = -1;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(PB_E_DEVICE, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(PB_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        addr[dev] = (double *)p;
    }
    return addr[dev];
}

// out[k] = (sum over chunks c, in order, of part[k C + c]) / (4 pi): the same
// sum, in the same order, as the host finish of pb_mesh_reaction_potential
__global__ void k_reaction_finish(int npts, int C, const double *__restrict__ part, double *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npts) return;
    double s = 0.0;
    for (int c = 0; c < C; ++c) s += part[(size_t)k * C + c];
    out[k] = s * kInv4Pi;
}

void reaction_potential_noalloc(DevMesh &d, const double *traces, int npts, const double *pts, double *out,
                                hipStream_t stream)
{
    const int C = red_chunks(d.hm.T);
    if ((size_t)npts * (size_t)C > kNoAllocScratchDoubles)
        fail(PB_E_INVALID_ARG, "npts x source chunks (" + std::to_string((size_t)npts * C) +
                                   ") exceeds the scratch of " + std::to_string(kNoAllocScratchDoubles) + " doubles");
    double *part = noalloc_scratch();
    struct StreamSwap {
        DevMesh &d;
        hipStream_t keep;
        StreamSwap(DevMesh &dm, hipStream_t s) : d(dm), keep(dm.stream) { if (s) d.stream = s; }
        ~StreamSwap() { d.stream = keep; }
    } swap(d, stream);
    launch_source_prep(d, traces, false);
    launch_reaction(d, npts, pts, part);
    hipLaunchKernelGGL(k_reaction_finish, dim3((npts + 255) / 256), dim3(256), 0, d.stream, npts, C, part, out);
    HIPCHECK(hipGetLastError());
}

}  // namespace pbm
