// FP64 Krylov building blocks for GMRES (Preconditioning; GMRES without
// restart): block dot products against the Arnoldi basis, basis updates and
// the final combination.  Every reduction has a fixed shape, so results do
// not depend on scheduling.
#include "pbm_internal.h"

namespace pbm {

constexpr int kKB = 256;

// out[i] = <V_i, w> for i < nvec; one block per basis vector.
__global__ __launch_bounds__(kDotThreads) void k_dots(int n, const double *__restrict__ Vb, size_t ldv,
                                                      const double *__restrict__ w, double *__restrict__ out)
{
    __shared__ double sh[kDotThreads];
    const double *v = Vb + (size_t)blockIdx.x * ldv;
    double acc = 0.0;
    for (int e = threadIdx.x; e < n; e += kDotThreads) acc += v[e] * w[e];
    const double r = dot_block_sum(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = r;
}

// w += sign * sum_i h[i] V_i
__global__ void k_update(int n, int nvec, const double *__restrict__ Vb, size_t ldv, const double *__restrict__ h,
                         double *__restrict__ w, double sign)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double acc = 0.0;
    for (int i = 0; i < nvec; ++i) acc += h[i] * Vb[(size_t)i * ldv + e];
    w[e] += sign * acc;
}

__global__ void k_combine(int n, int nvec, const double *__restrict__ Vb, size_t ldv, const double *__restrict__ y,
                          double *__restrict__ x)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double acc = 0.0;
    for (int i = 0; i < nvec; ++i) acc += y[i] * Vb[(size_t)i * ldv + e];
    x[e] = acc;
}

__global__ void k_scale_copy(int n, const double *__restrict__ x, double a, double *__restrict__ y)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] = a * x[e];
}

__global__ void k_axpy(int n, double a, const double *__restrict__ x, double *__restrict__ y)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] += a * x[e];
}

__global__ void k_precond(int V, const double *__restrict__ pinv, const double *__restrict__ x, double *__restrict__ y)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    const double *P = pinv + 4 * (size_t)i;
    const double a = x[i], b = x[V + i];
    y[i] = P[0] * a + P[1] * b;
    y[V + i] = P[2] * a + P[3] * b;
}

static inline dim3 g1(int n) { return dim3((n + kKB - 1) / kKB); }

void kr_dots(hipStream_t s, int n, int nvec, const double *V, size_t ldv, const double *w, double *out)
{
    hipLaunchKernelGGL(k_dots, dim3(nvec), dim3(kDotThreads), 0, s, n, V, ldv, w, out);
}
void kr_update(hipStream_t s, int n, int nvec, const double *V, size_t ldv, const double *h, double *w, double sign)
{
    hipLaunchKernelGGL(k_update, g1(n), dim3(kKB), 0, s, n, nvec, V, ldv, h, w, sign);
}
void kr_combine(hipStream_t s, int n, int nvec, const double *V, size_t ldv, const double *y, double *x)
{
    hipLaunchKernelGGL(k_combine, g1(n), dim3(kKB), 0, s, n, nvec, V, ldv, y, x);
}
void kr_scale_copy(hipStream_t s, int n, const double *x, double a, double *y)
{
    hipLaunchKernelGGL(k_scale_copy, g1(n), dim3(kKB), 0, s, n, x, a, y);
}
void kr_axpy(hipStream_t s, int n, double a, const double *x, double *y)
{
    hipLaunchKernelGGL(k_axpy, g1(n), dim3(kKB), 0, s, n, a, x, y);
}
void kr_precond(hipStream_t s, int V, const double *pinv, const double *x, double *y)
{
    hipLaunchKernelGGL(k_precond, g1(V), dim3(kKB), 0, s, V, pinv, x, y);
}

}  // namespace pbm

// ----------------------------------------------- captured GMRES iteration
// The iteration index and the stopping flag live in device memory, so one
// captured graph serves every iteration; blocks beyond the current basis size
// return at once.
namespace pbm {

__global__ __launch_bounds__(kDotThreads) void k_gdots(int n, const double *__restrict__ Vb,
                                                       const GState *__restrict__ st, double *__restrict__ out)
{
    __shared__ double sh[kDotThreads];
    const int i = blockIdx.x;
    if (st->done || i > st->j) return;
    const double *v = Vb + (size_t)i * n;
    const double *w = Vb + (size_t)(st->j + 1) * n;
    double acc = 0.0;
    for (int e = threadIdx.x; e < n; e += kDotThreads) acc += v[e] * w[e];
    const double r = dot_block_sum(acc, sh);
    if (threadIdx.x == 0) out[i] = r;
}

__global__ void k_gupdate(int n, const double *__restrict__ Vb, const GState *__restrict__ st,
                          const double *__restrict__ h)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n || st->done) return;
    const int j = st->j;
    double acc = 0.0;
    for (int i = 0; i <= j; ++i) acc += h[i] * Vb[(size_t)i * n + e];
    ((double *)Vb)[(size_t)(j + 1) * n + e] -= acc;
}

// |w|^2 with one block, same reduction shape as k_dots
__global__ __launch_bounds__(kDotThreads) void k_gnorm(int n, const double *__restrict__ Vb, GState *__restrict__ st)
{
    __shared__ double sh[kDotThreads];
    if (st->done) return;
    const double *w = Vb + (size_t)(st->j + 1) * n;
    double acc = 0.0;
    for (int e = threadIdx.x; e < n; e += kDotThreads) acc += w[e] * w[e];
    const double r = dot_block_sum(acc, sh);
    if (threadIdx.x == 0) st->nrm2 = r;
}

// Hessenberg column j = h1 + h2 (two Gram-Schmidt passes), previous Givens
// rotations, new rotation, residual estimate |g_{j+1}|; advances j.  The
// rotations are written with explicit fused multiply-adds, exactly as the host
// implementations are, so eager, batched and captured solves agree bitwise.
__global__ void k_givens(GState *__restrict__ st, double *__restrict__ H, double *__restrict__ cs,
                         double *__restrict__ sn, double *__restrict__ g, const double *__restrict__ h1,
                         const double *__restrict__ h2)
{
    if (threadIdx.x != 0 || st->done) return;
    const int j = st->j, m = st->m;
    double *col = H + (size_t)j * (m + 1);
    for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
    const double hn = sqrt(fmax(st->nrm2, 0.0));
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double a = fma(cs[i], col[i], sn[i] * col[i + 1]);
        col[i + 1] = fma(-sn[i], col[i], cs[i] * col[i + 1]);
        col[i] = a;
    }
    const double den = sqrt(fma(col[j], col[j], col[j + 1] * col[j + 1]));
    cs[j] = col[j] / den;
    sn[j] = col[j + 1] / den;
    col[j] = den;
    col[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    st->res = fabs(g[j + 1]);
    st->inv = hn > 0.0 ? 1.0 / hn : 0.0;
    st->j = j + 1;
    if (st->res <= st->tolb || !(den > 0.0) || j + 1 >= m) st->done = 1;
}

__global__ void k_gnormalize(int n, double *__restrict__ Vb, const GState *__restrict__ st)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n || st->done) return;
    Vb[(size_t)st->j * n + e] *= st->inv;
}

void kr_graph_iteration_tail(hipStream_t s, int n, int m, double *Vb, GState *st, double *H, double *cs, double *sn,
                             double *g, double *h1, double *h2)
{
    hipLaunchKernelGGL(k_gdots, dim3(m + 1), dim3(kDotThreads), 0, s, n, Vb, st, h1);
    hipLaunchKernelGGL(k_gupdate, g1(n), dim3(kKB), 0, s, n, Vb, st, h1);
    hipLaunchKernelGGL(k_gdots, dim3(m + 1), dim3(kDotThreads), 0, s, n, Vb, st, h2);
    hipLaunchKernelGGL(k_gupdate, g1(n), dim3(kKB), 0, s, n, Vb, st, h2);
    hipLaunchKernelGGL(k_gnorm, dim3(1), dim3(kDotThreads), 0, s, n, Vb, st);
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, s, st, H, cs, sn, g, h1, h2);
    hipLaunchKernelGGL(k_gnormalize, g1(n), dim3(kKB), 0, s, n, Vb, st);
}

}  // namespace pbm
