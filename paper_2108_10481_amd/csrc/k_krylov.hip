// FP64 Krylov building blocks for GMRES (Preconditioning; GMRES without
// restart): block dot products against the Arnoldi basis, basis updates and
// the final combination.  Every reduction has a fixed shape, so results do
// not depend on scheduling.
#include <algorithm>

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
// return at once.  Each kernel's work is a device function shared with the
// batched kernels below (several solves in one launch), so both round alike.
namespace pbm {

// h[i] = <V_i, w>, w = V_{j+1}: one block of kDotThreads threads
__device__ __forceinline__ void gdots_item(int n, const double *__restrict__ Vb, int j, int i,
                                           double *__restrict__ out, double *sh)
{
    const double *v = Vb + (size_t)i * n;
    const double *w = Vb + (size_t)(j + 1) * n;
    double acc = 0.0;
    for (int e = threadIdx.x; e < n; e += kDotThreads) acc += v[e] * w[e];
    const double r = dot_block_sum(acc, sh);
    if (threadIdx.x == 0) out[i] = r;
}

// w[e] -= sum_{i <= j} h[i] V_i[e]
__device__ __forceinline__ void gupdate_elem(int n, double *__restrict__ Vb, int j, const double *__restrict__ h,
                                             int e)
{
    double acc = 0.0;
    for (int i = 0; i <= j; ++i) acc += h[i] * Vb[(size_t)i * n + e];
    Vb[(size_t)(j + 1) * n + e] -= acc;
}

// |w|^2 with one block, same reduction shape as k_dots
__device__ __forceinline__ void gnorm_block(int n, const double *__restrict__ Vb, GState *__restrict__ st, double *sh)
{
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
// One thread.
__device__ __forceinline__ void givens_step(GState *__restrict__ st, double *__restrict__ H, double *__restrict__ cs,
                                            double *__restrict__ sn, double *__restrict__ g,
                                            const double *__restrict__ h1, const double *__restrict__ h2)
{
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

__global__ __launch_bounds__(kDotThreads) void k_gdots(int n, const double *__restrict__ Vb,
                                                       const GState *__restrict__ st, double *__restrict__ out)
{
    __shared__ double sh[kDotThreads];
    const int i = blockIdx.x;
    if (st->done || i > st->j) return;
    gdots_item(n, Vb, st->j, i, out, sh);
}

__global__ void k_gupdate(int n, const double *__restrict__ Vb, const GState *__restrict__ st,
                          const double *__restrict__ h)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n || st->done) return;
    gupdate_elem(n, (double *)Vb, st->j, h, e);
}

__global__ __launch_bounds__(kDotThreads) void k_gnorm(int n, const double *__restrict__ Vb, GState *__restrict__ st)
{
    __shared__ double sh[kDotThreads];
    if (st->done) return;
    gnorm_block(n, Vb, st, sh);
}

__global__ void k_givens(GState *__restrict__ st, double *__restrict__ H, double *__restrict__ cs,
                         double *__restrict__ sn, double *__restrict__ g, const double *__restrict__ h1,
                         const double *__restrict__ h2)
{
    if (threadIdx.x != 0 || st->done) return;
    givens_step(st, H, cs, sn, g, h1, h2);
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

// ------------------------------------ the same iteration tail, many solves
// One launch per step for every solve of a lockstep batch (KrylovReq per
// solve).  Element-wise steps give each solve ceil(n / kKB) blocks (block
// ranges in boff, a prefix over the solves); the dot products of all solves
// form one list of (solve, basis vector) items that the blocks stride over,
// each item done by one block exactly as k_gdots does it; norm and rotation
// take one block per solve.  A solve whose stop flag is set does nothing.

// solve owning block b of a prefix boff[0..R] (boff[0] = 0, boff[R] = blocks)
__device__ __forceinline__ int owner_of(const int *__restrict__ boff, int R, int b)
{
    int lo = 0, hi = R - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kDotThreads) void k_bgdots(int R, const KrylovReq *__restrict__ rq, int pass)
{
    __shared__ double sh[kDotThreads];
    __shared__ int pre[PB_MAX_BATCH_REQUESTS + 1];
    for (int r = threadIdx.x; r < R; r += kDotThreads) {
        const GState *st = rq[r].st;
        pre[r + 1] = st->done ? 0 : st->j + 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        pre[0] = 0;
        for (int r = 0; r < R; ++r) pre[r + 1] += pre[r];
    }
    __syncthreads();
    const int total = pre[R];
    for (int k = blockIdx.x; k < total; k += gridDim.x) {
        const int r = owner_of(pre, R, k);
        const KrylovReq &q = rq[r];
        __syncthreads();   // sh of the previous item is read
        gdots_item(q.n, q.Vb, q.st->j, k - pre[r], pass ? q.h2 : q.h1, sh);
    }
}

__global__ void k_bgupdate(int R, const KrylovReq *__restrict__ rq, const int *__restrict__ boff, int pass)
{
    const int r = owner_of(boff, R, blockIdx.x);
    const KrylovReq &q = rq[r];
    const int e = (blockIdx.x - boff[r]) * blockDim.x + threadIdx.x;
    if (e >= q.n || q.st->done) return;
    gupdate_elem(q.n, q.Vb, q.st->j, pass ? q.h2 : q.h1, e);
}

__global__ __launch_bounds__(kDotThreads) void k_bgnorm(const KrylovReq *__restrict__ rq)
{
    __shared__ double sh[kDotThreads];
    const KrylovReq &q = rq[blockIdx.x];
    if (q.st->done) return;
    gnorm_block(q.n, q.Vb, q.st, sh);
}

__global__ void k_bgivens(int R, const KrylovReq *__restrict__ rq)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const KrylovReq &q = rq[r];
    if (q.st->done) return;
    givens_step(q.st, q.H, q.cs, q.sn, q.g, q.h1, q.h2);
}

__global__ void k_bgnormalize(int R, const KrylovReq *__restrict__ rq, const int *__restrict__ boff)
{
    const int r = owner_of(boff, R, blockIdx.x);
    const KrylovReq &q = rq[r];
    const int e = (blockIdx.x - boff[r]) * blockDim.x + threadIdx.x;
    if (e >= q.n || q.st->done) return;
    q.Vb[(size_t)q.st->j * q.n + e] *= q.st->inv;
}

int kr_batch_blocks(int n) { return (n + kKB - 1) / kKB; }

void kr_batch_iteration_tail(hipStream_t s, int R, const KrylovReq *rq, const int *boff, int nblocks, int ndot)
{
    const dim3 gd((unsigned)std::max(1, std::min(ndot, 1024)));
    hipLaunchKernelGGL(k_bgdots, gd, dim3(kDotThreads), 0, s, R, rq, 0);
    hipLaunchKernelGGL(k_bgupdate, dim3(nblocks), dim3(kKB), 0, s, R, rq, boff, 0);
    hipLaunchKernelGGL(k_bgdots, gd, dim3(kDotThreads), 0, s, R, rq, 1);
    hipLaunchKernelGGL(k_bgupdate, dim3(nblocks), dim3(kKB), 0, s, R, rq, boff, 1);
    hipLaunchKernelGGL(k_bgnorm, dim3(R), dim3(kDotThreads), 0, s, rq);
    hipLaunchKernelGGL(k_bgivens, dim3((R + 63) / 64), dim3(64), 0, s, R, rq);
    hipLaunchKernelGGL(k_bgnormalize, dim3(nblocks), dim3(kKB), 0, s, R, rq, boff);
    HIPCHECK(hipGetLastError());
}

}  // namespace pbm
