// FP64 Krylov building blocks for GMRES (Preconditioning; GMRES without
// restart): block dot products against the Arnoldi basis, basis updates and
// the final combination.  Every reduction has a fixed shape, so results do
// not depend on scheduling.
#include "pbm_internal.h"

namespace pbm {

constexpr int kKB = 256;

// out[i] = <V_i, w> for i < nvec; one block per basis vector.
__global__ __launch_bounds__(kKB) void k_dots(int n, const double *__restrict__ Vb, size_t ldv,
                                              const double *__restrict__ w, double *__restrict__ out)
{
    __shared__ double sh[kKB];
    const double *v = Vb + (size_t)blockIdx.x * ldv;
    double acc = 0.0;
    for (int e = threadIdx.x; e < n; e += kKB) acc += v[e] * w[e];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kKB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
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
    hipLaunchKernelGGL(k_dots, dim3(nvec), dim3(kKB), 0, s, n, V, ldv, w, out);
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
