// Several right-hand sides (charge sets) on one resident mesh.
//
// The systems share the operator, so they advance together: one batched GMRES
// (independent Arnoldi processes in lock-step, one host synchronisation per
// iteration for all of them) whose operator product applies the 16-bit
// assembled far field to all right-hand sides in one MFMA GEMM,
//   Y (2V x 16) = A_far (2V x 2V, BF16 / FP16) X (2V x 16), FP32 accumulate.
// This is the one dense contraction on the path; it streams A once per product
// and is bound by HBM bandwidth, the matrix cores keep the VALU out of the way.
// Mixed modes wrap the batched inner solves in FP64 iterative refinement on the
// accurate (FP32-stored) operator, as for one right-hand side.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <functional>
#include <string>
#include <vector>

#include "dense.h"

namespace pbm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

pb_status finish_result(DevMesh &d, const pb_charges *ch, const double *pb, double *u, int its, int outer,
                        double t_rhs, double t_prec, double t_gmres, pb_result *res);
void charges_to_device(DevMesh &d, const pb_charges *c);
void check_charges_inside(DevMesh &d, int nq);

// ------------------------------------------------------------------ GEMM
// One wavefront per 16-row tile, all 16 right-hand sides.  v_mfma_f32_16x16x32
// operand layout (lane l): A[row l%16][k 8(l/16) .. +7], B[k 8(l/16) .. +7][col
// l%16]; result D[row 4(l/16) + i][col l%16], i = 0..3.  The two column blocks
// are accumulated separately so FP16 block scales can be undone per block.
template <int KIND>
__device__ __forceinline__ f32x4 mfma16(const uint16_t *a, const uint16_t *b, f32x4 c)
{
    if constexpr (KIND == 1)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(*(const bf16x8 *)a, *(const bf16x8 *)b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(*(const f16x8 *)a, *(const f16x8 *)b, c, 0, 0, 0);
}

// Row-major operand (used when the tiled copy below does not fit): RT row
// tiles of 16 per wavefront share each B (x) fragment.  Each load reads 64
// bytes of 16 rows.
template <int KIND, int RT>
__global__ __launch_bounds__(256) void k_gemm16(int n, int V, size_t Vp, size_t ld, const uint16_t *__restrict__ A,
                                                const uint16_t *__restrict__ X, float i0, float i1, float i2, float i3,
                                                double *__restrict__ Y)
{
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6;
    const int nwave = gridDim.x * 4;
    const int ntile = (n + 16 * RT - 1) / (16 * RT);
    const int kq = (lane >> 4) * 8;
    const int cl = lane & 15;
    const uint16_t *xrow = X + (size_t)cl * ld + kq;
    for (int tile = wave; tile < ntile; tile += nwave) {
        const int r0 = tile * 16 * RT;
        const uint16_t *arow[RT];
        f32x4 c0[RT], c1[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            // rows past n re-read row n-1; their results are dropped
            arow[t] = A + (size_t)min(r0 + 16 * t + cl, n - 1) * ld + kq;
            c0[t] = f32x4{0.f, 0.f, 0.f, 0.f};
            c1[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll 4
        for (size_t k = 0; k < Vp; k += 32)
#pragma unroll
            for (int t = 0; t < RT; ++t) c0[t] = mfma16<KIND>(arow[t] + k, xrow + k, c0[t]);
#pragma unroll 4
        for (size_t k = Vp; k < ld; k += 32)
#pragma unroll
            for (int t = 0; t < RT; ++t) c1[t] = mfma16<KIND>(arow[t] + k, xrow + k, c1[t]);
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = r0 + 16 * t + 4 * (lane >> 4) + i;
                if (r < n) {
                    const bool top = r < V;
                    Y[(size_t)cl * n + r] = (double)c0[t][i] * (top ? i0 : i2) + (double)c1[t][i] * (top ? i1 : i3);
                }
            }
    }
}

// Tiled operand: nk = ld / 32 steps per 16-row tile, the first nk0 = Vp / 32
// in the first column block; lane l reads the 16 bytes at (tile nk + s) 512 +
// 8 l, so a wavefront's load is 1 KB of consecutive bytes.  The MFMA sequence
// and every lane's operands are those of k_gemm16<KIND, 1>, so the results are
// bitwise the same.
template <int KIND>
__global__ __launch_bounds__(256) void k_gemm16t(int n, int V, int nk0, int nk, size_t ld,
                                                 const uint16_t *__restrict__ At, const uint16_t *__restrict__ X,
                                                 float i0, float i1, float i2, float i3, double *__restrict__ Y)
{
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6;
    const int nwave = gridDim.x * 4;
    const int ntile = (n + 15) / 16;
    const int kq = (lane >> 4) * 8;
    const int cl = lane & 15;
    const uint16_t *xrow = X + (size_t)cl * ld + kq;
    for (int tile = wave; tile < ntile; tile += nwave) {
        const uint16_t *at = At + (size_t)tile * nk * 512 + 8 * lane;
        f32x4 c0 = f32x4{0.f, 0.f, 0.f, 0.f}, c1 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int st = 0; st < nk0; ++st) c0 = mfma16<KIND>(at + (size_t)st * 512, xrow + (size_t)st * 32, c0);
#pragma unroll 4
        for (int st = nk0; st < nk; ++st) c1 = mfma16<KIND>(at + (size_t)st * 512, xrow + (size_t)st * 32, c1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = tile * 16 + 4 * (lane >> 4) + i;
            if (r < n) {
                const bool top = r < V;
                Y[(size_t)cl * n + r] = (double)c0[i] * (top ? i0 : i2) + (double)c1[i] * (top ? i1 : i3);
            }
        }
    }
}

// Row-major 16-bit copy -> tiled copy (k_gemm16t's operand order); rows past
// n are zero.  One 16-byte chunk per (tile, step, lane).
__global__ void k_tile16(int n, size_t ld, int ntile, int nk, const uint16_t *__restrict__ A,
                         uint16_t *__restrict__ At)
{
    const size_t total = (size_t)ntile * nk * 64;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < total; c += (size_t)gridDim.x * blockDim.x) {
        const int lane = (int)(c & 63);
        const size_t ts = c >> 6;                    // tile * nk + step
        const int tile = (int)(ts / (size_t)nk), st = (int)(ts % (size_t)nk);
        const int row = tile * 16 + (lane & 15);
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (row < n) v = *(const uint4 *)(A + (size_t)row * ld + (size_t)st * 32 + (lane >> 4) * 8);
        *(uint4 *)(At + c * 8) = v;
    }
}

__device__ __forceinline__ uint16_t f2bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// X16[c][k] in the padded column layout, c < nb from the FP64 systems, zero otherwise
__global__ void k_pad_batch(int V, int n, int nb, size_t Vp, size_t ld, int kind, const int32_t *__restrict__ vperm,
                            const double *__restrict__ Xs, uint16_t *__restrict__ X16)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (k >= ld) return;
    double v = 0.0;
    if (c < nb) {
        if (k < (size_t)V) v = Xs[(size_t)c * n + vperm[k]];
        else if (k >= Vp && k < Vp + (size_t)V) v = Xs[(size_t)c * n + V + vperm[k - Vp]];
    }
    uint16_t o;
    if (kind == 1) o = f2bf16((float)v);
    else o = __builtin_bit_cast(uint16_t, (_Float16)(float)v);
    X16[(size_t)c * ld + k] = o;
}

// per (vertex i, system s): far part from Y16, near-field CSR product,
// optional 2x2 preconditioner
__global__ void k_gather_batch(int V, int n, int precond, const int32_t *__restrict__ row_ptr,
                               const int32_t *__restrict__ col, const double *__restrict__ N, int64_t nnz,
                               const double *__restrict__ pinv, const int32_t *__restrict__ vpos,
                               const double *__restrict__ Yfar, const double *__restrict__ X, double *__restrict__ Y)
{
    // kRowLanes lanes per row, the same slot order and butterfly as k_gather
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes;
    const int c = threadIdx.x % kRowLanes;
    const int s = blockIdx.y;
    if (i >= V) return;
    const double *x = X + (size_t)s * n;
    double n1 = 0.0, n2 = 0.0;
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
    if (c != 0) return;
    const int r = vpos[i];   // dense row order
    double y1 = Yfar[(size_t)s * n + r], y2 = Yfar[(size_t)s * n + V + r];
    y1 += n1;
    y2 += n2;
    if (precond) {
        const double *P = pinv + 4 * (size_t)i;
        const double z1 = P[0] * y1 + P[1] * y2, z2 = P[2] * y1 + P[3] * y2;
        y1 = z1;
        y2 = z2;
    }
    Y[(size_t)s * n + i] = y1;
    Y[(size_t)s * n + V + i] = y2;
}

// ------------------------------------------------------- batched Krylov
// basis layout [vector i][system s][n]
__global__ __launch_bounds__(kDotThreads) void k_bdots(int n, int nb, const double *__restrict__ Vb,
                                                       const double *__restrict__ W, double *__restrict__ out,
                                                       int ostride)
{
    __shared__ double sh[kDotThreads];
    const int i = blockIdx.x, s = blockIdx.y;
    const double *v = Vb + ((size_t)i * nb + s) * n;
    const double *w = W + (size_t)s * n;
    double acc = 0.0;
    for (int e = threadIdx.x; e < n; e += kDotThreads) acc += v[e] * w[e];
    const double r = dot_block_sum(acc, sh);
    if (threadIdx.x == 0) out[(size_t)s * ostride + i] = r;
}

__global__ void k_bupdate(int n, int nvec, int nb, const double *__restrict__ Vb, const double *__restrict__ h,
                          int hstride, double *__restrict__ W, double sign)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (e >= n) return;
    double acc = 0.0;
    for (int i = 0; i < nvec; ++i) acc += h[(size_t)s * hstride + i] * Vb[((size_t)i * nb + s) * n + e];
    W[(size_t)s * n + e] += sign * acc;
}

// W[s] /= sqrt(nrm2[s]) when positive
__global__ void k_bnormalize(int n, const double *__restrict__ nrm2, int nstride, double *__restrict__ W)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (e >= n) return;
    const double q = nrm2[(size_t)s * nstride];
    if (q > 0.0) W[(size_t)s * n + e] *= 1.0 / sqrt(q);
}

__global__ void k_bscale(int n, const double *__restrict__ a, const double *__restrict__ X, double *__restrict__ Y)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (e >= n) return;
    Y[(size_t)s * n + e] = a[s] * X[(size_t)s * n + e];
}

// X[s] = sum_{i < kmax} y[s][i] basis[i][s]  (y zero-padded past each system's k)
__global__ void k_bcombine(int n, int kmax, int nb, const double *__restrict__ Vb, const double *__restrict__ y,
                           int ystride, double *__restrict__ X)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (e >= n) return;
    double acc = 0.0;
    for (int i = 0; i < kmax; ++i) acc += y[(size_t)s * ystride + i] * Vb[((size_t)i * nb + s) * n + e];
    X[(size_t)s * n + e] = acc;
}

// ------------------------------------------------------------- host side
struct BatchWork {
    int cap_m = 0, cap_nb = 0;
    double *basis = nullptr, *kbuf = nullptr, *y = nullptr, *sc = nullptr;
    double *B = nullptr, *PB = nullptr, *U = nullptr, *R = nullptr, *C = nullptr, *Z = nullptr;
};

static BatchWork &work(DevMesh &d, int m, int nb)
{
    BatchWork *w = d.bw;
    if (!w || w->cap_m < m || w->cap_nb < nb) {
        const size_t n = 2 * (size_t)d.hm.V;
        BatchWork nw;
        nw.cap_m = std::max(m, w ? w->cap_m : 0);
        nw.cap_nb = kMaxBatch;
        nw.basis = (double *)d.alloc(sizeof(double) * n * (nw.cap_m + 1) * kMaxBatch);
        nw.kbuf = (double *)d.alloc(sizeof(double) * (2 * (nw.cap_m + 1) + 1) * kMaxBatch);
        nw.y = (double *)d.alloc(sizeof(double) * (nw.cap_m + 1) * kMaxBatch);
        nw.sc = (double *)d.alloc(sizeof(double) * kMaxBatch);
        for (double **p : {&nw.B, &nw.PB, &nw.U, &nw.R, &nw.C, &nw.Z}) *p = (double *)d.alloc(sizeof(double) * n * kMaxBatch);
        if (!w) w = d.bw = new BatchWork();
        *w = nw;   // older buffers stay in the handle's allocation list until destroy
    }
    return *w;
}

void destroy_batch(DevMesh &d)
{
    delete d.bw;
    d.bw = nullptr;
}

// P^-1 A applied to nb systems: one MFMA GEMM on the 16-bit far field, or one
// accurate product per system.
static void apply_batch(DevMesh &d, int nb, const double *X, double *Y)
{
    const int V = d.hm.V, n = 2 * V;
    Dense *D = d.dense;
    if (D && D->level == 0 && D->A16) {
        if (!D->X16) {
            D->X16 = (uint16_t *)d.alloc(sizeof(uint16_t) * kMaxBatch * D->ld);
            D->Y16 = (double *)d.alloc(sizeof(double) * kMaxBatch * n);
        }
        hipLaunchKernelGGL(k_pad_batch, dim3((unsigned)((D->ld + 255) / 256), kMaxBatch), dim3(256), 0, d.stream, V, n,
                           nb, D->Vp, D->ld, D->kind16, D->vperm, X, D->X16);
        float inv[4] = {1.f, 1.f, 1.f, 1.f};
        if (D->kind16 == 2)
            for (int b = 0; b < 4; ++b) inv[b] = 1.f / D->scale16[b];
        const int ntile = (n + 15) / 16, nk = (int)(D->ld / 32), nk0 = (int)(D->Vp / 32);
        if (!D->A16t && !D->a16t_failed) {
            try {
                D->A16t = (uint16_t *)d.alloc(sizeof(uint16_t) * (size_t)ntile * nk * 512);
            } catch (const Error &) {
                (void)hipGetLastError();
                D->a16t_failed = true;
            }
        }
        if (D->A16t && D->a16t_version != D->a16_version) {
            hipLaunchKernelGGL(k_tile16, dim3(8192), dim3(256), 0, d.stream, n, D->ld, ntile, nk, D->A16, D->A16t);
            D->a16t_version = D->a16_version;
        }
        auto launch = [&]() {
            if (D->A16t) {
                const int nwg = std::min((ntile + 3) / 4, 4096);
                if (D->kind16 == 1)
                    hipLaunchKernelGGL((k_gemm16t<1>), dim3(nwg), dim3(256), 0, d.stream, n, V, nk0, nk, D->ld,
                                       D->A16t, D->X16, inv[0], inv[1], inv[2], inv[3], D->Y16);
                else
                    hipLaunchKernelGGL((k_gemm16t<2>), dim3(nwg), dim3(256), 0, d.stream, n, V, nk0, nk, D->ld,
                                       D->A16t, D->X16, inv[0], inv[1], inv[2], inv[3], D->Y16);
                return;
            }
            const int nt2 = (n + 31) / 32;
            const int nwg = std::min((nt2 + 3) / 4, 4096);
            if (D->kind16 == 1)
                hipLaunchKernelGGL((k_gemm16<1, 2>), dim3(nwg), dim3(256), 0, d.stream, n, V, D->Vp, D->ld, D->A16,
                                   D->X16, inv[0], inv[1], inv[2], inv[3], D->Y16);
            else
                hipLaunchKernelGGL((k_gemm16<2, 2>), dim3(nwg), dim3(256), 0, d.stream, n, V, D->Vp, D->ld, D->A16,
                                   D->X16, inv[0], inv[1], inv[2], inv[3], D->Y16);
        };
        Profiler &pf = d.prof;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (pf.on(0)) {
            HIPCHECK(hipEventCreate(&e0));
            HIPCHECK(hipEventCreate(&e1));
            HIPCHECK(hipEventRecord(e0, d.stream));
        }
        launch();
        if (pf.on(0)) {
            HIPCHECK(hipEventRecord(e1, d.stream));
            pf.record(0, e0, e1, (double)n * n * 2.0 + kMaxBatch * (double)n * (2.0 + 8.0));
        }
        if (mass_mode(d)) {
            hipLaunchKernelGGL(k_gather_batch, dim3((V + 256 / kRowLanes - 1) / (256 / kRowLanes), nb), dim3(256), 0, d.stream, V, n, 0, d.row_ptr,
                               d.col, d.N, d.nnz(), d.pinv, D->vpos, D->Y16, X, d.mtmp);
            mass_precond(d, nb, d.mtmp, Y, DevCtl());
        } else {
            hipLaunchKernelGGL(k_gather_batch, dim3((V + 256 / kRowLanes - 1) / (256 / kRowLanes), nb), dim3(256), 0, d.stream, V, n, 1, d.row_ptr,
                               d.col, d.N, d.nnz(), d.pinv, D->vpos, D->Y16, X, Y);
        }
        HIPCHECK(hipGetLastError());
    } else {
        for (int s = 0; s < nb; ++s) apply_operator(d, X + (size_t)s * n, Y + (size_t)s * n, PB_APPLY_PRECOND, nullptr);
    }
}

// Lock-step GMRES for nb systems sharing the operator (each its own Arnoldi
// process, CGS2, Givens rotations, stopping rule |r_k| <= tol_s |pb_s|).
static void gmres_batch(DevMesh &d, int nb, const double *PB, double *X, const std::vector<double> &tol, int max_iter,
                        std::vector<int> &its, std::vector<double> &est)
{
    const int n = 2 * d.hm.V;
    const int m = std::min(max_iter, n);
    BatchWork &w = work(d, m, nb);
    hipStream_t st = d.stream;
    const int ks = 2 * (m + 1) + 1;   // kbuf stride per system
    const dim3 gv((n + 255) / 256, nb), b256(256);
    hipLaunchKernelGGL(k_bdots, dim3(1, nb), dim3(kDotThreads), 0, st, n, 1, PB, PB, w.kbuf, ks);
    std::vector<double> hb((size_t)ks * nb);
    HIPCHECK(hipMemcpyAsync(hb.data(), w.kbuf, sizeof(double) * ks * nb, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    std::vector<double> beta(nb), inv(nb);
    std::vector<char> done(nb, 0);
    its.assign(nb, 0);
    est.assign(nb, 0.0);
    for (int s = 0; s < nb; ++s) {
        beta[s] = std::sqrt(std::max(hb[(size_t)s * ks], 0.0));
        inv[s] = beta[s] > 0 ? 1.0 / beta[s] : 0.0;
        if (!(beta[s] > 0)) done[s] = 1;
    }
    HIPCHECK(hipMemcpyAsync(w.sc, inv.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_bscale, gv, b256, 0, st, n, w.sc, PB, w.basis);
    std::vector<std::vector<double>> H(nb, std::vector<double>((size_t)(m + 1) * m, 0.0));
    std::vector<std::vector<double>> cs(nb, std::vector<double>(m)), sn(nb, std::vector<double>(m)),
        g(nb, std::vector<double>(m + 1, 0.0));
    for (int s = 0; s < nb; ++s) g[s][0] = beta[s];
    int j = 0;
    for (j = 0; j < m; ++j) {
        bool all = true;
        for (int s = 0; s < nb; ++s) all = all && done[s];
        if (all) break;
        double *Vj = w.basis + (size_t)j * nb * n, *Wn = w.basis + (size_t)(j + 1) * nb * n;
        apply_batch(d, nb, Vj, Wn);
        double *h1 = w.kbuf, *h2 = w.kbuf + (j + 1), *nr = w.kbuf + 2 * (j + 1);
        hipLaunchKernelGGL(k_bdots, dim3(j + 1, nb), dim3(kDotThreads), 0, st, n, nb, w.basis, Wn, h1, ks);
        hipLaunchKernelGGL(k_bupdate, gv, b256, 0, st, n, j + 1, nb, w.basis, h1, ks, Wn, -1.0);
        hipLaunchKernelGGL(k_bdots, dim3(j + 1, nb), dim3(kDotThreads), 0, st, n, nb, w.basis, Wn, h2, ks);
        hipLaunchKernelGGL(k_bupdate, gv, b256, 0, st, n, j + 1, nb, w.basis, h2, ks, Wn, -1.0);
        hipLaunchKernelGGL(k_bdots, dim3(1, nb), dim3(kDotThreads), 0, st, n, 1, Wn, Wn, nr, ks);
        hipLaunchKernelGGL(k_bnormalize, gv, b256, 0, st, n, nr, ks, Wn);
        HIPCHECK(hipMemcpyAsync(hb.data(), w.kbuf, sizeof(double) * ks * nb, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        for (int s = 0; s < nb; ++s) {
            if (done[s]) continue;
            const double *hs = &hb[(size_t)s * ks];
            double *col = &H[s][(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) col[i] = hs[i] + hs[j + 1 + i];
            col[j + 1] = std::sqrt(std::max(hs[2 * (j + 1)], 0.0));
            for (int i = 0; i < j; ++i) {   // explicit FMAs: same arithmetic as the device Givens kernel
                const double a = std::fma(cs[s][i], col[i], sn[s][i] * col[i + 1]);
                col[i + 1] = std::fma(-sn[s][i], col[i], cs[s][i] * col[i + 1]);
                col[i] = a;
            }
            const double den = std::sqrt(std::fma(col[j], col[j], col[j + 1] * col[j + 1]));
            cs[s][j] = col[j] / den;
            sn[s][j] = col[j + 1] / den;
            col[j] = den;
            col[j + 1] = 0.0;
            g[s][j + 1] = -sn[s][j] * g[s][j];
            g[s][j] = cs[s][j] * g[s][j];
            its[s] = j + 1;
            est[s] = std::fabs(g[s][j + 1]) / beta[s];
            if (std::fabs(g[s][j + 1]) <= tol[s] * beta[s] || !(den > 0.0)) done[s] = 1;
        }
    }
    const int kmax = std::max(1, *std::max_element(its.begin(), its.end()));
    std::vector<double> y((size_t)nb * (m + 1), 0.0);
    for (int s = 0; s < nb; ++s) {
        const int k = its[s];
        double *ys = &y[(size_t)s * (m + 1)];
        for (int i = k - 1; i >= 0; --i) {
            double a = g[s][i];
            for (int l = i + 1; l < k; ++l) a -= H[s][(size_t)l * (m + 1) + i] * ys[l];
            ys[i] = a / H[s][(size_t)i * (m + 1) + i];
        }
    }
    HIPCHECK(hipMemcpyAsync(w.y, y.data(), sizeof(double) * y.size(), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_bcombine, gv, b256, 0, st, n, kmax, nb, w.basis, w.y, m + 1, X);
    HIPCHECK(hipGetLastError());
}

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

pb_status solve_multi(DevMesh &d, int n_sets, const pb_charges *sets, pb_result *out)
{
    check_solvable(d);
    if (!d.dense) {   // matrix-free: the far field is recomputed per product anyway
        pb_status worst = PB_OK;
        for (int k = 0; k < n_sets; ++k) {
            pb_status st = solve_on_mesh(d, &sets[k], &out[k]);
            if (st < 0) return st;
            worst = std::max(worst, st);
        }
        return worst;
    }
    const int V = d.hm.V, n = 2 * V;
    Dense &D = *d.dense;
    hipStream_t st = d.stream;
    pb_status worst = PB_OK;
    for (int c0 = 0; c0 < n_sets; c0 += kMaxBatch) {
        const int nb = std::min(kMaxBatch, n_sets - c0);
        const int m = std::min(d.prm.precision >= PB_MIXED_BF16 ? d.opt.inner_max_iter : d.opt.max_iter, n);
        BatchWork &w = work(d, m, nb);
        const double t0 = now_s();
        for (int s = 0; s < nb; ++s) {
            charges_to_device(d, &sets[c0 + s]);
            check_charges_inside(d, sets[c0 + s].n);
            formulation_rhs(d, sets[c0 + s].n, d.qbuf, w.B + (size_t)s * n);
        }
        HIPCHECK(hipStreamSynchronize(st));
        const double t1 = now_s();
        if (mass_mode(d)) mass_precond(d, nb, w.B, w.PB, DevCtl());
        else
            for (int s = 0; s < nb; ++s) kr_precond(st, V, d.pinv, w.B + (size_t)s * n, w.PB + (size_t)s * n);
        HIPCHECK(hipStreamSynchronize(st));
        const double t2 = now_s();
        std::vector<int> its(nb, 0), itot(nb, 0), outer(nb, 1);
        std::vector<double> est(nb, 0.0);
        if (D.A16) {
            // iterative refinement: r = pb - P^-1 A_hi u; batched inner GMRES on the 16-bit far field
            HIPCHECK(hipMemsetAsync(w.U, 0, sizeof(double) * n * nb, st));
            HIPCHECK(hipMemcpyAsync(w.R, w.PB, sizeof(double) * n * nb, hipMemcpyDeviceToDevice, st));
            std::vector<double> nb2(nb), rel(nb, 1.0), tol(nb);
            hipLaunchKernelGGL(k_bdots, dim3(1, nb), dim3(kDotThreads), 0, st, n, 1, w.PB, w.PB, w.kbuf, 1);
            HIPCHECK(hipMemcpyAsync(nb2.data(), w.kbuf, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
            HIPCHECK(hipStreamSynchronize(st));
            std::vector<char> conv(nb, 0);
            for (int k = 1; k <= 30; ++k) {
                for (int s = 0; s < nb; ++s)
                    tol[s] = conv[s] ? 1.0 : std::max(d.opt.inner_tol, 0.5 * d.opt.tol / std::max(rel[s], 1e-300));
                D.level = 0;
                gmres_batch(d, nb, w.R, w.C, tol, m, its, est);
                D.level = 1;
                for (int s = 0; s < nb; ++s) {
                    if (conv[s]) continue;
                    itot[s] += its[s];
                    outer[s] = k;
                    kr_axpy(st, n, 1.0, w.C + (size_t)s * n, w.U + (size_t)s * n);
                    apply_operator(d, w.U + (size_t)s * n, w.R + (size_t)s * n, PB_APPLY_PRECOND, nullptr);
                    kr_scale_copy(st, n, w.R + (size_t)s * n, -1.0, w.R + (size_t)s * n);
                    kr_axpy(st, n, 1.0, w.PB + (size_t)s * n, w.R + (size_t)s * n);
                }
                hipLaunchKernelGGL(k_bdots, dim3(1, nb), dim3(kDotThreads), 0, st, n, 1, w.R, w.R, w.kbuf, 1);
                std::vector<double> r2(nb);
                HIPCHECK(hipMemcpyAsync(r2.data(), w.kbuf, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
                HIPCHECK(hipStreamSynchronize(st));
                bool all = true;
                for (int s = 0; s < nb; ++s) {
                    if (conv[s]) continue;
                    rel[s] = nb2[s] > 0 ? std::sqrt(r2[s] / nb2[s]) : 0.0;
                    if (rel[s] <= d.opt.tol || itot[s] >= d.opt.max_iter) conv[s] = 1;
                    else all = false;
                }
                // converged systems get a zero right-hand side in later sweeps
                for (int s = 0; s < nb; ++s)
                    if (conv[s]) HIPCHECK(hipMemsetAsync(w.R + (size_t)s * n, 0, sizeof(double) * n, st));
                if (all) break;
            }
        } else {
            std::vector<double> tol(nb, d.opt.tol);
            gmres_batch(d, nb, w.PB, w.U, tol, m, its, est);
            itot = its;
        }
        HIPCHECK(hipStreamSynchronize(st));
        const double t3 = now_s();
        for (int s = 0; s < nb; ++s) {
            pb_status r = finish_result(d, &sets[c0 + s], w.PB + (size_t)s * n, w.U + (size_t)s * n, itot[s], outer[s],
                                        (t1 - t0) / nb, (t2 - t1) / nb, (t3 - t2) / nb, &out[c0 + s]);
            if (r < 0) return r;
            worst = std::max(worst, r);
        }
    }
    return worst;
}

}  // namespace pbm
