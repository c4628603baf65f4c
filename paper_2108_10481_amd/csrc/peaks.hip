// Measured MI355X (gfx950) peaks for the roofline denominators: FP32 and FP64
// fused multiply-add, the two transcendentals of the far-field kernels
// (v_exp_f32, v_rsq_f32), exp mixed with FMAs that feed it and with FMAs of
// independent chains (whether the transcendental unit issues beside the FMA
// pipeline), the BF16 matrix-core
// instruction v_mfma_f32_16x16x32_bf16, and an HBM read stream and copy.
// Measurement only: no part of the solver calls this library.
//
// Every loop runs kChains independent dependency chains per lane so that the
// issue rate, not the latency, limits it; values stay bounded (x -> a x + b
// with |a| < 1, x -> 2^-x, x -> 1 / sqrt(x)) and every chain's result is
// stored, so no work can be removed.  Timing: HIP events around one launch
// after a warm-up launch, on a grid of 8 resident blocks of 256 lanes per CU.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 8;
constexpr int kBlock = 256;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int KIND>
__global__ __launch_bounds__(kBlock) void k_valu32(int iters, float a, float b, float *out)
{
    float x[kChains], y[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = y[c] = 0.25f + 1e-4f * (threadIdx.x + c);
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if (KIND == 0) {                    // 1 FMA
                x[c] = fmaf(x[c], a, b);
            } else if (KIND == 1) {             // 1 exp2 (negation is an input modifier)
                x[c] = __builtin_amdgcn_exp2f(-x[c]);
            } else if (KIND == 2) {             // 1 rsqrt
                x[c] = __builtin_amdgcn_rsqf(x[c]);
            } else if (KIND == 3) {             // 4 FMA + 1 exp2 of their result
                float z = fmaf(x[c], a, b);
                z = fmaf(z, a, b);
                z = fmaf(z, a, b);
                z = fmaf(z, a, b);
                x[c] = __builtin_amdgcn_exp2f(-z);
            } else if (KIND == 4) {             // 4 FMA, 1 exp2 of an independent chain
                float z = fmaf(x[c], a, b);
                z = fmaf(z, a, b);
                z = fmaf(z, a, b);
                x[c] = fmaf(z, a, b);
                y[c] = __builtin_amdgcn_exp2f(-y[c]);
            } else {                            // 1 FMA, 1 exp2 of an independent chain
                x[c] = fmaf(x[c], a, b);
                y[c] = __builtin_amdgcn_exp2f(-y[c]);
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c] + y[c];
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_fma64(int iters, double a, double b, double *out)
{
    double x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = 0.25 + 1e-4 * (threadIdx.x + c);
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = fma(x[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

// four independent 16 x 16 accumulators per wavefront, each updated by
// v_mfma_f32_16x16x32_bf16 (16 * 16 * 32 multiply-adds) once per iteration
__global__ __launch_bounds__(kBlock) void k_mfma_bf16(int iters, float *out)
{
    bf16x8 a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = (__bf16)(1e-3f * (threadIdx.x + k));
        b[k] = (__bf16)(1e-3f * (threadIdx.x - k));
    }
    f32x4 c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[j], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) s += c[j][0] + c[j][1] + c[j][2] + c[j][3];
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_read(size_t n4, const float4 *__restrict__ in, float *out)
{
    float s = 0.0f;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (size_t)gridDim.x * kBlock) {
        const float4 v = in[i];
        s += v.x + v.y + v.z + v.w;
    }
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_copy(size_t n4, const float4 *__restrict__ in, float4 *__restrict__ out)
{
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (size_t)gridDim.x * kBlock)
        out[i] = in[i];
}

int cu_count()
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, 0) != hipSuccess) return -1;
    return p.multiProcessorCount;
}

template <typename F>
int timed(F launch, float *ms)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
    launch();   // warm-up
    if (hipDeviceSynchronize() != hipSuccess) return -1;
    (void)hipEventRecord(e0, nullptr);
    launch();
    (void)hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess) return -1;
    (void)hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

extern "C" {

// Number of compute units of device 0 (-1 on error).
int pbk_cu_count(void) { return cu_count(); }

// kind 0..3: FP32 FMA, exp2, rsqrt, 4 FMA + 1 exp2 of their result; kind 4:
// FP64 FMA; kind 5: BF16 MFMA 16x16x32; kind 6: 4 FMA + 1 independent exp2;
// kind 7: 1 FMA + 1 independent exp2.  blocks_per_cu blocks of 256 lanes per CU,
// iters loop iterations.  *ms: duration of one timed launch; *lane_ops:
// instructions times lanes executed (MFMA: multiply-adds).  Returns 0 on
// success.
int pbk_compute(int kind, int blocks_per_cu, int iters, float *ms, double *lane_ops)
{
    const int cus = cu_count();
    if (cus <= 0 || blocks_per_cu < 1 || iters < 1 || kind < 0 || kind > 7) return -1;
    const int blocks = cus * blocks_per_cu;
    void *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * kBlock * sizeof(double)) != hipSuccess) return -1;
    const double lanes = (double)blocks * kBlock;
    int rc = 0;
    switch (kind) {
    case 0: rc = timed([&] { k_valu32<0><<<blocks, kBlock>>>(iters, 0.999f, 1e-3f, (float *)out); }, ms);
            *lane_ops = lanes * iters * kChains; break;
    case 1: rc = timed([&] { k_valu32<1><<<blocks, kBlock>>>(iters, 0.999f, 1e-3f, (float *)out); }, ms);
            *lane_ops = lanes * iters * kChains; break;
    case 2: rc = timed([&] { k_valu32<2><<<blocks, kBlock>>>(iters, 0.999f, 1e-3f, (float *)out); }, ms);
            *lane_ops = lanes * iters * kChains; break;
    case 3: rc = timed([&] { k_valu32<3><<<blocks, kBlock>>>(iters, 0.999f, 1e-3f, (float *)out); }, ms);
            *lane_ops = lanes * iters * kChains * 5.0; break;
    case 4: rc = timed([&] { k_fma64<<<blocks, kBlock>>>(iters, 0.999, 1e-3, (double *)out); }, ms);
            *lane_ops = lanes * iters * kChains; break;
    case 5: rc = timed([&] { k_mfma_bf16<<<blocks, kBlock>>>(iters, (float *)out); }, ms);
            *lane_ops = (double)blocks * (kBlock / 64) * iters * 4.0 * 16 * 16 * 32; break;
    case 6: rc = timed([&] { k_valu32<4><<<blocks, kBlock>>>(iters, 0.999f, 1e-3f, (float *)out); }, ms);
            *lane_ops = lanes * iters * kChains * 5.0; break;
    default: rc = timed([&] { k_valu32<5><<<blocks, kBlock>>>(iters, 0.999f, 1e-3f, (float *)out); }, ms);
            *lane_ops = lanes * iters * kChains * 2.0; break;
    }
    (void)hipFree(out);
    return rc;
}

// HBM: kind 0 reads `bytes` (a multiple of 16), kind 1 copies `bytes` into a
// second buffer.  *ms: one timed launch; the byte count moved is bytes (read)
// or 2 bytes (copy).
int pbk_stream(int kind, size_t bytes, float *ms)
{
    const int cus = cu_count();
    if (cus <= 0 || bytes < 16 || bytes % 16) return -1;
    const int blocks = cus * 8;
    void *a = nullptr, *b = nullptr, *o = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) return -1;
    if (hipMemset(a, 0, bytes) != hipSuccess) { (void)hipFree(a); return -1; }
    int rc;
    if (kind == 0) {
        if (hipMalloc(&o, (size_t)blocks * kBlock * sizeof(float)) != hipSuccess) { (void)hipFree(a); return -1; }
        rc = timed([&] { k_read<<<blocks, kBlock>>>(bytes / 16, (const float4 *)a, (float *)o); }, ms);
        (void)hipFree(o);
    } else {
        if (hipMalloc(&b, bytes) != hipSuccess) { (void)hipFree(a); return -1; }
        rc = timed([&] { k_copy<<<blocks, kBlock>>>(bytes / 16, (const float4 *)a, (float4 *)b); }, ms);
        (void)hipFree(b);
    }
    (void)hipFree(a);
    return rc;
}

}  // extern "C"
