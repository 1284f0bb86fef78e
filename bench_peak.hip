// Issue-rate microbenchmark of the vector ALU on gfx950, for the roofline peaks the benchmark divides
// by: single-precision FMA (v_fma_f32 / v_fmac_f32, compiled with packed FP32 disabled like the
// library) with a scalar operand and with vector operands only, double-precision FMA (v_fma_f64) and
// the single-precision reciprocal square root (v_rsq_f32).  Each lane runs 8 or 16 independent
// dependency chains so that issue, not latency, bounds the loop; the grid puts 8 workgroups of 4 waves
// on each compute unit (8 wavefronts per SIMD).  On gfx950 single-precision instructions whose
// operands are all vector registers issue at about twice the rate of those that read a scalar
// register; double-precision ones run at the lower rate either way.
//
// C ABI: pk_run(kind, iters, blocks, &ms) launches one kernel of `blocks` workgroups of 256 lanes,
// times it with HIP events and returns the operations executed (an FMA counts 2, other operations 1);
// kind 0 = FP32 FMA with a scalar operand, 1 = FP64 FMA, 2 = FP32 rsq, 3 = FP32 add, 4 = FP32 FMA with
// vector operands only, 5 = FP64 add.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

constexpr int kChains = 16;
constexpr int kBlock = 256;

template <typename T>
__global__ __launch_bounds__(kBlock) void fma_kernel(int iters, T a, T b, T *sink)
{
    T acc[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc[k] = (T)(threadIdx.x + k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) acc[k] = acc[k] * a + b;
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += acc[k];
    if (s == (T)-1.2345) sink[blockIdx.x] = s;  // never true for these inputs; keeps the chains live
}

// acc = acc * a + b with a, b per lane (every operand a vector register): eight accumulators updated
// round-robin, 32 v_fma_f32 per loop trip in a fixed order (inline assembly of plain VALU FMAs, so
// the compiler can neither move a scalar operand in nor reorder the chains)
#define PK_FMA(i) "v_fma_f32 %" #i ", %8, %9, %" #i "\n"
#define PK_FMA8 PK_FMA(0) PK_FMA(1) PK_FMA(2) PK_FMA(3) PK_FMA(4) PK_FMA(5) PK_FMA(6) PK_FMA(7)
__global__ __launch_bounds__(kBlock) void fma_vv_kernel(int iters, float a0, float b0, float *sink)
{
    float x0 = (float)threadIdx.x * 1e-3f + 1.0f, x1 = x0 + 1, x2 = x0 + 2, x3 = x0 + 3, x4 = x0 + 4, x5 = x0 + 5,
          x6 = x0 + 6, x7 = x0 + 7;
    const float a = a0 + (float)(threadIdx.x & 1) * 1e-9f, b = b0 + (float)(threadIdx.x & 2) * 1e-9f;
    for (int i = 0; i < iters; ++i)
        asm volatile(PK_FMA8 PK_FMA8 PK_FMA8 PK_FMA8
                     : "+v"(x0), "+v"(x1), "+v"(x2), "+v"(x3), "+v"(x4), "+v"(x5), "+v"(x6), "+v"(x7)
                     : "v"(a), "v"(b));
    const float s = x0 + x1 + x2 + x3 + x4 + x5 + x6 + x7;
    if (s == -1.2345f) sink[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void add_kernel(int iters, T b, T *sink)
{
    T acc[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc[k] = (T)(threadIdx.x + k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) acc[k] = acc[k] + b;
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += acc[k];
    if (s == (T)-1.2345) sink[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void rsq_kernel(int iters, float *sink)
{
    float acc[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc[k] = 1.0f + (float)(threadIdx.x + k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) acc[k] = __builtin_amdgcn_rsqf(acc[k]);
    }
    float s = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += acc[k];
    if (s == -1.2345f) sink[blockIdx.x] = s;
}

void *g_sink = nullptr;

}  // namespace

extern "C" double pk_run(int kind, int iters, int blocks, float *ms)
{
    if (!g_sink && hipMalloc(&g_sink, (size_t)blocks * sizeof(double) + 4096) != hipSuccess) return -1.0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
    (void)hipEventRecord(e0, nullptr);
    if (kind == 0)
        hipLaunchKernelGGL(fma_kernel<float>, dim3(blocks), dim3(kBlock), 0, nullptr, iters, 0.999999f, 1e-7f,
                           (float *)g_sink);
    else if (kind == 1)
        hipLaunchKernelGGL(fma_kernel<double>, dim3(blocks), dim3(kBlock), 0, nullptr, iters, 0.999999999,
                           1e-12, (double *)g_sink);
    else if (kind == 2)
        hipLaunchKernelGGL(rsq_kernel, dim3(blocks), dim3(kBlock), 0, nullptr, iters, (float *)g_sink);
    else if (kind == 3)
        hipLaunchKernelGGL(add_kernel<float>, dim3(blocks), dim3(kBlock), 0, nullptr, iters, 1e-7f, (float *)g_sink);
    else if (kind == 4)
        hipLaunchKernelGGL(fma_vv_kernel, dim3(blocks), dim3(kBlock), 0, nullptr, iters / 2, 0.999999f, 1e-7f,
                           (float *)g_sink);
    else
        hipLaunchKernelGGL(add_kernel<double>, dim3(blocks), dim3(kBlock), 0, nullptr, iters, 1e-12,
                           (double *)g_sink);
    (void)hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t;
    // kind 4 runs iters / 2 trips of 32 FMAs, the others iters trips of kChains operations
    const double per_lane = kind == 4 ? (double)(iters / 2) * 32 * 2.0
                                      : (double)iters * kChains * ((kind == 0 || kind == 1) ? 2.0 : 1.0);
    return per_lane * kBlock * (double)blocks;
}
