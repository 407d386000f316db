// Achievable device peaks measured by the library's own probe kernels (diagnostic):
// a streaming copy for the HBM bandwidth, and register-only matrix-core loops for the
// BF16 and FP64 matrix-core rates.  The roofline fractions of the benchmarks are
// reported against these and against the published figures.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "op.hpp"

namespace ige {

namespace {

typedef __bf16 pbf8 __attribute__((ext_vector_type(8)));
typedef float pf4 __attribute__((ext_vector_type(4)));
typedef double pd4 __attribute__((ext_vector_type(4)));

// grid-stride copy of n 16-byte words
__global__ __launch_bounds__(256) void k_probe_copy(const uint4 *src, uint4 *dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// iters rounds of 16 independent 16x16x32 BF16 products per wave (fewer chains per wave
// leave the matrix core idle between dependent products: 8 chains reached 1.2 of the
// 2.0 PFLOP/s that 16 reach, measured); one value per wave out
__global__ __launch_bounds__(256) void k_probe_bf16(int iters, float *out)
{
    const int lane = threadIdx.x & 63;
    pbf8 a, b;
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(0.001f * (lane + i));
        b[i] = (__bf16)(0.002f * (lane - i));
    }
    pf4 acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = pf4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    if (lane == 0) out[blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)] = s;
}

// the same with the 16x16x4 FP64 product (8 chains: 16 measured slower)
__global__ __launch_bounds__(256) void k_probe_f64(int iters, double *out)
{
    const int lane = threadIdx.x & 63;
    const double a = 0.001 * lane, b = 0.002 * (64 - lane);
    pd4 acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = pd4{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    if (lane == 0) out[blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)] = s;
}

// best of reps timed launches (after one warm-up), in seconds
template <typename F>
double time_best(hipStream_t s, int reps, F launch)
{
    hipEvent_t e0, e1;
    IGE_HIP(hipEventCreate(&e0));
    IGE_HIP(hipEventCreate(&e1));
    double best = 1e30;
    try {
        launch();
        for (int i = 0; i < reps; ++i) {
            IGE_HIP(hipEventRecord(e0, s));
            launch();
            IGE_HIP(hipEventRecord(e1, s));
            IGE_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            IGE_HIP(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, (double)ms * 1e-3);
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

}  // namespace

double peak_probe(hipStream_t s, int kind)
{
    int dev = 0, ncu = 0;
    IGE_HIP(hipGetDevice(&dev));
    IGE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (kind == 0) {   // HBM: 1 GiB read and 1 GiB written per launch
        const int64_t n = (int64_t)1 << 26;   // 16-byte words
        DBuf<uint4> a, b;
        a.alloc((size_t)n);
        b.alloc((size_t)n);
        IGE_HIP(hipMemsetAsync(a.p, 0, a.bytes(), s));
        const dim3 grid((unsigned)(ncu * 4)), blk(256);   // 4 workgroups per CU: the fastest shape measured
        const double t = time_best(s, 5, [&] {
            hipLaunchKernelGGL(k_probe_copy, grid, blk, 0, s, a.p, b.p, n);
            IGE_HIP(hipGetLastError());
        });
        return 2.0 * (double)n * 16.0 / t / 1e9;   // GB/s
    }
    // matrix cores: four waves per SIMD on every CU
    const int wgs = ncu * 4, waves = wgs * 4, iters = 2048;
    if (kind == 1) {
        DBuf<float> out;
        out.alloc((size_t)waves);
        const double t = time_best(s, 5, [&] {
            hipLaunchKernelGGL(k_probe_bf16, dim3(wgs), dim3(256), 0, s, iters, out.p);
            IGE_HIP(hipGetLastError());
        });
        return (double)waves * iters * 16 * (2.0 * 16 * 16 * 32) / t / 1e12;   // TFLOP/s
    }
    DBuf<double> out;
    out.alloc((size_t)waves);
    const double t = time_best(s, 5, [&] {
        hipLaunchKernelGGL(k_probe_f64, dim3(wgs), dim3(256), 0, s, iters, out.p);
        IGE_HIP(hipGetLastError());
    });
    return (double)waves * iters * 8 * (2.0 * 16 * 16 * 4) / t / 1e12;   // TFLOP/s
}

}  // namespace ige
