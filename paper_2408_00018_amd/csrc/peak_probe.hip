// Issue-rate probe for the VALU instruction classes the annealing step uses.
//
// Each kernel keeps 16 independent dependency chains per lane and runs `iters`
// rounds of one operation on each, so the measured rate is the instruction's
// throughput rather than its latency.  The results are written to `sink` so
// nothing is optimised away.  Used by the benchmark to check the per-class
// costs the ALU roofline assumes (full rate vs quarter rate).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa_device.hpp"
#include "sa_mlp_common.hpp"

namespace {

constexpr int kChains = 16;

enum Kind : int {
    kFmaF32 = 0,
    kMadU64 = 1,
    kMulHiU32 = 2,
    kXor3 = 3,
    kSinF32 = 4,
    kSqrtF32 = 5,
    kExp2F32 = 6,
    kFmaF64 = 7,
    kNumKinds = 8
};

__global__ void __launch_bounds__(256) probe_kernel(int kind, int iters, uint32_t *sink)
{
    extern __shared__ float lds_pad[];  // sized by the host to cap workgroups per CU
    if (threadIdx.x == 0 && iters < 0) lds_pad[0] = 0.0f;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t u[kChains];
    float f[kChains];
    double g[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        u[i] = tid * 2654435761u + i;
        f[i] = 0.25f + 1e-3f * (float)((tid + i) & 255);
        g[i] = 0.25 + 1e-3 * (double)((tid + i) & 255);
    }
    const uint32_t k1 = 0xD2511F53u, k2 = 0x9E3779B9u;
    switch (kind) {
    case kFmaF32:
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int i = 0; i < kChains; ++i) f[i] = fmaf(f[i], 0.999f, 1e-4f);
        break;
    case kMadU64:
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int i = 0; i < kChains; ++i) {
                const uint64_t p = (uint64_t)u[i] * k1;
                u[i] = (uint32_t)(p >> 32) ^ (uint32_t)p;
            }
        break;
    case kMulHiU32:
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int i = 0; i < kChains; ++i) u[i] = __umulhi(u[i], k1) + k2;
        break;
    case kXor3:
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int i = 0; i < kChains; ++i) u[i] = u[i] ^ u[(i + 1) % kChains] ^ (k2 + it);
        break;
    case kSinF32:
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int i = 0; i < kChains; ++i) f[i] = __builtin_amdgcn_sinf(f[i]);
        break;
    case kSqrtF32:
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int i = 0; i < kChains; ++i) f[i] = __builtin_amdgcn_sqrtf(f[i]);
        break;
    case kExp2F32:
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int i = 0; i < kChains; ++i) f[i] = __builtin_amdgcn_exp2f(-f[i]);
        break;
    case kFmaF64:
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int i = 0; i < kChains; ++i) g[i] = fma(g[i], 0.999, 1e-4);
        break;
    default:
        break;
    }
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) acc ^= u[i] ^ __float_as_uint(f[i]) ^ (uint32_t)__double_as_longlong(g[i]);
    sink[tid] = acc;
}

// One hardware transcendental per element: 0 sin(2 pi t), 1 cos(2 pi t) (the
// instructions take revolutions), 2 sqrt(t), 3 2^t; 4 e^t - 1 as the FP32
// Ackley increment computes it (sa::expm1_f32); 5 the FP32 GELU of the
// Gaussian proposal network and 6 its derivative (sa::mlp::act, act_grad);
// 7 log2(t) (v_log_f32); 8 1/t (v_rcp_f32, the centre families' terms).
__global__ void __launch_bounds__(256) accuracy_kernel(int op, const float *in, float *out, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float t = in[i];
    float r;
    switch (op) {
    case 0: r = __builtin_amdgcn_sinf(t); break;
    case 1: r = __builtin_amdgcn_cosf(t); break;
    case 2: r = __builtin_amdgcn_sqrtf(t); break;
    case 3: r = __builtin_amdgcn_exp2f(t); break;
    case 4: r = sa::expm1_f32(t); break;
    case 5: r = sa::mlp::act(t, sa::mlp::kNetGeluGauss); break;
    case 6: r = sa::mlp::act_grad(t, sa::mlp::kNetGeluGauss); break;
    case 7: r = __builtin_amdgcn_logf(t); break;
    default: r = __builtin_amdgcn_rcpf(t); break;
    }
    out[i] = r;
}

}  // namespace

extern "C" {

// Apply hardware transcendental `op` (see accuracy_kernel) to n FP32 values:
// in and out are device pointers to n floats.  Synchronises.  Used to measure
// the instructions' error against an FP64 evaluation of the same inputs.
int sa_peak_accuracy(int op, const float *in, float *out, uint32_t n)
{
    if (op < 0 || op > 8 || !in || !out) return -1;
    if (n == 0) return 0;
    hipLaunchKernelGGL(accuracy_kernel, dim3((n + 255) / 256), dim3(256), 0, 0, op, in, out, n);
    if (hipGetLastError() != hipSuccess) return -3;
    return hipDeviceSynchronize() == hipSuccess ? 0 : -3;
}

// Run `kind` on `blocks` x 256 lanes for `iters` rounds of 16 chains; return
// the elapsed milliseconds (HIP events on the null stream) in *ms.  The
// operation count is blocks * 256 * iters * 16 lane-operations.
int sa_peak_probe(int kind, int blocks, int iters, float *ms)
{
    if (kind < 0 || kind >= kNumKinds || blocks <= 0 || iters <= 0 || !ms) return -1;
    uint32_t *sink = nullptr;
    if (hipMalloc(&sink, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) return -2;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    hipLaunchKernelGGL(probe_kernel, dim3(blocks), dim3(256), 0, 0, kind, 1, sink);  // warm-up
    (void)hipEventRecord(a, 0);
    hipLaunchKernelGGL(probe_kernel, dim3(blocks), dim3(256), 0, 0, kind, iters, sink);
    (void)hipEventRecord(b, 0);
    hipError_t e = hipEventSynchronize(b);
    float t = 0.0f;
    (void)hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(sink);
    *ms = t;
    return e == hipSuccess ? 0 : -3;
}

// The same operation with one 64-lane workgroup per wave and enough dynamic
// LDS per workgroup that at most `waves_per_simd` waves share each SIMD of a
// 256-CU device (160 KiB LDS per CU): shows how many waves a SIMD needs to
// reach the instruction's issue rate.  Operation count:
// 256 * 4 * waves_per_simd * 64 * iters * 16.
int sa_peak_probe_occupancy(int kind, int waves_per_simd, int iters, float *ms)
{
    if (kind < 0 || kind >= kNumKinds || waves_per_simd < 1 || waves_per_simd > 8 || iters <= 0 || !ms) return -1;
    const int blocks = 256 * 4 * waves_per_simd;
    const size_t lds = (size_t)(160 * 1024) / (4 * (size_t)waves_per_simd) - 1024;
    uint32_t *sink = nullptr;
    if (hipMalloc(&sink, (size_t)blocks * 64 * sizeof(uint32_t)) != hipSuccess) return -2;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    hipLaunchKernelGGL(probe_kernel, dim3(blocks), dim3(64), lds, 0, kind, 1, sink);
    (void)hipEventRecord(a, 0);
    hipLaunchKernelGGL(probe_kernel, dim3(blocks), dim3(64), lds, 0, kind, iters, sink);
    (void)hipEventRecord(b, 0);
    hipError_t e = hipEventSynchronize(b);
    float t = 0.0f;
    (void)hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(sink);
    *ms = t;
    return e == hipSuccess ? 0 : -3;
}

}  // extern "C"
