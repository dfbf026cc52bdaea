// Shapes, parameter layout and scalar helpers of the learned proposal network,
// shared by its training kernels and the annealing kernels that run it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sa {
namespace mlp {

constexpr int kInputs = 6;   // features of the chosen coordinate
constexpr int kHidden = 128; // width of both hidden layers
constexpr int kRecord = 7;   // captured record: 6 features + accepted scaled displacement

// Parameter vector layout: W1 [6][128], b1 [128], W2 [128][128], b2 [128],
// W3 [128][2], b3 [2] (row-major [in][out]).
constexpr uint32_t kOffW1 = 0;
constexpr uint32_t kOffB1 = kOffW1 + kInputs * kHidden;
constexpr uint32_t kOffW2 = kOffB1 + kHidden;
constexpr uint32_t kOffB2 = kOffW2 + kHidden * kHidden;
constexpr uint32_t kOffW3 = kOffB2 + kHidden;
constexpr uint32_t kOffB3 = kOffW3 + kHidden * 2;
constexpr uint32_t kNumParams = kOffB3 + 2;
static_assert(kNumParams == 17666, "parameter count");

// Network kinds (include/sa.h SA_NET_*): relu hidden activations with a
// Cauchy distribution over the scaled displacement and log-magnitude history
// features, or GELU activations with a Gaussian distribution (mean, log
// standard deviation) and the history's scaled displacements as they are.
enum NetKind : int { kNetReluCauchy = 0, kNetGeluGauss = 1 };

// Standard normal density phi(x) and the upper tail 1 - Phi(|x|) by the
// rational approximation 26.2.17 of Abramowitz and Stegun (Handbook of
// Mathematical Functions, 1964): 1 - Phi(x) = phi(x) (b1 t + ... + b5 t^5),
// t = 1 / (1 + p x), x >= 0, absolute error below 7.5e-8; FP32 with the
// hardware reciprocal and base-2 exponential.
__device__ __forceinline__ float normal_pdf(float x)
{
    return 0.398942280401432678f * __builtin_amdgcn_exp2f((x * x) * -0.721347520444481703f);
}

__device__ __forceinline__ float normal_upper_tail(float ax, float pdf)
{
    const float t = __builtin_amdgcn_rcpf(fmaf(0.2316419f, ax, 1.0f));
    float q = fmaf(t, 1.330274429f, -1.821255978f);
    q = fmaf(t, q, 1.781477937f);
    q = fmaf(t, q, -0.356563782f);
    q = fmaf(t, q, 0.319381530f);
    return pdf * (t * q);
}

// Phi(a) for any a.
__device__ __forceinline__ float normal_cdf(float a)
{
    const float ax = fminf(fabsf(a), 16.0f);
    const float tail = normal_upper_tail(ax, normal_pdf(ax));
    return a >= 0.0f ? 1.0f - tail : tail;
}

// Hidden activation of a kind: relu (derivative 0 at 0), or GELU
// a Phi(a) with derivative Phi(a) + a phi(a).
__device__ __forceinline__ float act(float a, int kind = kNetReluCauchy)
{
    if (kind == kNetGeluGauss) return a * normal_cdf(a);
    return fmaxf(a, 0.0f);
}

__device__ __forceinline__ float act_grad(float a, int kind = kNetReluCauchy)
{
    if (kind == kNetGeluGauss) {
        const float ax = fminf(fabsf(a), 16.0f);
        const float pdf = normal_pdf(ax);
        const float tail = normal_upper_tail(ax, pdf);
        return (a >= 0.0f ? 1.0f - tail : tail) + a * pdf;
    }
    return a > 0.0f ? 1.0f : 0.0f;
}

// FP32 <-> BF16 (round to nearest even; NaN stays NaN).
__host__ __device__ __forceinline__ uint16_t f32_to_bf16_bits(float f)
{
    const uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__host__ __device__ __forceinline__ float bf16_bits_to_f32(uint16_t b)
{
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}

}  // namespace mlp
}  // namespace sa
