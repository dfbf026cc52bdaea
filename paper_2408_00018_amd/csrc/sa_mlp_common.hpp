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

// GELU, tanh form: a/2 (1 + tanh(sqrt(2/pi) (a + 0.044715 a^3))), with
// tanh(u) = 1 - 2 / (exp(2u) + 1).
__host__ __device__ __forceinline__ float gelu(float a)
{
    const float u = 0.7978845608028654f * fmaf(0.044715f * a, a * a, a);
    const float t = 1.0f - 2.0f / (__expf(2.0f * u) + 1.0f);
    return 0.5f * a * (1.0f + t);
}

__host__ __device__ __forceinline__ float gelu_grad(float a)
{
    const float u = 0.7978845608028654f * fmaf(0.044715f * a, a * a, a);
    const float t = 1.0f - 2.0f / (__expf(2.0f * u) + 1.0f);
    const float du = 0.7978845608028654f * fmaf(3.0f * 0.044715f, a * a, 1.0f);
    return 0.5f * (1.0f + t) + 0.5f * a * (1.0f - t * t) * du;
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
