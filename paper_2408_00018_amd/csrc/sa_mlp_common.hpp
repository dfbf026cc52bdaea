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

// Hidden activation: relu, with derivative 0 at 0.
__host__ __device__ __forceinline__ float act(float a) { return fmaxf(a, 0.0f); }

__host__ __device__ __forceinline__ float act_grad(float a) { return a > 0.0f ? 1.0f : 0.0f; }

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
