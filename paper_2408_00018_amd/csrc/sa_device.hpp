// Device-side building blocks of the gfx950 annealing kernels: the
// counter-based generator, the uniform/coordinate maps and the cost terms.
//
// Everything here is written for wave64 CDNA hardware.  FP32 code calls the
// hardware transcendental instructions directly (v_sin_f32/v_cos_f32 take
// their argument in revolutions, v_sqrt_f32, v_exp_f32); FP64 code uses the
// device math library so that the FP64 path follows the same arithmetic as a
// plain FP64 evaluation of the definitions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sa {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11).  Ten rounds of two 32x32->64 multiplies; the key is
// bumped by the Weyl constants between rounds.  The key is wave-uniform, so
// its schedule lives in scalar registers.
// ---------------------------------------------------------------------------
struct Ctr {
    uint32_t w0, w1, w2, w3;
};

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Three-input XOR in one VALU instruction: CDNA4's v_bitop3_b32 with truth
// table 0x96 (A ^ B ^ C).  Left to itself the compiler emits two v_xor_b32.
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t key)
{
    return __builtin_amdgcn_bitop3_b32(a, b, key, 0x96);
}

__device__ __forceinline__ Ctr philox4x32_10(Ctr c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c.w0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c.w2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        // Rounds 1-2 use plain XORs: where their inputs are wave-uniform (a
        // uniform counter word) the compiler keeps them on the scalar unit;
        // the later rounds use the single-instruction three-input XOR.
        if (round < 2)
            c = Ctr{hi1 ^ c.w1 ^ k0, lo1, hi0 ^ c.w3 ^ k1, lo0};
        else
            c = Ctr{xor3_key(hi1, c.w1, k0), lo1, xor3_key(hi0, c.w3, k1), lo0};
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return c;
}

constexpr uint32_t kTagMove = 0u;
constexpr uint32_t kTagInit = 1u;
constexpr uint32_t kTagSos = 5u;  // stochastic exchange decision
constexpr uint32_t kTagLearn = 3u;  // draws of the learned proposal
constexpr uint32_t kInitLevel = 0xFFFFFFFFu;

// Uniform in [0,1) from the top 24 bits (exact in FP32 and FP64).
__device__ __forceinline__ float u24f(uint32_t r) { return (float)(r >> 8) * 0x1p-24f; }
__device__ __forceinline__ double u24d(uint32_t r) { return (double)(r >> 8) * 0x1p-24; }
template <typename R> __device__ __forceinline__ R u24(uint32_t r);
template <> __device__ __forceinline__ float u24<float>(uint32_t r) { return u24f(r); }
template <> __device__ __forceinline__ double u24<double>(uint32_t r) { return u24d(r); }

// Coordinate index in [0,n): high word of r * n.
__device__ __forceinline__ uint32_t pick(uint32_t r, uint32_t n) { return __umulhi(r, n); }

// ---------------------------------------------------------------------------
// FP32 hardware transcendentals.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// sin(2 pi t) and cos(2 pi t): the hardware instructions take revolutions.
__device__ __forceinline__ float hw_sin_rev(float t) { return __builtin_amdgcn_sinf(t); }
__device__ __forceinline__ float hw_cos_rev(float t) { return __builtin_amdgcn_cosf(t); }
// 2^t and log2(t)
__device__ __forceinline__ float hw_exp2(float t) { return __builtin_amdgcn_exp2f(t); }
__device__ __forceinline__ float hw_log2(float t) { return __builtin_amdgcn_logf(t); }

// e^x - 1 in FP32 (Ackley's increment): for |x| <= 1/2 the Taylor polynomial
// through x^9/9! in Horner form (truncation below 2^-26 relative, a few ulps
// of rounding), beyond it 2^(x log2 e) - 1 on the hardware exponential
// (|e^x - 1| >= 0.39 there, so the subtraction costs at most two bits).  Both
// forms are evaluated and one selected, so the lanes of a wave do not split.
__device__ __forceinline__ float expm1_f32(float x)
{
    float p = fmaf(x, 1.0f / 362880.0f, 1.0f / 40320.0f);
    p = fmaf(x, p, 1.0f / 5040.0f);
    p = fmaf(x, p, 1.0f / 720.0f);
    p = fmaf(x, p, 1.0f / 120.0f);
    p = fmaf(x, p, 1.0f / 24.0f);
    p = fmaf(x, p, 1.0f / 6.0f);
    p = fmaf(x, p, 0.5f);
    p = fmaf(x, p, 1.0f);
    const float small = x * p;
    const float large = hw_exp2(x * 1.44269504088896341f) - 1.0f;
    return fabsf(x) <= 0.5f ? small : large;
}

constexpr float kInv2Pi = 0.159154943091895335768883763372514362f;
constexpr float kInv4Pi2 = 0.0253302959105844428049187623077562f;  // 1 / (4 pi^2)
constexpr float kLog2e = 1.44269504088896340735992468100189214f;
constexpr float kLn2 = 0.693147180559945309417232121458176568f;
constexpr double kPi = 3.14159265358979323846;
constexpr double kE = 2.71828182845904523536;

// ---------------------------------------------------------------------------
// FP64 terms: written exactly as the definitions, in the order the full
// evaluation sums them (coordinate 0 first).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double schwefel_term_d(double y) { return y * sin(sqrt(fabs(y))); }
__device__ __forceinline__ double rastrigin_term_d(double y) { return y * y - 10.0 * cos(2.0 * kPi * y); }
__device__ __forceinline__ double ackley_from_sums_d(double s1, double s2, uint32_t n)
{
    const double dn = (double)n;
    return -20.0 * exp(-0.2 * sqrt(s1 / dn)) - exp(s2 / dn) + 20.0 + kE;
}

// ---------------------------------------------------------------------------
// FP32 increments, written without cancellation:
//   Schwefel   h(y) = y sin(sqrt|y|),  df = (h(y) - h(y')) / n
//   Rastrigin  g(y) = y^2 + 20 sin^2(pi y)   (= y^2 - 10 cos 2 pi y + 10)
//              g(y') - g(y) = dl*sg + 20 sin(pi dl) sin(pi sg),
//              dl = y' - y, sg = y' + y
//   Ackley     S1 += dl*sg;  S2 += cos 2pi y' - cos 2pi y = -2 sin(pi sg) sin(pi dl)
//              df = -20 e^a expm1(a' - a) - e^b expm1(dS2/n),
//              a = -0.2 sqrt(S1/n), b = S2/n,
//              a' - a = -0.2 (dS1/n) / (sqrt(S1'/n) + sqrt(S1/n))
// ---------------------------------------------------------------------------
__device__ __forceinline__ float schwefel_h(float y)
{
    return y * hw_sin_rev(hw_sqrt(fabsf(y)) * kInv2Pi);
}

}  // namespace sa
