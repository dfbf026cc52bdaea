// Inference of the learned proposal network inside a wavefront, on BF16
// MFMA with FP32 accumulation, shared by the annealing kernels and the
// network's own inference entry point.
//
// The 64 lanes of a wave each bring one feature vector (their chain's chosen
// coordinate).  The wave evaluates the transposed network
//     H1^T = act(W1^T Z^T + b1),  H2^T = act(W2^T H1^T + b2),  O^T = W3^T H2^T + b3
// (act = relu, or GELU for the Gaussian network kind)
// on v_mfma_f32_16x16x32_bf16 in four column tiles of 16 chains, so that the
// accumulator layout of one layer (lane l holds rows 4(l/16)+j, j<4, of column
// l%16) is already the B-operand layout of the next: the K index of a layer's
// operand element i in lane group g is relabelled as
//     kperm(g, i) = 4g + i (i < 4),  16 + 4g + (i - 4) (i >= 4)
// inside each 32-wide K block, and the weights (the A operands) are packed
// with the same relabelling.  Hidden activations therefore never leave
// registers.  Features enter layer 1 split into a BF16 high part (lane group 0)
// and a BF16 remainder (lane group 1) against the same weights, so the input
// layer sees them to about 16 bits; biases are added in FP32 as the
// accumulator's initial value.  Hidden activations are rounded to BF16 before
// each product, as in the training kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa_mlp_common.hpp"

namespace sa {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Packed network: MFMA A-operand fragments (64 lanes x 8 BF16 = 1 KiB each)
// followed by the FP32 biases.
constexpr uint32_t kFrag = 64 * 16;
constexpr uint32_t kNetL1 = 0;                      // 8 fragments: row tile rt
constexpr uint32_t kNetL2 = kNetL1 + 8 * kFrag;     // 32 fragments: [rt][kb]
constexpr uint32_t kNetL3 = kNetL2 + 32 * kFrag;    // 4 fragments: [kb]
constexpr uint32_t kNetB1 = kNetL3 + 4 * kFrag;     // 128 floats
constexpr uint32_t kNetB2 = kNetB1 + kHidden * 4;   // 128 floats
constexpr uint32_t kNetB3 = kNetB2 + kHidden * 4;   // 4 floats (b3, 0, 0)
constexpr uint32_t kNetBytes = kNetB3 + 16;
static_assert(kNetBytes % 16 == 0, "packed network must be a whole number of 16-byte words");

__host__ __device__ __forceinline__ uint32_t kperm(uint32_t g, uint32_t i)
{
    return i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4);
}

// BF16 bits of element i of lane `lane` of packed fragment `frag` (0..43),
// from the FP32 parameter vector (layout in sa_mlp_common.hpp).
__host__ __device__ __forceinline__ uint16_t pack_element(const float *theta, uint32_t frag, uint32_t lane,
                                                          uint32_t i)
{
    const uint32_t g = lane >> 4, m = lane & 15;
    float v = 0.0f;
    if (frag < 8) {  // layer 1, row tile frag: W1[i][16 rt + m] for the high and remainder groups
        if (g < 2 && i < (uint32_t)kInputs) v = theta[kOffW1 + i * kHidden + 16 * frag + m];
    } else if (frag < 40) {  // layer 2, [rt][kb]
        const uint32_t rt = (frag - 8) >> 2, kb = (frag - 8) & 3;
        v = theta[kOffW2 + (32 * kb + kperm(g, i)) * kHidden + 16 * rt + m];
    } else {  // layer 3, [kb]: rows 0 (mu) and 1 (s)
        const uint32_t kb = frag - 40;
        if (m < 2) v = theta[kOffW3 + (32 * kb + kperm(g, i)) * 2 + m];
    }
    return f32_to_bf16_bits(v);
}

__device__ __forceinline__ bf16x8 frag_at(const unsigned char *net, uint32_t off, uint32_t lane)
{
    return *reinterpret_cast<const bf16x8 *>(net + off + 16 * lane);
}

__device__ __forceinline__ floatx4 f4_at(const unsigned char *net, uint32_t off)
{
    return *reinterpret_cast<const floatx4 *>(net + off);
}

__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }

typedef short short2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Two FP32 values as a word of two BF16 (one v_cvt_pk_bf16_f32, round to
// nearest even), relu applied as a signed 16-bit integer max of the bit
// patterns (one v_pk_max_i16; a negative value, -0 included, has the sign bit
// set, and rounding keeps the sign, so relu(bf16(a)) = bf16(relu(a))).
__device__ __forceinline__ uint32_t relu_pack(float a, float b)
{
    const bf16x2 h = __builtin_convertvector(float2v{a, b}, bf16x2);
    const short2v m = __builtin_elementwise_max(__builtin_bit_cast(short2v, h), short2v{0, 0});
    return __builtin_bit_cast(uint32_t, m);
}

// Two FP32 pre-activations as a word of two BF16 GELU values (GELU in FP32,
// then one v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t gelu_pack(float a, float b)
{
    const bf16x2 h = __builtin_convertvector(float2v{act(a, kNetGeluGauss), act(b, kNetGeluGauss)}, bf16x2);
    return __builtin_bit_cast(uint32_t, h);
}

template <int KIND> __device__ __forceinline__ uint32_t act_pack(float a, float b)
{
    if constexpr (KIND == kNetGeluGauss) return gelu_pack(a, b);
    else return relu_pack(a, b);
}

__device__ __forceinline__ bf16x8 words(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3)
{
    return __builtin_bit_cast(bf16x8, u32x4{w0, w1, w2, w3});
}

// (mu, s) of this lane's feature vector z[0..5].  Every lane of the wave must
// call it (the products are wave-wide).  `net` is the packed network in LDS;
// KIND selects the hidden activation (NetKind).
template <int KIND = kNetReluCauchy>
__device__ __forceinline__ void net_forward(const unsigned char *net, const float (&z)[kInputs], float &mu, float &s)
{
    const uint32_t lane = threadIdx.x & 63u, g = lane >> 4, col = lane & 15u;

    // Layer-1 B operands: features of chains 16 ct + col, high part in group 0
    // and BF16 remainder in group 1.
    bf16x8 b1[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
#pragma unroll
        for (int i = 0; i < 8; ++i) b1[ct][i] = to_bf16(0.0f);
#pragma unroll
        for (int i = 0; i < kInputs; ++i) {
            const float v = __shfl(z[i], 16 * ct + col, 64);
            const __bf16 hi = to_bf16(v);
            const __bf16 lo = to_bf16(v - (float)hi);
            b1[ct][i] = g == 0 ? hi : (g == 1 ? lo : to_bf16(0.0f));
        }
    }

    // Layer 1 -> layer-2 B operands: word (rt & 1) * 2 + j / 2 of h1[ct][rt / 2]
    // holds rows 4g + j, j + 1 of row tile rt.
    uint32_t h1[4][4][4];
#pragma unroll
    for (int rt = 0; rt < 8; ++rt) {
        const bf16x8 a = frag_at(net, kNetL1 + rt * kFrag, lane);
        const floatx4 bias = f4_at(net, kNetB1 + 4 * (16 * rt + 4 * g));
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1[ct], bias, 0, 0, 0);
            h1[ct][rt >> 1][(rt & 1) * 2 + 0] = act_pack<KIND>(acc[0], acc[1]);
            h1[ct][rt >> 1][(rt & 1) * 2 + 1] = act_pack<KIND>(acc[2], acc[3]);
        }
    }

    // Layer 2 -> layer-3 B operands h2[ct][kb], same packing.
    uint32_t h2[4][4][4];
#pragma unroll
    for (int rt = 0; rt < 8; ++rt) {
        const floatx4 bias = f4_at(net, kNetB2 + 4 * (16 * rt + 4 * g));
        floatx4 acc[4] = {bias, bias, bias, bias};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const bf16x8 a = frag_at(net, kNetL2 + (rt * 4 + kb) * kFrag, lane);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    a, words(h1[ct][kb][0], h1[ct][kb][1], h1[ct][kb][2], h1[ct][kb][3]), acc[ct], 0, 0, 0);
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            h2[ct][rt >> 1][(rt & 1) * 2 + 0] = act_pack<KIND>(acc[ct][0], acc[ct][1]);
            h2[ct][rt >> 1][(rt & 1) * 2 + 1] = act_pack<KIND>(acc[ct][2], acc[ct][3]);
        }
    }

    // Layer 3: rows 0 and 1 of the single row tile are mu and s.
    const floatx4 b3 = f4_at(net, kNetB3);
    const floatx4 init = g == 0 ? floatx4{b3[0], b3[1], 0.0f, 0.0f} : floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    floatx4 o[4] = {init, init, init, init};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const bf16x8 a = frag_at(net, kNetL3 + kb * kFrag, lane);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
            o[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                a, words(h2[ct][kb][0], h2[ct][kb][1], h2[ct][kb][2], h2[ct][kb][3]), o[ct], 0, 0, 0);
    }

    // Lane c's outputs sit in lane c % 16 of column tile c / 16.
    mu = 0.0f;
    s = 0.0f;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const float m = __shfl(o[ct][0], (int)col, 64);
        const float v = __shfl(o[ct][1], (int)col, 64);
        if ((lane >> 4) == (uint32_t)ct) {
            mu = m;
            s = v;
        }
    }
}

// Copy the packed network from global memory into LDS (whole workgroup).
__device__ __forceinline__ void stage_net(unsigned char *lds, const unsigned char *net)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(net);
    uint4 *dst = reinterpret_cast<uint4 *>(lds);
    for (uint32_t i = threadIdx.x; i < kNetBytes / 16; i += blockDim.x) dst[i] = src[i];
}

}  // namespace mlp

// Pack the FP32 parameter vector `theta` (device) into `net` (device,
// mlp::kNetBytes bytes) on stream s.
hipError_t launch_pack_net(const float *theta, unsigned char *net, hipStream_t s);

}  // namespace sa
