// Training of the learned proposal network on gfx950 (sa_mlp_* in
// include/sa.h).
//
// Network (per chosen coordinate): z (6 features) -> 128 (act) -> 128
// (act) -> 2 outputs (location and log scale of a distribution over the
// coordinate's scaled displacement); loss = negative log-likelihood of
// accepted displacements.  Two kinds (NetKind): relu with a Cauchy
// distribution, GELU with a Gaussian one.  Master parameters and Adam
// moments are FP32; the three weight matrices are used in BF16.  The
// 128x128 layer and its two backward products run on BF16 MFMA
// (v_mfma_f32_16x16x32_bf16, FP32 accumulate); the 6-wide input layer and
// the 2-wide output layer, whose shapes waste a matrix tile, run on VALU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "sa_device.hpp"
#include "sa_host.hpp"
#include "sa_mlp_common.hpp"
#include "sa_mlp_net.hpp"

using sa::fail;

namespace {

using namespace sa::mlp;


// ---------------------------------------------------------------------------
// One training pass (forward, loss, backward, gradient) fused per block of
// kRows minibatch rows: a workgroup of four waves takes blocks
// blockIdx.x, blockIdx.x + gridDim.x, ... and keeps its running sums of every
// parameter's gradient in registers; the reduction kernel adds the
// workgroups' sums in workgroup order.  Per block, in LDS:
//   z (gathered features), a1 = z W1 + b1 (FP32, VALU), h1 = bf16(act(a1))
//   row-major and transposed;
//   a2 = h1 W2 + b2 on MFMA (B operand: the transposed BF16 W2, staged in
//   LDS once per workgroup, 16-byte reads), h2 = bf16(act(a2)) (kept as FP32);
//   outputs, loss and d(loss)/d(outputs) per row (VALU, wave reductions);
//   da2 = (W3 dO) act'(a2), FP32 and BF16 (row-major and transposed);
//   dW2 += h1^T da2 on MFMA (K = the block's rows; accumulators stay in
//   registers across blocks);
//   da1 = (da2 W2^T) act'(a1) on MFMA (B operand: the staged W2 read
//   column-wise, eight 2-byte reads per fragment);
//   the small gradients (W1, b1, b2, W3, b3) and the loss, summed over the
//   block's rows by the thread that owns each.
// Every weight and bias a thread uses is loaded once, before the first
// block's rows are gathered, so their latency overlaps the gather's.
// The mean over the minibatch enters through inv_b in d(loss)/d(outputs).
// MFMA v_mfma_f32_16x16x32_bf16 operand layout: lane l holds A[l%16][8(l/16)
// + i] and B[8(l/16) + i][l%16], i < 8; the accumulator holds C[4(l/16) +
// j][l%16], j < 4.
// ---------------------------------------------------------------------------
constexpr int kRows = 32;                     // minibatch rows per block
constexpr int kLdF = kHidden + 4;             // FP32 row stride (bank spread)
constexpr int kLdH = kHidden + 8;             // BF16 row stride, [row][hidden]
constexpr int kLdT = kRows + 8;               // BF16 row stride, [hidden][row]
constexpr uint32_t kSmallGrads = kInputs * kHidden + kHidden + kHidden + 2 * kHidden + 2;  // W1, b1, b2, W3, b3
static_assert(kSmallGrads == kNumParams - kHidden * kHidden, "every parameter but W2");
constexpr uint32_t kPartStride = kNumParams + 1;  // per workgroup: every gradient, then the loss sum
constexpr int kSmallPerThread = (int)((kSmallGrads + 1 + 255) / 256);

struct TrainLds {
    uint16_t w2t[kHidden][kHidden + 8];  // BF16 W2 transposed, [out][in] (padded rows)
    float w3[kHidden][2];
    float z[kRows][8];
    float delta[kRows];
    float dmu[kRows], ds[kRows], loss[kRows];
    float a1[kRows][kLdF];
    float a2[kRows][kLdF];   // a2, then da1
    float h2[kRows][kLdF];
    float da2[kRows][kLdF];
    uint16_t h1[kRows][kLdH], h1t[kHidden][kLdT];
    uint16_t da2b[kRows][kLdH], da2t[kHidden][kLdT];
};

// Parameter index of the small-gradient slot q (0 .. kSmallGrads; the last
// slot is the loss, index kNumParams).
__device__ __forceinline__ uint32_t small_param(uint32_t q)
{
    if (q < kOffB1 + kHidden) return q;                                   // W1, b1
    if (q < kOffB1 + 2 * kHidden) return kOffB2 + (q - kOffB1 - kHidden);  // b2
    if (q < kOffB1 + 4 * kHidden) return kOffW3 + (q - kOffB1 - 2 * kHidden);  // W3
    if (q < kSmallGrads) return kOffB3 + (q - kOffB1 - 4 * kHidden);     // b3
    return kNumParams;                                                    // loss
}

__device__ __forceinline__ bf16x8 lds8(const uint16_t *p) { return *reinterpret_cast<const bf16x8 *>(p); }

// Minibatch row r of training step t: a record index drawn with replacement
// (Philox counters (r, t, 0, 4) under the training seed), or idx[r].
__device__ __forceinline__ uint32_t row_record(const uint32_t *idx, uint32_t r, uint32_t t, uint64_t nrec, uint32_t k0,
                                               uint32_t k1)
{
    if (idx) return idx[r];
    const sa::Ctr c = sa::philox4x32_10(sa::Ctr{r, t, 0u, 4u}, k0, k1);
    const uint64_t wide = ((uint64_t)c.w0 << 32) | c.w1;
    return (uint32_t)__umul64hi(wide, nrec);
}

template <int KIND>
__global__ void __launch_bounds__(256)
    train_rows(const float *records, uint64_t nrec, const uint32_t *idx, uint32_t batch, uint32_t t, uint32_t k0,
               uint32_t k1, float inv_b, const float *theta, const uint16_t *W1b, const uint16_t *W2t,
               const uint16_t *W3b, float *partial)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    TrainLds &L = *reinterpret_cast<TrainLds *>(lds_raw);
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, g = lane >> 4, c16 = lane & 15u;
    // ---- weights: W2^T into LDS (all eight 16-byte loads of a thread in
    // flight before the first LDS store), the rest into registers
    constexpr uint32_t kStage = kHidden * kHidden / 8 / 256;
    uint4 w2v[kStage];
#pragma unroll
    for (uint32_t k = 0; k < kStage; ++k) {
        const uint32_t e = tid + 256u * k, row = e / (kHidden / 8), c8 = e % (kHidden / 8);
        w2v[k] = *reinterpret_cast<const uint4 *>(W2t + row * kHidden + 8 * c8);
    }
#pragma unroll
    for (uint32_t k = 0; k < kStage; ++k) {
        const uint32_t e = tid + 256u * k, row = e / (kHidden / 8), c8 = e % (kHidden / 8);
        *reinterpret_cast<uint4 *>(&L.w2t[row][8 * c8]) = w2v[k];
    }
    const uint32_t jt = tid & (kHidden - 1);  // hidden unit of this thread in the elementwise steps
    float w1[kInputs];
#pragma unroll
    for (int i = 0; i < kInputs; ++i) w1[i] = bf16_bits_to_f32(W1b[i * kHidden + jt]);
    const float b1j = theta[kOffB1 + jt];
    const float w3j0 = bf16_bits_to_f32(W3b[2 * jt + 0]), w3j1 = bf16_bits_to_f32(W3b[2 * jt + 1]);
    if (tid < 2u * kHidden) L.w3[tid >> 1][tid & 1u] = bf16_bits_to_f32(W3b[tid]);
    const float b2c[2] = {theta[kOffB2 + 16 * (2 * wave) + c16], theta[kOffB2 + 16 * (2 * wave + 1) + c16]};
    const float b30 = theta[kOffB3 + 0], b31 = theta[kOffB3 + 1];

    floatx4 dw2[16];  // this wave's 16 tiles of dW2: tile q -> (mt, nt) = (4 wave + q / 4, 4 (q % 4) ... )
#pragma unroll
    for (int q = 0; q < 16; ++q) dw2[q] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    float small[kSmallPerThread];
#pragma unroll
    for (int k = 0; k < kSmallPerThread; ++k) small[k] = 0.0f;

    const uint32_t blocks = batch / kRows;
    for (uint32_t blk = blockIdx.x; blk < blocks; blk += gridDim.x) {
        const uint32_t r0 = blk * kRows;
        // ---- gather
        if (tid < (uint32_t)kRows) {
            const float *rec = records + (size_t)row_record(idx, r0 + tid, t, nrec, k0, k1) * kRecord;
#pragma unroll
            for (int i = 0; i < kInputs; ++i) L.z[tid][i] = rec[i];
            L.delta[tid] = rec[kInputs];
        }
        __syncthreads();
        // ---- layer 1 (VALU): thread -> hidden j, rows (tid / 128) * 16 + k
        {
            const uint32_t j = jt, rb = (tid >> 7) * (kRows / 2);
            for (uint32_t k = 0; k < (uint32_t)kRows / 2; ++k) {
                const uint32_t r = rb + k;
                float a = b1j;
#pragma unroll
                for (int i = 0; i < kInputs; ++i) a = fmaf(L.z[r][i], w1[i], a);
                L.a1[r][j] = a;
                const uint16_t h = f32_to_bf16_bits(act(a, KIND));
                L.h1[r][j] = h;
                L.h1t[j][r] = h;
            }
        }
        __syncthreads();
        // ---- layer 2 (MFMA): wave -> column tiles 2 wave, 2 wave + 1 of both row tiles
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t rt = q >> 1, ct = 2 * wave + (q & 1);
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kb = 0; kb < kHidden / 32; ++kb) {
                const bf16x8 a = lds8(&L.h1[16 * rt + c16][32 * kb + 8 * g]);
                const bf16x8 b = lds8(&L.w2t[16 * ct + c16][32 * kb + 8 * g]);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const uint32_t r = 16 * rt + 4 * g + jj, col = 16 * ct + c16;
                const float v = acc[jj] + b2c[q & 1];
                L.a2[r][col] = v;
                L.h2[r][col] = bf16_bits_to_f32(f32_to_bf16_bits(act(v, KIND)));
            }
        }
        __syncthreads();
        // ---- outputs and loss: wave -> rows 8 wave + lane / 8, eight lanes per
        // row (hidden units sub, sub + 8, ...), then a three-step lane reduction
        {
            const uint32_t r = 8 * wave + (lane >> 3), sub = lane & 7u;
            float o0 = 0.0f, o1 = 0.0f;
#pragma unroll
            for (uint32_t q = 0; q < (uint32_t)kHidden / 8; ++q) {
                const uint32_t j = sub + 8 * q;
                o0 = fmaf(L.h2[r][j], L.w3[j][0], o0);
                o1 = fmaf(L.h2[r][j], L.w3[j][1], o1);
            }
#pragma unroll
            for (int off = 4; off > 0; off >>= 1) {
                o0 += __shfl_xor(o0, off, 64);
                o1 += __shfl_xor(o1, off, 64);
            }
            if (sub == 0) {
                const float mu = o0 + b30, sl = o1 + b31;
                const float is = expf(-sl);
                const float rr = (L.delta[r] - mu) * is;  // standardised residual
                float dmu, dsl, lr;
                if (KIND == kNetGeluGauss) {  // s + ln sqrt(2 pi) + r^2 / 2
                    dmu = -rr * is * inv_b;
                    dsl = (1.0f - rr * rr) * inv_b;
                    lr = sl + 0.918938533204672742f + 0.5f * rr * rr;
                } else {  // s + ln pi + ln(1 + r^2)
                    const float qq = 1.0f + rr * rr;
                    dmu = -2.0f * rr * is / qq * inv_b;
                    dsl = (1.0f - 2.0f * rr * rr / qq) * inv_b;
                    lr = sl + 1.14472988584940017f + logf(qq);
                }
                L.dmu[r] = dmu;
                L.ds[r] = dsl;
                L.loss[r] = lr;
            }
        }
        __syncthreads();
        // ---- da2 = (W3 dO) act'(a2): thread -> hidden j, rows (tid / 128) * 16 + k
        {
            const uint32_t j = jt, rb = (tid >> 7) * (kRows / 2);
            for (uint32_t k = 0; k < (uint32_t)kRows / 2; ++k) {
                const uint32_t r = rb + k;
                const float dh = w3j0 * L.dmu[r] + w3j1 * L.ds[r];
                const float da = dh * act_grad(L.a2[r][j], KIND);
                L.da2[r][j] = da;
                const uint16_t b = f32_to_bf16_bits(da);
                L.da2b[r][j] = b;
                L.da2t[j][r] = b;
            }
        }
        __syncthreads();
        // ---- dW2 += h1^T da2 (K = the block's rows): wave -> row tiles 2 wave, 2 wave + 1 (of 8)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const uint32_t mt = 2 * wave + (q >> 3), nt = q & 7;
            const bf16x8 a = lds8(&L.h1t[16 * mt + c16][8 * g]);
            const bf16x8 b = lds8(&L.da2t[16 * nt + c16][8 * g]);
            dw2[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, dw2[q], 0, 0, 0);
        }
        // ---- da1 = (da2 W2^T) act'(a1), into the a2 buffer
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t rt = q >> 1, ct = 2 * wave + (q & 1);
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kb = 0; kb < kHidden / 32; ++kb) {
                const bf16x8 a = lds8(&L.da2b[16 * rt + c16][32 * kb + 8 * g]);
                // B(k = out, n = in) = W2[in][out] = w2t[out][in]
                bf16x8 b;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    b[e] = __builtin_bit_cast(__bf16, L.w2t[32 * kb + 8 * g + e][16 * ct + c16]);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
            }
            // (a2 was last read by the da2 step, before the barrier above)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const uint32_t r = 16 * rt + 4 * g + jj, col = 16 * ct + c16;
                L.a2[r][col] = acc[jj] * act_grad(L.a1[r][col], KIND);
            }
        }
        __syncthreads();
        // ---- the small gradients and the loss, summed over the block's rows
        // (the a2 buffer now holds da1)
#pragma unroll
        for (int k = 0; k < kSmallPerThread; ++k) {
            const uint32_t qs = tid + 256u * k;
            if (qs > kSmallGrads) break;
            float sacc = 0.0f;
            if (qs < kOffB1) {  // W1[i][j]
                const uint32_t i = qs / kHidden, j = qs % kHidden;
                for (int r = 0; r < kRows; ++r) sacc = fmaf(L.z[r][i], L.a2[r][j], sacc);
            } else if (qs < kOffB1 + kHidden) {  // b1
                const uint32_t j = qs - kOffB1;
                for (int r = 0; r < kRows; ++r) sacc += L.a2[r][j];
            } else if (qs < kOffB1 + 2 * kHidden) {  // b2
                const uint32_t j = qs - kOffB1 - kHidden;
                for (int r = 0; r < kRows; ++r) sacc += L.da2[r][j];
            } else if (qs < kOffB1 + 4 * kHidden) {  // W3[j][c]
                const uint32_t u = qs - kOffB1 - 2 * kHidden, j = u / 2, c = u % 2;
                for (int r = 0; r < kRows; ++r) sacc = fmaf(L.h2[r][j], c ? L.ds[r] : L.dmu[r], sacc);
            } else if (qs < kSmallGrads) {  // b3
                const uint32_t c = qs - kOffB1 - 4 * kHidden;
                for (int r = 0; r < kRows; ++r) sacc += c ? L.ds[r] : L.dmu[r];
            } else {  // loss
                for (int r = 0; r < kRows; ++r) sacc += L.loss[r];
            }
            small[k] += sacc;
        }
        __syncthreads();
    }
    // ---- this workgroup's sums
    float *out = partial + (size_t)blockIdx.x * kPartStride;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint32_t mt = 2 * wave + (q >> 3), nt = q & 7;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
            out[kOffW2 + (16 * mt + 4 * g + jj) * kHidden + 16 * nt + c16] = dw2[q][jj];
    }
#pragma unroll
    for (int k = 0; k < kSmallPerThread; ++k) {
        const uint32_t qs = tid + 256u * k;
        if (qs <= kSmallGrads) out[small_param(qs)] = small[k];
    }
}

enum ReduceMode { kReduceGrad = 0, kReduceAdam = 1, kReduceRefresh = 2 };

constexpr uint32_t kReduceWaves = 8;  // waves per reduction workgroup, 64 parameters each

// Sum the workgroups' partial gradients (kReduceGrad: into g; the loss sum /
// batch into *loss), or also take an Adam step (Kingma & Ba) on the FP32
// master parameters (kReduceAdam; the mean loss also goes to
// loss_trace[step] when given), or neither (kReduceRefresh).  A workgroup
// takes 64 parameters (one per lane); wave w adds the partials of workgroups
// w, w + 8, ... into four running sums (a fixed order), and wave 0 adds the
// eight wave sums in order: the result does not depend on timing.
// Every mode refreshes the BF16 weight matrices: W1, W2 (transposed,
// [out][in]), W3.
__global__ void __launch_bounds__(64 * kReduceWaves)
    reduce_step(int mode, const float *partial, uint32_t groups, float inv_b, float *theta, float *g, float *m,
                float *v, float lr, float beta1, float beta2, float eps, float c1, float c2, float *loss,
                float *loss_trace, uint32_t step, uint16_t *W1b, uint16_t *W2t, uint16_t *W3b)
{
    __shared__ float part[kReduceWaves][64];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t i = blockIdx.x * 64u + lane;
    const bool live = i <= kNumParams;
    if (mode != kReduceRefresh) {
        // four running sums (workgroups w, w + 8, w + 16, w + 24 of each step
        // of 32), so four loads are in flight at a time
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
        if (live) {
            const float *pp = partial + i;
            const size_t st = (size_t)kReduceWaves * kPartStride;
            uint32_t w = wave;
            for (; w + 3 * kReduceWaves < groups; w += 4 * kReduceWaves) {
                a0 += pp[(size_t)w * kPartStride];
                a1 += pp[(size_t)w * kPartStride + st];
                a2 += pp[(size_t)w * kPartStride + 2 * st];
                a3 += pp[(size_t)w * kPartStride + 3 * st];
            }
            for (; w < groups; w += kReduceWaves) a0 += pp[(size_t)w * kPartStride];
        }
        part[wave][lane] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
    if (wave != 0 || !live) return;
    if (mode != kReduceRefresh) {
        float s = 0.0f;
#pragma unroll
        for (uint32_t w = 0; w < kReduceWaves; ++w) s += part[w][lane];
        if (i == kNumParams) {
            const float mean = s * inv_b;
            loss[0] = mean;
            if (loss_trace) loss_trace[step] = mean;
            return;
        }
        g[i] = s;
        if (mode == kReduceAdam) {
            const float mi = beta1 * m[i] + (1.0f - beta1) * s;
            const float vi = beta2 * v[i] + (1.0f - beta2) * s * s;
            m[i] = mi;
            v[i] = vi;
            theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        }
    }
    if (i == kNumParams) return;
    const uint16_t b = f32_to_bf16_bits(theta[i]);
    if (i < kOffB1) {
        W1b[i - kOffW1] = b;
    } else if (i >= kOffW2 && i < kOffB2) {
        const uint32_t e = i - kOffW2;
        W2t[(e % kHidden) * kHidden + e / kHidden] = b;
    } else if (i >= kOffW3 && i < kOffB3) {
        W3b[i - kOffW3] = b;
    }
}

// Pack theta into MFMA fragment order (one thread per fragment lane) and copy
// the biases.
__global__ void pack_net(const float *theta, unsigned char *net)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 44 * 64) {
        const uint32_t frag = t >> 6, lane = t & 63;
        uint16_t *dst = reinterpret_cast<uint16_t *>(net + frag * kFrag + 16 * lane);
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) dst[i] = pack_element(theta, frag, lane, i);
    }
    float *b = reinterpret_cast<float *>(net + kNetB1);
    if (t < 2 * kHidden) b[t] = t < kHidden ? theta[kOffB1 + t] : theta[kOffB2 + t - kHidden];
    if (t < 4) reinterpret_cast<float *>(net + kNetB3)[t] = t < 2 ? theta[kOffB3 + t] : 0.0f;
}

// (mu, s) for `rows` feature vectors Z[rows][6], one chain per lane as in the
// annealing kernels.
template <int KIND>
__global__ void __launch_bounds__(256) infer_rows(const unsigned char *net, const float *Z, uint32_t rows, float *out)
{
    __shared__ __align__(16) unsigned char lds[kNetBytes];
    stage_net(lds, net);
    __syncthreads();
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = r < rows;
    float z[kInputs];
#pragma unroll
    for (int i = 0; i < kInputs; ++i) z[i] = live ? Z[(size_t)r * kInputs + i] : 0.0f;
    float mu, s;
    net_forward<KIND>(lds, z, mu, s);
    if (live) {
        out[2 * (size_t)r + 0] = mu;
        out[2 * (size_t)r + 1] = s;
    }
}

}  // namespace

namespace sa {
hipError_t launch_pack_net(const float *theta, unsigned char *net, hipStream_t s)
{
    hipLaunchKernelGGL(pack_net, dim3(11), dim3(256), 0, s, theta, net);
    return hipGetLastError();
}
}  // namespace sa

struct sa_mlp {
    hipStream_t stream = nullptr;
    uint32_t max_batch = 0;
    unsigned char *ws = nullptr;
    float *theta, *g, *m, *v, *loss;
    uint16_t *W1b, *W2t, *W3b;        // BF16 weight matrices (W2 transposed: [out][in])
    uint32_t *idx;                    // explicit minibatch indices (sa_mlp_grad)
    unsigned char *net;               // packed copy for inference
    float *partial;                   // per workgroup: gradient sums and the loss sum
    float *trace;                     // kTraceChunk per-step mean losses, copied out chunk by chunk
    uint32_t t = 0;                   // Adam steps taken
    int kind = kNetReluCauchy;
};

namespace {

constexpr uint32_t kTraceChunk = 4096;

// Workgroups of a training pass over `batch` rows.
uint32_t train_groups(uint32_t batch) { return std::min<uint32_t>(batch / kRows, 256u); }

sa_status mlp_alloc(sa_mlp *p)
{
    const size_t H = kHidden;
    size_t off = 0;
    std::vector<std::pair<void **, size_t>> parts = {
        {(void **)&p->theta, kNumParams * 4}, {(void **)&p->g, kNumParams * 4}, {(void **)&p->m, kNumParams * 4},
        {(void **)&p->v, kNumParams * 4},     {(void **)&p->loss, 4},            {(void **)&p->W1b, kInputs * H * 2},
        {(void **)&p->W2t, H * H * 2},        {(void **)&p->W3b, H * 2 * 2},
        {(void **)&p->idx, (size_t)p->max_batch * 4}, {(void **)&p->net, kNetBytes},
        {(void **)&p->partial, (size_t)train_groups(p->max_batch) * kPartStride * 4},
        {(void **)&p->trace, kTraceChunk * 4}};
    std::vector<size_t> at;
    for (auto &q : parts) {
        at.push_back(off);
        off = sa::align_up(off + q.second);
    }
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&p->ws), off);
    if (e != hipSuccess) return fail(SA_ERR_NOMEM, "hipMalloc(%zu): %s", off, hipGetErrorString(e));
    for (size_t i = 0; i < parts.size(); ++i) *parts[i].first = p->ws + at[i];
    SA_HIP(hipMemsetAsync(p->ws, 0, off, p->stream));
    return SA_OK;
}

// One fused forward/backward pass over a minibatch (rows from idx, or drawn
// for step t) into the per-workgroup partial sums.
sa_status mlp_rows(sa_mlp *p, const float *records, uint64_t nrec, const uint32_t *idx, uint32_t batch, uint32_t t,
                   uint64_t seed)
{
    const uint32_t groups = train_groups(batch);
    const float inv_b = 1.0f / (float)batch;
    const size_t lds = sizeof(TrainLds);
    if (p->kind == kNetGeluGauss)
        hipLaunchKernelGGL(train_rows<kNetGeluGauss>, dim3(groups), dim3(256), lds, p->stream, records, nrec, idx,
                           batch, t, (uint32_t)seed, (uint32_t)(seed >> 32), inv_b, p->theta, p->W1b, p->W2t,
                           p->W3b, p->partial);
    else
        hipLaunchKernelGGL(train_rows<kNetReluCauchy>, dim3(groups), dim3(256), lds, p->stream, records, nrec, idx,
                           batch, t, (uint32_t)seed, (uint32_t)(seed >> 32), inv_b, p->theta, p->W1b, p->W2t,
                           p->W3b, p->partial);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

sa_status mlp_reduce(sa_mlp *p, int mode, uint32_t batch, float lr, float *loss_trace, uint32_t step)
{
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    float c1 = 1.0f, c2 = 1.0f;
    if (mode == kReduceAdam) {
        c1 = 1.0f - std::pow(beta1, (float)(p->t + 1));
        c2 = 1.0f - std::pow(beta2, (float)(p->t + 1));
    }
    const uint32_t groups = batch ? train_groups(batch) : 0;
    const float inv_b = batch ? 1.0f / (float)batch : 0.0f;
    hipLaunchKernelGGL(reduce_step, dim3((kNumParams + 1 + 63) / 64), dim3(64 * kReduceWaves), 0, p->stream, mode,
                       p->partial, groups, inv_b, p->theta, p->g, p->m, p->v, lr, beta1, beta2, eps, c1, c2, p->loss, loss_trace,
                       step, p->W1b, p->W2t, p->W3b);
    SA_HIP(hipGetLastError());
    if (mode == kReduceAdam) p->t += 1;
    return SA_OK;
}

}  // namespace

extern "C" {

sa_status sa_mlp_create(uint32_t max_batch, void *stream, sa_mlp **out)
{
    sa::g_last_error.clear();
    if (!out) return fail(SA_ERR_INVALID, "out must not be NULL");
    *out = nullptr;
    if (max_batch == 0 || max_batch % 32 || max_batch > (1u << 20))
        return fail(SA_ERR_INVALID, "max_batch must be a multiple of 32 in [32, 2^20]");
    SA_FAULT_CHECK(sa::kFaultAlloc);
    sa_mlp *p = new (std::nothrow) sa_mlp;
    if (!p) return fail(SA_ERR_NOMEM, "host allocation failed");
    p->stream = reinterpret_cast<hipStream_t>(stream);
    p->max_batch = max_batch;
    if (sa_status st = mlp_alloc(p); st != SA_OK) {
        delete p;
        return st;
    }
    *out = p;
    return SA_OK;
}

sa_status sa_mlp_set_params(sa_mlp *p, const float *params)
{
    sa::g_last_error.clear();
    if (!p || !params) return fail(SA_ERR_INVALID, "null argument");
    SA_HIP(hipMemcpyAsync(p->theta, params, kNumParams * sizeof(float), hipMemcpyHostToDevice, p->stream));
    SA_HIP(hipMemsetAsync(p->m, 0, kNumParams * sizeof(float), p->stream));
    SA_HIP(hipMemsetAsync(p->v, 0, kNumParams * sizeof(float), p->stream));
    p->t = 0;
    if (sa_status st = mlp_reduce(p, kReduceRefresh, 0, 0.0f, nullptr, 0); st != SA_OK) return st;
    SA_HIP(hipStreamSynchronize(p->stream));
    return SA_OK;
}

sa_status sa_mlp_get_params(sa_mlp *p, float *params)
{
    sa::g_last_error.clear();
    if (!p || !params) return fail(SA_ERR_INVALID, "null argument");
    SA_HIP(hipStreamSynchronize(p->stream));
    SA_HIP(hipMemcpy(params, p->theta, kNumParams * sizeof(float), hipMemcpyDeviceToHost));
    return SA_OK;
}

sa_status sa_mlp_grad(sa_mlp *p, const float *records, uint64_t nrec, const uint32_t *idx, uint32_t batch,
                      float *grad, float *loss)
{
    sa::g_last_error.clear();
    if (!p || !records || !idx) return fail(SA_ERR_INVALID, "null argument");
    if (batch == 0 || batch % 32 || batch > p->max_batch)
        return fail(SA_ERR_INVALID, "batch must be a multiple of 32 and at most max_batch");
    for (uint32_t r = 0; r < batch; ++r)
        if (idx[r] >= nrec) return fail(SA_ERR_INVALID, "index %u out of range", r);
    SA_FAULT_CHECK(sa::kFaultLaunch);
    SA_HIP(hipMemcpyAsync(p->idx, idx, batch * sizeof(uint32_t), hipMemcpyHostToDevice, p->stream));
    if (sa_status st = mlp_rows(p, records, nrec, p->idx, batch, 0, 0); st != SA_OK) return st;
    if (sa_status st = mlp_reduce(p, kReduceGrad, batch, 0.0f, nullptr, 0); st != SA_OK) return st;
    SA_HIP(hipStreamSynchronize(p->stream));
    if (grad) SA_HIP(hipMemcpy(grad, p->g, kNumParams * sizeof(float), hipMemcpyDeviceToHost));
    if (loss) SA_HIP(hipMemcpy(loss, p->loss, sizeof(float), hipMemcpyDeviceToHost));
    return SA_OK;
}

sa_status sa_mlp_train(sa_mlp *p, const float *records, uint64_t nrec, uint32_t batch, uint32_t steps, float lr,
                       uint64_t seed, float *loss_trace)
{
    sa::g_last_error.clear();
    if (!p || !records) return fail(SA_ERR_INVALID, "null argument");
    if (nrec == 0 || nrec > 0xFFFFFFFFull) return fail(SA_ERR_INVALID, "nrec must be in [1, 2^32)");
    if (batch == 0 || batch % 32 || batch > p->max_batch)
        return fail(SA_ERR_INVALID, "batch must be a multiple of 32 and at most max_batch");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(SA_ERR_INVALID, "lr must be finite and > 0");
    SA_FAULT_CHECK(sa::kFaultLaunch);
    for (uint32_t s0 = 0; s0 < steps; s0 += kTraceChunk) {
        const uint32_t n = std::min(kTraceChunk, steps - s0);
        for (uint32_t k = 0; k < n; ++k) {
            if (sa_status st = mlp_rows(p, records, nrec, nullptr, batch, p->t, seed); st != SA_OK) return st;
            if (sa_status st = mlp_reduce(p, kReduceAdam, batch, lr, loss_trace ? p->trace : nullptr, k); st != SA_OK)
                return st;
        }
        if (loss_trace) {
            SA_HIP(hipStreamSynchronize(p->stream));
            SA_HIP(hipMemcpy(loss_trace + s0, p->trace, n * sizeof(float), hipMemcpyDeviceToHost));
        }
    }
    SA_HIP(hipStreamSynchronize(p->stream));
    return SA_OK;
}

sa_status sa_mlp_infer(sa_mlp *p, const float *Z, uint32_t rows, float *out)
{
    sa::g_last_error.clear();
    if (!p || !Z || !out) return fail(SA_ERR_INVALID, "null argument");
    if (rows == 0) return SA_OK;
    SA_FAULT_CHECK(sa::kFaultLaunch);
    hipError_t e = sa::launch_pack_net(p->theta, p->net, p->stream);
    if (e != hipSuccess) return fail(SA_ERR_DEVICE, "pack launch: %s", hipGetErrorString(e));
    if (p->kind == kNetGeluGauss)
        hipLaunchKernelGGL(infer_rows<kNetGeluGauss>, dim3((rows + 255) / 256), dim3(256), 0, p->stream, p->net, Z,
                           rows, out);
    else
        hipLaunchKernelGGL(infer_rows<kNetReluCauchy>, dim3((rows + 255) / 256), dim3(256), 0, p->stream, p->net, Z,
                           rows, out);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

sa_status sa_mlp_set_kind(sa_mlp *p, int kind)
{
    sa::g_last_error.clear();
    if (!p) return fail(SA_ERR_INVALID, "null trainer");
    if (kind != SA_NET_RELU_CAUCHY && kind != SA_NET_GELU_GAUSS) return fail(SA_ERR_INVALID, "unknown network kind %d", kind);
    p->kind = kind;
    return SA_OK;
}

void sa_mlp_destroy(sa_mlp *p)
{
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    if (p->ws) (void)hipFree(p->ws);
    delete p;
}

}  // extern "C"
