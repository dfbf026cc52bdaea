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


__device__ __forceinline__ __bf16 bf16_of_bits(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

// k index of element i (0..7) of lane l in a 16x16x32 MFMA operand.
__device__ __forceinline__ int mfma_k(int lane, int i) { return (lane >> 4) * 8 + i; }

enum Epilogue { kEpiStore = 0, kEpiBiasAct = 1, kEpiActBwd = 2 };

// C(m, n) = sum_k A(m, k) B(k, n) with A(m,k) = A[m*am + k*ak] and
// B(k,n) = B[k*bk + n*bn] (BF16 bits), FP32 accumulate; one wave per 16x16
// tile; M, N multiples of 16, K a multiple of 32.  Epilogues:
//   kEpiStore     C = acc
//   kEpiBiasAct  C = acc + bias[n] (pre-activation), H = act(C)
//   kEpiActBwd   C = acc * act'(aux(m, n))
template <int EPI>
__global__ void __launch_bounds__(256)
    gemm_bf16(int M, int N, int K, const uint16_t *A, int am, int ak, const uint16_t *B, int bk, int bn, float *C,
              int ldc, const float *bias, const float *aux, float *H, int kind)
{
    const int lane = threadIdx.x & 63;
    const int tile = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const int tiles_n = N >> 4;
    if (tile >= (M >> 4) * tiles_n) return;
    const int tm = tile / tiles_n, tn = tile % tiles_n;
    const int row = (tm << 4) + (lane & 15), col = (tn << 4) + (lane & 15);
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = k0 + mfma_k(lane, i);
            a[i] = bf16_of_bits(A[(size_t)row * am + (size_t)k * ak]);
            b[i] = bf16_of_bits(B[(size_t)k * bk + (size_t)col * bn]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = (tm << 4) + (lane >> 4) * 4 + j, c = (tn << 4) + (lane & 15);
        float v = acc[j];
        if (EPI == kEpiBiasAct) {
            v += bias[c];
            H[(size_t)r * ldc + c] = bf16_bits_to_f32(f32_to_bf16_bits(act(v, kind)));
        }
        if (EPI == kEpiActBwd) v *= act_grad(aux[(size_t)r * ldc + c], kind);
        C[(size_t)r * ldc + c] = v;
    }
}

// Minibatch indices drawn with replacement from the records (Philox counters
// (r, step, 0, 4) under the training seed).
__global__ void sample_index(uint32_t *idx, uint32_t batch, uint64_t nrec, uint32_t step, uint32_t k0, uint32_t k1)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= batch) return;
    const sa::Ctr c = sa::philox4x32_10(sa::Ctr{r, step, 0u, 4u}, k0, k1);
    const uint64_t wide = ((uint64_t)c.w0 << 32) | c.w1;
    idx[r] = (uint32_t)__umul64hi(wide, nrec);
}

// Layer 1 (VALU): gather the minibatch, a1 = z W1 + b1, h1 = act(a1) in BF16.
__global__ void layer1_forward(const float *records, const uint32_t *idx, uint32_t batch, const uint16_t *W1b,
                               const float *b1, float *Z, float *delta, float *A1, uint16_t *H1b, int kind)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= batch * kHidden) return;
    const uint32_t r = t / kHidden, j = t % kHidden;
    const float *rec = records + (size_t)idx[r] * kRecord;
    float a = b1[j];
#pragma unroll
    for (int i = 0; i < kInputs; ++i) a = fmaf(rec[i], bf16_bits_to_f32(W1b[i * kHidden + j]), a);
    A1[(size_t)r * kHidden + j] = a;
    H1b[(size_t)r * kHidden + j] = f32_to_bf16_bits(act(a, kind));
    if (j < kInputs) Z[(size_t)r * kInputs + j] = rec[j];
    if (j == kInputs) delta[r] = rec[kInputs];
}

// Layer 3 (VALU, one wave per record): outputs, loss, d(loss)/d(outputs) and
// the gradient back into layer 2's pre-activation (FP32 and BF16).
__global__ void __launch_bounds__(256) layer3_loss(const float *H2, const float *A2, const uint16_t *W3b,
                                                   const float *b3, const float *delta, uint32_t batch, float inv_b,
                                                   float *loss_r, float *dO, float *dA2, uint16_t *dA2b, int kind)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= batch) return;
    float o0 = 0.0f, o1 = 0.0f;
    for (uint32_t j = lane; j < kHidden; j += 64) {
        const float h = H2[(size_t)r * kHidden + j];
        o0 = fmaf(h, bf16_bits_to_f32(W3b[2 * j + 0]), o0);
        o1 = fmaf(h, bf16_bits_to_f32(W3b[2 * j + 1]), o1);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        o0 += __shfl_xor(o0, off, 64);
        o1 += __shfl_xor(o1, off, 64);
    }
    const float mu = o0 + b3[0], s = o1 + b3[1];
    const float is = expf(-s);
    const float rr = (delta[r] - mu) * is;  // standardised residual
    float dmu, ds, lr;
    if (kind == kNetGeluGauss) {  // s + ln sqrt(2 pi) + r^2 / 2
        dmu = -rr * is * inv_b;
        ds = (1.0f - rr * rr) * inv_b;
        lr = s + 0.918938533204672742f + 0.5f * rr * rr;
    } else {  // s + ln pi + ln(1 + r^2)
        const float q = 1.0f + rr * rr;
        dmu = -2.0f * rr * is / q * inv_b;
        ds = (1.0f - 2.0f * rr * rr / q) * inv_b;
        lr = s + 1.14472988584940017f + logf(q);
    }
    if (lane == 0) {
        loss_r[r] = lr;
        dO[2 * r + 0] = dmu;
        dO[2 * r + 1] = ds;
    }
    for (uint32_t j = lane; j < kHidden; j += 64) {
        const float dh = bf16_bits_to_f32(W3b[2 * j + 0]) * dmu + bf16_bits_to_f32(W3b[2 * j + 1]) * ds;
        const float da = dh * act_grad(A2[(size_t)r * kHidden + j], kind);
        dA2[(size_t)r * kHidden + j] = da;
        dA2b[(size_t)r * kHidden + j] = f32_to_bf16_bits(da);
    }
}

// The small gradients (W1, b1, b2, W3, b3): 1282 sums over the minibatch.
// Pass 1: one thread per (parameter, chunk of kGradChunk records) sums its
// chunk in record order; pass 2 adds the chunks in order.  W2's gradient comes
// from MFMA.
constexpr uint32_t kSmallGrads = kInputs * kHidden + kHidden + kHidden + 2 * kHidden + 2;  // W1, b1, b2, W3, b3
static_assert(kSmallGrads == kNumParams - kHidden * kHidden, "every parameter but W2");
constexpr uint32_t kGradChunk = 128;

__global__ void small_grads_partial(const float *Z, const float *dA1, const float *dA2, const float *H2,
                                    const float *dO, uint32_t batch, float *partial)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kSmallGrads) return;
    const uint32_t r0 = blockIdx.y * kGradChunk, r1 = min(batch, r0 + kGradChunk);
    float s = 0.0f;
    if (t < kOffB1) {  // W1[i][j]
        const uint32_t i = t / kHidden, j = t % kHidden;
        for (uint32_t r = r0; r < r1; ++r) s = fmaf(Z[(size_t)r * kInputs + i], dA1[(size_t)r * kHidden + j], s);
    } else if (t < kOffB1 + kHidden) {  // b1
        const uint32_t j = t - kOffB1;
        for (uint32_t r = r0; r < r1; ++r) s += dA1[(size_t)r * kHidden + j];
    } else if (t < kOffB1 + 2 * kHidden) {  // b2
        const uint32_t j = t - kOffB1 - kHidden;
        for (uint32_t r = r0; r < r1; ++r) s += dA2[(size_t)r * kHidden + j];
    } else if (t < kOffB1 + 4 * kHidden) {  // W3[j][k]
        const uint32_t q = t - kOffB1 - 2 * kHidden, j = q / 2, k = q % 2;
        for (uint32_t r = r0; r < r1; ++r) s = fmaf(H2[(size_t)r * kHidden + j], dO[2 * r + k], s);
    } else {  // b3
        const uint32_t k = t - kOffB1 - 4 * kHidden;
        for (uint32_t r = r0; r < r1; ++r) s += dO[2 * r + k];
    }
    partial[(size_t)blockIdx.y * kSmallGrads + t] = s;
}

__global__ void small_grads_sum(const float *partial, uint32_t chunks, float *g)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kSmallGrads) return;
    float s = 0.0f;
    for (uint32_t c = 0; c < chunks; ++c) s += partial[(size_t)c * kSmallGrads + t];
    uint32_t at;
    if (t < kOffB1 + kHidden) at = t;                                   // W1, b1
    else if (t < kOffB1 + 2 * kHidden) at = kOffB2 + (t - kOffB1 - kHidden);  // b2
    else if (t < kOffB1 + 4 * kHidden) at = kOffW3 + (t - kOffB1 - 2 * kHidden);  // W3
    else at = kOffB3 + (t - kOffB1 - 4 * kHidden);                       // b3
    g[at] = s;
}

// Mean of the per-record losses (one workgroup, fixed order).
__global__ void __launch_bounds__(256) loss_mean(const float *loss_r, uint32_t batch, float *out)
{
    __shared__ double part[256];
    double s = 0.0;
    for (uint32_t r = threadIdx.x; r < batch; r += blockDim.x) s += loss_r[r];
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)(part[0] / (double)batch);
}

// Adam (Kingma & Ba) on the FP32 master parameters; refresh the BF16 weights.
__global__ void adam_update(float *theta, const float *g, float *m, float *v, float lr, float beta1, float beta2,
                            float eps, float c1, float c2, uint16_t *W1b, uint16_t *W2b, uint16_t *W3b)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNumParams) return;
    if (lr > 0.0f) {
        const float mi = beta1 * m[i] + (1.0f - beta1) * g[i];
        const float vi = beta2 * v[i] + (1.0f - beta2) * g[i] * g[i];
        m[i] = mi;
        v[i] = vi;
        theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
    const uint16_t b = f32_to_bf16_bits(theta[i]);
    if (i < kOffB1) W1b[i - kOffW1] = b;
    else if (i >= kOffW2 && i < kOffB2) W2b[i - kOffW2] = b;
    else if (i >= kOffW3 && i < kOffB3) W3b[i - kOffW3] = b;
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
    float *theta, *g, *m, *v, *Z, *delta, *A1, *A2, *H2, *dA2, *dA1, *loss_r, *dO, *loss;
    uint16_t *W1b, *W2b, *W3b, *H1b, *dA2b;
    uint32_t *idx;
    unsigned char *net;  // packed copy for inference
    float *partial;      // chunk partial sums of the small gradients
    uint32_t t = 0;  // Adam steps taken
    int kind = kNetReluCauchy;
};

namespace {

sa_status mlp_alloc(sa_mlp *p)
{
    const size_t B = p->max_batch, H = kHidden;
    size_t off = 0;
    std::vector<std::pair<void **, size_t>> parts = {
        {(void **)&p->theta, kNumParams * 4}, {(void **)&p->g, kNumParams * 4}, {(void **)&p->m, kNumParams * 4},
        {(void **)&p->v, kNumParams * 4},     {(void **)&p->Z, B * kInputs * 4}, {(void **)&p->delta, B * 4},
        {(void **)&p->A1, B * H * 4},         {(void **)&p->A2, B * H * 4},      {(void **)&p->H2, B * H * 4},
        {(void **)&p->dA2, B * H * 4},        {(void **)&p->dA1, B * H * 4},     {(void **)&p->loss_r, B * 4},
        {(void **)&p->dO, B * 2 * 4},         {(void **)&p->loss, 4},            {(void **)&p->W1b, kInputs * H * 2},
        {(void **)&p->W2b, H * H * 2},        {(void **)&p->W3b, H * 2 * 2},     {(void **)&p->H1b, B * H * 2},
        {(void **)&p->dA2b, B * H * 2},       {(void **)&p->idx, B * 4},         {(void **)&p->net, kNetBytes},
        {(void **)&p->partial, ((B + kGradChunk - 1) / kGradChunk) * kSmallGrads * 4}};
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

// One forward/backward pass over the minibatch in p->idx; the gradient of the
// mean loss ends in p->g, the mean loss in p->loss.
sa_status mlp_grad_pass(sa_mlp *p, const float *records, uint32_t batch)
{
    const dim3 blk(256);
    const float inv_b = 1.0f / (float)batch;
    hipLaunchKernelGGL(layer1_forward, dim3((batch * kHidden + 255) / 256), blk, 0, p->stream, records, p->idx,
                       batch, p->W1b, p->theta + kOffB1, p->Z, p->delta, p->A1, p->H1b, p->kind);
    // a2 = h1 W2 + b2, h2 = act(a2)
    const int tiles_bh = (int)(batch / 16) * (kHidden / 16);
    hipLaunchKernelGGL((gemm_bf16<kEpiBiasAct>), dim3((tiles_bh + 3) / 4), blk, 0, p->stream, (int)batch, kHidden,
                       kHidden, p->H1b, kHidden, 1, p->W2b, kHidden, 1, p->A2, kHidden, p->theta + kOffB2,
                       (const float *)nullptr, p->H2, p->kind);
    hipLaunchKernelGGL(layer3_loss, dim3((batch + 3) / 4), blk, 0, p->stream, p->H2, p->A2, p->W3b,
                       p->theta + kOffB3, p->delta, batch, inv_b, p->loss_r, p->dO, p->dA2, p->dA2b, p->kind);
    // dW2 = h1^T da2  (M = N = 128, K = batch)
    hipLaunchKernelGGL((gemm_bf16<kEpiStore>), dim3((64 + 3) / 4), blk, 0, p->stream, kHidden, kHidden, (int)batch,
                       p->H1b, 1, kHidden, p->dA2b, kHidden, 1, p->g + kOffW2, kHidden, (const float *)nullptr,
                       (const float *)nullptr, (float *)nullptr, p->kind);
    // da1 = (da2 W2^T) * act'(a1)
    hipLaunchKernelGGL((gemm_bf16<kEpiActBwd>), dim3((tiles_bh + 3) / 4), blk, 0, p->stream, (int)batch, kHidden,
                       kHidden, p->dA2b, kHidden, 1, p->W2b, 1, kHidden, p->dA1, kHidden, (const float *)nullptr,
                       p->A1, (float *)nullptr, p->kind);
    const uint32_t chunks = (batch + kGradChunk - 1) / kGradChunk;
    hipLaunchKernelGGL(small_grads_partial, dim3((kSmallGrads + 255) / 256, chunks), blk, 0, p->stream, p->Z,
                       p->dA1, p->dA2, p->H2, p->dO, batch, p->partial);
    hipLaunchKernelGGL(small_grads_sum, dim3((kSmallGrads + 255) / 256), blk, 0, p->stream, p->partial, chunks,
                       p->g);
    hipLaunchKernelGGL(loss_mean, dim3(1), blk, 0, p->stream, p->loss_r, batch, p->loss);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

sa_status refresh_bf16(sa_mlp *p)
{
    hipLaunchKernelGGL(adam_update, dim3((kNumParams + 255) / 256), dim3(256), 0, p->stream, p->theta, p->g, p->m,
                       p->v, 0.0f, 0.0f, 0.0f, 0.0f, 1.0f, 1.0f, p->W1b, p->W2b, p->W3b);
    SA_HIP(hipGetLastError());
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
    if (sa_status st = refresh_bf16(p); st != SA_OK) return st;
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
    if (sa_status st = mlp_grad_pass(p, records, batch); st != SA_OK) return st;
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
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    std::vector<float> trace(loss_trace ? steps : 0);
    for (uint32_t s = 0; s < steps; ++s) {
        hipLaunchKernelGGL(sample_index, dim3((batch + 255) / 256), dim3(256), 0, p->stream, p->idx, batch, nrec,
                           p->t, (uint32_t)seed, (uint32_t)(seed >> 32));
        if (sa_status st = mlp_grad_pass(p, records, batch); st != SA_OK) return st;
        p->t += 1;
        const float c1 = 1.0f - std::pow(beta1, (float)p->t), c2 = 1.0f - std::pow(beta2, (float)p->t);
        hipLaunchKernelGGL(adam_update, dim3((kNumParams + 255) / 256), dim3(256), 0, p->stream, p->theta, p->g,
                           p->m, p->v, lr, beta1, beta2, eps, c1, c2, p->W1b, p->W2b, p->W3b);
        SA_HIP(hipGetLastError());
        if (loss_trace) SA_HIP(hipMemcpyAsync(&trace[s], p->loss, sizeof(float), hipMemcpyDeviceToHost, p->stream));
    }
    SA_HIP(hipStreamSynchronize(p->stream));
    if (loss_trace) std::memcpy(loss_trace, trace.data(), steps * sizeof(float));
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
