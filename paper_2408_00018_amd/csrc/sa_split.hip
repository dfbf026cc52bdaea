// FP32 plain level kernel with the generator split off into its own waves.
//
// With one 64-chain wave per SIMD (65536 chains on 256 CUs) the step loop is
// limited by how fast a single wave issues, not by the SIMD: two waves issue
// ~1.8x the instructions of one.  So each workgroup runs 256 chains with
// eight waves: four state waves (one chain per lane, states in LDS as in the
// dense kernel) and four generator waves that compute the same Philox blocks
// -- coordinate and both uniforms of each move -- into an LDS ring, a chunk of
// C moves ahead.  Generator wave w + 4 serves state wave w and shares its
// SIMD.  A workgroup barrier separates chunks (the ring is double-buffered).
// A chunk is one group of four moves of the plain move stream (three
// generator blocks).  The moves are the dense kernel's moves, value for value.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sa_device.hpp"
#include "sa_internal.hpp"
#include "sa_level_common.hpp"
#include "sa_step.hpp"

namespace sa {

namespace {

constexpr uint32_t kChains = 256;  // chains per workgroup (state lanes)
constexpr uint32_t kChunk = 4;     // moves per ring half: one group of the move stream
static_assert(kChunk == 4, "a chunk is one four-move group of the move stream");

// One move's draws in a 16-byte ring entry: coordinate, the change uniform,
// the acceptance word's top 24 bits as a float (FP32 bit patterns), unused.
typedef uint4 Draw;

}  // namespace

// LDS: ring[2][kChunk][kChains] Draw | xs[n][kChains] | xw[n] | xb[n] | tab[n][4] (TABLE only)
template <int F, bool TABLE, int MOVE>
__global__ void __launch_bounds__(512) split_level_kernel(const LevelArgs<float> a, const uint32_t level,
                                                          const uint32_t prev_groups)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Slot<float> wave_slot[8];
    __shared__ uint64_t wave_acc[8];
    __shared__ double sh_part[8][2];
    __shared__ double sh_start[3];

    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const bool gen = tid >= kChains;
    const uint32_t col = gen ? tid - kChains : tid;  // chain column this thread serves
    const uint32_t G = gridDim.x, n = a.n;
    Draw *ring = reinterpret_cast<Draw *>(lds_raw);
    float *xs = reinterpret_cast<float *>(ring + 2 * kChunk * kChains);
    float *xw = xs + (size_t)n * kChains;
    float *xb = xw + n;
    float *tab = xb + n;
    // The level's constant is loaded before the hand-off (latency overlap).
    const float nl2T = -kLog2e * a.inv_T[level];

    if (TABLE) {
        for (uint32_t i = tid; i < 4 * n; i += blockDim.x) tab[i] = a.table[i];
    }
    if (level == a.start_level) {
        for (uint32_t i = tid; i < n; i += blockDim.x) xw[i] = a.x_start[i];
        __syncthreads();
        const Full v = full_eval_wg<float, F, TABLE>(a, tab, xw, sh_part);
        if (tid == 0) {
            sh_start[0] = v.f;
            sh_start[1] = v.s1;
            sh_start[2] = v.s2;
        }
    } else if (level > 0) {
        adopt_winner<float>(a, level - 1, prev_groups, xw, sh_start, blockIdx.x == 0, wave_slot, wave_acc);
    }
    __syncthreads();

    const uint32_t k0 = a.seed_lo, k1 = a.seed_hi;
    const uint32_t ctr3 = kTagMove | (a.problem << 8);
    const Full start{sh_start[0], sh_start[1], sh_start[2]};
    const uint32_t steps = a.steps, nchunks = (steps + kChunk - 1) / kChunk;
    float wf = widen_inf<float>();
    uint32_t wc = 0xFFFFFFFFu;
    uint32_t accepted = 0;
    // The workgroup's best state: copied to xb while another tile follows,
    // read in place (column of xs) when it comes from the last tile.
    const float *best = xb;
    uint32_t best_stride = 1;

    for (uint32_t tile = blockIdx.x; tile < a.tiles; tile += G) {
        const uint32_t chain = tile * kChains + col;
        Cost<float, F> cost;
        if (!gen) {
            if (level == 0) {
                FullAcc<F> acc;
                Ctr r{};
                for (uint32_t i = 0; i < n; ++i) {
                    if ((i & 3u) == 0)
                        r = philox4x32_10(Ctr{i >> 2, kInitLevel, chain, kTagInit | (a.problem << 8)}, k0, k1);
                    const uint32_t w = (i & 3u) == 0 ? r.w0 : (i & 3u) == 1 ? r.w1 : (i & 3u) == 2 ? r.w2 : r.w3;
                    const Coord<float> c = coord<float, TABLE>(a, tab, i);
                    float xi = c.lo + (c.hi - c.lo) * u24<float>(w);
                    if (xi > c.hi) xi = c.hi;
                    if (xi < c.lo) xi = c.lo;
                    xs[i * kChains + col] = xi;
                    acc.add((double)xi - (double)c.sh);
                }
                cost.set(acc.finish(n), n);
            } else {
                fill_tile_c<kChains>(xs, col, xw, n);
                cost.set(start, n);
            }
        }

        // Generator: draws of chunk k (group k of the move stream) into ring
        // half k & 1.
        const auto produce = [&](uint32_t k) {
            Draw *half = ring + (k & 1u) * kChunk * kChains;
            const MoveGroup m = move_group(k, level, chain, ctr3, k0, k1);
#pragma unroll
            for (uint32_t j = 0; j < kChunk; ++j) {
                const uint32_t step = k * kChunk + j;
                if (step < steps) {
                    uint32_t wd, w1, w2;
                    move_words(m, j, wd, w1, w2);
                    half[j * kChains + col] = make_uint4(pick(wd, n), __float_as_uint(u24f(w1)),
                                                         __float_as_uint((float)(w2 >> 8)), 0u);
                }
            }
        };
        if (gen) produce(0);
        __syncthreads();
        for (uint32_t k = 0; k < nchunks; ++k) {
            if (gen) {
                if (k + 1 < nchunks) produce(k + 1);
            } else {
                // The chunk's draws and the states at their coordinates are read
                // up front (one LDS round trip); a coordinate a later move of the
                // chunk repeats is forwarded from the earlier move's result.
                const Draw *half = ring + (k & 1u) * kChunk * kChains;
                const uint32_t valid = min(kChunk, steps - k * kChunk);
                uint32_t d[kChunk];
                float u1[kChunk], k2[kChunk], xv[kChunk];
#pragma unroll
                for (uint32_t j = 0; j < kChunk; ++j) {
                    const Draw e = half[(j < valid ? j : 0u) * kChains + col];
                    d[j] = e.x;
                    u1[j] = __uint_as_float(e.y);
                    k2[j] = __uint_as_float(e.z);
                }
#pragma unroll
                for (uint32_t j = 0; j < kChunk; ++j) xv[j] = xs[__umul24(d[j], kChains) + col];
#pragma unroll
                for (uint32_t j = 0; j < kChunk; ++j) {
                    if (j < valid) {
                        const Coord<float> c = coord<float, TABLE>(a, tab, d[j]);
                        const float xn = neighbour<MOVE>(xv[j], c, u1[j]);
                        const bool take = cost.step(xv[j], xn, c.sh, k2[j], nl2T, a.inv_n);
                        const float xwr = take ? xn : xv[j];
                        xs[__umul24(d[j], kChains) + col] = xwr;
                        cost.commit(take, a.inv_n);
                        accepted += take ? 1u : 0u;
#pragma unroll
                        for (uint32_t m = j + 1; m < kChunk; ++m) xv[m] = d[m] == d[j] ? xwr : xv[m];
                    }
                }
            }
            __syncthreads();
        }

        // ---- tile argmin over the state waves; keep the workgroup's best
        float bf = gen ? widen_inf<float>() : cost.f;
        uint32_t bc = gen ? 0xFFFFFFFFu : chain;
        wave_best(bf, bc);
        if (lane == 0) wave_slot[wave] = Slot<float>{bf, bc, 0u, 0u, 0.0, 0.0, 0.0};
        __syncthreads();
        float tf = wave_slot[0].f;
        uint32_t tc = wave_slot[0].chain;
        for (uint32_t w = 1; w < kChains / 64; ++w) best_of(tf, tc, wave_slot[w].f, wave_slot[w].chain);
        float nf = wf;
        uint32_t nc = wc;
        best_of(nf, nc, tf, tc);
        const bool last = tile + G >= a.tiles;
        if (nc != wc) {
            const uint32_t bcol = tc - tile * kChains;
            if (last) {
                best = xs + bcol;
                best_stride = kChains;
            } else {
                for (uint32_t i = tid; i < n; i += blockDim.x) xb[i] = xs[i * kChains + bcol];
                best = xb;
                best_stride = 1;
            }
            wf = nf;
            wc = nc;
        }
        if (!last) __syncthreads();  // xs, xb, the ring and wave_slot are reused by the next tile
    }

    // the evaluation's barriers also order the per-wave acceptance counts
    const uint32_t wacc = wave_sum(accepted);
    if (lane == 0) wave_acc[wave] = wacc;
    const Full fr = full_eval_wg<float, F, TABLE>(a, tab, best, sh_part, best_stride);
    const size_t slot = (size_t)(level & 1u) * a.tiles + blockIdx.x;
    if (tid == 0) {
        uint32_t acc = 0;
        for (uint32_t w = 0; w < kChains / 64; ++w) acc += (uint32_t)wave_acc[w];
        a.slots[slot] = Slot<float>{wf, wc, acc, 0u, fr.f, fr.s1, fr.s2};
    }
    for (uint32_t i = tid; i < n; i += blockDim.x) a.slot_x[slot * n + i] = best[i * best_stride];
}

size_t split_lds_bytes(uint32_t n, bool table)
{
    return 2 * kChunk * kChains * sizeof(Draw) + ((size_t)n * kChains + 2 * (size_t)n + (table ? 4 * (size_t)n : 0)) *
                                                     sizeof(float);
}

namespace {

template <int F, bool TABLE, int MOVE>
hipError_t launch_split(const LevelArgs<float> &a, uint32_t level, uint32_t prev_groups, uint32_t *groups,
                        hipStream_t s)
{
    auto kern = split_level_kernel<F, TABLE, MOVE>;
    const size_t lds = split_lds_bytes(a.n, TABLE);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 512, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)per_cu * a.num_cus, a.tiles);
    *groups = grid;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(512), lds, s, a, level, prev_groups);
    return hipGetLastError();
}

template <int F>
hipError_t split_dispatch_f(bool table, const LevelArgs<float> &a, uint32_t level, uint32_t prev, uint32_t *groups,
                            hipStream_t s)
{
    if (a.move == SA_MOVE_RADIUS)
        return table ? launch_split<F, true, SA_MOVE_RADIUS>(a, level, prev, groups, s)
                     : launch_split<F, false, SA_MOVE_RADIUS>(a, level, prev, groups, s);
    return table ? launch_split<F, true, SA_MOVE_RESAMPLE>(a, level, prev, groups, s)
                 : launch_split<F, false, SA_MOVE_RESAMPLE>(a, level, prev, groups, s);
}

}  // namespace

hipError_t launch_split_level_f32(int func, bool table, const LevelArgs<float> &a, uint32_t level,
                                  uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    if (a.wg != kChains) return hipErrorInvalidValue;
    switch (func) {
    case kSchwefel: return split_dispatch_f<kSchwefel>(table, a, level, prev_groups, groups, s);
    case kRastrigin: return split_dispatch_f<kRastrigin>(table, a, level, prev_groups, groups, s);
    case kAckley: return split_dispatch_f<kAckley>(table, a, level, prev_groups, groups, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sa
