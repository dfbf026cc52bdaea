// Batched synchronous parallel simulated annealing: many independent
// box-constrained problems of uneven dimension advance one temperature level
// per launch.
//
// Each wave owns one tile of 64 chains of one problem and an LDS region of
// its own (states x[d][lane], the problem's start state and its {l,u,rho,s}
// table), so nothing in a launch synchronises beyond a single wave.  Every
// wave publishes its tile's best chain (carried cost, chain, a full
// re-evaluation and the state); at the next level's launch every tile of a
// problem reduces its problem's candidates to the same winner and starts
// from it (Sec. 2.2.2), and the problem's first tile publishes the trace and
// the record.  The host packs tiles of different problems into workgroups
// so that their LDS regions fill the 160 KiB of a CU.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa_device.hpp"
#include "sa_internal.hpp"
#include "sa_step.hpp"

namespace sa {

namespace {

// LDS accesses of one wave made visible to the whole wave.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R> __device__ __forceinline__ Coord<R> table_coord(const R *tab, uint32_t d)
{
    return Coord<R>{tab[4 * d + 0], tab[4 * d + 1], tab[4 * d + 2], tab[4 * d + 3]};
}

// Full evaluation of an LDS state by one wave, FP64 arithmetic: FP64 runs sum
// in coordinate order on lane 0 (the order of a plain evaluation), FP32 runs
// in a fixed lane-strided order.
template <typename R, int F> __device__ Full wave_full_eval(const R *x, const R *tab, uint32_t n)
{
    const uint32_t lane = threadIdx.x & 63u;
    if (sizeof(R) == sizeof(double)) {
        Full v{0.0, 0.0, 0.0};
        if (lane == 0) {
            FullAcc<F> acc;
            for (uint32_t i = 0; i < n; ++i) acc.add((double)x[i] - (double)tab[4 * i + 3]);
            v = acc.finish(n);
        }
        return Full{__shfl(v.f, 0, 64), __shfl(v.s1, 0, 64), __shfl(v.s2, 0, 64)};
    }
    FullAcc<F> acc;
    for (uint32_t i = lane; i < n; i += 64) acc.add((double)x[i] - (double)tab[4 * i + 3]);
    FullAcc<F> tot;
    tot.a = wave_sum_d(acc.a);
    tot.b = wave_sum_d(acc.b);
    return tot.finish(n);
}

// Reduce problem p's candidates of level `lvl` to its winner (lowest carried
// cost, ties to the lowest chain); load the winner into xw and its full
// re-evaluation into start.  With `publish` also write the trace entry, the
// record and the broadcast state of problem p.
template <typename R>
__device__ void batch_adopt(const BatchArgs<R> &a, const BatchProblem &P, uint32_t p, uint32_t lvl, R *xw,
                            double *start, bool publish)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t n = P.n, tiles = P.chains >> 6;
    const size_t sbase = (size_t)(lvl & 1u) * a.ntiles;
    const double rec_prev = publish ? a.rec[p] : 0.0;  // loaded with the candidates
    R gf = widen_inf<R>();
    uint32_t gc = 0xFFFFFFFFu, gj = P.first_tile;
    uint64_t gacc = 0;
    for (uint32_t j = lane; j < tiles; j += 64) {
        const Slot<R> s = a.slots[sbase + P.first_tile + j];
        if (s.f < gf || (s.f == gf && s.chain < gc)) {
            gf = s.f;
            gc = s.chain;
            gj = P.first_tile + j;
        }
        gacc += s.accepts;
    }
    wave_best(gf, gc, gj);
    gacc = wave_sum(gacc);
    gj = __builtin_amdgcn_readfirstlane(gj);
    if (gj < P.first_tile || gj >= P.first_tile + tiles) gj = P.first_tile;  // all-NaN guard
    const size_t xoff = (size_t)(lvl & 1u) * a.slot_x_stride + a.tile_xoff[gj];
    for (uint32_t i = lane; i < n; i += 64) xw[i] = a.slot_x[xoff + i];
    const Slot<R> ws = a.slots[sbase + gj];
    start[0] = ws.ff;
    start[1] = ws.s1;
    start[2] = ws.s2;
    if (publish) {
        const bool improved = ws.ff < rec_prev;
        for (uint32_t i = lane; i < n; i += 64) {
            const R v = a.slot_x[xoff + i];
            a.x_best[P.x_off + i] = v;
            if (a.trace_x) a.trace_x[(size_t)a.levels * P.x_off + (size_t)lvl * n + i] = v;
            if (improved) a.x_rec[P.x_off + i] = v;
        }
        if (lane == 0) {
            if (improved) {
                a.rec[p] = ws.ff;
                a.rec_level[p] = lvl;
            }
            sa_level t;
            t.win_chain = gc;
            t.reserved = 0;
            t.f_win = (double)gf;
            t.f_best = ws.ff;
            t.f_rec = improved ? ws.ff : rec_prev;
            t.accepts = gacc;
            t.t_ns = wall_clock64();  // ticks here; sa_batch_trace converts them to ns
            a.trace[(size_t)p * a.levels + lvl] = t;
        }
    }
    wave_sync();
}

// One level of one tile (64 chains of problem p).
template <typename R, int F, int MOVE, bool LOG>
__device__ void batch_tile(const BatchArgs<R> &a, const BatchProblem &P, uint32_t p, uint32_t tile, R *xs, R *xw,
                           const R *tab, uint32_t level, const double *start, double T, float nl2T)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t n = P.n;
    const uint32_t chain = ((tile - P.first_tile) << 6) + lane;
    const uint32_t k0 = a.seed_lo, k1 = a.seed_hi;
    Cost<R, F> cost;
    if (level == 0) {
        FullAcc<F> acc;
        Ctr r{};
        for (uint32_t i = 0; i < n; ++i) {
            if ((i & 3u) == 0) r = philox4x32_10(Ctr{i >> 2, kInitLevel, chain, kTagInit | (p << 8)}, k0, k1);
            const uint32_t w = (i & 3u) == 0 ? r.w0 : (i & 3u) == 1 ? r.w1 : (i & 3u) == 2 ? r.w2 : r.w3;
            const Coord<R> c = table_coord(tab, i);
            R xi = c.lo + (c.hi - c.lo) * u24<R>(w);
            if (xi > c.hi) xi = c.hi;
            if (xi < c.lo) xi = c.lo;
            xs[(i << 6) + lane] = xi;
            acc.add((double)xi - (double)c.sh);
        }
        cost.set(acc.finish(n), n);
    } else {
        fill_tile(xs, 64u, lane, xw, n);
        cost.set(Full{start[0], start[1], start[2]}, n);
    }
    const bool log_level = LOG && p == a.log_problem && level >= a.log_level && level - a.log_level < a.log_levels;
    const bool logging = log_level && chain < a.log_chains;
    const auto coordf = [&](uint32_t d) { return table_coord(tab, d); };
    const auto logf = [&](uint32_t step, uint32_t d, bool take, R xd, R xn, R df) {
        if (LOG && logging) {
            sa_move_rec m;
            m.d = d;
            m.accept = take ? 1u : 0u;
            m.x_old = (double)xd;
            m.x_new = (double)xn;
            m.df = (double)df;
            a.log[((size_t)(level - a.log_level) * a.log_chains + chain) * a.steps + step] = m;
        }
    };
    const uint32_t accepted = run_steps<R, F, MOVE>(xs, 64u, lane, cost, coordf, logf, n, a.steps, level, chain,
                                                    kTagMove | (p << 8), k0, k1, T, nl2T, P.inv_n);
    if (LOG && log_level) a.log_final[(size_t)(level - a.log_level) * P.chains + chain] = (double)cost.f;

    // tile argmin; the winning column becomes the tile's candidate state
    R bf = cost.f;
    uint32_t bc = chain;
    wave_best(bf, bc);
    const uint32_t acc = wave_sum(accepted);
    wave_sync();
    const uint32_t col = bc & 63u;
    for (uint32_t i = lane; i < n; i += 64) xw[i] = xs[(i << 6) + col];
    wave_sync();
    const Full fr = wave_full_eval<R, F>(xw, tab, n);
    const size_t slot = (size_t)(level & 1u) * a.ntiles + tile;
    if (lane == 0) a.slots[slot] = Slot<R>{bf, bc, acc, 0u, fr.f, fr.s1, fr.s2};
    const size_t xoff = (size_t)(level & 1u) * a.slot_x_stride + a.tile_xoff[tile];
    for (uint32_t i = lane; i < n; i += 64) a.slot_x[xoff + i] = xw[i];
}

template <typename R, int MOVE, bool LOG>
__global__ void __launch_bounds__(256) batch_level_kernel(const BatchArgs<R> a, const uint32_t level)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t slot = blockIdx.x * a.waves_per_group + wave;
    const uint32_t tile = __builtin_amdgcn_readfirstlane(a.wg_tile[slot]);
    if (tile == 0xFFFFFFFFu) return;
    const uint64_t t_start = wall_clock64();
    const uint32_t p = __builtin_amdgcn_readfirstlane(a.tile_prob[tile]);
    const BatchProblem P = a.probs[p];
    // The level's constants are loaded before the hand-off (latency overlap).
    const double T = a.T[level];
    const float nl2T = -kLog2e * a.inv_T[level];
    R *xs = reinterpret_cast<R *>(lds_raw + __builtin_amdgcn_readfirstlane(a.wg_lds[slot]));
    R *xw = xs + ((size_t)P.n << 6);
    R *tab = xw + P.n;
    for (uint32_t i = lane; i < 4 * P.n; i += 64) tab[i] = a.table[4 * (size_t)P.tab_off + i];
    double start[3] = {0.0, 0.0, 0.0};
    wave_sync();
    if (level > 0) batch_adopt<R>(a, P, p, level - 1, xw, start, tile == P.first_tile);
    wave_sync();
    switch (P.func) {
    case kSchwefel: batch_tile<R, kSchwefel, MOVE, LOG>(a, P, p, tile, xs, xw, tab, level, start, T, nl2T); break;
    case kRastrigin: batch_tile<R, kRastrigin, MOVE, LOG>(a, P, p, tile, xs, xw, tab, level, start, T, nl2T); break;
    default: batch_tile<R, kAckley, MOVE, LOG>(a, P, p, tile, xs, xw, tab, level, start, T, nl2T); break;
    }
    if (a.clock && level - a.clock_level < a.clock_levels && lane == 0) {
        uint64_t *c = a.clock + ((size_t)(level - a.clock_level) * a.ntiles + tile) * 2u;
        c[0] = t_start;
        c[1] = wall_clock64();
    }
}

// One wave per problem: publish level `level` from its candidates.
template <typename R>
__global__ void __launch_bounds__(256) batch_finalize_kernel(const BatchArgs<R> a, const uint32_t level,
                                                             const uint32_t max_n)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t p = blockIdx.x * 4u + wave;
    if (p >= a.nprob) return;
    const BatchProblem P = a.probs[p];
    R *xw = reinterpret_cast<R *>(lds_raw) + (size_t)wave * max_n;
    double start[3];
    batch_adopt<R>(a, P, p, level, xw, start, true);
}

__global__ void batch_reset_kernel(double *rec, uint32_t *rec_level, uint32_t nprob)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) {
        rec[p] = __builtin_inf();
        rec_level[p] = 0xFFFFFFFFu;
    }
}

template <typename R>
hipError_t launch_level(const BatchArgs<R> &a, uint32_t groups, size_t lds, bool log, uint32_t level, hipStream_t s)
{
    const dim3 grid(groups), block(64 * a.waves_per_group);
    if (a.move == SA_MOVE_RADIUS) {
        if (log)
            hipLaunchKernelGGL((batch_level_kernel<R, SA_MOVE_RADIUS, true>), grid, block, lds, s, a, level);
        else
            hipLaunchKernelGGL((batch_level_kernel<R, SA_MOVE_RADIUS, false>), grid, block, lds, s, a, level);
    } else {
        if (log)
            hipLaunchKernelGGL((batch_level_kernel<R, SA_MOVE_RESAMPLE, true>), grid, block, lds, s, a, level);
        else
            hipLaunchKernelGGL((batch_level_kernel<R, SA_MOVE_RESAMPLE, false>), grid, block, lds, s, a, level);
    }
    return hipGetLastError();
}

}  // namespace

size_t batch_wave_lds_bytes(uint32_t n, size_t real_size) { return ((size_t)n * 64 + (size_t)n + 4 * (size_t)n) * real_size; }

hipError_t launch_batch_level_f32(const BatchArgs<float> &a, uint32_t groups, size_t lds, bool log, uint32_t level,
                                  hipStream_t s)
{
    return launch_level<float>(a, groups, lds, log, level, s);
}

hipError_t launch_batch_level_f64(const BatchArgs<double> &a, uint32_t groups, size_t lds, bool log, uint32_t level,
                                  hipStream_t s)
{
    return launch_level<double>(a, groups, lds, log, level, s);
}

hipError_t launch_batch_finalize_f32(const BatchArgs<float> &a, uint32_t level, uint32_t max_n, hipStream_t s)
{
    hipLaunchKernelGGL(batch_finalize_kernel<float>, dim3((a.nprob + 3) / 4), dim3(256), 4 * (size_t)max_n * sizeof(float),
                       s, a, level, max_n);
    return hipGetLastError();
}

hipError_t launch_batch_finalize_f64(const BatchArgs<double> &a, uint32_t level, uint32_t max_n, hipStream_t s)
{
    hipLaunchKernelGGL(batch_finalize_kernel<double>, dim3((a.nprob + 3) / 4), dim3(256),
                       4 * (size_t)max_n * sizeof(double), s, a, level, max_n);
    return hipGetLastError();
}

hipError_t launch_batch_reset(double *rec, uint32_t *rec_level, uint32_t nprob, hipStream_t s)
{
    hipLaunchKernelGGL(batch_reset_kernel, dim3((nprob + 255) / 256), dim3(256), 0, s, rec, rec_level, nprob);
    return hipGetLastError();
}

}  // namespace sa
