// Level kernel of synchronous parallel simulated annealing for gfx950.
//
// One Markov chain per lane.  A workgroup of WG lanes keeps a tile of chains'
// states in LDS as x[d][lane] (coordinate-major), so a per-lane random
// coordinate d is a bank-conflict-free LDS access.  One launch runs one
// temperature level (Sec. 2.2.2: every chain runs N Metropolis steps at a
// fixed T and the lowest final state starts every chain at the next level).
// Each workgroup runs its tiles of chains, keeps its best chain, re-evaluates
// that state in full and publishes it as a candidate with plain stores; the
// kernel boundary makes the candidates visible, and every workgroup of the
// next level's launch reduces them to the same winner before it starts.
// There is no cross-workgroup synchronisation inside a launch: on gfx950 a
// grid-wide barrier (or a last-workgroup hand-off with agent-scope fences)
// costs several times the ~1.5 us of a graph-replayed launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "sa_device.hpp"
#include "sa_internal.hpp"
#include "sa_step.hpp"
#include "sa_level_common.hpp"

namespace sa {

// ---------------------------------------------------------------------------
// The level kernel.  prev_groups: candidates the previous level's launch
// published (unused at level 0 and at the start level).  UNSHIFTED: the box
// is uniform, the shift is zero and every level starts from a broadcast, all
// known at compile time, so the steps skip the x - s subtractions (x - 0 is x
// exactly: the same bits as the general kernel, two fewer operations per move)
// and the kernel carries no own-state paths.
// LDS: [net (learned modes)] | xs[n][WG] tile states | xw[n] level start |
//      xb[n] workgroup best | tab[n][4] per-coordinate box/shift (TABLE only)
// ---------------------------------------------------------------------------
template <typename R, int F, bool TABLE, int MODE, int MOVE, bool UNSHIFTED = false>
__global__ void __launch_bounds__(256)
    level_kernel(const LevelArgs<R> a, const uint32_t level, const uint32_t prev_groups)
{
    constexpr bool LOG = MODE == kModeLog || MODE == kModeLearnLog;
    constexpr bool LEARN = MODE == kModeLearn || MODE == kModeLearnLog;
    constexpr bool CAPTURE = MODE == kModeCapture;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Slot<R> wave_slot[4];
    __shared__ uint64_t wave_acc[4];
    __shared__ double sh_part[4][2];
    __shared__ double sh_start[3];

    const uint32_t WG = blockDim.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t nwaves = WG >> 6;
    const uint32_t G = gridDim.x;
    const uint32_t n = a.n;
    unsigned char *net_lds = lds_raw;
    R *xs = reinterpret_cast<R *>(lds_raw + (LEARN ? mlp::kNetBytes : 0u));
    R *xw = xs + (size_t)n * WG;
    R *xb = xw + n;
    R *tab = xb + n;

    // The level's constants are loaded first, so their latency overlaps the
    // hand-off's loads instead of following it.
    const double T = a.T[level];
    const float nl2T = -kLog2e * a.inv_T[level];
    const float featT = (LEARN || CAPTURE) ? a.featT[level] : 0.0f;
    if (LEARN) mlp::stage_net(net_lds, a.net);
    if (TABLE) {
        for (uint32_t i = tid; i < 4 * n; i += WG) tab[i] = a.table[i];
    }
    if (level == a.start_level) {
        for (uint32_t i = tid; i < n; i += WG) xw[i] = a.x_start[i];
        __syncthreads();
        const Full v = full_eval_wg<R, F, TABLE>(a, tab, xw, sh_part);
        if (tid == 0) {
            sh_start[0] = v.f;
            sh_start[1] = v.s1;
            sh_start[2] = v.s2;
        }
    } else if (level > 0) {
        adopt_winner<R>(a, level - 1, prev_groups, xw, sh_start, blockIdx.x == 0, wave_slot, wave_acc);
    }
    __syncthreads();

    const uint32_t k0 = a.seed_lo, k1 = a.seed_hi;
    const uint32_t ctr3 = kTagMove | (a.problem << 8);
    const bool log_level = LOG && level >= a.log_level && level - a.log_level < a.log_levels;
    const Full start{sh_start[0], sh_start[1], sh_start[2]};
    // Without a broadcast at this level's start every chain continues from its
    // own state and carried cost; they are kept at the end unless the next
    // level starts from a broadcast.
    const uint32_t ex = a.exchange;
    const bool own = !UNSHIFTED && level > 0 && level != a.start_level && !(ex != 0 && level % ex == 0);
    const bool keep = !UNSHIFTED && ex != 1 && !(ex != 0 && (level + 1) % ex == 0);
    R wf = widen_inf<R>();
    uint32_t wc = 0xFFFFFFFFu;
    uint32_t accepted = 0;
    // The workgroup's best state: copied to xb while another tile follows,
    // read in place (column of xs) when it comes from the last tile.
    const R *best = xb;
    uint32_t best_stride = 1;

    for (uint32_t tile = blockIdx.x; tile < a.tiles; tile += G) {
        const uint32_t chain = tile * WG + tid;
        // ---- tile start: own random point at level 0, else the level's start state
        Cost<R, F> cost;
        if (level == 0) {
            FullAcc<F> acc;
            Ctr r{};
            for (uint32_t i = 0; i < n; ++i) {
                if ((i & 3u) == 0)
                    r = philox4x32_10(Ctr{i >> 2, kInitLevel, chain, kTagInit | (a.problem << 8)}, k0, k1);
                const uint32_t w = (i & 3u) == 0 ? r.w0 : (i & 3u) == 1 ? r.w1 : (i & 3u) == 2 ? r.w2 : r.w3;
                const Coord<R> c = coord<R, TABLE>(a, tab, i);
                R xi = c.lo + (c.hi - c.lo) * u24<R>(w);
                if (xi > c.hi) xi = c.hi;
                if (xi < c.lo) xi = c.lo;
                xs[i * WG + tid] = xi;
                acc.add((double)xi - (double)c.sh);
            }
            cost.set(acc.finish(n), n);
        } else if (own) {
            load_column(xs, WG, tid, a.chain_x + chain, a.chains, n);
            cost.load(a.chain_cost + chain, a.chains);
        } else {
            if (WG == 256)
                fill_tile_c<256>(xs, tid, xw, n);
            else
                fill_tile(xs, WG, tid, xw, n);
            cost.set(start, n);
        }

        // ---- N steps
        const bool logging = log_level && chain < a.log_chains;
        const auto coordf = [&](uint32_t d) {
            Coord<R> c = coord<R, TABLE>(a, tab, d);
            if constexpr (UNSHIFTED) c.sh = R(0);
            return c;
        };
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
        R hist[4] = {R(0), R(0), R(0), R(0)};  // last four accepted scaled displacements
        if constexpr (LEARN) {
            float h[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            accepted += run_learned_steps<F>(xs, WG, tid, cost, coordf, logf, n, a.steps, level, chain, ctr3,
                                             kTagLearn | (a.problem << 8), k0, k1, nl2T, a.inv_n, featT, a.eps,
                                             net_lds, h);
        } else if constexpr (CAPTURE) {
            // Record (features at x, scaled displacement) of every accepted move;
            // one counter update per wave and step.
            const auto capf = [&](uint32_t, uint32_t d, bool take, R xd, R xn, R) {
                const Coord<R> c = coordf(d);
                const R w = c.hi - c.lo;
                const R z0 = (xd - c.lo) / w;
                const R dl = (xn - xd) / w;
                const uint64_t mask = __ballot(take);
                if (mask) {
                    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1u;
                    unsigned long long base = 0;
                    if (lane == leader) base = atomicAdd(a.cap_count, (unsigned long long)__popcll(mask));
                    const uint32_t lo = __shfl((uint32_t)base, (int)leader, 64);
                    const uint32_t hi = __shfl((uint32_t)(base >> 32), (int)leader, 64);
                    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                    const uint64_t slot = (((uint64_t)hi << 32) | lo) + rank;
                    if (take && slot < a.cap_capacity) {
                        float *rec = a.cap_rec + slot * 7u;
                        rec[0] = (float)z0;
                        rec[1] = featT;
                        rec[2] = (float)hist_feature(hist[0]);
                        rec[3] = (float)hist_feature(hist[1]);
                        rec[4] = (float)hist_feature(hist[2]);
                        rec[5] = (float)hist_feature(hist[3]);
                        rec[6] = (float)dl;
                    }
                }
                if (take) {
                    hist[3] = hist[2];
                    hist[2] = hist[1];
                    hist[1] = hist[0];
                    hist[0] = dl;
                }
            };
            accepted += run_steps<R, F, MOVE>(xs, WG, tid, cost, coordf, capf, n, a.steps, level, chain, ctr3, k0,
                                              k1, T, nl2T, a.inv_n);
        } else {
            accepted += run_steps<R, F, MOVE>(xs, WG, tid, cost, coordf, logf, n, a.steps, level, chain, ctr3, k0,
                                              k1, T, nl2T, a.inv_n);
        }
        if (LOG && log_level) a.log_final[(size_t)(level - a.log_level) * a.chains + chain] = (double)cost.f;
        if (keep) {
            store_column(xs, WG, tid, a.chain_x + chain, a.chains, n);
            cost.save(a.chain_cost + chain, a.chains);
        }

        // ---- tile argmin of (final cost, chain); keep the workgroup's best
        R bf = cost.f;
        uint32_t bc = chain;
        wave_best(bf, bc);
        if (lane == 0) wave_slot[wave] = Slot<R>{bf, bc, 0u, 0u, 0.0, 0.0, 0.0};
        __syncthreads();
        R tf = wave_slot[0].f;
        uint32_t tc = wave_slot[0].chain;
        for (uint32_t w = 1; w < nwaves; ++w) best_of(tf, tc, wave_slot[w].f, wave_slot[w].chain);
        R nf = wf;
        uint32_t nc = wc;
        best_of(nf, nc, tf, tc);
        const bool last = tile + G >= a.tiles;
        if (nc != wc) {
            const uint32_t col = tc - tile * WG;
            if (last) {
                best = xs + col;
                best_stride = WG;
            } else {
                for (uint32_t i = tid; i < n; i += WG) xb[i] = xs[i * WG + col];
                best = xb;
                best_stride = 1;
            }
            wf = nf;
            wc = nc;
        }
        if (!last) __syncthreads();  // xs, xb and wave_slot are reused by the next tile
    }

    // ---- publish this workgroup's candidate, re-evaluated in full; the
    // evaluation's barriers also order the per-wave acceptance counts
    const uint32_t wacc = wave_sum(accepted);
    if (lane == 0) wave_acc[wave] = wacc;
    const Full fr = full_eval_wg<R, F, TABLE>(a, tab, best, sh_part, best_stride);
    const size_t slot = (size_t)(level & 1u) * a.tiles + blockIdx.x;
    if (tid == 0) {
        uint32_t acc = 0;
        for (uint32_t w = 0; w < nwaves; ++w) acc += (uint32_t)wave_acc[w];
        a.slots[slot] = Slot<R>{wf, wc, acc, 0u, fr.f, fr.s1, fr.s2};
    }
    for (uint32_t i = tid; i < n; i += WG) a.slot_x[slot * n + i] = best[i * best_stride];
}

// Close a run of levels: reduce the last level's candidates and publish its
// trace entry, record and broadcast state.
template <typename R>
__global__ void __launch_bounds__(256) finalize_kernel(const LevelArgs<R> a, const uint32_t level,
                                                        const uint32_t groups)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Slot<R> wave_slot[4];
    __shared__ uint64_t wave_acc[4];
    __shared__ double sh_start[3];
    adopt_winner<R>(a, level, groups, reinterpret_cast<R *>(lds_raw), sh_start, true, wave_slot, wave_acc);
}

__global__ void reset_kernel(double *rec, uint32_t *rec_level)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        rec[0] = __builtin_inf();
        *rec_level = 0xFFFFFFFFu;
    }
}

size_t level_lds_bytes(uint32_t n, uint32_t wg, size_t real_size, bool table, bool learn)
{
    return ((size_t)n * wg + 2 * (size_t)n + (table ? 4 * (size_t)n : 0)) * real_size +
           (learn ? (size_t)mlp::kNetBytes : 0);
}

template <typename R, int F, bool TABLE, int MODE, int MOVE, bool UNSHIFTED = false>
static hipError_t launch_one(const LevelArgs<R> &a, uint32_t level, uint32_t prev_groups, uint32_t *groups,
                             hipStream_t s)
{
    auto kern = level_kernel<R, F, TABLE, MODE, MOVE, UNSHIFTED>;
    const size_t lds =
        level_lds_bytes(a.n, a.wg, sizeof(R), TABLE, MODE == kModeLearn || MODE == kModeLearnLog);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, (int)a.wg, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)per_cu * a.num_cus, a.tiles);
    *groups = grid;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(a.wg), lds, s, a, level, prev_groups);
    return hipGetLastError();
}

template <typename R, int F, bool TABLE, int MOVE>
static hipError_t launch_mode(int mode, const LevelArgs<R> &a, uint32_t level, uint32_t prev, uint32_t *groups,
                              hipStream_t s)
{
    switch (mode) {
    case kModePlain:
        if constexpr (!TABLE && sizeof(R) == sizeof(float)) {
            if (a.sh == R(0) && !std::signbit(a.sh) && a.exchange == 1)  // +0 exactly, synchronous
                return launch_one<R, F, TABLE, kModePlain, MOVE, true>(a, level, prev, groups, s);
        }
        return launch_one<R, F, TABLE, kModePlain, MOVE>(a, level, prev, groups, s);
    case kModeLog: return launch_one<R, F, TABLE, kModeLog, MOVE>(a, level, prev, groups, s);
    case kModeCapture: return launch_one<R, F, TABLE, kModeCapture, MOVE>(a, level, prev, groups, s);
    default: break;
    }
    if constexpr (sizeof(R) == sizeof(float) && MOVE == SA_MOVE_RADIUS) {
        if (mode == kModeLearn) return launch_one<R, F, TABLE, kModeLearn, MOVE>(a, level, prev, groups, s);
        if (mode == kModeLearnLog) return launch_one<R, F, TABLE, kModeLearnLog, MOVE>(a, level, prev, groups, s);
    }
    return hipErrorInvalidValue;
}

template <typename R, int F>
static hipError_t dispatch_f(bool table, int mode, const LevelArgs<R> &a, uint32_t level, uint32_t prev,
                             uint32_t *groups, hipStream_t s)
{
    if (a.move == SA_MOVE_RADIUS)
        return table ? launch_mode<R, F, true, SA_MOVE_RADIUS>(mode, a, level, prev, groups, s)
                     : launch_mode<R, F, false, SA_MOVE_RADIUS>(mode, a, level, prev, groups, s);
    return table ? launch_mode<R, F, true, SA_MOVE_RESAMPLE>(mode, a, level, prev, groups, s)
                 : launch_mode<R, F, false, SA_MOVE_RESAMPLE>(mode, a, level, prev, groups, s);
}

template <typename R>
static hipError_t dispatch(int func, bool table, int mode, const LevelArgs<R> &a, uint32_t level, uint32_t prev,
                           uint32_t *groups, hipStream_t s)
{
    switch (func) {
    case kSchwefel: return dispatch_f<R, kSchwefel>(table, mode, a, level, prev, groups, s);
    case kRastrigin: return dispatch_f<R, kRastrigin>(table, mode, a, level, prev, groups, s);
    case kAckley: return dispatch_f<R, kAckley>(table, mode, a, level, prev, groups, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_level_f32(int func, bool table, int mode, const LevelArgs<float> &a, uint32_t level,
                            uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    return dispatch<float>(func, table, mode, a, level, prev_groups, groups, s);
}

hipError_t launch_level_f64(int func, bool table, int mode, const LevelArgs<double> &a, uint32_t level,
                            uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    return dispatch<double>(func, table, mode, a, level, prev_groups, groups, s);
}

hipError_t launch_finalize_f32(const LevelArgs<float> &a, uint32_t level, uint32_t groups, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel<float>, dim3(1), dim3(256), a.n * sizeof(float), s, a, level, groups);
    return hipGetLastError();
}

hipError_t launch_finalize_f64(const LevelArgs<double> &a, uint32_t level, uint32_t groups, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel<double>, dim3(1), dim3(256), a.n * sizeof(double), s, a, level, groups);
    return hipGetLastError();
}

hipError_t launch_reset(double *rec, uint32_t *rec_level, hipStream_t s)
{
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, rec, rec_level);
    return hipGetLastError();
}

}  // namespace sa
