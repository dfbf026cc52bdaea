// Level kernel with a base-plus-overlay chain state, for dimensions whose
// dense per-lane state x[n][WG] does not fit in LDS beside enough waves
// (n = 512 leaves one wave per CU; n = 1024 does not fit at all).
//
// Within a level every chain starts from the same state (the previous level's
// winner, Sec. 2.2.2) and changes at most N coordinates.  So the workgroup
// keeps that start state once, xw[n], and each lane keeps only the
// coordinates its chain has changed, in an open-addressing table of K slots
// (16-bit coordinate key, value; linear probing; K > N, so a probe always
// ends).  Reading x_d probes the lane's table and falls back to xw[d]; an
// accepted move writes the slot the probe ended on.  At level 0 the fallback
// is the chain's own uniform start point, regenerated from its start counters.
// Slot h of lane t sits at h * WG + t, so lanes probing different slots still
// hit distinct banks.  The arithmetic of a move is the dense kernel's, so the
// trajectories are identical.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sa_device.hpp"
#include "sa_internal.hpp"
#include "sa_level_common.hpp"
#include "sa_step.hpp"

namespace sa {

namespace {

constexpr uint32_t kEmptyKey = 0xFFFFu;

// First slot of coordinate d in a table of K slots (Fibonacci hashing).
__device__ __forceinline__ uint32_t slot_of(uint32_t d, uint32_t K) { return __umulhi(d * 2654435761u, K); }

// Value of coordinate d before the chain has changed it: its own uniform start
// at level 0 (the dense kernel's formula), else the level's start state.
template <typename R, bool TABLE>
__device__ __forceinline__ R start_coord(const LevelArgs<R> &a, const R *tab, const R *xw, uint32_t level,
                                         uint32_t chain, uint32_t d)
{
    if (level != 0) return xw[d];
    const Ctr r = philox4x32_10(Ctr{d >> 2, kInitLevel, chain, kTagInit | (a.problem << 8)}, a.seed_lo, a.seed_hi);
    const uint32_t w = (d & 3u) == 0 ? r.w0 : (d & 3u) == 1 ? r.w1 : (d & 3u) == 2 ? r.w2 : r.w3;
    const Coord<R> c = coord<R, TABLE>(a, tab, d);
    R xi = c.lo + (c.hi - c.lo) * u24<R>(w);
    if (xi > c.hi) xi = c.hi;
    if (xi < c.lo) xi = c.lo;
    return xi;
}

// N Metropolis steps of one chain per lane on the overlay state.  The next
// group's generator blocks are computed a group ahead as independent work.
template <typename R, int F, bool TABLE, int MOVE, typename LogFn>
__device__ __forceinline__ uint32_t run_overlay_steps(const LevelArgs<R> &a, const R *tab, const R *xw,
                                                      uint16_t *keys, R *vals, uint32_t K, uint32_t WG, uint32_t tid,
                                                      Cost<R, F> &cost, const LogFn &logf, uint32_t level,
                                                      uint32_t chain, double T, float nl2T)
{
    const uint32_t n = a.n, k0 = a.seed_lo, k1 = a.seed_hi;
    const uint32_t ctr3 = kTagMove | (a.problem << 8);
    uint32_t accepted = 0;
    MoveGroup m = move_group(0u, level, chain, ctr3, k0, k1);
    const uint32_t steps = a.steps;
    for (uint32_t g = 0; 4u * g < steps; ++g) {
        const MoveGroup next = move_group(g + 1u, level, chain, ctr3, k0, k1);
#pragma unroll
        for (uint32_t j = 0; j < 4u; ++j) {
            const uint32_t step = 4u * g + j;
            if (step >= steps) break;
            uint32_t wd, w1, w2;
            move_words(m, j, wd, w1, w2);
            const uint32_t d = pick(wd, n);
            // the coordinate's box/shift entry is read before the probe, so the
            // two LDS round trips overlap
            const Coord<R> c = coord<R, TABLE>(a, tab, d);
            uint32_t h = slot_of(d, K);
            // the home slot's key and value and the start-state fallback are
            // read together (one LDS round trip when the home slot decides,
            // the common case); a collision continues the probe
            const uint32_t key0 = keys[h * WG + tid];
            const R val0 = vals[h * WG + tid];
            const R base0 = level != 0 ? xw[d] : R(0);
            // kh, vh: key and value of the slot the probe ends on (vh is not
            // read for an empty slot; an empty slot's value is never used)
            uint32_t kh = key0;
            R vh = val0;
            R xd = key0 == d ? val0 : base0;
            if (key0 != d && key0 != kEmptyKey) {
                for (;;) {
                    h = h + 1u == K ? 0u : h + 1u;
                    kh = keys[h * WG + tid];
                    if (kh == d) {
                        vh = vals[h * WG + tid];
                        xd = vh;
                        break;
                    }
                    if (kh == kEmptyKey) {
                        xd = base0;
                        break;
                    }
                }
            }
            if (level == 0 && kh == kEmptyKey) xd = start_coord<R, TABLE>(a, tab, xw, level, chain, d);
            const R xn = neighbour_w<MOVE>(xd, c, w1);
            R df;
            bool take;
            if constexpr (sizeof(R) == sizeof(float)) {
                take = cost.step(xd, xn, c.sh, (float)(w2 >> 8), nl2T, a.inv_n);
                df = cost.df_;
            } else {
                df = cost.delta(xd - c.sh, xn - c.sh, n, a.inv_n);
                take = metropolis_w(df, w2, T, nl2T);
            }
            logf(step, d, take, xd, xn, df);
            // the slot's new contents, or its old ones: no branch on the decision
            keys[h * WG + tid] = (uint16_t)(take ? d : kh);
            vals[h * WG + tid] = take ? xn : vh;
            cost.commit(take, a.inv_n);
            accepted += take ? 1u : 0u;
        }
        m = next;
    }
    return accepted;
}

}  // namespace

// ---------------------------------------------------------------------------
// LDS: xw[n] level start | xb[n] workgroup best | tab[n][4] (TABLE only) |
//      vals[K][WG] | keys[K][WG] (16-bit)
// ---------------------------------------------------------------------------
template <typename R, int F, bool TABLE, bool LOG, int MOVE>
__global__ void __launch_bounds__(256)
    overlay_level_kernel(const LevelArgs<R> a, const uint32_t level, const uint32_t prev_groups)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Slot<R> wave_slot[4];
    __shared__ uint64_t wave_acc[4];
    __shared__ double sh_part[4][2];
    __shared__ double sh_start[3];

    const uint32_t WG = blockDim.x, tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nwaves = WG >> 6;
    const uint32_t G = gridDim.x, n = a.n, K = a.ov_slots;
    R *xw = reinterpret_cast<R *>(lds_raw);
    R *xb = xw + n;
    R *tab = xb + n;
    R *vals = tab + (TABLE ? 4 * n : 0);
    uint16_t *keys = reinterpret_cast<uint16_t *>(vals + (size_t)K * WG);
    // The level's constants are loaded before the hand-off (latency overlap).
    const double T = a.T[level];
    const float nl2T = -kLog2e * a.inv_T[level];

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

    const bool log_level = LOG && level >= a.log_level && level - a.log_level < a.log_levels;
    const Full start{sh_start[0], sh_start[1], sh_start[2]};
    R wf = widen_inf<R>();
    uint32_t wc = 0xFFFFFFFFu;
    uint32_t accepted = 0;

    for (uint32_t tile = blockIdx.x; tile < a.tiles; tile += G) {
        const uint32_t chain = tile * WG + tid;
        for (uint32_t k = 0; k < K; ++k) keys[k * WG + tid] = (uint16_t)kEmptyKey;
        Cost<R, F> cost;
        if (level == 0) {
            FullAcc<F> acc;
            for (uint32_t i = 0; i < n; ++i)
                acc.add((double)start_coord<R, TABLE>(a, tab, xw, 0u, chain, i) -
                        (double)coord<R, TABLE>(a, tab, i).sh);
            cost.set(acc.finish(n), n);
        } else {
            cost.set(start, n);
        }

        const bool logging = log_level && chain < a.log_chains;
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
        accepted += run_overlay_steps<R, F, TABLE, MOVE>(a, tab, xw, keys, vals, K, WG, tid, cost, logf, level, chain,
                                                          T, nl2T);
        if (LOG && log_level) a.log_final[(size_t)(level - a.log_level) * a.chains + chain] = (double)cost.f;

        // ---- tile argmin; materialise a new workgroup best: start values, then its changes
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
        if (nc != wc) {
            const uint32_t col = tc - tile * WG;
            for (uint32_t i = tid; i < n; i += WG) xb[i] = start_coord<R, TABLE>(a, tab, xw, level, tc, i);
            __syncthreads();
            for (uint32_t k = tid; k < K; k += WG) {
                const uint32_t key = keys[k * WG + col];
                if (key != kEmptyKey) xb[key] = vals[k * WG + col];
            }
            wf = nf;
            wc = nc;
        }
        __syncthreads();
    }

    // the evaluation's barriers also order the per-wave acceptance counts
    const uint32_t wacc = wave_sum(accepted);
    if (lane == 0) wave_acc[wave] = wacc;
    const Full fr = full_eval_wg<R, F, TABLE>(a, tab, xb, sh_part);
    const size_t slot = (size_t)(level & 1u) * a.tiles + blockIdx.x;
    if (tid == 0) {
        uint32_t acc = 0;
        for (uint32_t w = 0; w < nwaves; ++w) acc += (uint32_t)wave_acc[w];
        a.slots[slot] = Slot<R>{wf, wc, acc, 0u, fr.f, fr.s1, fr.s2};
    }
    for (uint32_t i = tid; i < n; i += WG) a.slot_x[slot * n + i] = xb[i];
}

size_t overlay_lds_bytes(uint32_t n, uint32_t wg, uint32_t slots, size_t real_size, bool table)
{
    return (2 * (size_t)n + (table ? 4 * (size_t)n : 0)) * real_size + (size_t)slots * wg * (real_size + 2);
}

namespace {

template <typename R, int F, bool TABLE, bool LOG, int MOVE>
hipError_t launch_ov(const LevelArgs<R> &a, uint32_t level, uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    auto kern = overlay_level_kernel<R, F, TABLE, LOG, MOVE>;
    const size_t lds = overlay_lds_bytes(a.n, a.wg, a.ov_slots, sizeof(R), TABLE);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, (int)a.wg, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)per_cu * a.num_cus, a.tiles);
    *groups = grid;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(a.wg), lds, s, a, level, prev_groups);
    return hipGetLastError();
}

template <typename R, int F>
hipError_t ov_dispatch_f(bool table, bool log, const LevelArgs<R> &a, uint32_t level, uint32_t prev,
                         uint32_t *groups, hipStream_t s)
{
    if (a.move == SA_MOVE_RADIUS) {
        if (table)
            return log ? launch_ov<R, F, true, true, SA_MOVE_RADIUS>(a, level, prev, groups, s)
                       : launch_ov<R, F, true, false, SA_MOVE_RADIUS>(a, level, prev, groups, s);
        return log ? launch_ov<R, F, false, true, SA_MOVE_RADIUS>(a, level, prev, groups, s)
                   : launch_ov<R, F, false, false, SA_MOVE_RADIUS>(a, level, prev, groups, s);
    }
    if (table)
        return log ? launch_ov<R, F, true, true, SA_MOVE_RESAMPLE>(a, level, prev, groups, s)
                   : launch_ov<R, F, true, false, SA_MOVE_RESAMPLE>(a, level, prev, groups, s);
    return log ? launch_ov<R, F, false, true, SA_MOVE_RESAMPLE>(a, level, prev, groups, s)
               : launch_ov<R, F, false, false, SA_MOVE_RESAMPLE>(a, level, prev, groups, s);
}

template <typename R>
hipError_t ov_dispatch(int func, bool table, bool log, const LevelArgs<R> &a, uint32_t level, uint32_t prev,
                       uint32_t *groups, hipStream_t s)
{
    switch (func) {
    case kSchwefel: return ov_dispatch_f<R, kSchwefel>(table, log, a, level, prev, groups, s);
    case kRastrigin: return ov_dispatch_f<R, kRastrigin>(table, log, a, level, prev, groups, s);
    case kAckley: return ov_dispatch_f<R, kAckley>(table, log, a, level, prev, groups, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_overlay_level_f32(int func, bool table, bool log, const LevelArgs<float> &a, uint32_t level,
                                    uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    return ov_dispatch<float>(func, table, log, a, level, prev_groups, groups, s);
}

hipError_t launch_overlay_level_f64(int func, bool table, bool log, const LevelArgs<double> &a, uint32_t level,
                                    uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    return ov_dispatch<double>(func, table, log, a, level, prev_groups, groups, s);
}

}  // namespace sa
