// The level kernel of synchronous parallel simulated annealing (one launch
// per temperature level), shared by the plain launchers (sa_kernels.hip) and
// the exchange-variant launchers (sa_variant.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa_device.hpp"
#include "sa_internal.hpp"
#include "sa_step.hpp"
#include "sa_level_common.hpp"
#include "sa_mlp_net.hpp"

namespace sa {

// ---------------------------------------------------------------------------
// Best-seen variant: rebuild the best-seen state of chain tc (its tile's
// candidate) into xb.  Its start state -- its own random point at level 0,
// its own state of the previous level if it continued from it, else the
// level's start state xw -- then its first bs_s moves (the move count that
// reached its lowest cost, held by the candidate's lane) re-applied where
// its accept bits say they were taken.  Lanes compute the moves' coordinates
// and change words in parallel; each coordinate then replays its own changes
// in move order on one lane.  Contains workgroup barriers.
// ---------------------------------------------------------------------------
template <typename R, int F, bool TABLE, int MOVE, typename CoordFn>
__device__ void rebuild_best_seen(const LevelArgs<R> &a, const R *tab, const R *xw, R *xb, const uint32_t *maskl,
                                  uint32_t *rd, uint32_t *rw, uint32_t *sh_cand, uint32_t tile, uint32_t tc,
                                  uint32_t bs_s, bool own_lane, uint32_t level, uint32_t ctr3, const CoordFn &coordf)
{
    const uint32_t WG = blockDim.x, tid = threadIdx.x, n = a.n;
    const uint32_t col = tc - tile * WG;
    if (tid == col) {
        sh_cand[0] = bs_s;
        sh_cand[1] = own_lane ? 1u : 0u;
    }
    __syncthreads();
    const uint32_t ns = sh_cand[0];
    const bool cown = sh_cand[1] != 0u;
    const uint32_t k0 = a.seed_lo, k1 = a.seed_hi;
    for (uint32_t i = tid; i < n; i += WG) {
        R v;
        if (level == 0) {
            const Ctr r = philox4x32_10(Ctr{i >> 2, kInitLevel, tc, kTagInit | (a.problem << 8)}, k0, k1);
            const uint32_t w = (i & 3u) == 0 ? r.w0 : (i & 3u) == 1 ? r.w1 : (i & 3u) == 2 ? r.w2 : r.w3;
            const Coord<R> c = coord<R, TABLE>(a, tab, i);
            v = c.lo + (c.hi - c.lo) * u24<R>(w);
            if (v > c.hi) v = c.hi;
            if (v < c.lo) v = c.lo;
        } else if (cown) {
            v = a.chain_x[(size_t)i * a.chains + tc];
        } else {
            v = xw[i];
        }
        xb[i] = v;
    }
    for (uint32_t t = tid; t < ns; t += WG) {
        uint32_t wd, w1, w2;
        move_words(move_group(t >> 2, level, tc, ctr3, k0, k1), t & 3u, wd, w1, w2);
        const bool taken = ((maskl[(t >> 5) * WG + col] >> (t & 31u)) & 1u) != 0u;
        rd[t] = taken ? pick(wd, n) : n;
        rw[t] = w1;
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += WG) {
        R v = xb[i];
        const Coord<R> c = coordf(i);
        for (uint32_t t = 0; t < ns; ++t)
            if (rd[t] == i) v = neighbour_w<MOVE>(v, c, rw[t]);
        xb[i] = v;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// The level kernel.  prev_groups: candidates the previous level's launch
// published (unused at level 0 and at the start level).  UNSHIFTED: the box
// is uniform, the shift is zero and every level starts from a broadcast, all
// known at compile time, so the steps skip the x - s subtractions (x - 0 is x
// exactly: the same bits as the general kernel, two fewer operations per move)
// and the kernel carries no own-state paths.
// VAR (plain and logged moves on the general kernel only): kVarSos -- the
// stochastic exchange: at a level that starts with an exchange each chain
// keeps its own state and carried cost iff U < exp(-(f_own - f_win)/T_prev)
// (U from word 0 of the block (0, level, chain, kTagSos), the test of the
// Metropolis step), else it starts from the winner; every chain's state is
// kept at every level.  kVarBest -- each chain's best-seen state of the level
// (the first state of lowest carried cost among its start state and its
// states after each accepted move) stands in for its final state in the
// level's argmin: the lane tracks the lowest cost and its move count and
// records its accept bits in LDS; for the tile's candidate the workgroup
// rebuilds that state from the chain's start state by re-applying its
// accepted moves (each coordinate on its own lane, in move order: the move
// stream is counter-based, so the changes are recomputed exactly).
// LDS: [net (learned modes)] | xs[n][WG] tile states | xw[n] level start |
//      xb[n] workgroup best | tab[n][4] per-coordinate box/shift (TABLE only)
//      | kVarBest: accept bits [words][WG], replay coordinates[steps], change
//      words[steps]
// ---------------------------------------------------------------------------
template <typename R, int F, bool TABLE, int MODE, int MOVE, bool UNSHIFTED = false, int VAR = 0>
__global__ void __launch_bounds__(256)
    level_kernel(const LevelArgs<R> a, const uint32_t level, const uint32_t prev_groups)
{
    constexpr bool SOS = (VAR & kVarSos) != 0;
    constexpr bool BEST = (VAR & kVarBest) != 0;
    static_assert(VAR == 0 || (!UNSHIFTED && (MODE == kModePlain || MODE == kModeLog)),
                  "exchange variants run plain or logged moves on the general kernel");
    constexpr bool LOG = MODE == kModeLog || MODE == kModeLearnLog || MODE == kModeLearnLogG;
    constexpr bool LEARN = MODE == kModeLearn || MODE == kModeLearnLog || MODE == kModeLearnG || MODE == kModeLearnLogG;
    constexpr int KIND = (MODE == kModeLearnG || MODE == kModeLearnLogG) ? mlp::kNetGeluGauss : mlp::kNetReluCauchy;
    constexpr bool CAPTURE = MODE == kModeCapture;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Slot<R> wave_slot[4];
    __shared__ uint64_t wave_acc[4];
    __shared__ double sh_part[4][2];
    __shared__ double sh_start[4];  // start cost (f, S1, S2); [3] the winner's carried cost (kVarSos)
    __shared__ uint32_t sh_cand[2];  // kVarBest: the candidate's moves to re-apply, own-start flag

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
    // kVarBest scratch after the table
    uint32_t *maskl = reinterpret_cast<uint32_t *>(tab + (TABLE ? 4 * (size_t)n : 0));
    uint32_t *rd = maskl + (size_t)((a.steps + 31u) >> 5) * WG;
    uint32_t *rw = rd + a.steps;

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
        adopt_winner<R>(a, level - 1, prev_groups, xw, sh_start, blockIdx.x == 0, wave_slot, wave_acc,
                        SOS ? &sh_start[3] : nullptr);
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
    const bool keep = !UNSHIFTED && (SOS || (ex != 1 && !(ex != 0 && (level + 1) % ex == 0)));
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
        bool own_lane = own;
        if constexpr (SOS) {
            if (level > 0 && level != a.start_level && !own) {  // a level that starts with an exchange
                const R dfo = a.chain_cost[chain] - (R)sh_start[3];
                const uint32_t u = philox4x32_10(Ctr{0u, level, chain, kTagSos | (a.problem << 8)}, k0, k1).w0;
                if constexpr (sizeof(R) == sizeof(float))
                    own_lane = metropolis_k(dfo, (float)(u >> 8), -kLog2e * a.inv_T[level - 1]);
                else
                    own_lane = metropolis_w(dfo, u, a.T[level - 1], 0.0f);
            }
        }
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
        } else if (own_lane) {
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
        // kVarBest: lowest carried cost so far, the move count that reached it, accept bits
        R bs_f = cost.f;
        uint32_t bs_s = 0u, accw = 0u;
        const auto bestf = [&](uint32_t step, bool take, R f) {
            if constexpr (BEST) {
                accw |= (take ? 1u : 0u) << (step & 31u);
                if ((step & 31u) == 31u) {
                    maskl[(step >> 5) * WG + tid] = accw;
                    accw = 0u;
                }
                if (f < bs_f) {
                    bs_f = f;
                    bs_s = step + 1u;
                }
            }
        };
        if constexpr (LEARN) {
            float h[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            accepted += run_learned_steps<F, KIND>(xs, WG, tid, cost, coordf, logf, n, a.steps, level, chain, ctr3,
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
                        const bool raw = a.net_kind == mlp::kNetGeluGauss;
#pragma unroll
                        for (int k = 0; k < 4; ++k) rec[2 + k] = raw ? (float)hist[k] : (float)hist_feature(hist[k]);
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
        } else if constexpr (BEST) {
            accepted += run_steps<R, F, MOVE>(xs, WG, tid, cost, coordf, logf, n, a.steps, level, chain, ctr3, k0,
                                              k1, T, nl2T, a.inv_n, bestf);
            if (a.steps & 31u) maskl[(a.steps >> 5) * WG + tid] = accw;
        } else {
            accepted += run_steps<R, F, MOVE>(xs, WG, tid, cost, coordf, logf, n, a.steps, level, chain, ctr3, k0,
                                              k1, T, nl2T, a.inv_n);
        }
        // the value the level's argmin runs over: the final or the best-seen cost
        const R rf = BEST ? bs_f : cost.f;
        if (LOG && log_level) a.log_final[(size_t)(level - a.log_level) * a.chains + chain] = (double)rf;
        // (kVarBest stores after the candidate is rebuilt: its own start state is read from chain_x)
        if (!BEST && keep) {
            store_column(xs, WG, tid, a.chain_x + chain, a.chains, n);
            cost.save(a.chain_cost + chain, a.chains);
        }

        // ---- tile argmin of (final cost, chain); keep the workgroup's best
        R bf = rf;
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
        if constexpr (BEST) {
            if (nc != wc) {
                rebuild_best_seen<R, F, TABLE, MOVE>(a, tab, xw, xb, maskl, rd, rw, sh_cand, tile, tc, bs_s, own_lane,
                                                     level, ctr3, coordf);
                best = xb;
                best_stride = 1;
                wf = nf;
                wc = nc;
            }
            if (keep) {
                store_column(xs, WG, tid, a.chain_x + chain, a.chains, n);
                cost.save(a.chain_cost + chain, a.chains);
            }
        } else if (nc != wc) {
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


}  // namespace sa
