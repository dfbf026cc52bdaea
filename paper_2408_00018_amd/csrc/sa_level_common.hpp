// Level-boundary pieces shared by the level kernels (dense and overlay state
// layouts): per-coordinate parameters, the workgroup's full evaluation of a
// state in LDS, and the reduction of the previous level's candidates to the
// winner every chain starts from (Sec. 2.2.2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa_device.hpp"
#include "sa_internal.hpp"
#include "sa_step.hpp"

namespace sa {

template <typename R, bool TABLE>
__device__ __forceinline__ Coord<R> coord(const LevelArgs<R> &a, const R *tab, uint32_t d)
{
    if (TABLE) return Coord<R>{tab[4 * d + 0], tab[4 * d + 1], tab[4 * d + 2], tab[4 * d + 3]};
    return Coord<R>{a.lo, a.hi, a.rho, a.sh};
}

// ---------------------------------------------------------------------------
// Full evaluation of a state held in LDS (coordinate i at x[i * stride]),
// FP64 arithmetic.  FP64 runs sum in coordinate order on one lane (the order
// of a plain sequential evaluation); FP32 runs use a fixed parallel order.
// Contains workgroup barriers: LDS writes made before the call are visible to
// every thread of the workgroup after it.
// ---------------------------------------------------------------------------
template <typename R, int F, bool TABLE>
__device__ Full full_eval_wg(const LevelArgs<R> &a, const R *tab, const R *x, double (*part)[2],
                             uint32_t stride = 1)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nwaves = blockDim.x >> 6;
    const uint32_t n = a.n;
    if (sizeof(R) == sizeof(double)) {
        if (tid == 0) {
            FullAcc<F> acc;
            for (uint32_t i = 0; i < n; ++i) acc.add((double)x[i * stride] - (double)coord<R, TABLE>(a, tab, i).sh);
            const Full v = acc.finish(n);
            part[0][0] = v.f;
            part[0][1] = v.s1;
            part[1][0] = v.s2;
        }
        __syncthreads();
        const Full v{part[0][0], part[0][1], part[1][0]};
        __syncthreads();
        return v;
    }
    FullAcc<F> acc;
    for (uint32_t i = tid; i < n; i += blockDim.x)
        acc.add((double)x[i * stride] - (double)coord<R, TABLE>(a, tab, i).sh);
    const double pa = wave_sum_d(acc.a), pb = wave_sum_d(acc.b);
    if (lane == 0) {
        part[wave][0] = pa;
        part[wave][1] = pb;
    }
    __syncthreads();
    FullAcc<F> tot;
    for (uint32_t w = 0; w < nwaves; ++w) {
        tot.a += part[w][0];
        tot.b += part[w][1];
    }
    __syncthreads();
    return tot.finish(n);
}

// ---------------------------------------------------------------------------
// Reduce the candidates level `lvl` published (`groups` of them) to the
// level's winner: lowest carried cost, ties to the lowest chain.  Every
// workgroup that calls this gets the same winner; its state goes to xw and
// its full re-evaluation to start -- or, for an elitist run, the record's
// (the winner if it improves the record after level lvl - 1, else that
// record, read from the mirror the previous launch wrote).  With `publish`
// the workgroup also writes the level's trace entry, the record, the
// winner's state and the record's mirror for the next launch.  win_f
// (optional, LDS) gets the winner's carried cost.
// ---------------------------------------------------------------------------
template <typename R>
__device__ void adopt_winner(const LevelArgs<R> &a, uint32_t lvl, uint32_t groups, R *xw, double *start,
                             bool publish, Slot<R> *wave_slot, uint64_t *wave_acc, double *win_f = nullptr)
{
    const uint32_t WG = blockDim.x, tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nwaves = WG >> 6;
    const uint32_t n = a.n;
    const size_t base = (size_t)(lvl & 1u) * a.tiles;
    // The record the previous launch left is loaded together with the
    // candidates, not after the winner is known (one global round trip fewer
    // on the publishing workgroup's path).
    const double rec_prev = publish ? a.rec[0] : 0.0;
    R gf = widen_inf<R>();
    uint32_t gc = 0xFFFFFFFFu, gj = 0;
    uint64_t gacc = 0;
    for (uint32_t j = tid; j < groups; j += WG) {
        const Slot<R> s = a.slots[base + j];
        if (s.f < gf || (s.f == gf && s.chain < gc)) {
            gf = s.f;
            gc = s.chain;
            gj = j;
        }
        gacc += s.accepts;
    }
    wave_best(gf, gc, gj);
    gacc = wave_sum(gacc);
    __syncthreads();
    if (lane == 0) {
        wave_slot[wave] = Slot<R>{gf, gc, gj, 0u, 0.0, 0.0, 0.0};
        wave_acc[wave] = gacc;
    }
    __syncthreads();
    gf = wave_slot[0].f;
    gc = wave_slot[0].chain;
    gj = wave_slot[0].accepts;
    gacc = wave_acc[0];
    for (uint32_t w = 1; w < nwaves; ++w) {
        if (wave_slot[w].f < gf || (wave_slot[w].f == gf && wave_slot[w].chain < gc)) {
            gf = wave_slot[w].f;
            gc = wave_slot[w].chain;
            gj = wave_slot[w].accepts;
        }
        gacc += wave_acc[w];
    }
    if (gj >= groups) gj = 0;  // only if every candidate cost were NaN; keeps the index in range
    const size_t w = base + gj;
    const Slot<R> ws = a.slots[w];
    const bool improved = publish && ws.ff < rec_prev;
    // elitist: the record after level lvl - 1 (mirror (lvl + 1) & 1; +inf
    // after a reset) and the one after level lvl (mirror lvl & 1)
    const uint32_t e_in = (lvl + 1u) & 1u, e_out = lvl & 1u;
    const bool elite_keeps = a.elitist && !(ws.ff < a.elite_f[3 * e_in]);
    for (uint32_t i = tid; i < n; i += WG) {
        const R v = a.slot_x[w * n + i];
        const R e = elite_keeps ? a.elite_x[(size_t)e_in * n + i] : v;
        xw[i] = e;
        if (publish) {
            a.x_best[i] = v;
            if (a.trace_x) a.trace_x[(size_t)lvl * n + i] = v;
            if (improved) a.x_rec[i] = v;
            if (a.elitist) a.elite_x[(size_t)e_out * n + i] = e;
        }
    }
    if (tid == 0) {
        const double *ef = a.elite_f + 3 * e_in;
        start[0] = elite_keeps ? ef[0] : ws.ff;
        start[1] = elite_keeps ? ef[1] : ws.s1;
        start[2] = elite_keeps ? ef[2] : ws.s2;
        if (win_f) *win_f = (double)gf;
        if (publish && a.elitist) {
            a.elite_f[3 * e_out + 0] = start[0];
            a.elite_f[3 * e_out + 1] = start[1];
            a.elite_f[3 * e_out + 2] = start[2];
        }
    }
    if (publish) {
        if (tid == 0) {
            if (improved) {
                a.rec[0] = ws.ff;
                *a.rec_level = lvl;
            }
            sa_level t;
            t.win_chain = gc;
            t.reserved = 0;
            t.f_win = (double)gf;
            t.f_best = ws.ff;
            t.f_rec = improved ? ws.ff : rec_prev;
            t.accepts = gacc;
            t.t_ns = wall_clock64();  // ticks here; sa_trace converts them to ns
            a.trace[lvl] = t;
        }
    }
    __syncthreads();
}

}  // namespace sa
