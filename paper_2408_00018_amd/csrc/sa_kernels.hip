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

#include "sa_device.hpp"
#include "sa_internal.hpp"

namespace sa {

// ---------------------------------------------------------------------------
// Per-chain cost state.  delta() returns the increment of changing one
// coordinate from y to yn (shifted coordinates) and stages the new state;
// commit() installs it when the move is accepted.
// ---------------------------------------------------------------------------
template <typename R, int F> struct Cost;

// FP64: the increments are the definitions, evaluated in the same order as a
// plain FP64 implementation would (the FP64 path is checked move for move).
template <> struct Cost<double, kSchwefel> {
    double f, fn;
    __device__ void set(const Full &v, uint32_t) { f = v.f; }
    __device__ double delta(double y, double yn, uint32_t n, float)
    {
        const double df = -(schwefel_term_d(yn) - schwefel_term_d(y)) / (double)n;
        fn = f + df;
        return df;
    }
    __device__ void commit(bool take, float) { f = take ? fn : f; }
};

template <> struct Cost<double, kRastrigin> {
    double f, fn;
    __device__ void set(const Full &v, uint32_t) { f = v.f; }
    __device__ double delta(double y, double yn, uint32_t, float)
    {
        const double df = rastrigin_term_d(yn) - rastrigin_term_d(y);
        fn = f + df;
        return df;
    }
    __device__ void commit(bool take, float) { f = take ? fn : f; }
};

template <> struct Cost<double, kAckley> {
    double f, s1, s2, fn, s1n, s2n;
    __device__ void set(const Full &v, uint32_t)
    {
        f = v.f;
        s1 = v.s1;
        s2 = v.s2;
    }
    __device__ double delta(double y, double yn, uint32_t n, float)
    {
        s1n = s1 + (yn * yn - y * y);
        s2n = s2 + (cos(2.0 * kPi * yn) - cos(2.0 * kPi * y));
        fn = ackley_from_sums_d(s1n, s2n, n);
        return fn - f;
    }
    __device__ void commit(bool take, float)
    {
        f = take ? fn : f;
        s1 = take ? s1n : s1;
        s2 = take ? s2n : s2;
    }
};

// FP32: cancellation-free increments on the hardware transcendentals.
//   Schwefel   df = (h(y) - h(y')) / n,  h(y) = y sin(sqrt|y|)
//   Rastrigin  g(y) = y^2 + 20 sin^2(pi y)  (equal to y^2 - 10 cos 2 pi y + 10)
//              g(y') - g(y) = dl sg + 20 sin(pi dl) sin(pi sg),  dl = y'-y, sg = y'+y
//   Ackley     dS1 = dl sg,  dS2 = cos 2pi y' - cos 2pi y = -2 sin(pi sg) sin(pi dl)
//              df = -20 e^a expm1(a'-a) - e^b expm1(dS2/n)
//              a = -0.2 sqrt(S1/n), b = S2/n, a'-a = -0.2 (dS1/n) / (sqrt(S1'/n) + sqrt(S1/n))
template <> struct Cost<float, kSchwefel> {
    float f, df_;
    __device__ void set(const Full &v, uint32_t) { f = (float)v.f; }
    __device__ float delta(float y, float yn, uint32_t, float inv_n)
    {
        df_ = (schwefel_h(y) - schwefel_h(yn)) * inv_n;
        return df_;
    }
    __device__ void commit(bool take, float) { f = take ? f + df_ : f; }
};

template <> struct Cost<float, kRastrigin> {
    float f, df_;
    __device__ void set(const Full &v, uint32_t) { f = (float)v.f; }
    __device__ float delta(float y, float yn, uint32_t, float)
    {
        const float dl = yn - y, sg = yn + y;
        df_ = fmaf(dl, sg, 20.0f * hw_sin_rev(0.5f * dl) * hw_sin_rev(0.5f * sg));
        return df_;
    }
    __device__ void commit(bool take, float) { f = take ? f + df_ : f; }
};

template <> struct Cost<float, kAckley> {
    float f, s1, s2, q, ea, eb;  // q = sqrt(S1/n), ea = exp(-0.2 q), eb = exp(S2/n)
    float df_, s1n_, s2n_, qn_;
    __device__ void set(const Full &v, uint32_t n)
    {
        f = (float)v.f;
        s1 = (float)v.s1;
        s2 = (float)v.s2;
        const double qd = sqrt(v.s1 / (double)n);
        q = (float)qd;
        ea = (float)exp(-0.2 * qd);
        eb = (float)exp(v.s2 / (double)n);
    }
    __device__ float delta(float y, float yn, uint32_t, float inv_n)
    {
        const float dl = yn - y, sg = yn + y;
        const float ds1 = dl * sg;
        const float ds2 = -2.0f * hw_sin_rev(0.5f * sg) * hw_sin_rev(0.5f * dl);
        s1n_ = fmaxf(s1 + ds1, 0.0f);
        s2n_ = s2 + ds2;
        qn_ = hw_sqrt(s1n_ * inv_n);
        const float den = qn_ + q;
        const float da = den > 0.0f ? (-0.2f * (ds1 * inv_n)) / den : 0.0f;
        df_ = -20.0f * ea * expm1f(da) - eb * expm1f(ds2 * inv_n);
        return df_;
    }
    __device__ void commit(bool take, float inv_n)
    {
        if (take) {
            f += df_;
            s1 = s1n_;
            s2 = s2n_;
            q = qn_;
            ea = hw_exp2((-0.2f * kLog2e) * qn_);
            eb = hw_exp2(kLog2e * (s2n_ * inv_n));
        }
    }
};

// ---------------------------------------------------------------------------
// Full evaluation in FP64 arithmetic, definition form, coordinates summed in
// order 0..n-1 (the order of a plain sequential evaluation).
// ---------------------------------------------------------------------------
template <int F> struct FullAcc {
    double a = 0.0, b = 0.0;
    __device__ void add(double y)
    {
        if (F == kSchwefel) {
            a += schwefel_term_d(y);
        } else if (F == kRastrigin) {
            a += rastrigin_term_d(y);
        } else {
            a += y * y;
            b += cos(2.0 * kPi * y);
        }
    }
    __device__ Full finish(uint32_t n) const
    {
        if (F == kSchwefel) return Full{-a / (double)n, 0.0, 0.0};
        if (F == kRastrigin) return Full{10.0 * (double)n + a, 0.0, 0.0};
        return Full{ackley_from_sums_d(a, b, n), a, b};
    }
};

// Per-coordinate parameters {l, u, rho, s}.
template <typename R> struct Coord {
    R lo, hi, rho, sh;
};

template <typename R, bool TABLE>
__device__ __forceinline__ Coord<R> coord(const LevelArgs<R> &a, const R *tab, uint32_t d)
{
    if (TABLE) return Coord<R>{tab[4 * d + 0], tab[4 * d + 1], tab[4 * d + 2], tab[4 * d + 3]};
    return Coord<R>{a.lo, a.hi, a.rho, a.sh};
}

// Neighbour of one coordinate: x + rho (2U - 1) (radius rule) or l + (u - l) U
// (resampling), clamped to [l, u].  FP32 clamps with one v_med3_f32.
template <int MOVE> __device__ __forceinline__ float neighbour(float xd, const Coord<float> &c, float u1)
{
    const float xn = MOVE == SA_MOVE_RADIUS ? fmaf(c.rho, fmaf(2.0f, u1, -1.0f), xd) : fmaf(c.rho, u1, c.lo);
    return __builtin_amdgcn_fmed3f(xn, c.lo, c.hi);
}
template <int MOVE> __device__ __forceinline__ double neighbour(double xd, const Coord<double> &c, double u1)
{
    double xn = MOVE == SA_MOVE_RADIUS ? xd + c.rho * (2.0 * u1 - 1.0) : c.lo + c.rho * u1;
    if (xn > c.hi) xn = c.hi;
    if (xn < c.lo) xn = c.lo;
    return xn;
}

// Metropolis acceptance (eq. (5), k_b = 1): always downhill, else U < exp(-df/T).
__device__ __forceinline__ bool metropolis(float df, float u2, double, float neg_log2e_inv_T)
{
    return df <= 0.0f || u2 < hw_exp2(df * neg_log2e_inv_T);
}
__device__ __forceinline__ bool metropolis(double df, double u2, double T, float)
{
    return df <= 0.0 || u2 < exp(-df / T);
}

// Lexicographic (cost, chain) minimum: ties go to the lower chain index.
template <typename R> __device__ __forceinline__ void best_of(R &f, uint32_t &c, R f2, uint32_t c2)
{
    if (f2 < f || (f2 == f && c2 < c)) {
        f = f2;
        c = c2;
    }
}

template <typename R> __device__ __forceinline__ void wave_best(R &f, uint32_t &c)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const R f2 = __shfl_xor(f, off, 64);
        const uint32_t c2 = __shfl_xor(c, off, 64);
        best_of(f, c, f2, c2);
    }
}

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename R> __device__ __forceinline__ R widen_inf();
template <> __device__ __forceinline__ float widen_inf<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double widen_inf<double>() { return __builtin_inf(); }

// ---------------------------------------------------------------------------
// Full evaluation of a state held in LDS, FP64 arithmetic.  FP64 runs sum in
// coordinate order on one lane (the order of a plain sequential
// evaluation); FP32 runs use a fixed parallel order.
// ---------------------------------------------------------------------------
template <typename R, int F, bool TABLE>
__device__ Full full_eval_wg(const LevelArgs<R> &a, const R *tab, const R *x, double (*part)[2])
{
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nwaves = blockDim.x >> 6;
    const uint32_t n = a.n;
    if (sizeof(R) == sizeof(double)) {
        if (tid == 0) {
            FullAcc<F> acc;
            for (uint32_t i = 0; i < n; ++i) acc.add((double)x[i] - (double)coord<R, TABLE>(a, tab, i).sh);
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
    for (uint32_t i = tid; i < n; i += blockDim.x) acc.add((double)x[i] - (double)coord<R, TABLE>(a, tab, i).sh);
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
// its full re-evaluation to start.  With `publish` the workgroup also writes
// the level's trace entry, the record and the broadcast state.
// ---------------------------------------------------------------------------
template <typename R>
__device__ void adopt_winner(const LevelArgs<R> &a, uint32_t lvl, uint32_t groups, R *xw, double *start,
                             bool publish, Slot<R> *wave_slot, uint64_t *wave_acc)
{
    const uint32_t WG = blockDim.x, tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nwaves = WG >> 6;
    const uint32_t n = a.n;
    const size_t base = (size_t)(lvl & 1u) * a.tiles;
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
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const R f2 = __shfl_xor(gf, off, 64);
        const uint32_t c2 = __shfl_xor(gc, off, 64);
        const uint32_t j2 = __shfl_xor(gj, off, 64);
        if (f2 < gf || (f2 == gf && c2 < gc)) {
            gf = f2;
            gc = c2;
            gj = j2;
        }
    }
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
    for (uint32_t i = tid; i < n; i += WG) xw[i] = a.slot_x[w * n + i];
    const Slot<R> ws = a.slots[w];
    if (tid == 0) {
        start[0] = ws.ff;
        start[1] = ws.s1;
        start[2] = ws.s2;
    }
    if (publish) {
        const bool improved = ws.ff < a.rec[0];
        __syncthreads();
        for (uint32_t i = tid; i < n; i += WG) {
            const R v = a.slot_x[w * n + i];
            a.x_best[i] = v;
            if (a.trace_x) a.trace_x[(size_t)lvl * n + i] = v;
            if (improved) a.x_rec[i] = v;
        }
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
            t.f_rec = improved ? ws.ff : a.rec[0];
            t.accepts = gacc;
            t.t_ticks = wall_clock64();
            a.trace[lvl] = t;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// The level kernel.  prev_groups: candidates the previous level's launch
// published (unused at level 0).
// LDS: xs[n][WG] tile states | xw[n] level start | xb[n] workgroup best |
//      tab[n][4] per-coordinate box/shift (TABLE only)
// ---------------------------------------------------------------------------
template <typename R, int F, bool TABLE, bool LOG, int MOVE>
__global__ void __launch_bounds__(256)
    level_kernel(const LevelArgs<R> a, const uint32_t level, const uint32_t prev_groups)
{
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
    R *xs = reinterpret_cast<R *>(lds_raw);
    R *xw = xs + (size_t)n * WG;
    R *xb = xw + n;
    R *tab = xb + n;

    if (TABLE) {
        for (uint32_t i = tid; i < 4 * n; i += WG) tab[i] = a.table[i];
    }
    if (level > 0) adopt_winner<R>(a, level - 1, prev_groups, xw, sh_start, blockIdx.x == 0, wave_slot, wave_acc);
    __syncthreads();

    const uint32_t k0 = a.seed_lo, k1 = a.seed_hi;
    const uint32_t ctr3 = kTagMove | (a.problem << 8);
    const double T = a.T[level];
    const float nl2T = -kLog2e * a.inv_T[level];
    const bool log_level = LOG && level >= a.log_level && level - a.log_level < a.log_levels;
    const Full start{sh_start[0], sh_start[1], sh_start[2]};
    R wf = widen_inf<R>();
    uint32_t wc = 0xFFFFFFFFu;
    uint32_t accepted = 0;

    for (uint32_t tile = blockIdx.x; tile < a.tiles; tile += G) {
        const uint32_t chain = tile * WG + tid;
        // ---- tile start: own random point at level 0, else the winner
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
        } else {
            for (uint32_t i = 0; i < n; ++i) xs[i * WG + tid] = xw[i];
            cost.set(start, n);
        }

        // ---- N Metropolis steps, software-pipelined two moves deep: at the
        // top of move s the (old) value of move s+1's coordinate is read from
        // LDS and move s+2's draws are computed, so neither the LDS latency
        // nor the generator's dependent rounds sit on move s's critical path.
        // If move s+1 picks the coordinate move s writes, the written value is
        // forwarded.
        const bool logging = log_level && chain < a.log_chains;
        Ctr r = philox4x32_10(Ctr{0u, level, chain, ctr3}, k0, k1);
        Ctr r1 = philox4x32_10(Ctr{1u, level, chain, ctr3}, k0, k1);
        uint32_t d = pick(r.w0, n);
        uint32_t d1 = pick(r1.w0, n);
        R xd = xs[__umul24(d, WG) + tid];
        for (uint32_t step = 0; step < a.steps; ++step) {
            const R x1_lds = xs[__umul24(d1, WG) + tid];
            const Ctr r2 = philox4x32_10(Ctr{step + 2u, level, chain, ctr3}, k0, k1);
            const Coord<R> c = coord<R, TABLE>(a, tab, d);
            const R xn = neighbour<MOVE>(xd, c, u24<R>(r.w1));
            const R df = cost.delta(xd - c.sh, xn - c.sh, n, a.inv_n);
            const bool take = metropolis(df, u24<R>(r.w2), T, nl2T);
            if (LOG && logging) {
                sa_move_rec m;
                m.d = d;
                m.accept = take ? 1u : 0u;
                m.x_old = (double)xd;
                m.x_new = (double)xn;
                m.df = (double)df;
                a.log[((size_t)(level - a.log_level) * a.log_chains + chain) * a.steps + step] = m;
            }
            const R xwr = take ? xn : xd;
            xs[__umul24(d, WG) + tid] = xwr;
            cost.commit(take, a.inv_n);
            accepted += take ? 1u : 0u;
            xd = d1 == d ? xwr : x1_lds;
            d = d1;
            r = r1;
            r1 = r2;
            d1 = pick(r2.w0, n);
        }
        if (LOG && log_level) a.log_final[(size_t)(level - a.log_level) * a.chains + chain] = (double)cost.f;

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
        if (nc != wc) {
            const uint32_t col = tc - tile * WG;
            for (uint32_t i = tid; i < n; i += WG) xb[i] = xs[i * WG + col];
            wf = nf;
            wc = nc;
        }
        __syncthreads();
    }

    // ---- publish this workgroup's candidate, re-evaluated in full
    const Full fr = full_eval_wg<R, F, TABLE>(a, tab, xb, sh_part);
    const uint32_t wacc = wave_sum(accepted);
    if (lane == 0) wave_acc[wave] = wacc;
    __syncthreads();
    const size_t slot = (size_t)(level & 1u) * a.tiles + blockIdx.x;
    if (tid == 0) {
        uint32_t acc = 0;
        for (uint32_t w = 0; w < nwaves; ++w) acc += (uint32_t)wave_acc[w];
        a.slots[slot] = Slot<R>{wf, wc, acc, 0u, fr.f, fr.s1, fr.s2};
    }
    for (uint32_t i = tid; i < n; i += WG) a.slot_x[slot * n + i] = xb[i];
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

size_t level_lds_bytes(uint32_t n, uint32_t wg, size_t real_size, bool table)
{
    return ((size_t)n * wg + 2 * (size_t)n + (table ? 4 * (size_t)n : 0)) * real_size;
}

template <typename R, int F, bool TABLE, bool LOG, int MOVE>
static hipError_t launch_one(const LevelArgs<R> &a, uint32_t level, uint32_t prev_groups, uint32_t *groups,
                             hipStream_t s)
{
    auto kern = level_kernel<R, F, TABLE, LOG, MOVE>;
    const size_t lds = level_lds_bytes(a.n, a.wg, sizeof(R), TABLE);
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
static hipError_t dispatch_f(bool table, bool log, const LevelArgs<R> &a, uint32_t level, uint32_t prev,
                             uint32_t *groups, hipStream_t s)
{
    if (a.move == SA_MOVE_RADIUS) {
        if (table)
            return log ? launch_one<R, F, true, true, SA_MOVE_RADIUS>(a, level, prev, groups, s)
                       : launch_one<R, F, true, false, SA_MOVE_RADIUS>(a, level, prev, groups, s);
        return log ? launch_one<R, F, false, true, SA_MOVE_RADIUS>(a, level, prev, groups, s)
                   : launch_one<R, F, false, false, SA_MOVE_RADIUS>(a, level, prev, groups, s);
    }
    if (table)
        return log ? launch_one<R, F, true, true, SA_MOVE_RESAMPLE>(a, level, prev, groups, s)
                   : launch_one<R, F, true, false, SA_MOVE_RESAMPLE>(a, level, prev, groups, s);
    return log ? launch_one<R, F, false, true, SA_MOVE_RESAMPLE>(a, level, prev, groups, s)
               : launch_one<R, F, false, false, SA_MOVE_RESAMPLE>(a, level, prev, groups, s);
}

template <typename R>
static hipError_t dispatch(int func, bool table, bool log, const LevelArgs<R> &a, uint32_t level, uint32_t prev,
                           uint32_t *groups, hipStream_t s)
{
    switch (func) {
    case kSchwefel: return dispatch_f<R, kSchwefel>(table, log, a, level, prev, groups, s);
    case kRastrigin: return dispatch_f<R, kRastrigin>(table, log, a, level, prev, groups, s);
    case kAckley: return dispatch_f<R, kAckley>(table, log, a, level, prev, groups, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_level_f32(int func, bool table, bool log, const LevelArgs<float> &a, uint32_t level,
                            uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    return dispatch<float>(func, table, log, a, level, prev_groups, groups, s);
}

hipError_t launch_level_f64(int func, bool table, bool log, const LevelArgs<double> &a, uint32_t level,
                            uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    return dispatch<double>(func, table, log, a, level, prev_groups, groups, s);
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
