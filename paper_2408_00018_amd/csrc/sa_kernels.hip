// Level kernel of synchronous parallel simulated annealing for gfx950.
//
// One Markov chain per lane.  A workgroup of WG lanes keeps its chains'
// states in LDS as x[d][lane] (coordinate-major), so a per-lane random
// coordinate d is a bank-conflict-free LDS access.  One launch runs one
// temperature level (Sec. 2.2.2: every chain runs N Metropolis steps at a
// fixed T) and ends with the device-wide argmin and broadcast that start the
// next level: every workgroup publishes its best chain and that chain's
// state, and the last workgroup to finish picks the global winner,
// re-evaluates it in full, updates the record and the trace and publishes
// the winner as the next level's start.
#include <hip/hip_runtime.h>
#include <stdint.h>

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
// The level kernel.
// ---------------------------------------------------------------------------
template <typename R, int F, bool TABLE, bool LOG, int MOVE>
__global__ void __launch_bounds__(256) level_kernel(const LevelArgs<R> a, const uint32_t level)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Slot<R> wave_slot[4];
    __shared__ uint64_t wave_acc[4];
    __shared__ uint32_t sh_flag;
    __shared__ double sh_part[4][2];

    const uint32_t WG = a.wg;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t nwaves = WG >> 6;
    const uint32_t chain = blockIdx.x * WG + tid;
    const uint32_t n = a.n;
    R *xs = reinterpret_cast<R *>(lds_raw);
    R *tab = xs + (size_t)n * WG;

    if (TABLE) {
        for (uint32_t i = tid; i < 4 * n; i += WG) tab[i] = a.table[i];
        __syncthreads();
    }

    // ---- level start: own random point at level 0, else the broadcast winner
    Cost<R, F> cost;
    if (level == 0) {
        FullAcc<F> acc;
        Ctr r{};
        for (uint32_t i = 0; i < n; ++i) {
            if ((i & 3u) == 0)
                r = philox4x32_10(Ctr{i >> 2, kInitLevel, chain, kTagInit | (a.problem << 8)}, a.seed_lo, a.seed_hi);
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
        for (uint32_t i = 0; i < n; ++i) xs[i * WG + tid] = a.x_best[i];
        cost.set(Full{a.start[0], a.start[1], a.start[2]}, n);
    }

    // ---- N Metropolis steps at T_level
    const double T = a.T[level];
    const float nl2T = -kLog2e * a.inv_T[level];
    const uint32_t ctr3 = kTagMove | (a.problem << 8);
    const bool logging = LOG && chain < a.log_chains && level >= a.log_level && level - a.log_level < a.log_levels;
    // Software-pipelined two steps deep: at the top of step s the (old) value
    // of step s+1's coordinate is read from LDS and step s+2's draws are
    // computed, so neither the LDS latency nor the generator's dependent
    // rounds sit on step s's critical path.  If step s+1 picks the coordinate
    // step s writes, the written value is forwarded.
    uint32_t accepted = 0;
    const uint32_t k0 = a.seed_lo, k1 = a.seed_hi;
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
        const R xw = take ? xn : xd;
        xs[__umul24(d, WG) + tid] = xw;
        cost.commit(take, a.inv_n);
        accepted += take ? 1u : 0u;
        xd = d1 == d ? xw : x1_lds;
        d = d1;
        r = r1;
        r1 = r2;
        d1 = pick(r2.w0, n);
    }
    if (LOG && level >= a.log_level && level - a.log_level < a.log_levels)
        a.log_final[(size_t)(level - a.log_level) * a.chains + chain] = (double)cost.f;

    // ---- workgroup argmin of (final cost, chain) and accepted-move count
    R bf = cost.f;
    uint32_t bc = chain;
    wave_best(bf, bc);
    const uint32_t wacc = wave_sum(accepted);
    if (lane == 0) {
        wave_slot[wave] = Slot<R>{bf, bc, wacc};
    }
    __syncthreads();
    if (tid == 0) {
        Slot<R> s = wave_slot[0];
        for (uint32_t w = 1; w < nwaves; ++w) {
            best_of(s.f, s.chain, wave_slot[w].f, wave_slot[w].chain);
            s.accepts += wave_slot[w].accepts;
        }
        a.slots[blockIdx.x] = s;
        sh_flag = s.chain - blockIdx.x * WG;
    }
    __syncthreads();
    {
        const uint32_t wl = sh_flag;
        R *dst = a.slot_x + (size_t)blockIdx.x * n;
        for (uint32_t i = tid; i < n; i += WG) dst[i] = xs[i * WG + wl];
    }
    // Publish the slot, then count this workgroup as arrived.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) {
        const uint32_t prev = __hip_atomic_fetch_add(a.arrive, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        sh_flag = (prev == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (sh_flag == 0) return;

    // ---- last workgroup: global winner, broadcast, full re-evaluation, record
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    R gf = widen_inf<R>();
    uint32_t gc = 0xFFFFFFFFu;
    uint64_t gacc = 0;
    for (uint32_t j = tid; j < gridDim.x; j += WG) {
        const Slot<R> s = a.slots[j];
        best_of(gf, gc, s.f, s.chain);
        gacc += s.accepts;
    }
    wave_best(gf, gc);
    gacc = wave_sum(gacc);
    __syncthreads();
    if (lane == 0) {
        wave_slot[wave] = Slot<R>{gf, gc, 0u};
        wave_acc[wave] = gacc;
    }
    __syncthreads();
    gf = wave_slot[0].f;
    gc = wave_slot[0].chain;
    gacc = wave_acc[0];
    for (uint32_t w = 1; w < nwaves; ++w) {
        best_of(gf, gc, wave_slot[w].f, wave_slot[w].chain);
        gacc += wave_acc[w];
    }
    if (gc >= a.chains) gc = 0;  // only if every final cost were NaN; keeps the index in range
    const uint32_t wslot = gc / WG;
    R *xw = xs;  // reuse LDS column 0 as the winner's state
    __syncthreads();
    for (uint32_t i = tid; i < n; i += WG) {
        const R v = a.slot_x[(size_t)wslot * n + i];
        xw[i] = v;
        a.x_best[i] = v;
        if (a.trace_x) a.trace_x[(size_t)level * n + i] = v;
    }
    __syncthreads();

    Full fresh;
    if (sizeof(R) == sizeof(double)) {
        // FP64 runs: the sequential order of a plain evaluation.
        if (tid == 0) {
            FullAcc<F> acc;
            for (uint32_t i = 0; i < n; ++i) {
                const Coord<R> c = coord<R, TABLE>(a, tab, i);
                acc.add((double)xw[i] - (double)c.sh);
            }
            fresh = acc.finish(n);
            sh_part[0][0] = fresh.f;
            sh_part[0][1] = fresh.s1;
            sh_part[1][0] = fresh.s2;
        }
        __syncthreads();
        fresh = Full{sh_part[0][0], sh_part[0][1], sh_part[1][0]};
    } else {
        // FP32 runs: FP64 arithmetic, fixed parallel order.
        FullAcc<F> acc;
        for (uint32_t i = tid; i < n; i += WG) {
            const Coord<R> c = coord<R, TABLE>(a, tab, i);
            acc.add((double)xw[i] - (double)c.sh);
        }
        const double pa = wave_sum_d(acc.a), pb = wave_sum_d(acc.b);
        if (lane == 0) {
            sh_part[wave][0] = pa;
            sh_part[wave][1] = pb;
        }
        __syncthreads();
        FullAcc<F> tot;
        for (uint32_t w = 0; w < nwaves; ++w) {
            tot.a += sh_part[w][0];
            tot.b += sh_part[w][1];
        }
        fresh = tot.finish(n);
    }

    const bool improved = fresh.f < a.rec[0];
    if (improved) {
        for (uint32_t i = tid; i < n; i += WG) a.x_rec[i] = xw[i];
    }
    __syncthreads();
    if (tid == 0) {
        if (improved) {
            a.rec[0] = fresh.f;
            *a.rec_level = level;
        }
        a.start[0] = fresh.f;
        a.start[1] = fresh.s1;
        a.start[2] = fresh.s2;
        sa_level t;
        t.win_chain = gc;
        t.reserved = 0;
        t.f_win = (double)gf;
        t.f_best = fresh.f;
        t.f_rec = improved ? fresh.f : a.rec[0];
        t.accepts = gacc;
        t.t_ticks = wall_clock64();
        a.trace[level] = t;
        __hip_atomic_store(a.arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void reset_kernel(double *rec, uint32_t *rec_level, uint32_t *arrive)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        rec[0] = __builtin_inf();
        *rec_level = 0xFFFFFFFFu;
        *arrive = 0u;
    }
}

size_t level_lds_bytes(uint32_t n, uint32_t wg, size_t real_size, bool table)
{
    return ((size_t)n * wg + (table ? 4 * (size_t)n : 0)) * real_size;
}

template <typename R, int F, bool TABLE, bool LOG>
static hipError_t launch_one(const LevelArgs<R> &a, uint32_t level, hipStream_t s)
{
    const size_t lds = level_lds_bytes(a.n, a.wg, sizeof(R), TABLE);
    if (a.move == SA_MOVE_RADIUS)
        hipLaunchKernelGGL((level_kernel<R, F, TABLE, LOG, SA_MOVE_RADIUS>), dim3(a.chains / a.wg), dim3(a.wg), lds,
                           s, a, level);
    else
        hipLaunchKernelGGL((level_kernel<R, F, TABLE, LOG, SA_MOVE_RESAMPLE>), dim3(a.chains / a.wg), dim3(a.wg),
                           lds, s, a, level);
    return hipGetLastError();
}

template <typename R, int F>
static hipError_t dispatch_tl(bool table, bool log, const LevelArgs<R> &a, uint32_t level, hipStream_t s)
{
    if (table) return log ? launch_one<R, F, true, true>(a, level, s) : launch_one<R, F, true, false>(a, level, s);
    return log ? launch_one<R, F, false, true>(a, level, s) : launch_one<R, F, false, false>(a, level, s);
}

template <typename R>
static hipError_t dispatch(int func, bool table, bool log, const LevelArgs<R> &a, uint32_t level, hipStream_t s)
{
    switch (func) {
    case kSchwefel: return dispatch_tl<R, kSchwefel>(table, log, a, level, s);
    case kRastrigin: return dispatch_tl<R, kRastrigin>(table, log, a, level, s);
    case kAckley: return dispatch_tl<R, kAckley>(table, log, a, level, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_level_f32(int func, bool table, bool log, const LevelArgs<float> &a, uint32_t level,
                            hipStream_t s)
{
    return dispatch<float>(func, table, log, a, level, s);
}

hipError_t launch_level_f64(int func, bool table, bool log, const LevelArgs<double> &a, uint32_t level,
                            hipStream_t s)
{
    return dispatch<double>(func, table, log, a, level, s);
}

hipError_t launch_reset(double *rec, uint32_t *rec_level, uint32_t *arrive, hipStream_t s)
{
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, rec, rec_level, arrive);
    return hipGetLastError();
}

}  // namespace sa
