// Level kernel for the non-separable test functions of the paper's suite
// (Appendix: Test 8 Griewank, Test 10 Levy-Montalvo, Test 14 generalized
// Rosenbrock).  No cost term belongs to one coordinate alone, so every move
// evaluates f(x') in full, as the paper's kernel does for every function
// (Sec. 3.3, synchronous kernel: f at the neighbour each step).  The same
// kernel runs the separable families (Schwefel, Rastrigin, Ackley) with that
// full evaluation when a run asks for it instead of their increment.
//
// Layout and level structure as the separable level kernel: one chain per
// lane, a tile's states in LDS as x[d][lane] (coordinate-major), one launch
// per temperature level, the previous level's per-workgroup candidates
// reduced to the winner at the start (Sec. 2.2.2).  A move writes x'_d into
// the chain's column, evaluates the column in full (n LDS reads on the
// lane's own bank, the coordinate constants on the scalar unit), and
// restores x_d if the move is rejected.
//
// Forms (y = x - s):
//   Schwefel        -(1/n) sum y_i sin(sqrt|y_i|)
//   Rastrigin       sum y_i^2 + 20 sin^2(pi y_i)   (= 10 n + sum y_i^2 - 10 cos(2 pi y_i))
//   Ackley          -20 expm1(-0.2 sqrt(S1/n)) - e expm1(-2 D/n),
//                   S1 = sum y_i^2, D = sum sin^2(pi y_i)  (sum cos(2 pi y_i) = n - 2 D)
//   Griewank        1 + sum y_i^2 / 4000 - prod cos(y_i / sqrt(i))
//   Levy-Montalvo   (pi/n) [10 sin^2(pi w_1) + sum_{i<n} (w_i - 1)^2
//                   (1 + 10 sin^2(pi w_{i+1})) + (w_n - 1)^2],  w = 1 + (y + 1)/4
//   Rosenbrock      sum_{i<n} [100 (y_{i+1} - y_i^2)^2 + (1 - y_i)^2]
//   Shekel (m = 5, 7, 10), foxholes, Langerman: sums over table centres
//                   (sa_centres.hpp), Appendix Tests 18, 19, 11
// The printed Griewank puts the product inside the sum and the printed
// Rosenbrock squares (y_{i+1} - y_i); both are read as the named functions
// (the forms above), whose stated minima (0 at the origin, 0 at (1,...,1))
// they then have.
// FP64 runs evaluate the definitions term by term in coordinate order, as a
// plain sequential evaluation does (the separable families in their printed
// forms).  FP32 runs use the hardware transcendentals: cos(y/sqrt(i)) =
// cos_rev(y c_i) with c_i = 1/(2 pi sqrt(i)) from a per-coordinate table,
// sin^2(pi w) = sin_rev((w - 1)/2)^2, sin(sqrt|y|) = sin_rev(sqrt(|y|/(4 pi^2))),
// and the separable families in the cancellation-free forms above.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "sa_device.hpp"
#include "sa_internal.hpp"
#include "sa_step.hpp"
#include "sa_level_common.hpp"
#include "sa_centres.hpp"

namespace sa {

// ---------------------------------------------------------------------------
// FP64 full evaluation of a coupled function, definition order; y(i) returns
// shifted coordinate i.
// ---------------------------------------------------------------------------
template <int F> constexpr bool kSeparable = F == kSchwefel || F == kRastrigin || F == kAckley;

template <int F, typename YFn> __device__ double coupled_f64(uint32_t n, const YFn &y)
{
    if constexpr (kSeparable<F>) {
        FullAcc<F> acc;
        for (uint32_t i = 0; i < n; ++i) acc.add(y(i));
        return acc.finish(n).f;
    } else if constexpr (F == kGriewank) {
        double sum = 0.0, prod = 1.0;
        for (uint32_t i = 0; i < n; ++i) {
            const double v = y(i);
            sum += v * v / 4000.0;
            prod *= cos(v / sqrt((double)(i + 1)));
        }
        return 1.0 + sum - prod;
    } else if constexpr (F == kLevyMontalvo) {
        double w0 = 1.0 + (y(0) + 1.0) / 4.0;
        const double sp = sin(kPi * w0);
        double acc = 10.0 * sp * sp;
        for (uint32_t i = 0; i + 1 < n; ++i) {
            const double w1 = 1.0 + (y(i + 1) + 1.0) / 4.0;
            const double sn = sin(kPi * w1);
            acc += (w0 - 1.0) * (w0 - 1.0) * (1.0 + 10.0 * sn * sn);
            w0 = w1;
        }
        acc += (w0 - 1.0) * (w0 - 1.0);
        return kPi / (double)n * acc;
    } else if constexpr (kCentreFamily<F>) {
        double acc = 0.0;
        for (uint32_t i = 0; i < kCentres<F>; ++i) {
            double d = 0.0;
            for (uint32_t j = 0; j < n; ++j) {
                const double t = y(j) - centre_a64<F>(i, j);
                d += t * t;
            }
            acc += centre_term64<F>(i, d);
        }
        return -acc;
    } else {
        double acc = 0.0;
        for (uint32_t i = 0; i + 1 < n; ++i) {
            const double a = y(i), b = y(i + 1);
            acc += 100.0 * (b - a * a) * (b - a * a) + (1.0 - a) * (1.0 - a);
        }
        return acc;
    }
}

// FP32 term i of a centre family from its squared distance d: 1/(d + c_i) on
// the hardware reciprocal, or Langerman's c_i e^(-d/pi) cos(pi d) with
// cos(pi d) = cos_rev(d/2) taken on the argument reduced to [-1/2, 1/2]
// revolutions (exact: d/2 minus its nearest integer).
template <int F> __device__ __forceinline__ float centre_term32(uint32_t i, float d)
{
    if constexpr (F == kLangerman) {
        constexpr float kNegLog2eOverPi = (float)(-1.44269504088896340736 / 3.14159265358979323846);
        const float h = 0.5f * d;
        const float r = h - __builtin_rintf(h);
        return centre_c32<F>(i) * hw_exp2(d * kNegLog2eOverPi) * hw_cos_rev(r);
    } else {
        return __builtin_amdgcn_rcpf(d + centre_c32<F>(i));
    }
}

// FP64 term i of the sum-form families (Levy-Montalvo without its pi/n
// factor, Rosenbrock), for evaluations split over lanes.
template <int F, typename YFn> __device__ double coupled_term_f64(uint32_t n, uint32_t i, const YFn &y)
{
    if constexpr (F == kLevyMontalvo) {
        const double wi = 1.0 + (y(i) + 1.0) / 4.0;
        double t = 0.0;
        if (i == 0) {
            const double s0 = sin(kPi * wi);
            t += 10.0 * s0 * s0;
        }
        if (i + 1 < n) {
            const double sn = sin(kPi * (1.0 + (y(i + 1) + 1.0) / 4.0));
            t += (wi - 1.0) * (wi - 1.0) * (1.0 + 10.0 * sn * sn);
        } else {
            t += (wi - 1.0) * (wi - 1.0);
        }
        return t;
    } else {
        if (i + 1 >= n) return 0.0;
        const double a = y(i), b = y(i + 1);
        return 100.0 * (b - a * a) * (b - a * a) + (1.0 - a) * (1.0 - a);
    }
}

template <typename T> __device__ __forceinline__ T wave_prod(T v)
{
    over_lane_steps([&](auto k) {
        T a, b;
        lane_pair<decltype(k)::value>(v, a, b);
        v = a * b;
    });
    return v;
}

// FP32 evaluation of a centre family at one chain's column, J >= n columns:
// the coordinates in registers, then the centres in table order, fully
// unrolled so every table entry is an instruction constant (no scalar-load
// round trip per coefficient) and the centres' independent distance sums
// interleave; columns j >= n are computed and then dropped by a select, so
// d is the same as a sum over j < n.
template <int F, uint32_t J, typename ShFn>
__device__ __forceinline__ float centre_f32(const float *col, uint32_t st, uint32_t n, const ShFn &sh)
{
    float yv[J];
#pragma unroll
    for (uint32_t j = 0; j < J; ++j) yv[j] = j < n ? col[j * st] - sh(j) : 0.0f;
    float acc = 0.0f;
#pragma unroll
    for (uint32_t i = 0; i < kCentres<F>; ++i) {
        float d = 0.0f;
#pragma unroll
        for (uint32_t j = 0; j < J; ++j) {
            const float t = yv[j] - centre_a32<F>(i, j);
            const float dn = fmaf(t, t, d);
            d = j < n ? dn : d;
        }
        acc += centre_term32<F>(i, d);
    }
    return -acc;
}

// ---------------------------------------------------------------------------
// FP32 full evaluation of one chain's column (coordinate i at col[i * STRIDE],
// STRIDE = 0: the run-time `stride`).  sh(i) returns coordinate i's shift;
// gco: Griewank's c_i = 1/(2 pi sqrt(i+1)), FP32, wave-uniform loads;
// scale, rounded to FP32: Levy-Montalvo's pi/n, Schwefel's -1/n, Ackley's 1/n.
// ---------------------------------------------------------------------------
template <int F, uint32_t STRIDE, typename ShFn>
__device__ __forceinline__ float coupled_f32(const float *col, uint32_t stride, uint32_t n, const ShFn &sh,
                                             const float *__restrict__ gco, float scale)
{
    const uint32_t st = STRIDE ? STRIDE : stride;
    if constexpr (F == kSchwefel) {
        float acc = 0.0f;
#pragma unroll 4
        for (uint32_t i = 0; i < n; ++i) {
            const float y = col[i * st] - sh(i);
            acc = fmaf(y, hw_sin_rev(hw_sqrt(fabsf(y) * kInv4Pi2)), acc);
        }
        return acc * scale;
    } else if constexpr (F == kRastrigin) {
        float acc = 0.0f;
#pragma unroll 4
        for (uint32_t i = 0; i < n; ++i) {
            const float y = col[i * st] - sh(i);
            const float sp = hw_sin_rev(0.5f * y);
            acc = fmaf(y, y, fmaf(20.0f * sp, sp, acc));
        }
        return acc;
    } else if constexpr (F == kAckley) {
        float s1 = 0.0f, dd = 0.0f;
#pragma unroll 4
        for (uint32_t i = 0; i < n; ++i) {
            const float y = col[i * st] - sh(i);
            const float sp = hw_sin_rev(0.5f * y);
            s1 = fmaf(y, y, s1);
            dd = fmaf(sp, sp, dd);
        }
        const float ea = expm1_f32(-0.2f * hw_sqrt(s1 * scale));
        const float eb = expm1_f32(-2.0f * (dd * scale));
        return fmaf(-20.0f, ea, -(float)kE * eb);
    } else if constexpr (F == kGriewank) {
        float s = 0.0f, p = 1.0f;
#pragma unroll 4
        for (uint32_t i = 0; i < n; ++i) {
            const float y = col[i * st] - sh(i);
            s = fmaf(y, y, s);
            p *= hw_cos_rev(y * gco[i]);
        }
        return fmaf(s, 2.5e-4f, 1.0f) - p;
    } else if constexpr (F == kLevyMontalvo) {
        // v_i = w_i - 1 = (y_i + 1)/4; sin^2(pi w_i) = sin^2(pi v_i) = sin_rev(v_i/2)^2
        const float h0 = fmaf(col[0] - sh(0), 0.125f, 0.125f);  // v_0 / 2
        const float s0 = hw_sin_rev(h0);
        float acc = 10.0f * s0 * s0;
        float vp = 2.0f * h0;
#pragma unroll 4
        for (uint32_t i = 1; i < n; ++i) {
            const float h = fmaf(col[i * st] - sh(i), 0.125f, 0.125f);
            const float si = hw_sin_rev(h);
            acc = fmaf(vp * vp, fmaf(10.0f * si, si, 1.0f), acc);
            vp = 2.0f * h;
        }
        acc = fmaf(vp, vp, acc);
        return acc * scale;
    } else if constexpr (kCentreFamily<F>) {
        // compile-time column counts, chosen by n (wave-uniform)
        if constexpr (kShekelTable<F>) return centre_f32<F, 4>(col, st, n, sh);
        else if (n <= 2) return centre_f32<F, 2>(col, st, n, sh);
        else if (n <= 5) return centre_f32<F, 5>(col, st, n, sh);
        else return centre_f32<F, 10>(col, st, n, sh);
    } else {
        float acc = 0.0f;
        float a = col[0] - sh(0);
#pragma unroll 4
        for (uint32_t i = 1; i < n; ++i) {
            const float b = col[i * st] - sh(i);
            const float t = fmaf(-a, a, b);
            const float u = 1.0f - a;
            acc = fmaf(100.0f * t, t, acc);
            acc = fmaf(u, u, acc);
            a = b;
        }
        return acc;
    }
}

// ---------------------------------------------------------------------------
// Full FP64 evaluation of a state in LDS (x[i * stride]) by the workgroup:
// FP64 runs in definition order on one lane; FP32 runs split over the first
// wave (Griewank: a sum and a product; Ackley: its two sums; the others: a
// sum of per-coordinate terms).  Contains workgroup barriers.
// ---------------------------------------------------------------------------
template <typename R, int F, bool TABLE>
__device__ double coupled_full_wg(const LevelArgs<R> &a, const R *tab, const R *x, double *part, uint32_t stride = 1)
{
    const uint32_t tid = threadIdx.x, n = a.n;
    const auto y = [&](uint32_t i) { return (double)x[i * stride] - (double)coord<R, TABLE>(a, tab, i).sh; };
    if (sizeof(R) == sizeof(double)) {
        if (tid == 0) part[0] = coupled_f64<F>(n, y);
    } else if (tid < 64) {
        double v;
        if constexpr (kSeparable<F>) {
            FullAcc<F> acc;
            for (uint32_t i = tid; i < n; i += 64) acc.add(y(i));
            acc.a = wave_sum_d(acc.a);
            acc.b = wave_sum_d(acc.b);
            v = acc.finish(n).f;
        } else if constexpr (kCentreFamily<F>) {
            // lanes over the centres
            double s = 0.0;
            for (uint32_t i = tid; i < kCentres<F>; i += 64) {
                double d = 0.0;
                for (uint32_t j = 0; j < n; ++j) {
                    const double t = y(j) - centre_a64<F>(i, j);
                    d += t * t;
                }
                s += centre_term64<F>(i, d);
            }
            v = -wave_sum_d(s);
        } else if constexpr (F == kGriewank) {
            double s = 0.0, p = 1.0;
            for (uint32_t i = tid; i < n; i += 64) {
                const double yi = y(i);
                s += yi * yi / 4000.0;
                p *= cos(yi / sqrt((double)(i + 1)));
            }
            s = wave_sum_d(s);
            p = wave_prod(p);
            v = 1.0 + s - p;
        } else {
            double s = 0.0;
            for (uint32_t i = tid; i < n; i += 64) s += coupled_term_f64<F>(n, i, y);
            s = wave_sum_d(s);
            v = F == kLevyMontalvo ? kPi / (double)n * s : s;
        }
        if (tid == 0) part[0] = v;
    }
    __syncthreads();
    const double r = part[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// N Metropolis steps of one chain per lane (Sec. 2.1, Steps 2-4) with full
// re-evaluation.  The move stream is the plain one (three words per move,
// blocks (b, level, chain, tag) in order).  evalf() evaluates the lane's
// column in full.
// ---------------------------------------------------------------------------
template <typename R, int MOVE, typename CoordFn, typename EvalFn, typename LogFn>
__device__ __forceinline__ uint32_t run_full_steps(R *xs, uint32_t stride, uint32_t lane_off, R &f,
                                                   const CoordFn &coordf, const EvalFn &evalf, const LogFn &logf,
                                                   uint32_t n, uint32_t steps, uint32_t level, uint32_t chain,
                                                   uint32_t ctr3, uint32_t k0, uint32_t k1, double T, float nl2T)
{
    uint32_t accepted = 0;
    MoveGroup m{};
    for (uint32_t step = 0; step < steps; ++step) {
        if ((step & 3u) == 0) m = move_group(step >> 2, level, chain, ctr3, k0, k1);
        uint32_t wd, w1, w2;
        move_words(m, step & 3u, wd, w1, w2);
        const uint32_t d = pick(wd, n);
        const Coord<R> c = coordf(d);
        const uint32_t at = __umul24(d, stride) + lane_off;
        const R xd = xs[at];
        const R xn = neighbour_w<MOVE>(xd, c, w1);
        xs[at] = xn;
        const R fn = evalf();
        const R df = fn - f;
        bool take;
        if constexpr (sizeof(R) == sizeof(float))
            take = metropolis_k(df, (float)(w2 >> 8), nl2T);
        else
            take = metropolis_w(df, w2, T, nl2T);
        logf(step, d, take, xd, xn, df);
        xs[at] = take ? xn : xd;
        f = take ? fn : f;
        accepted += take ? 1u : 0u;
    }
    return accepted;
}

// ---------------------------------------------------------------------------
// The level kernel (plain or logged moves).  UNSHIFTED: uniform box, zero
// shift, a broadcast at every level (the shift subtraction is left out:
// x - 0 is x exactly).
// LDS: xs[n][WG] tile states | xw[n] level start | xb[n] workgroup best |
//      tab[n][4] per-coordinate box/shift (TABLE only) | gco[n] (FP32 Griewank)
// ---------------------------------------------------------------------------
template <typename R, int F, bool TABLE, int MODE, int MOVE, bool UNSHIFTED>
__global__ void __launch_bounds__(256)
    coupled_level_kernel(const LevelArgs<R> a, const uint32_t level, const uint32_t prev_groups)
{
    constexpr bool LOG = MODE == kModeLog;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Slot<R> wave_slot[4];
    __shared__ uint64_t wave_acc[4];
    __shared__ double sh_part[2];
    __shared__ double sh_start[3];

    const uint32_t WG = blockDim.x, tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nwaves = WG >> 6;
    const uint32_t G = gridDim.x, n = a.n;
    R *xs = reinterpret_cast<R *>(lds_raw);
    R *xw = xs + (size_t)n * WG;
    R *xb = xw + n;
    R *tab = xb + n;
    // FP32 Griewank: the n factors c_i staged in LDS after the table (read
    // from global memory in the step loop they cost a load round trip per
    // four coordinates)
    float *gco = reinterpret_cast<float *>(tab + (TABLE ? 4 * (size_t)n : 0));
    constexpr bool kStageGco = F == kGriewank && sizeof(R) == sizeof(float);

    const double T = a.T[level];
    const float nl2T = -kLog2e * a.inv_T[level];
    if (kStageGco) {
        for (uint32_t i = tid; i < n; i += WG) gco[i] = a.gcoef[i];
    }
    if (TABLE) {
        for (uint32_t i = tid; i < 4 * n; i += WG) tab[i] = a.table[i];
    }
    if (level == a.start_level) {
        for (uint32_t i = tid; i < n; i += WG) xw[i] = a.x_start[i];
        __syncthreads();
        const double v = coupled_full_wg<R, F, TABLE>(a, tab, xw, sh_part);
        if (tid == 0) sh_start[0] = v;
    } else if (level > 0) {
        adopt_winner<R>(a, level - 1, prev_groups, xw, sh_start, blockIdx.x == 0, wave_slot, wave_acc);
    }
    __syncthreads();

    const uint32_t k0 = a.seed_lo, k1 = a.seed_hi;
    const uint32_t ctr3 = kTagMove | (a.problem << 8);
    const bool log_level = LOG && level >= a.log_level && level - a.log_level < a.log_levels;
    const double start = sh_start[0];
    const uint32_t ex = a.exchange;
    const bool own = !UNSHIFTED && level > 0 && level != a.start_level && !(ex != 0 && level % ex == 0);
    const bool keep = !UNSHIFTED && ex != 1 && !(ex != 0 && (level + 1) % ex == 0);
    R wf = widen_inf<R>();
    uint32_t wc = 0xFFFFFFFFu;
    uint32_t accepted = 0;
    const R *best = xb;
    uint32_t best_stride = 1;

    const auto coordf = [&](uint32_t d) {
        Coord<R> c = coord<R, TABLE>(a, tab, d);
        if constexpr (UNSHIFTED) c.sh = R(0);
        return c;
    };
    const auto shf = [&](uint32_t i) -> float {
        if constexpr (UNSHIFTED) return 0.0f;
        else if constexpr (TABLE) return (float)tab[4 * i + 3];
        else return (float)a.sh;
    };

    for (uint32_t tile = blockIdx.x; tile < a.tiles; tile += G) {
        const uint32_t chain = tile * WG + tid;
        R f;
        if (level == 0) {
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
            }
            f = (R)coupled_f64<F>(n, [&](uint32_t i) {
                return (double)xs[i * WG + tid] - (double)coord<R, TABLE>(a, tab, i).sh;
            });
        } else if (own) {
            load_column(xs, WG, tid, a.chain_x + chain, a.chains, n);
            f = a.chain_cost[chain];
        } else {
            if (WG == 256)
                fill_tile_c<256>(xs, tid, xw, n);
            else
                fill_tile(xs, WG, tid, xw, n);
            f = (R)start;
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
        const auto evalf = [&]() -> R {
            if constexpr (sizeof(R) == sizeof(float)) {
                if (WG == 256) return coupled_f32<F, 256>(xs + tid, 256, n, shf, gco, a.cscale);
                return coupled_f32<F, 0>(xs + tid, WG, n, shf, gco, a.cscale);
            } else {
                return coupled_f64<F>(n, [&](uint32_t i) { return xs[i * WG + tid] - coordf(i).sh; });
            }
        };
        accepted += run_full_steps<R, MOVE>(xs, WG, tid, f, coordf, evalf, logf, n, a.steps, level, chain, ctr3, k0,
                                            k1, T, nl2T);
        if (LOG && log_level) a.log_final[(size_t)(level - a.log_level) * a.chains + chain] = (double)f;
        if (keep) {
            store_column(xs, WG, tid, a.chain_x + chain, a.chains, n);
            a.chain_cost[chain] = f;
        }

        // ---- tile argmin of (final cost, chain); keep the workgroup's best
        R bf = f;
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
        if (!last) __syncthreads();
    }

    const uint32_t wacc = wave_sum(accepted);
    if (lane == 0) wave_acc[wave] = wacc;
    const double fr = coupled_full_wg<R, F, TABLE>(a, tab, best, sh_part, best_stride);
    const size_t slot = (size_t)(level & 1u) * a.tiles + blockIdx.x;
    if (tid == 0) {
        uint32_t acc = 0;
        for (uint32_t w = 0; w < nwaves; ++w) acc += (uint32_t)wave_acc[w];
        a.slots[slot] = Slot<R>{wf, wc, acc, 0u, fr, 0.0, 0.0};
    }
    for (uint32_t i = tid; i < n; i += WG) a.slot_x[slot * n + i] = best[i * best_stride];
}

template <typename R, int F, bool TABLE, int MODE, int MOVE, bool UNSHIFTED = false>
static hipError_t launch_one(const LevelArgs<R> &a, uint32_t level, uint32_t prev_groups, uint32_t *groups,
                             hipStream_t s)
{
    auto kern = coupled_level_kernel<R, F, TABLE, MODE, MOVE, UNSHIFTED>;
    const size_t lds = level_lds_bytes(a.n, a.wg, sizeof(R), TABLE, false) +
                       (F == kGriewank && sizeof(R) == sizeof(float) ? (size_t)a.n * sizeof(float) : 0);
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
static hipError_t launch_mode(bool log, const LevelArgs<R> &a, uint32_t level, uint32_t prev, uint32_t *groups,
                              hipStream_t s)
{
    if (log) return launch_one<R, F, TABLE, kModeLog, MOVE>(a, level, prev, groups, s);
    if constexpr (!TABLE && sizeof(R) == sizeof(float)) {
        if (a.sh == R(0) && !std::signbit(a.sh) && a.exchange == 1)
            return launch_one<R, F, TABLE, kModePlain, MOVE, true>(a, level, prev, groups, s);
    }
    return launch_one<R, F, TABLE, kModePlain, MOVE>(a, level, prev, groups, s);
}

template <typename R, int F>
static hipError_t dispatch_f(bool table, bool log, const LevelArgs<R> &a, uint32_t level, uint32_t prev,
                             uint32_t *groups, hipStream_t s)
{
    if (a.move == SA_MOVE_RADIUS)
        return table ? launch_mode<R, F, true, SA_MOVE_RADIUS>(log, a, level, prev, groups, s)
                     : launch_mode<R, F, false, SA_MOVE_RADIUS>(log, a, level, prev, groups, s);
    return table ? launch_mode<R, F, true, SA_MOVE_RESAMPLE>(log, a, level, prev, groups, s)
                 : launch_mode<R, F, false, SA_MOVE_RESAMPLE>(log, a, level, prev, groups, s);
}

template <typename R>
static hipError_t dispatch(int func, bool table, bool log, const LevelArgs<R> &a, uint32_t level, uint32_t prev,
                           uint32_t *groups, hipStream_t s)
{
    switch (func) {
    case kSchwefel: return dispatch_f<R, kSchwefel>(table, log, a, level, prev, groups, s);
    case kRastrigin: return dispatch_f<R, kRastrigin>(table, log, a, level, prev, groups, s);
    case kAckley: return dispatch_f<R, kAckley>(table, log, a, level, prev, groups, s);
    case kGriewank: return dispatch_f<R, kGriewank>(table, log, a, level, prev, groups, s);
    case kLevyMontalvo: return dispatch_f<R, kLevyMontalvo>(table, log, a, level, prev, groups, s);
    case kRosenbrock: return dispatch_f<R, kRosenbrock>(table, log, a, level, prev, groups, s);
    case kShekel5: return dispatch_f<R, kShekel5>(table, log, a, level, prev, groups, s);
    case kShekel7: return dispatch_f<R, kShekel7>(table, log, a, level, prev, groups, s);
    case kShekel10: return dispatch_f<R, kShekel10>(table, log, a, level, prev, groups, s);
    case kFoxholes: return dispatch_f<R, kFoxholes>(table, log, a, level, prev, groups, s);
    case kLangerman: return dispatch_f<R, kLangerman>(table, log, a, level, prev, groups, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_coupled_level_f32(int func, bool table, bool log, const LevelArgs<float> &a, uint32_t level,
                                    uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    return dispatch<float>(func, table, log, a, level, prev_groups, groups, s);
}

hipError_t launch_coupled_level_f64(int func, bool table, bool log, const LevelArgs<double> &a, uint32_t level,
                                    uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    return dispatch<double>(func, table, log, a, level, prev_groups, groups, s);
}

}  // namespace sa
