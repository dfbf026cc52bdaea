// Per-move machinery shared by the single-problem and the batched kernels:
// per-chain cost state and increments, full evaluation, the neighbour, the
// Metropolis test, wave reductions, and the software-pipelined step loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "sa_device.hpp"
#include "sa_internal.hpp"
#include "sa_mlp_net.hpp"

namespace sa {

// ---------------------------------------------------------------------------
// Per-chain cost state.  delta() returns the increment of changing one
// coordinate from y to yn (shifted coordinates) and stages the new state;
// commit() installs it when the move is accepted.
// ---------------------------------------------------------------------------
template <typename R, int F> struct Cost;

// FP32 Metropolis test (eq. (5), k_b = 1) on k = (w >> 8) as a float, where
// U = k 2^-24 is the acceptance uniform: accept iff df <= 0 or
// k < 2^(24 - df log2(e) / T).
__device__ __forceinline__ bool metropolis_k(float df, float k, float neg_log2e_inv_T)
{
    return df <= 0.0f || k < hw_exp2(fmaf(df, neg_log2e_inv_T, 24.0f));
}

// FP64: the increments are the definitions, evaluated in the same order as a
// plain FP64 implementation would (the FP64 path is checked move for move).
template <> struct Cost<double, kSchwefel> {
    double f, fn;
    // Carried state between levels that start without a broadcast: word k of
    // a chain's record at p[k * stride].
    __device__ void save(double *p, uint32_t) const { p[0] = f; }
    __device__ void load(const double *p, uint32_t) { f = p[0]; }
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
    // Carried state between levels that start without a broadcast: word k of
    // a chain's record at p[k * stride].
    __device__ void save(double *p, uint32_t) const { p[0] = f; }
    __device__ void load(const double *p, uint32_t) { f = p[0]; }
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
    // Carried state between levels that start without a broadcast: word k of
    // a chain's record at p[k * stride].
    __device__ void save(double *p, uint32_t stride) const
    {
        p[0] = f;
        p[stride] = s1;
        p[2 * stride] = s2;
    }
    __device__ void load(const double *p, uint32_t stride)
    {
        f = p[0];
        s1 = p[stride];
        s2 = p[2 * stride];
    }
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
    // Carried state between levels that start without a broadcast: word k of
    // a chain's record at p[k * stride].
    __device__ void save(float *p, uint32_t) const { p[0] = f; }
    __device__ void load(const float *p, uint32_t) { f = p[0]; }
    __device__ void set(const Full &v, uint32_t) { f = (float)v.f; }
    __device__ float delta(float y, float yn, uint32_t, float inv_n)
    {
        df_ = (schwefel_h(y) - schwefel_h(yn)) * inv_n;
        return df_;
    }
    // Increment and acceptance of x_d: xd -> xn (shift sh, acceptance k), with
    // as few dependent operations after xn as the arithmetic allows: the sine's
    // argument in revolutions is sqrt|y / (4 pi^2)| with y / (4 pi^2) one
    // multiply-add from x, the difference of the terms one more, and 1/n
    // is folded into the exponent of the acceptance test.
    __device__ bool step(float xd, float xn, float sh, float k, float nl2T, float inv_n)
    {
        const float shs = -sh * kInv4Pi2;
        const float y = xd - sh, yn = xn - sh;
        const float so = hw_sin_rev(hw_sqrt(fabsf(fmaf(xd, kInv4Pi2, shs))));
        const float sn = hw_sin_rev(hw_sqrt(fabsf(fmaf(xn, kInv4Pi2, shs))));
        const float d = fmaf(-yn, sn, y * so);  // h(y) - h(y'), so df = d / n
        df_ = d * inv_n;
        return d <= 0.0f || k < hw_exp2(fmaf(d, nl2T * inv_n, 24.0f));
    }
    __device__ void commit(bool take, float) { f = take ? f + df_ : f; }
};

template <> struct Cost<float, kRastrigin> {
    float f, df_;
    // Carried state between levels that start without a broadcast: word k of
    // a chain's record at p[k * stride].
    __device__ void save(float *p, uint32_t) const { p[0] = f; }
    __device__ void load(const float *p, uint32_t) { f = p[0]; }
    __device__ void set(const Full &v, uint32_t) { f = (float)v.f; }
    __device__ float delta(float y, float yn, uint32_t, float)
    {
        const float dl = yn - y, sg = yn + y;
        df_ = fmaf(dl, sg, 20.0f * hw_sin_rev(0.5f * dl) * hw_sin_rev(0.5f * sg));
        return df_;
    }
    __device__ bool step(float xd, float xn, float sh, float k, float nl2T, float inv_n)
    {
        return metropolis_k(delta(xd - sh, xn - sh, 0u, inv_n), k, nl2T);
    }
    __device__ void commit(bool take, float) { f = take ? f + df_ : f; }
};

template <> struct Cost<float, kAckley> {
    float f, s1, s2, q, ea, eb;  // q = sqrt(S1/n), ea = exp(-0.2 q), eb = exp(S2/n)
    // Carried state between levels that start without a broadcast: word k of
    // a chain's record at p[k * stride].
    __device__ void save(float *p, uint32_t stride) const
    {
        p[0] = f;
        p[stride] = s1;
        p[2 * stride] = s2;
        p[3 * stride] = q;
        p[4 * stride] = ea;
        p[5 * stride] = eb;
    }
    __device__ void load(const float *p, uint32_t stride)
    {
        f = p[0];
        s1 = p[stride];
        s2 = p[2 * stride];
        q = p[3 * stride];
        ea = p[4 * stride];
        eb = p[5 * stride];
    }
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
        const float da = den > 0.0f ? (-0.2f * (ds1 * inv_n)) * __builtin_amdgcn_rcpf(den) : 0.0f;
        df_ = -20.0f * ea * expm1_f32(da) - eb * expm1_f32(ds2 * inv_n);
        return df_;
    }
    __device__ bool step(float xd, float xn, float sh, float k, float nl2T, float inv_n)
    {
        return metropolis_k(delta(xd - sh, xn - sh, 0u, inv_n), k, nl2T);
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

// FP32 radius neighbour straight from the generator word w (U = (w >> 8) 2^-24):
// 2U - 1 = (w >> 8) 2^-23 - 1 in one exact multiply-add, so the result is
// neighbour<SA_MOVE_RADIUS>(xd, c, U) bit for bit.
__device__ __forceinline__ float radius_neighbour_w(float xd, const Coord<float> &c, uint32_t w)
{
    const float t = fmaf((float)(w >> 8), 0x1p-23f, -1.0f);
    return __builtin_amdgcn_fmed3f(fmaf(c.rho, t, xd), c.lo, c.hi);
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
// Neighbour and FP64 acceptance straight from the move's generator words.
template <int MOVE> __device__ __forceinline__ float neighbour_w(float xd, const Coord<float> &c, uint32_t w)
{
    if constexpr (MOVE == SA_MOVE_RADIUS) return radius_neighbour_w(xd, c, w);
    return neighbour<MOVE>(xd, c, u24f(w));
}
template <int MOVE> __device__ __forceinline__ double neighbour_w(double xd, const Coord<double> &c, uint32_t w)
{
    return neighbour<MOVE>(xd, c, u24<double>(w));
}
__device__ __forceinline__ bool metropolis_w(double df, uint32_t w, double T, float)
{
    return metropolis(df, u24<double>(w), T, 0.0f);
}

// Lexicographic (cost, chain) minimum: ties go to the lower chain index.
template <typename R> __device__ __forceinline__ void best_of(R &f, uint32_t &c, R f2, uint32_t c2)
{
    if (f2 < f || (f2 == f && c2 < c)) {
        f = f2;
        c = c2;
    }
}

// ---------------------------------------------------------------------------
// Wave-wide reductions without the LDS crossbar.  Step k (k = 0..5) hands
// every lane two operands a, b whose combination covers the lane's group of
// 2^(k+1) lanes: steps 0-3 pair a lane with a partner in its 16-lane row
// through DPP (quad permutations, half-row and row mirrors), steps 4 and 5
// exchange whole rows and half-waves with gfx950's permlane16/permlane32
// swaps (both operands are then swapped copies; their combination is the
// same).  For a commutative, associative combination every lane ends with the
// wave's result.
// ---------------------------------------------------------------------------
template <int K> __device__ __forceinline__ void lane_pair(uint32_t v, uint32_t &a, uint32_t &b)
{
    if constexpr (K < 4) {
        constexpr int ctrl = K == 0 ? 0xB1 : K == 1 ? 0x4E : K == 2 ? 0x141 : 0x140;
        a = v;
        b = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, 0xF, 0xF, false);
    } else if constexpr (K == 4) {
        const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        a = p[0];
        b = p[1];
    } else {
        const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        a = p[0];
        b = p[1];
    }
}

template <int K> __device__ __forceinline__ void lane_pair(float v, float &a, float &b)
{
    uint32_t ua, ub;
    lane_pair<K>(__float_as_uint(v), ua, ub);
    a = __uint_as_float(ua);
    b = __uint_as_float(ub);
}

template <int K> __device__ __forceinline__ void lane_pair(uint64_t v, uint64_t &a, uint64_t &b)
{
    uint32_t alo, blo, ahi, bhi;
    lane_pair<K>((uint32_t)v, alo, blo);
    lane_pair<K>((uint32_t)(v >> 32), ahi, bhi);
    a = ((uint64_t)ahi << 32) | alo;
    b = ((uint64_t)bhi << 32) | blo;
}

template <int K> __device__ __forceinline__ void lane_pair(double v, double &a, double &b)
{
    uint64_t ua, ub;
    lane_pair<K>((uint64_t)__double_as_longlong(v), ua, ub);
    a = __longlong_as_double((long long)ua);
    b = __longlong_as_double((long long)ub);
}

// Calls f(integral_constant<int, K>) for K = 0..5.
template <typename Fn> __device__ __forceinline__ void over_lane_steps(Fn &&f)
{
    f(std::integral_constant<int, 0>{});
    f(std::integral_constant<int, 1>{});
    f(std::integral_constant<int, 2>{});
    f(std::integral_constant<int, 3>{});
    f(std::integral_constant<int, 4>{});
    f(std::integral_constant<int, 5>{});
}

// Lexicographic (cost, chain) minimum over the wave; every lane gets it.
template <typename R> __device__ __forceinline__ void wave_best(R &f, uint32_t &c)
{
    over_lane_steps([&](auto k) {
        constexpr int K = decltype(k)::value;
        R fa, fb;
        uint32_t ca, cb;
        lane_pair<K>(f, fa, fb);
        lane_pair<K>(c, ca, cb);
        best_of(fa, ca, fb, cb);
        f = fa;
        c = ca;
    });
}

// The same with a payload j that travels with the chosen (cost, chain).
template <typename R> __device__ __forceinline__ void wave_best(R &f, uint32_t &c, uint32_t &j)
{
    over_lane_steps([&](auto k) {
        constexpr int K = decltype(k)::value;
        R fa, fb;
        uint32_t ca, cb, ja, jb;
        lane_pair<K>(f, fa, fb);
        lane_pair<K>(c, ca, cb);
        lane_pair<K>(j, ja, jb);
        if (fb < fa || (fb == fa && cb < ca)) {
            fa = fb;
            ca = cb;
            ja = jb;
        }
        f = fa;
        c = ca;
        j = ja;
    });
}

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
    over_lane_steps([&](auto k) {
        T a, b;
        lane_pair<decltype(k)::value>(v, a, b);
        v = a + b;
    });
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v) { return wave_sum<double>(v); }

// History feature of the learned proposal: a scaled displacement h enters the
// network as sign(h) ln(1 + 2^24 |h|) / 16 (a signed log magnitude, so a step
// size proportional to recent accepted steps is a linear map of it).
__device__ __forceinline__ float hist_feature(float h)
{
    return copysignf(hw_log2(fmaf(0x1p24f, fabsf(h), 1.0f)) * (kLn2 / 16.0f), h);
}
__device__ __forceinline__ double hist_feature(double h) { return copysign(log(1.0 + 0x1p24 * fabs(h)) / 16.0, h); }

template <typename R> __device__ __forceinline__ R widen_inf();
template <> __device__ __forceinline__ float widen_inf<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double widen_inf<double>() { return __builtin_inf(); }

// ---------------------------------------------------------------------------
// Start every chain of a tile from the level's start state:
// xs[i * stride + col] = xw[i] for i < n.  The reads are issued sixteen (then
// four) at a time, so the loop waits for one LDS round trip per batch instead
// of one per coordinate.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void fill_tile(R *xs, uint32_t stride, uint32_t col, const R *xw, uint32_t n)
{
    uint32_t i = 0;
    for (; i + 16u <= n; i += 16u) {
        R v[16];
#pragma unroll
        for (uint32_t k = 0; k < 16u; ++k) v[k] = xw[i + k];
#pragma unroll
        for (uint32_t k = 0; k < 16u; ++k) xs[(i + k) * stride + col] = v[k];
    }
    for (; i + 4u <= n; i += 4u) {
        R v[4];
#pragma unroll
        for (uint32_t k = 0; k < 4u; ++k) v[k] = xw[i + k];
#pragma unroll
        for (uint32_t k = 0; k < 4u; ++k) xs[(i + k) * stride + col] = v[k];
    }
    for (; i < n; ++i) xs[i * stride + col] = xw[i];
}

// The same with the row stride a compile-time constant: every store of a
// batch is an immediate offset from one address (measured 0.8% faster per
// level than the run-time stride on 256-chain tiles; writing whole rows with
// 16-byte stores, which needs a barrier, was not faster).
template <uint32_t STRIDE, typename R>
__device__ __forceinline__ void fill_tile_c(R *xs, uint32_t col, const R *xw, uint32_t n)
{
    R *c = xs + col;
    uint32_t i = 0;
    for (; i + 16u <= n; i += 16u) {
        R v[16];
#pragma unroll
        for (uint32_t k = 0; k < 16u; ++k) v[k] = xw[i + k];
#pragma unroll
        for (uint32_t k = 0; k < 16u; ++k) c[(i + k) * STRIDE] = v[k];
    }
    for (; i + 4u <= n; i += 4u) {
        R v[4];
#pragma unroll
        for (uint32_t k = 0; k < 4u; ++k) v[k] = xw[i + k];
#pragma unroll
        for (uint32_t k = 0; k < 4u; ++k) c[(i + k) * STRIDE] = v[k];
    }
    for (; i < n; ++i) c[i * STRIDE] = xw[i];
}

// A chain's own state between levels without a broadcast: its column of a
// coordinate-major global array (row stride `gstride`) to and from its LDS
// column.  Loads are issued 16 at a time.
template <typename R>
__device__ __forceinline__ void load_column(R *xs, uint32_t stride, uint32_t col, const R *src, uint32_t gstride,
                                            uint32_t n)
{
    uint32_t i = 0;
    for (; i + 16u <= n; i += 16u) {
        R v[16];
#pragma unroll
        for (uint32_t k = 0; k < 16u; ++k) v[k] = src[(size_t)(i + k) * gstride];
#pragma unroll
        for (uint32_t k = 0; k < 16u; ++k) xs[(i + k) * stride + col] = v[k];
    }
    for (; i < n; ++i) xs[i * stride + col] = src[(size_t)i * gstride];
}
template <typename R>
__device__ __forceinline__ void store_column(const R *xs, uint32_t stride, uint32_t col, R *dst, uint32_t gstride,
                                             uint32_t n)
{
    for (uint32_t i = 0; i < n; ++i) dst[(size_t)i * gstride] = xs[i * stride + col];
}

// ---------------------------------------------------------------------------
// The plain move stream of one chain at one level.  The words of the Philox
// blocks (b, level, chain, tag), b = 0, 1, ..., are taken in order, three per
// move: coordinate, change, acceptance.  Four moves use three blocks, so
// moves 4g .. 4g+3 read blocks 3g, 3g+1, 3g+2:
//   move 4g    b0.w0  b0.w1  b0.w2
//   move 4g+1  b0.w3  b1.w0  b1.w1
//   move 4g+2  b1.w2  b1.w3  b2.w0
//   move 4g+3  b2.w1  b2.w2  b2.w3
// ---------------------------------------------------------------------------
struct MoveGroup {
    Ctr b0, b1, b2;
};

__device__ __forceinline__ MoveGroup move_group(uint32_t g, uint32_t level, uint32_t chain, uint32_t ctr3,
                                                uint32_t k0, uint32_t k1)
{
    const uint32_t b = 3u * g;
    return MoveGroup{philox4x32_10(Ctr{b, level, chain, ctr3}, k0, k1),
                     philox4x32_10(Ctr{b + 1u, level, chain, ctr3}, k0, k1),
                     philox4x32_10(Ctr{b + 2u, level, chain, ctr3}, k0, k1)};
}

// The three words of move j (0-3) of a group.
__device__ __forceinline__ void move_words(const MoveGroup &m, uint32_t j, uint32_t &wd, uint32_t &w1, uint32_t &w2)
{
    switch (j) {
    case 0: wd = m.b0.w0; w1 = m.b0.w1; w2 = m.b0.w2; break;
    case 1: wd = m.b0.w3; w1 = m.b1.w0; w2 = m.b1.w1; break;
    case 2: wd = m.b1.w2; w1 = m.b1.w3; w2 = m.b2.w0; break;
    default: wd = m.b2.w1; w1 = m.b2.w2; w2 = m.b2.w3; break;
    }
}

// ---------------------------------------------------------------------------
// N Metropolis steps of one chain per lane at temperature T (Sec. 2.1, Steps
// 2-4), state in LDS at xs[d * stride + lane_off].  Software-pipelined: at
// the top of move s the (old) value of move s+1's coordinate is read from
// LDS, and each generator block of the next group of four moves is computed
// as soon as the current group has consumed the block it replaces, so
// neither the LDS latency nor the generator's dependent rounds sit on a
// move's critical path.  If move s+1 picks the coordinate move s writes, the
// written value is forwarded.  coordf(d) returns coordinate d's
// {l, u, rho, s}; logf(step, d, take, x_old, x_new, df) is called for every
// move (a no-op unless logging).  Returns the number of accepted moves.
// ---------------------------------------------------------------------------
struct NoPost {
    template <typename R> __device__ __forceinline__ void operator()(uint32_t, bool, R) const {}
};

template <typename R, int F, int MOVE, typename CoordFn, typename LogFn, typename PostFn = NoPost>
__device__ __forceinline__ uint32_t run_steps(R *xs, uint32_t stride, uint32_t lane_off, Cost<R, F> &cost,
                                              const CoordFn &coordf, const LogFn &logf, uint32_t n, uint32_t steps,
                                              uint32_t level, uint32_t chain, uint32_t ctr3, uint32_t k0,
                                              uint32_t k1, double T, float nl2T, float inv_n,
                                              const PostFn &post = PostFn{})
{
    uint32_t accepted = 0;
    Ctr b0 = philox4x32_10(Ctr{0u, level, chain, ctr3}, k0, k1);
    Ctr b1 = philox4x32_10(Ctr{1u, level, chain, ctr3}, k0, k1);
    Ctr b2 = philox4x32_10(Ctr{2u, level, chain, ctr3}, k0, k1);
    uint32_t d = pick(b0.w0, n);
    uint32_t at = __umul24(d, stride) + lane_off;  // LDS index of the current move's coordinate
    R xd = xs[at];
    Coord<R> c = coordf(d);
    // One move on the change and acceptance words (w1, w2); dn is the next
    // move's coordinate, whose value and box/shift entry are read ahead.
    const auto move = [&](uint32_t step, uint32_t w1, uint32_t w2, uint32_t dn) {
        const uint32_t at_n = __umul24(dn, stride) + lane_off;
        const R xn_lds = xs[at_n];
        const Coord<R> c_n = coordf(dn);
        const R xn = neighbour_w<MOVE>(xd, c, w1);
        R df;
        bool take;
        if constexpr (sizeof(R) == sizeof(float)) {
            take = cost.step(xd, xn, c.sh, (float)(w2 >> 8), nl2T, inv_n);
            df = cost.df_;
        } else {
            df = cost.delta(xd - c.sh, xn - c.sh, n, inv_n);
            take = metropolis_w(df, w2, T, nl2T);
        }
        logf(step, d, take, xd, xn, df);
        const R xwr = take ? xn : xd;
        xs[at] = xwr;
        cost.commit(take, inv_n);
        post(step, take, cost.f);
        accepted += take ? 1u : 0u;
        // the next move's value, forwarded from this move when it picks the
        // same coordinate (same 32-bit LDS index); selecting after the
        // decision keeps the read-ahead value's first use at the end of the
        // move (measured: forming both candidates before the decision made
        // the level 6% slower)
        xd = at_n == at ? xwr : xn_lds;
        d = dn;
        at = at_n;
        c = c_n;
    };
    // One group of four moves per iteration; each block variable is
    // overwritten by its successor in the next group once its last word is
    // consumed, so the rotation needs no register copies.
    uint32_t step = 0, blk = 3;
    for (; step + 4 <= steps; step += 4, blk += 3) {
        move(step, b0.w1, b0.w2, pick(b0.w3, n));
        b0 = philox4x32_10(Ctr{blk, level, chain, ctr3}, k0, k1);
        move(step + 1, b1.w0, b1.w1, pick(b1.w2, n));
        move(step + 2, b1.w3, b2.w0, pick(b2.w1, n));
        b1 = philox4x32_10(Ctr{blk + 1u, level, chain, ctr3}, k0, k1);
        move(step + 3, b2.w2, b2.w3, pick(b0.w0, n));
        b2 = philox4x32_10(Ctr{blk + 2u, level, chain, ctr3}, k0, k1);
    }
    // The last one to three moves, on the blocks of their group (already drawn).
    if (step < steps) move(step, b0.w1, b0.w2, pick(b0.w3, n));
    if (step + 1 < steps) move(step + 1, b1.w0, b1.w1, pick(b1.w2, n));
    if (step + 2 < steps) move(step + 2, b1.w3, b2.w0, pick(b2.w1, n));
    return accepted;
}

// ---------------------------------------------------------------------------
// N steps of the learned-proposal mixture, FP32 (an extension of the method,
// not in the paper).  Per move, with the move's three words (wd, w1, w2) of
// the plain move stream and the learned block q (counter (step, level,
// chain, kTagLearn)):
//   d from wd; a plain move with probability eps (U(q1) < eps): the radius
//   neighbour from w1 and the Metropolis test on w2, as in run_steps;
//   otherwise the network gives (mu, s) at the features of x_d, the scaled
//   displacement is dl = mu + e^s t with t a standard draw of the network's
//   distribution -- Cauchy: t = tan(pi (U(q0) - 1/2)) by inversion; Gaussian:
//   t = sqrt(-2 ln(1 - U(q0))) cos(2 pi U(q2)) (Box-Muller) --,
//   x'_d = x_d + dl (u_d - l_d); a proposal outside [l_d, u_d] is rejected;
//   otherwise the network is evaluated again at x'_d (same history) and the
//   move is taken iff
//       U(w2) < exp(-df/T + ln q(x | x') - ln q(x' | x))
//   (Metropolis-Hastings.  For a fixed history each component, and so their
//   state-independent mixture, is reversible with respect to exp(-f/T); an
//   accepted move changes the history the next proposal sees, so the chain
//   is adaptive and the invariance holds only approximately.)
// h holds the history features of the chain's last four accepted scaled
// displacements (most recent first); every accepted move, plain or learned,
// pushes the feature of (x'_d - x_d)/(u_d - l_d): hist_feature of it for the
// Cauchy kind, the value itself for the Gaussian kind.
// All lanes of the wave run every step (the network runs on wave-wide MFMA).
// ---------------------------------------------------------------------------
template <int F, int KIND, typename CoordFn, typename LogFn>
__device__ __forceinline__ uint32_t run_learned_steps(float *xs, uint32_t stride, uint32_t lane_off,
                                                      Cost<float, F> &cost, const CoordFn &coordf, const LogFn &logf,
                                                      uint32_t n, uint32_t steps, uint32_t level, uint32_t chain,
                                                      uint32_t ctr_move, uint32_t ctr_learn, uint32_t k0, uint32_t k1,
                                                      float nl2T, float inv_n, float featT, float eps,
                                                      const unsigned char *net, float (&h)[4])
{
    uint32_t accepted = 0;
    MoveGroup m{};
    for (uint32_t step = 0; step < steps; ++step) {
        if ((step & 3u) == 0) m = move_group(step >> 2, level, chain, ctr_move, k0, k1);
        uint32_t wd, w1, w2;
        move_words(m, step & 3u, wd, w1, w2);
        const Ctr q = philox4x32_10(Ctr{step, level, chain, ctr_learn}, k0, k1);
        const uint32_t d = pick(wd, n);
        const Coord<float> c = coordf(d);
        const uint32_t at = __umul24(d, stride) + lane_off;
        const float xd = xs[at];
        const float w = c.hi - c.lo;
        const float inv_w = 1.0f / w;
        const bool plain = u24f(q.w1) < eps;

        float z[mlp::kInputs] = {(xd - c.lo) * inv_w, featT, h[0], h[1], h[2], h[3]};
        float mu, s;
        mlp::net_forward<KIND>(net, z, mu, s);
        float t;
        if constexpr (KIND == mlp::kNetGeluGauss) {
            // 1 - U(q0) lies in [2^-24, 1]: the logarithm is finite
            const float rad = __builtin_sqrtf(-2.0f * kLn2 * hw_log2(1.0f - u24f(q.w0)));
            t = rad * hw_cos_rev(u24f(q.w2));
        } else {
            // tan(pi a) = sin(2 pi a/2) / cos(2 pi a/2) on the revolution-based units
            const float half = 0.5f * (u24f(q.w0) - 0.5f);
            t = hw_sin_rev(half) / hw_cos_rev(half);
        }
        const float dl = fmaf(hw_exp2(kLog2e * s), t, mu);
        const float xl = fmaf(dl, w, xd);
        const bool inbox = xl >= c.lo && xl <= c.hi;
        z[0] = inbox ? (xl - c.lo) * inv_w : 0.5f;
        float mu2, s2;
        mlp::net_forward<KIND>(net, z, mu2, s2);
        // ln q(x | x') - ln q(x' | x); the forward standardised residual is t,
        // the reverse one -(dl + mu2) e^-s2
        const float e2 = (dl + mu2) * hw_exp2(-kLog2e * s2);
        float lq;
        if constexpr (KIND == mlp::kNetGeluGauss) lq = (s - s2) + 0.5f * (t * t - e2 * e2);
        else lq = (s - s2) + kLn2 * (hw_log2(fmaf(t, t, 1.0f)) - hw_log2(fmaf(e2, e2, 1.0f)));

        const float xp = neighbour<SA_MOVE_RADIUS>(xd, c, u24f(w1));
        const float xn = plain ? xp : xl;
        const bool valid = plain || inbox;
        const float df = cost.delta(xd - c.sh, (valid ? xn : xd) - c.sh, n, inv_n);
        const float u2 = u24f(w2);
        const bool take = plain ? metropolis(df, u2, 0.0, nl2T) : (inbox && u2 < hw_exp2(fmaf(df, nl2T, kLog2e * lq)));
        logf(step, d, take, xd, xn, df);
        xs[at] = take ? xn : xd;
        cost.commit(take, inv_n);
        if (take) {
            h[3] = h[2];
            h[2] = h[1];
            h[1] = h[0];
            const float hs = (xn - xd) * inv_w;
            h[0] = KIND == mlp::kNetGeluGauss ? hs : hist_feature(hs);
        }
        accepted += take ? 1u : 0u;
    }
    return accepted;
}

}  // namespace sa
