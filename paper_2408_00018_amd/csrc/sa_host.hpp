// Host-side helpers shared by the single-problem and the batched runtimes:
// error reporting, validation, FP32 inward rounding.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "../../include/sa.h"

namespace sa {

extern thread_local std::string g_last_error;

// LDS available to one workgroup on gfx950; workspace alignment.
constexpr size_t kLdsPerWorkgroup = 160 * 1024;
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

inline sa_status fail(sa_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

// Fault injection for tests of the error paths, from the environment
// variable SA_FAULT (read at every call):
//   "alloc"   every call that would allocate device memory fails with
//             SA_ERR_NOMEM once its arguments are validated, before it
//             touches the device;
//   "launch"  every call that would enqueue kernels fails with SA_ERR_DEVICE
//             before it enqueues anything, leaving the context as it was.
// Any other value, or none, injects nothing.
enum Fault { kFaultAlloc = 0, kFaultLaunch = 1 };

inline sa_status injected_fault(Fault f)
{
    const char *v = std::getenv("SA_FAULT");
    if (!v) return SA_OK;
    if (f == kFaultAlloc && std::strcmp(v, "alloc") == 0)
        return fail(SA_ERR_NOMEM, "device allocation refused (SA_FAULT=alloc)");
    if (f == kFaultLaunch && std::strcmp(v, "launch") == 0)
        return fail(SA_ERR_DEVICE, "kernel launch refused (SA_FAULT=launch)");
    return SA_OK;
}

#define SA_FAULT_CHECK(kind)                                            \
    do {                                                                \
        if (sa_status st_ = sa::injected_fault(kind); st_ != SA_OK) return st_; \
    } while (0)

#define SA_HIP(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) return sa::fail(SA_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Convert the kernels' constant-clock stamps (ticks of `khz` kHz) in the
// per-level records to nanoseconds, in place.
inline void stamps_to_ns(sa_level *rec, uint32_t count, int khz)
{
    for (uint32_t k = 0; k < count; ++k)
        rec[k].t_ns = khz > 0 ? (uint64_t)((unsigned __int128)rec[k].t_ns * 1000000u / (unsigned)khz) : 0;
}

// Families whose cost is a sum of per-coordinate terms (a move updates it
// incrementally); the others are re-evaluated in full at every move.
inline bool separable(uint32_t func) { return func <= SA_ACKLEY; }

// One problem: known function, n >= 1, finite box with lower < upper, finite shift.
inline sa_status validate_problem(const sa_problem *p, uint32_t index)
{
    if (!p) return fail(SA_ERR_INVALID, "problem %u is NULL", index);
    if (p->func > SA_LANGERMAN) return fail(SA_ERR_INVALID, "problem %u: unknown function id %u", index, p->func);
    if (p->n == 0) return fail(SA_ERR_INVALID, "problem %u: dimension n must be >= 1", index);
    if (p->func >= SA_SHEKEL5 && p->func <= SA_SHEKEL10 && p->n != 4)
        return fail(SA_ERR_INVALID, "problem %u: the Shekel functions take n = 4 (got %u)", index, p->n);
    if ((p->func == SA_FOXHOLES || p->func == SA_LANGERMAN) && p->n > 10)
        return fail(SA_ERR_INVALID, "problem %u: the foxholes and Langerman tables hold n <= 10 (got %u)", index,
                    p->n);
    if (!p->lower || !p->upper) return fail(SA_ERR_INVALID, "problem %u: lower/upper must not be NULL", index);
    for (uint32_t i = 0; i < p->n; ++i) {
        if (!std::isfinite(p->lower[i]) || !std::isfinite(p->upper[i]))
            return fail(SA_ERR_INVALID, "problem %u: box bound %u is not finite", index, i);
        if (!(p->lower[i] < p->upper[i]))
            return fail(SA_ERR_INVALID, "problem %u: box %u has lower >= upper", index, i);
        if (p->shift && !std::isfinite(p->shift[i]))
            return fail(SA_ERR_INVALID, "problem %u: shift %u is not finite", index, i);
    }
    return SA_OK;
}

inline sa_status validate_schedule(uint32_t levels, uint32_t steps, uint32_t precision, uint32_t move, double T0,
                                   double alpha, double radius_frac)
{
    if (levels == 0) return fail(SA_ERR_INVALID, "levels must be >= 1");
    if (steps == 0) return fail(SA_ERR_INVALID, "steps must be >= 1");
    if (precision > SA_FP64) return fail(SA_ERR_INVALID, "unknown precision %u", precision);
    if (move > SA_MOVE_RESAMPLE) return fail(SA_ERR_INVALID, "unknown move rule %u", move);
    if (!(T0 > 0.0) || !std::isfinite(T0)) return fail(SA_ERR_INVALID, "T0 must be finite and > 0");
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(SA_ERR_INVALID, "alpha must be in (0, 1]");
    if (!(radius_frac > 0.0) || !std::isfinite(radius_frac))
        return fail(SA_ERR_INVALID, "radius_frac must be finite and > 0");
    return SA_OK;
}

// Round a box inward to FP32 so every FP32 state lies in the FP64 box.
inline float round_up_f(double v)
{
    float f = (float)v;
    if ((double)f < v) f = std::nextafter(f, INFINITY);
    return f;
}
inline float round_down_f(double v)
{
    float f = (float)v;
    if ((double)f > v) f = std::nextafter(f, -INFINITY);
    return f;
}

// Box/shift values {l, u, rho, s} of one coordinate in the run's precision:
// FP32 runs round the box inward; rho = radius_frac (u - l) for the radius
// rule, u - l for resampling.
inline void coord_values(double lo, double hi, double sh, bool fp64, uint32_t move, double radius_frac, double out[4])
{
    if (fp64) {
        out[0] = lo;
        out[1] = hi;
        out[2] = move == SA_MOVE_RADIUS ? radius_frac * (hi - lo) : hi - lo;
        out[3] = sh;
    } else {
        const float l32 = round_up_f(lo), u32 = round_down_f(hi);
        const double w = (double)u32 - (double)l32;
        out[0] = l32;
        out[1] = u32;
        out[2] = (float)(move == SA_MOVE_RADIUS ? radius_frac * w : w);
        out[3] = (float)sh;
    }
}

}  // namespace sa
