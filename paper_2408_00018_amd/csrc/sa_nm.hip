// Nelder-Mead polish of annealing results on the device (the paper's hybrid
// strategy: a local minimizer started where the annealing stopped, Sec. 4.2
// and its hybrid results table).  The paper names the method, not its
// details; the steps are the standard simplex method with the coefficients of
// Lagarias, Reeds, Wright and Wright (SIAM J. Optim. 9, 1998): reflection 1,
// expansion 2, contraction 1/2, shrink 1/2, every trial point projected onto
// the box (the problem is box-constrained and the method is not).
//
// One wave per start point, FP64 throughout.  The simplex (n + 1 vertices of
// n coordinates) lives in device memory, vertex-major; the centroid, the
// trial points and the cost terms live in LDS.  Every elementwise step (trial
// points, shrink, spread) is spread over the lanes by coordinate; the
// centroid sums each coordinate over the vertices in vertex order on its
// lane; a cost evaluation computes the per-coordinate terms on the lanes and
// adds them in coordinate order on lane 0 -- the operation order of a plain
// sequential evaluation, so a run follows the same steps as one on the host.
//
// Per iteration: b = lowest cost (ties: lowest vertex), w = highest cost
// among the others (ties: lowest vertex), s = highest cost among all but w;
// stop when f_w - f_b <= ftol and every vertex lies within xtol of x_b in
// every coordinate, or after maxiter iterations.  xm = mean of all vertices
// but w; xr = xm + (xm - x_w):
//   f_b <= fr < f_s          take xr (reflect)
//   fr < f_b                 xe = xm + 2 (xm - x_w); take xe if fe < fr, else xr (expand)
//   f_s <= fr < f_w          xc = xm + (xr - xm)/2; take xc if fc <= fr (outside contraction)
//   fr >= f_w                xc = xm - (xm - x_w)/2; take xc if fc < f_w (inside contraction)
//   otherwise (no take)      every vertex v but b becomes x_b + (v - x_b)/2 (shrink)
// A taken point replaces vertex w.  Start: vertex 0 = x0, vertex i = x0 +
// h_i e_i with h_i = x0_i / 20 (0.00025 where x0_i = 0), reflected to x0 -
// h_i e_i when x0 + h_i e_i leaves the box, then clamped.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sa_centres.hpp"
#include "sa_host.hpp"

namespace {

using sa::fail;

constexpr double kPi = 3.14159265358979323846;
constexpr double kE = 2.71828182845904523536;
constexpr uint32_t kLanes = 64;

struct NmArgs {
    uint32_t func, n, maxiter, log_steps, nterms;
    double ftol, xtol;
    const double *lower, *upper, *shift;  // n each (shift may be null)
    const double *x0;                     // starts x n
    double *V;                            // starts x (n + 1) x n simplices
    double *x_out, *f_out;                // starts x n, starts
    uint32_t *iters, *evals;              // starts
    uint8_t *steps;                       // starts x maxiter step codes, or null
};

__device__ __forceinline__ double y_of(const NmArgs &a, const double *x, uint32_t i)
{
    return a.shift ? x[i] - a.shift[i] : x[i];
}

// Cost of the point x (device memory or LDS, n doubles): the per-coordinate
// terms on the lanes into t0/t1 (LDS), their sum in coordinate order on lane
// 0.  Returns the cost on every lane.
template <int F>
__device__ double nm_eval(const NmArgs &a, const double *x, double *t0, double *t1, double *bcast)
{
    const uint32_t lane = threadIdx.x, n = a.n;
    if constexpr (sa::kCentreFamily<F>) {
        // centre families: term i (one per table centre) on lane i
        for (uint32_t i = lane; i < sa::kCentres<F>; i += kLanes) {
            double d = 0.0;
            for (uint32_t j = 0; j < n; ++j) {
                const double t = y_of(a, x, j) - sa::centre_a64<F>(i, j);
                d += t * t;
            }
            t0[i] = sa::centre_term64<F>(i, d);
        }
    }
    for (uint32_t i = lane; i < (sa::kCentreFamily<F> ? 0u : n); i += kLanes) {
        const double y = y_of(a, x, i);
        if constexpr (F == SA_SCHWEFEL) {
            t0[i] = y * sin(sqrt(fabs(y)));
        } else if constexpr (F == SA_RASTRIGIN) {
            t0[i] = y * y - 10.0 * cos(2.0 * kPi * y);
        } else if constexpr (F == SA_ACKLEY) {
            t0[i] = y * y;
            t1[i] = cos(2.0 * kPi * y);
        } else if constexpr (F == SA_GRIEWANK) {
            t0[i] = y * y / 4000.0;
            t1[i] = cos(y / sqrt((double)(i + 1)));
        } else if constexpr (F == SA_LEVY_MONTALVO) {
            // term i < n-1: (w_i - 1)^2 (1 + 10 sin^2(pi w_{i+1})); t1[i] = w_i
            const double wi = 1.0 + (y + 1.0) / 4.0;
            t1[i] = wi;
            if (i + 1 < n) {
                const double w1 = 1.0 + (y_of(a, x, i + 1) + 1.0) / 4.0;
                const double sn = sin(kPi * w1);
                t0[i] = (wi - 1.0) * (wi - 1.0) * (1.0 + 10.0 * sn * sn);
            }
        } else {  // Rosenbrock: term i < n-1
            if (i + 1 < n) {
                const double b = y_of(a, x, i + 1);
                t0[i] = 100.0 * (b - y * y) * (b - y * y) + (1.0 - y) * (1.0 - y);
            }
        }
    }
    __syncthreads();
    if (lane == 0) {
        double v;
        if constexpr (F == SA_SCHWEFEL) {
            double acc = 0.0;
            for (uint32_t i = 0; i < n; ++i) acc += t0[i];
            v = -acc / (double)n;
        } else if constexpr (F == SA_RASTRIGIN) {
            double acc = 0.0;
            for (uint32_t i = 0; i < n; ++i) acc += t0[i];
            v = 10.0 * (double)n + acc;
        } else if constexpr (F == SA_ACKLEY) {
            double s1 = 0.0, s2 = 0.0;
            for (uint32_t i = 0; i < n; ++i) {
                s1 += t0[i];
                s2 += t1[i];
            }
            const double dn = (double)n;
            v = -20.0 * exp(-0.2 * sqrt(s1 / dn)) - exp(s2 / dn) + 20.0 + kE;
        } else if constexpr (F == SA_GRIEWANK) {
            double sum = 0.0, prod = 1.0;
            for (uint32_t i = 0; i < n; ++i) {
                sum += t0[i];
                prod *= t1[i];
            }
            v = 1.0 + sum - prod;
        } else if constexpr (sa::kCentreFamily<F>) {
            double acc = 0.0;
            for (uint32_t i = 0; i < sa::kCentres<F>; ++i) acc += t0[i];
            v = -acc;
        } else if constexpr (F == SA_LEVY_MONTALVO) {
            const double sp = sin(kPi * t1[0]);
            double acc = 10.0 * sp * sp;
            for (uint32_t i = 0; i + 1 < n; ++i) acc += t0[i];
            acc += (t1[n - 1] - 1.0) * (t1[n - 1] - 1.0);
            v = kPi / (double)n * acc;
        } else {
            double acc = 0.0;
            for (uint32_t i = 0; i + 1 < n; ++i) acc += t0[i];
            v = acc;
        }
        *bcast = v;
    }
    __syncthreads();
    const double v = *bcast;
    __syncthreads();
    return v;
}

// out = xm + t (xm - xw), projected onto the box (lanes over coordinates).
__device__ __forceinline__ void nm_point(const NmArgs &a, const double *xm, const double *xw, double t, double *out)
{
    for (uint32_t j = threadIdx.x; j < a.n; j += kLanes) {
        double v = xm[j] + t * (xm[j] - xw[j]);
        if (v > a.upper[j]) v = a.upper[j];
        if (v < a.lower[j]) v = a.lower[j];
        out[j] = v;
    }
}

// Lowest index holding the extreme of F[i] over i != skip (MAX: largest,
// else smallest); ties go to the lowest index, as a sequential scan that
// replaces only on a strict improvement gives.
template <bool MAX>
__device__ uint32_t nm_select(const double *F, uint32_t m, uint32_t skip)
{
    double bv = MAX ? -INFINITY : INFINITY;
    uint32_t bi = 0xFFFFFFFFu;
    for (uint32_t i = threadIdx.x; i < m; i += kLanes) {
        if (i == skip) continue;
        const double v = F[i];
        const bool better = bi == 0xFFFFFFFFu || (MAX ? v > bv : v < bv);
        if (better) {
            bv = v;
            bi = i;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(bv, off, kLanes);
        const uint32_t oi = __shfl_xor(bi, off, kLanes);
        const bool take = oi != 0xFFFFFFFFu &&
                          (bi == 0xFFFFFFFFu || (MAX ? ov > bv : ov < bv) || (ov == bv && oi < bi));
        if (take) {
            bv = ov;
            bi = oi;
        }
    }
    return __shfl(bi, 0, kLanes);
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kLanes));
    return v;
}

template <int F>
__global__ void __launch_bounds__(64) nm_kernel(const NmArgs a)
{
    extern __shared__ __align__(16) double lds[];
    const uint32_t n = a.n, m = n + 1, lane = threadIdx.x, k = blockIdx.x;
    double *xm = lds;        // n
    double *xr = xm + n;     // n
    double *xt = xr + n;     // n
    double *t0 = xt + n;     // terms (nm_terms(n))
    double *t1 = t0 + a.nterms;
    double *fv = t1 + a.nterms;  // n + 1 vertex costs
    double *bc = fv + m;     // 1
    double *V = a.V + (size_t)k * m * n;
    const double *x0 = a.x0 + (size_t)k * n;

    uint32_t evals = 0;
    // start simplex
    for (uint32_t i = 0; i < m; ++i) {
        double *v = V + (size_t)i * n;
        for (uint32_t j = lane; j < n; j += kLanes) {
            double val = x0[j];
            if (i > 0 && j == i - 1) {
                const double h = x0[j] != 0.0 ? x0[j] / 20.0 : 0.00025;
                val = x0[j] + h;
                if (val > a.upper[j] || val < a.lower[j]) val = x0[j] - h;
                if (val > a.upper[j]) val = a.upper[j];
                if (val < a.lower[j]) val = a.lower[j];
            }
            v[j] = val;
        }
        __syncthreads();
        const double f = nm_eval<F>(a, v, t0, t1, bc);
        if (lane == 0) fv[i] = f;
        ++evals;
    }
    __syncthreads();

    uint32_t it = 0;
    for (; it < a.maxiter; ++it) {
        const uint32_t b = nm_select<false>(fv, m, 0xFFFFFFFFu);
        const uint32_t w = nm_select<true>(fv, m, b);
        const uint32_t s = nm_select<true>(fv, m, w);
        const double *xb = V + (size_t)b * n;
        const double *xw = V + (size_t)w * n;
        // convergence (the spread is needed only when the costs pass)
        if (fv[w] - fv[b] <= a.ftol) {
            double spread = 0.0;
            for (uint32_t i = 0; i < m; ++i) {
                const double *v = V + (size_t)i * n;
                for (uint32_t j = lane; j < n; j += kLanes) spread = fmax(spread, fabs(v[j] - xb[j]));
            }
            spread = wave_max(spread);
            if (spread <= a.xtol) break;
        }
        // centroid of every vertex but w, summed in vertex order per coordinate
        for (uint32_t j = lane; j < n; j += kLanes) {
            double acc = 0.0;
            for (uint32_t i = 0; i < m; ++i)
                if (i != w) acc += V[(size_t)i * n + j];
            xm[j] = acc / (double)n;
        }
        __syncthreads();
        nm_point(a, xm, xw, 1.0, xr);
        __syncthreads();
        const double fr = nm_eval<F>(a, xr, t0, t1, bc);
        ++evals;
        const double fb = fv[b], fs = fv[s], fw = fv[w];
        uint32_t code;
        const double *take = nullptr;
        double ftake = 0.0;
        if (fr < fb) {
            nm_point(a, xm, xw, 2.0, xt);
            __syncthreads();
            const double fe = nm_eval<F>(a, xt, t0, t1, bc);
            ++evals;
            code = 1;
            if (fe < fr) {
                take = xt;
                ftake = fe;
            } else {
                take = xr;
                ftake = fr;
            }
        } else if (fr < fs) {
            code = 0;
            take = xr;
            ftake = fr;
        } else if (fr < fw) {
            nm_point(a, xm, xw, 0.5, xt);
            __syncthreads();
            const double fc = nm_eval<F>(a, xt, t0, t1, bc);
            ++evals;
            code = 2;
            if (fc <= fr) {
                take = xt;
                ftake = fc;
            }
        } else {
            nm_point(a, xm, xw, -0.5, xt);
            __syncthreads();
            const double fc = nm_eval<F>(a, xt, t0, t1, bc);
            ++evals;
            code = 3;
            if (fc < fw) {
                take = xt;
                ftake = fc;
            }
        }
        if (take) {
            double *dst = V + (size_t)w * n;
            for (uint32_t j = lane; j < n; j += kLanes) dst[j] = take[j];
            if (lane == 0) fv[w] = ftake;
            __syncthreads();
        } else {
            code = 4;
            for (uint32_t i = 0; i < m; ++i) {
                if (i == b) continue;
                double *v = V + (size_t)i * n;
                for (uint32_t j = lane; j < n; j += kLanes) v[j] = xb[j] + 0.5 * (v[j] - xb[j]);
                __syncthreads();
                const double f = nm_eval<F>(a, v, t0, t1, bc);
                if (lane == 0) fv[i] = f;
                ++evals;
            }
            __syncthreads();
        }
        if (a.steps && lane == 0) a.steps[(size_t)k * a.log_steps + it] = (uint8_t)code;
    }
    const uint32_t b = nm_select<false>(fv, m, 0xFFFFFFFFu);
    const double *xb = V + (size_t)b * n;
    for (uint32_t j = lane; j < n; j += kLanes) a.x_out[(size_t)k * n + j] = xb[j];
    if (lane == 0) {
        a.f_out[k] = fv[b];
        a.iters[k] = it;
        a.evals[k] = evals;
    }
}

// Per-term scratch (t0, t1): one entry per coordinate, or per centre of the
// centre families (at most 30).
uint32_t nm_terms(uint32_t n) { return std::max<uint32_t>(n, 30u); }
size_t nm_lds_bytes(uint32_t n) { return (4 * (size_t)n + 2 * (size_t)nm_terms(n) + 2) * sizeof(double); }

struct NmLayout {
    size_t lower, upper, shift, x0, V, x_out, f_out, iters, evals, steps, total;
};

NmLayout nm_layout(uint32_t n, uint32_t starts, uint32_t log_steps, bool shift)
{
    NmLayout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = sa::align_up(off + (bytes ? bytes : 1));
        return at;
    };
    l.lower = take(n * sizeof(double));
    l.upper = take(n * sizeof(double));
    l.shift = take(shift ? n * sizeof(double) : 0);
    l.x0 = take((size_t)starts * n * sizeof(double));
    l.V = take((size_t)starts * (n + 1) * n * sizeof(double));
    l.x_out = take((size_t)starts * n * sizeof(double));
    l.f_out = take((size_t)starts * sizeof(double));
    l.iters = take((size_t)starts * sizeof(uint32_t));
    l.evals = take((size_t)starts * sizeof(uint32_t));
    l.steps = take((size_t)starts * log_steps);
    l.total = off;
    return l;
}

constexpr uint32_t kNmMaxN = 2048;

sa_status nm_validate(const sa_problem *prob, uint32_t starts, const sa_nm_config *cfg)
{
    if (!prob || !cfg) return fail(SA_ERR_INVALID, "null problem or config");
    if (sa_status st = sa::validate_problem(prob, 0); st != SA_OK) return st;
    if (prob->n > kNmMaxN) return fail(SA_ERR_UNSUPPORTED, "Nelder-Mead polish: n = %u exceeds %u", prob->n, kNmMaxN);
    if (starts == 0) return fail(SA_ERR_INVALID, "starts must be >= 1");
    if (!(cfg->ftol >= 0.0) || !(cfg->xtol >= 0.0)) return fail(SA_ERR_INVALID, "ftol and xtol must be >= 0");
    return SA_OK;
}

template <int F> hipError_t launch_f(const NmArgs &a, uint32_t starts, hipStream_t s)
{
    hipLaunchKernelGGL(nm_kernel<F>, dim3(starts), dim3(kLanes), nm_lds_bytes(a.n), s, a);
    return hipGetLastError();
}

hipError_t launch(const NmArgs &a, uint32_t starts, hipStream_t s)
{
    switch (a.func) {
    case SA_SCHWEFEL: return launch_f<SA_SCHWEFEL>(a, starts, s);
    case SA_RASTRIGIN: return launch_f<SA_RASTRIGIN>(a, starts, s);
    case SA_ACKLEY: return launch_f<SA_ACKLEY>(a, starts, s);
    case SA_GRIEWANK: return launch_f<SA_GRIEWANK>(a, starts, s);
    case SA_LEVY_MONTALVO: return launch_f<SA_LEVY_MONTALVO>(a, starts, s);
    case SA_ROSENBROCK: return launch_f<SA_ROSENBROCK>(a, starts, s);
    case SA_SHEKEL5: return launch_f<SA_SHEKEL5>(a, starts, s);
    case SA_SHEKEL7: return launch_f<SA_SHEKEL7>(a, starts, s);
    case SA_SHEKEL10: return launch_f<SA_SHEKEL10>(a, starts, s);
    case SA_FOXHOLES: return launch_f<SA_FOXHOLES>(a, starts, s);
    default: return launch_f<SA_LANGERMAN>(a, starts, s);
    }
}

}  // namespace

extern "C" {

sa_status sa_nm_workspace_bytes(const sa_problem *prob, uint32_t starts, const sa_nm_config *cfg, size_t *bytes)
{
    sa::g_last_error.clear();
    if (!bytes) return fail(SA_ERR_INVALID, "bytes must not be NULL");
    sa_status st = nm_validate(prob, starts, cfg);
    if (st != SA_OK) return st;
    *bytes = nm_layout(prob->n, starts, cfg->log_steps ? cfg->maxiter : 0, prob->shift != nullptr).total;
    return SA_OK;
}

sa_status sa_nm_polish(const sa_problem *prob, const double *x0, uint32_t starts, const sa_nm_config *cfg,
                       void *stream, void *workspace, size_t ws_bytes, double *x_out, double *f_out,
                       uint32_t *iters_out, uint32_t *evals_out, uint8_t *step_log)
{
    sa::g_last_error.clear();
    sa_status st = nm_validate(prob, starts, cfg);
    if (st != SA_OK) return st;
    if (!x0) return fail(SA_ERR_INVALID, "x0 must not be NULL");
    if (step_log && !cfg->log_steps) return fail(SA_ERR_INVALID, "step_log needs cfg->log_steps");
    const uint32_t n = prob->n;
    for (size_t i = 0; i < (size_t)starts * n; ++i) {
        const uint32_t j = (uint32_t)(i % n);
        if (!(x0[i] >= prob->lower[j] && x0[i] <= prob->upper[j]))
            return fail(SA_ERR_INVALID, "start %zu, coordinate %u lies outside the box", i / n, j);
    }
    const uint32_t log_steps = cfg->log_steps ? cfg->maxiter : 0;
    const NmLayout l = nm_layout(n, starts, log_steps, prob->shift != nullptr);
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    SA_FAULT_CHECK(sa::kFaultLaunch);
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    bool own = false;
    if (ws) {
        if (ws_bytes < l.total)
            return fail(SA_ERR_INVALID, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, l.total);
        if (reinterpret_cast<uintptr_t>(ws) % sa::kAlign)
            return fail(SA_ERR_INVALID, "workspace must be %zu-byte aligned", sa::kAlign);
    } else {
        SA_FAULT_CHECK(sa::kFaultAlloc);
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&ws), l.total);
        if (e != hipSuccess) return fail(SA_ERR_NOMEM, "hipMalloc(%zu): %s", l.total, hipGetErrorString(e));
        own = true;
    }
    auto done = [&](sa_status r) {
        if (own) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(ws);
        }
        return r;
    };
#define NM_HIP(call)                                                                                    \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) return done(fail(SA_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_))); \
    } while (0)
    NM_HIP(hipMemcpyAsync(ws + l.lower, prob->lower, n * sizeof(double), hipMemcpyHostToDevice, s));
    NM_HIP(hipMemcpyAsync(ws + l.upper, prob->upper, n * sizeof(double), hipMemcpyHostToDevice, s));
    if (prob->shift)
        NM_HIP(hipMemcpyAsync(ws + l.shift, prob->shift, n * sizeof(double), hipMemcpyHostToDevice, s));
    NM_HIP(hipMemcpyAsync(ws + l.x0, x0, (size_t)starts * n * sizeof(double), hipMemcpyHostToDevice, s));
    NmArgs a{};
    a.func = prob->func;
    a.n = n;
    a.nterms = nm_terms(n);
    a.maxiter = cfg->maxiter;
    a.log_steps = log_steps;
    a.ftol = cfg->ftol;
    a.xtol = cfg->xtol;
    a.lower = reinterpret_cast<const double *>(ws + l.lower);
    a.upper = reinterpret_cast<const double *>(ws + l.upper);
    a.shift = prob->shift ? reinterpret_cast<const double *>(ws + l.shift) : nullptr;
    a.x0 = reinterpret_cast<const double *>(ws + l.x0);
    a.V = reinterpret_cast<double *>(ws + l.V);
    a.x_out = reinterpret_cast<double *>(ws + l.x_out);
    a.f_out = reinterpret_cast<double *>(ws + l.f_out);
    a.iters = reinterpret_cast<uint32_t *>(ws + l.iters);
    a.evals = reinterpret_cast<uint32_t *>(ws + l.evals);
    a.steps = log_steps ? reinterpret_cast<uint8_t *>(ws + l.steps) : nullptr;
    hipError_t e = launch(a, starts, s);
    if (e != hipSuccess) return done(fail(SA_ERR_DEVICE, "Nelder-Mead launch: %s", hipGetErrorString(e)));
    NM_HIP(hipStreamSynchronize(s));
    if (x_out) NM_HIP(hipMemcpy(x_out, ws + l.x_out, (size_t)starts * n * sizeof(double), hipMemcpyDeviceToHost));
    if (f_out) NM_HIP(hipMemcpy(f_out, ws + l.f_out, (size_t)starts * sizeof(double), hipMemcpyDeviceToHost));
    if (iters_out) NM_HIP(hipMemcpy(iters_out, ws + l.iters, (size_t)starts * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (evals_out) NM_HIP(hipMemcpy(evals_out, ws + l.evals, (size_t)starts * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (step_log) NM_HIP(hipMemcpy(step_log, ws + l.steps, (size_t)starts * log_steps, hipMemcpyDeviceToHost));
#undef NM_HIP
    return done(SA_OK);
}

}  // extern "C"
