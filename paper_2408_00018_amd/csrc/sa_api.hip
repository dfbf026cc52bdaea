// Host runtime and C ABI (include/sa.h) of the gfx950 annealing library.
//
// The host validates the problem, lays out one device workspace, builds the
// temperature table (T_{k+1} = alpha T_k, Sec. 2.1 Step 5) and enqueues one
// level kernel per temperature level, plus one finalising kernel per sa_run,
// on the caller's stream -- eagerly, or from a captured HIP graph.  No host
// work happens between levels: each level's launch reduces the previous
// level's candidates to the winner on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "sa_host.hpp"
#include "sa_internal.hpp"
#include "sa_mlp_net.hpp"

namespace sa {
thread_local std::string g_last_error;
}  // namespace sa

namespace {

using sa::align_up;
using sa::fail;
using sa::kAlign;
using sa::kLdsPerWorkgroup;

// Exchange variant of a config (sa::kVarSos / sa::kVarBest bits).
int variant_of(const sa_config *c)
{
    return ((c->flags & SA_FLAG_SOS) ? sa::kVarSos : 0) | ((c->flags & SA_FLAG_BEST_SEEN) ? sa::kVarBest : 0);
}

// Whether every move evaluates f in full (the non-separable families always;
// the separable ones under SA_FLAG_FULL_EVAL) rather than by its increment.
bool full_eval(const sa_problem *p, const sa_config *c)
{
    return !sa::separable(p->func) || (c->flags & SA_FLAG_FULL_EVAL);
}

// Dynamic LDS of a dense level launch (learned: the packed network too;
// best-seen: its accept bits and replay lists).
size_t dense_lds_bytes(uint32_t n, uint32_t wg, size_t real_size, bool table, bool learn, int var, uint32_t steps)
{
    return var ? sa::variant_lds_bytes(n, wg, real_size, table, (var & sa::kVarBest) != 0, steps)
               : sa::level_lds_bytes(n, wg, real_size, table, learn);
}

// Largest workgroup (4, 2 or 1 waves) that divides `chains` and whose state
// (and, for learned runs, the packed network) fits in LDS.  0 if none fits.
uint32_t pick_wg(uint32_t n, uint32_t chains, size_t real_size, bool table, bool learn, int var, uint32_t steps,
                 size_t lds_limit)
{
    for (uint32_t wg = 256; wg >= 64; wg >>= 1) {
        if (chains % wg) continue;
        if (dense_lds_bytes(n, wg, real_size, table, learn, var, steps) <= lds_limit) return wg;
    }
    return 0;
}

// Overlay layout: the largest workgroup (4, 2 or 1 waves) dividing `chains`
// whose tables hold at least 1.25 N + 1 slots per chain (probe lengths stay
// short), with up to 2N slots.  Coordinates are 16-bit keys.
bool pick_overlay(uint32_t n, uint32_t chains, uint32_t steps, size_t real_size, bool table, size_t lds_limit,
                  uint32_t *wg_out, uint32_t *slots_out)
{
    if (n >= 0xFFFFu) return false;
    const uint32_t want = std::max<uint32_t>(32u, (2 * steps + 7) / 8 * 8);
    const uint32_t need = (steps + steps / 4 + 8) / 8 * 8;
    for (uint32_t wg = 256; wg >= 64; wg >>= 1) {
        if (chains % wg) continue;
        const size_t fixed = sa::overlay_lds_bytes(n, wg, 0, real_size, table);
        if (fixed >= lds_limit) continue;
        size_t slots = (lds_limit - fixed) / ((size_t)wg * (real_size + 2)) / 8 * 8;
        slots = std::min<size_t>(slots, want);
        if (slots >= need && slots > steps) {
            *wg_out = wg;
            *slots_out = (uint32_t)slots;
            return true;
        }
    }
    return false;
}

constexpr uint32_t kNoStart = 0xFFFFFFFFu;

struct Layout {
    size_t table, T, inv_T, featT, x_best, slots, slot_x, x_rec, rec, rec_level, elite_x, elite_f, trace, trace_x, log,
        log_final;
    size_t x_start, theta, net, cap_count, chain_x, chain_cost, gcoef, total;
};

struct Plan {
    bool table = false;
    bool overlay = false;
    uint32_t ov_slots = 0;
    uint32_t wg = 0, groups = 0;
    size_t real = 0;
    Layout lay{};
};

sa_status validate(const sa_problem *p, const sa_config *c)
{
    if (!p || !c) return fail(SA_ERR_INVALID, "null problem or config");
    if (sa_status st = sa::validate_problem(p, 0); st != SA_OK) return st;
    if (c->chains == 0 || c->chains % 64) return fail(SA_ERR_INVALID, "chains must be a positive multiple of 64");
    if (sa_status st = sa::validate_schedule(c->levels, c->steps, c->precision, c->move, c->T0, c->alpha,
                                             c->radius_frac);
        st != SA_OK)
        return st;
    if (c->flags & ~(SA_FLAG_TRACE_X | SA_FLAG_GRAPH | SA_FLAG_LEARNED | SA_FLAG_OVERLAY | SA_FLAG_SOS |
                     SA_FLAG_BEST_SEEN | SA_FLAG_ELITIST | SA_FLAG_FULL_EVAL))
        return fail(SA_ERR_INVALID, "unknown flag bits");
    if ((c->flags & SA_FLAG_ELITIST) && (c->flags & SA_FLAG_SOS))
        return fail(SA_ERR_UNSUPPORTED, "the stochastic exchange compares chains with the winner; not with SA_FLAG_ELITIST");
    const bool full = full_eval(p, c);
    if ((c->flags & (SA_FLAG_SOS | SA_FLAG_BEST_SEEN)) && ((c->flags & (SA_FLAG_LEARNED | SA_FLAG_OVERLAY)) || full))
        return fail(SA_ERR_UNSUPPORTED,
                    "the exchange variants run plain or logged moves of the separable families on the dense layout");
    if ((c->flags & SA_FLAG_LEARNED) && (c->flags & SA_FLAG_OVERLAY))
        return fail(SA_ERR_UNSUPPORTED, "the learned proposal runs on the dense state layout");
    if (c->exchange > 1 && (c->flags & SA_FLAG_LEARNED))
        return fail(SA_ERR_UNSUPPORTED, "an exchange period other than 1 runs plain or logged moves only");
    if (c->exchange > 1 && (c->flags & SA_FLAG_OVERLAY))
        return fail(SA_ERR_UNSUPPORTED, "an exchange period other than 1 needs the dense state layout");
    if ((c->flags & SA_FLAG_LEARNED) && (c->precision != SA_FP32 || c->move != SA_MOVE_RADIUS))
        return fail(SA_ERR_UNSUPPORTED, "the learned proposal runs in FP32 with the radius move as its plain part");
    if (full && (c->flags & (SA_FLAG_LEARNED | SA_FLAG_OVERLAY)))
        return fail(SA_ERR_UNSUPPORTED,
                    "full evaluation per move (the non-separable families, SA_FLAG_FULL_EVAL) runs plain or logged "
                    "moves on the dense layout");
    if (c->log_chains) {
        if (c->log_chains > c->chains) return fail(SA_ERR_INVALID, "log_chains exceeds chains");
        if (c->log_levels == 0 || c->log_level >= c->levels || c->log_levels > c->levels - c->log_level)
            return fail(SA_ERR_INVALID, "logged level range outside [0, levels)");
    }
    return SA_OK;
}

bool uniform_box(const sa_problem *p)
{
    for (uint32_t i = 1; i < p->n; ++i) {
        if (p->lower[i] != p->lower[0] || p->upper[i] != p->upper[0]) return false;
        if (p->shift && p->shift[i] != p->shift[0]) return false;
    }
    return true;
}

sa_status plan(const sa_problem *p, const sa_config *c, size_t lds_limit, Plan *out)
{
    Plan pl;
    pl.table = !uniform_box(p);
    pl.real = c->precision == SA_FP64 ? sizeof(double) : sizeof(float);
    const bool learn = (c->flags & SA_FLAG_LEARNED) != 0;
    const int var = variant_of(c);
    // FP32 Griewank runs also stage their n cosine factors in LDS
    const size_t coef_lds = p->func == SA_GRIEWANK && c->precision == SA_FP32 ? p->n * sizeof(float) : 0;
    pl.wg = pick_wg(p->n, c->chains, pl.real, pl.table, learn, var, c->steps,
                    coef_lds < lds_limit ? lds_limit - coef_lds : 0);
    // Waves a layout keeps in flight on the device: its workgroups per CU (LDS
    // and the 32-wave limit) times the CUs, capped by its tiles.  The plan
    // counts the 256 CUs of the target device rather than querying it, so the
    // workspace size does not depend on which device answers.
    constexpr uint64_t kPlanCus = 256;
    const auto in_flight = [&](uint32_t wg, size_t lds) -> uint64_t {
        if (wg == 0 || lds == 0 || lds > lds_limit) return 0;
        const uint64_t per_cu = std::min<uint64_t>(lds_limit / lds, 2048u / wg);
        return std::min<uint64_t>(c->chains / wg, per_cu * kPlanCus) * (wg / 64);
    };
    const uint64_t dense_flight =
        pl.wg ? in_flight(pl.wg, dense_lds_bytes(p->n, pl.wg, pl.real, pl.table, learn, var, c->steps)) : 0;
    // Chains that keep their own state between levels need the dense layout.
    const bool periodic = c->exchange > 1 || (var & sa::kVarSos);
    // A shared level-start state plus per-chain tables of the changed
    // coordinates where the dense state does not fit or where the tables keep
    // at least twice as many waves in flight (their lookups cost a few
    // operations per move; measured at n = 512: 1.7x faster than the dense
    // layout with 131072 chains, 2.8x slower with 16384, where both put 256
    // waves in flight).
    if (!learn && !periodic && !var && !full_eval(p, c)) {
        uint32_t ov_wg = 0, ov_slots = 0;
        const bool ov_fits = pick_overlay(p->n, c->chains, c->steps, pl.real, pl.table, lds_limit, &ov_wg, &ov_slots);
        const uint64_t ov_flight =
            ov_fits ? in_flight(ov_wg, sa::overlay_lds_bytes(p->n, ov_wg, ov_slots, pl.real, pl.table)) : 0;
        if ((c->flags & SA_FLAG_OVERLAY) || dense_flight == 0 || ov_flight >= 2 * dense_flight) {
            if (!ov_fits)
                return fail(SA_ERR_UNSUPPORTED, "n=%u with %u steps fits neither state layout in LDS", p->n, c->steps);
            pl.wg = ov_wg;
            pl.ov_slots = ov_slots;
            pl.overlay = true;
        }
    }
    if (pl.wg == 0)
        return fail(SA_ERR_UNSUPPORTED, "state of n=%u does not fit in LDS for a 64-lane workgroup", p->n);
    pl.groups = c->chains / pl.wg;
    const size_t n = p->n, L = c->levels, R = pl.real;
    Layout &l = pl.lay;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + (bytes ? bytes : 1));
        return at;
    };
    l.table = take(pl.table ? 4 * n * R : 0);
    l.T = take(L * sizeof(double));
    l.inv_T = take(L * sizeof(float));
    l.featT = take(L * sizeof(float));
    l.x_best = take(n * R);
    // candidates are double-buffered by level parity; at most one per tile
    l.slots = take(2 * (size_t)pl.groups * sizeof(sa::Slot<double>));
    l.slot_x = take(2 * (size_t)pl.groups * n * R);
    l.x_rec = take(n * R);
    l.rec = take(2 * sizeof(double));
    l.rec_level = take(sizeof(uint32_t));
    l.elite_x = take((c->flags & SA_FLAG_ELITIST) ? 2 * n * R : 0);
    l.elite_f = take(6 * sizeof(double));
    l.trace = take(L * sizeof(sa_level));
    l.trace_x = take((c->flags & SA_FLAG_TRACE_X) ? L * n * R : 0);
    const size_t log_moves = c->log_chains ? (size_t)c->log_levels * c->log_chains * c->steps : 0;
    l.log = take(log_moves * sizeof(sa_move_rec));
    l.log_final = take(c->log_chains ? (size_t)c->log_levels * c->chains * sizeof(double) : 0);
    l.x_start = take(n * R);
    l.theta = take(learn ? sa::mlp::kNumParams * sizeof(float) : 0);
    l.net = take(learn ? sa::mlp::kNetBytes : 0);
    l.cap_count = take(sizeof(unsigned long long));
    l.chain_x = take(periodic ? (size_t)c->chains * n * R : 0);
    l.chain_cost = take(periodic ? (size_t)sa::kCostWords * c->chains * R : 0);
    l.gcoef = take(p->func == SA_GRIEWANK ? n * sizeof(float) : 0);
    l.total = off;
    *out = pl;
    return SA_OK;
}

}  // namespace

struct sa_ctx {
    int device = 0;
    int clock_khz = 0;  // rate of the device's constant clock
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    sa_problem prob{};
    sa_config cfg{};
    std::vector<double> lower, upper, shift;
    Plan pl;
    unsigned char *ws = nullptr;
    bool own_ws = false;
    uint32_t next_level = 0;
    uint64_t seed = 0;
    uint32_t groups = 0;  // candidates published by the last level enqueued
    uint32_t first_level = 0;  // first level of the current run (the start level, or 0)
    bool fp64 = false;
    bool learned = false;  // a proposal network is set
    int net_kind = SA_NET_RELU_CAUCHY;  // kind of the proposal network (and of captured features)
    bool capturing = false;  // accepted moves are being recorded
    sa::LevelArgs<float> a32{};
    sa::LevelArgs<double> a64{};
    struct Graph {
        hipGraph_t g = nullptr;
        hipGraphExec_t exec = nullptr;
        uint32_t groups = 0;  // candidates the captured run's last level publishes
    };
    std::map<std::tuple<uint32_t, uint32_t, uint32_t>, Graph> graphs;
};

namespace {

template <typename R> void fill_args(sa_ctx *c, sa::LevelArgs<R> &a)
{
    const Layout &l = c->pl.lay;
    unsigned char *w = c->ws;
    a.n = c->prob.n;
    a.chains = c->cfg.chains;
    a.steps = c->cfg.steps;
    a.move = c->cfg.move;
    a.problem = 0;
    a.seed_lo = (uint32_t)c->seed;
    a.seed_hi = (uint32_t)(c->seed >> 32);
    a.wg = c->pl.wg;
    a.tiles = c->pl.groups;
    a.ov_slots = c->pl.overlay ? c->pl.ov_slots : 0;
    a.table = c->pl.table ? reinterpret_cast<const R *>(w + l.table) : nullptr;
    a.inv_n = (float)(1.0 / (double)c->prob.n);
    a.T = reinterpret_cast<const double *>(w + l.T);
    a.inv_T = reinterpret_cast<const float *>(w + l.inv_T);
    a.x_best = reinterpret_cast<R *>(w + l.x_best);
    a.slots = reinterpret_cast<sa::Slot<R> *>(w + l.slots);
    a.slot_x = reinterpret_cast<R *>(w + l.slot_x);
    a.x_rec = reinterpret_cast<R *>(w + l.x_rec);
    a.rec = reinterpret_cast<double *>(w + l.rec);
    a.rec_level = reinterpret_cast<uint32_t *>(w + l.rec_level);
    a.elitist = (c->cfg.flags & SA_FLAG_ELITIST) ? 1u : 0u;
    a.elite_x = a.elitist ? reinterpret_cast<R *>(w + l.elite_x) : nullptr;
    a.elite_f = reinterpret_cast<double *>(w + l.elite_f);
    a.exchange = c->cfg.exchange <= 1 ? 1u : c->cfg.exchange == SA_EXCHANGE_NEVER ? 0u : c->cfg.exchange;
    const bool own_state = a.exchange != 1 || (c->cfg.flags & SA_FLAG_SOS);
    a.chain_x = own_state ? reinterpret_cast<R *>(w + l.chain_x) : nullptr;
    a.chain_cost = own_state ? reinterpret_cast<R *>(w + l.chain_cost) : nullptr;
    a.trace = reinterpret_cast<sa_level *>(w + l.trace);
    a.trace_x = (c->cfg.flags & SA_FLAG_TRACE_X) ? reinterpret_cast<R *>(w + l.trace_x) : nullptr;
    a.log = c->cfg.log_chains ? reinterpret_cast<sa_move_rec *>(w + l.log) : nullptr;
    a.log_final = c->cfg.log_chains ? reinterpret_cast<double *>(w + l.log_final) : nullptr;
    a.log_chains = c->cfg.log_chains;
    a.log_level = c->cfg.log_level;
    a.log_levels = c->cfg.log_chains ? c->cfg.log_levels : 0;
    a.x_start = reinterpret_cast<const R *>(w + l.x_start);
    a.start_level = kNoStart;
    a.featT = reinterpret_cast<const float *>(w + l.featT);
    a.net = (c->cfg.flags & SA_FLAG_LEARNED) ? w + l.net : nullptr;
    a.eps = 1.0f;
    a.cap_rec = nullptr;
    a.cap_count = reinterpret_cast<unsigned long long *>(w + l.cap_count);
    a.cap_capacity = 0;
    a.gcoef = reinterpret_cast<const float *>(w + l.gcoef);
    const double dn = (double)c->prob.n;
    a.cscale = (float)(c->prob.func == SA_SCHWEFEL  ? -1.0 / dn
                       : c->prob.func == SA_ACKLEY ? 1.0 / dn
                                                   : 3.14159265358979323846 / dn);
    a.net_kind = c->net_kind;
}

// Temperature feature of the proposal network: ln(tau T), tau = n for the
// objectives normalised by n (Schwefel, Ackley), 1 for Rastrigin.
// The Gaussian network kind takes ln T itself (tau = 1).
double feature_tau(const sa_problem &p) { return p.func == SA_RASTRIGIN ? 1.0 : (double)p.n; }

double feature_temperature_scale(const sa_ctx *c)
{
    return c->net_kind == SA_NET_GELU_GAUSS ? 1.0 : feature_tau(c->prob);
}

// Box/shift values of coordinate i in the run's precision: (l, u, rho, s).
void coord_values(const sa_ctx *c, uint32_t i, double out[4])
{
    sa::coord_values(c->prob.lower[i], c->prob.upper[i], c->prob.shift ? c->prob.shift[i] : 0.0, c->fp64, c->cfg.move,
                     c->cfg.radius_frac, out);
}

// Host memory the tables are built in before their copies to the device:
// T (levels doubles), inv_T and featT (levels floats each), tab (4 n reals of
// the run's precision, used with a per-coordinate table), gco (n floats,
// Griewank).  It must stay untouched until upload_tables returns.
struct Staging {
    double *T;
    float *inv_T, *featT;
    void *tab;
    float *gco;
};

sa_status upload_tables(sa_ctx *c, const Staging &hs)
{
    const Layout &l = c->pl.lay;
    const uint32_t n = c->prob.n, L = c->cfg.levels;
    const double tau = feature_temperature_scale(c);
    double t = c->cfg.T0;
    for (uint32_t k = 0; k < L; ++k) {
        hs.T[k] = t;
        hs.inv_T[k] = (float)(1.0 / t);
        hs.featT[k] = (float)std::log(tau * t);
        t = t * c->cfg.alpha;
    }
    SA_HIP(hipMemcpyAsync(c->ws + l.T, hs.T, L * sizeof(double), hipMemcpyHostToDevice, c->stream));
    SA_HIP(hipMemcpyAsync(c->ws + l.inv_T, hs.inv_T, L * sizeof(float), hipMemcpyHostToDevice, c->stream));
    SA_HIP(hipMemcpyAsync(c->ws + l.featT, hs.featT, L * sizeof(float), hipMemcpyHostToDevice, c->stream));
    double v[4];
    if (c->pl.table) {
        if (c->fp64) {
            double *tab = static_cast<double *>(hs.tab);
            for (uint32_t i = 0; i < n; ++i) {
                coord_values(c, i, v);
                for (int k = 0; k < 4; ++k) tab[4 * i + k] = v[k];
            }
            SA_HIP(hipMemcpyAsync(c->ws + l.table, tab, 4 * (size_t)n * sizeof(double), hipMemcpyHostToDevice,
                                  c->stream));
        } else {
            float *tab = static_cast<float *>(hs.tab);
            for (uint32_t i = 0; i < n; ++i) {
                coord_values(c, i, v);
                for (int k = 0; k < 4; ++k) tab[4 * i + k] = (float)v[k];
            }
            SA_HIP(hipMemcpyAsync(c->ws + l.table, tab, 4 * (size_t)n * sizeof(float), hipMemcpyHostToDevice,
                                  c->stream));
        }
    }
    if (c->prob.func == SA_GRIEWANK) {
        // Griewank's cos(y_i / sqrt(i)) in revolutions: y_i c_i, c_i = 1/(2 pi sqrt(i)), i = 1..n
        for (uint32_t i = 0; i < n; ++i)
            hs.gco[i] = (float)(1.0 / (2.0 * 3.14159265358979323846 * std::sqrt(i + 1.0)));
        SA_HIP(hipMemcpyAsync(c->ws + l.gcoef, hs.gco, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
    }
    coord_values(c, 0, v);
    if (c->fp64) {
        c->a64.lo = v[0];
        c->a64.hi = v[1];
        c->a64.rho = v[2];
        c->a64.sh = v[3];
    } else {
        c->a32.lo = (float)v[0];
        c->a32.hi = (float)v[1];
        c->a32.rho = (float)v[2];
        c->a32.sh = (float)v[3];
    }
    // The copies above read pageable host memory; finish them before the
    // staging memory is reused or released.
    SA_HIP(hipStreamSynchronize(c->stream));
    return SA_OK;
}

// upload_tables with staging in host vectors of the right sizes.
sa_status upload_tables(sa_ctx *c)
{
    const size_t n = c->prob.n, L = c->cfg.levels;
    std::vector<double> T(L), tab(4 * n);
    std::vector<float> inv_T(L), featT(L), gco(n);
    return upload_tables(c, Staging{T.data(), inv_T.data(), featT.data(), tab.data(), gco.data()});
}

// Enqueue levels [first, first + count), one launch each (the logged levels
// use the logging variant), then the launch that publishes the last level.
// *groups carries the candidate count of the level before `first` in and
// that of the last level out.
sa_status enqueue_levels(sa_ctx *c, uint32_t first, uint32_t count, hipStream_t s, uint32_t *groups)
{
    const uint32_t lg0 = c->cfg.log_level, lg1 = c->cfg.log_chains ? c->cfg.log_level + c->cfg.log_levels : 0;
    for (uint32_t k = first; k < first + count; ++k) {
        const bool log = k >= lg0 && k < lg1;
        const bool gauss = c->net_kind == SA_NET_GELU_GAUSS;
        const int mode = c->learned ? (log ? (gauss ? sa::kModeLearnLogG : sa::kModeLearnLog)
                                           : (gauss ? sa::kModeLearnG : sa::kModeLearn))
                                    : (log ? sa::kModeLog : (c->capturing ? sa::kModeCapture : sa::kModePlain));
        uint32_t g = 0;
        hipError_t e;
        if (const int var = variant_of(&c->cfg))
            e = c->fp64 ? sa::launch_variant_level_f64(c->prob.func, c->pl.table, var, log, c->a64, k, *groups, &g, s)
                        : sa::launch_variant_level_f32(c->prob.func, c->pl.table, var, log, c->a32, k, *groups, &g, s);
        else if (full_eval(&c->prob, &c->cfg))
            e = c->fp64 ? sa::launch_coupled_level_f64(c->prob.func, c->pl.table, log, c->a64, k, *groups, &g, s)
                        : sa::launch_coupled_level_f32(c->prob.func, c->pl.table, log, c->a32, k, *groups, &g, s);
        else if (c->pl.overlay)
            e = c->fp64 ? sa::launch_overlay_level_f64(c->prob.func, c->pl.table, log, c->a64, k, *groups, &g, s)
                        : sa::launch_overlay_level_f32(c->prob.func, c->pl.table, log, c->a32, k, *groups, &g, s);
        else
            e = c->fp64 ? sa::launch_level_f64(c->prob.func, c->pl.table, mode, c->a64, k, *groups, &g, s)
                        : sa::launch_level_f32(c->prob.func, c->pl.table, mode, c->a32, k, *groups, &g, s);
        if (e != hipSuccess) return fail(SA_ERR_DEVICE, "level %u launch: %s", k, hipGetErrorString(e));
        *groups = g;
    }
    const uint32_t last = first + count - 1;
    hipError_t e = c->fp64 ? sa::launch_finalize_f64(c->a64, last, *groups, s)
                           : sa::launch_finalize_f32(c->a32, last, *groups, s);
    if (e != hipSuccess) return fail(SA_ERR_DEVICE, "finalise launch: %s", hipGetErrorString(e));
    return SA_OK;
}

void drop_graphs(sa_ctx *c)
{
    for (auto &g : c->graphs) {
        if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
        if (g.second.g) (void)hipGraphDestroy(g.second.g);
    }
    c->graphs.clear();
}

sa_status enqueue_reset(sa_ctx *c)
{
    hipError_t e = sa::launch_reset(reinterpret_cast<double *>(c->ws + c->pl.lay.rec),
                                    reinterpret_cast<uint32_t *>(c->ws + c->pl.lay.rec_level),
                                    reinterpret_cast<double *>(c->ws + c->pl.lay.elite_f), c->stream);
    if (e != hipSuccess) return fail(SA_ERR_DEVICE, "reset launch: %s", hipGetErrorString(e));
    c->groups = 0;
    c->next_level = 0;
    c->first_level = 0;
    if (c->a32.start_level != kNoStart || c->a64.start_level != kNoStart) {
        drop_graphs(c);  // captured launches hold the start level
        c->a32.start_level = c->a64.start_level = kNoStart;
    }
    return SA_OK;
}

template <typename R>
sa_status read_candidates(sa_ctx *c, uint32_t k, double *x_out, double *f_out, uint32_t *chains_out)
{
    const Layout &l = c->pl.lay;
    const uint32_t n = c->prob.n, G = c->groups, last = c->next_level - 1;
    const size_t base = (size_t)(last & 1u) * c->pl.groups;
    std::vector<sa::Slot<R>> slots(G);
    SA_HIP(hipMemcpy(slots.data(), c->ws + l.slots + base * sizeof(sa::Slot<R>), G * sizeof(sa::Slot<R>),
                     hipMemcpyDeviceToHost));
    std::vector<uint32_t> order(G);
    for (uint32_t j = 0; j < G; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t p, uint32_t q) {
        return slots[p].f < slots[q].f || (slots[p].f == slots[q].f && slots[p].chain < slots[q].chain);
    });
    std::vector<R> x(n);
    for (uint32_t r = 0; r < k; ++r) {
        const sa::Slot<R> &sl = slots[order[r]];
        if (f_out) f_out[r] = sl.ff;
        if (chains_out) chains_out[r] = sl.chain;
        if (x_out) {
            SA_HIP(hipMemcpy(x.data(), c->ws + l.slot_x + ((base + order[r]) * n) * sizeof(R), n * sizeof(R),
                             hipMemcpyDeviceToHost));
            for (uint32_t i = 0; i < n; ++i) x_out[(size_t)r * n + i] = (double)x[i];
        }
    }
    return SA_OK;
}

}  // namespace

extern "C" {

const char *sa_last_error(void) { return sa::g_last_error.c_str(); }

sa_status sa_workspace_bytes(const sa_problem *prob, const sa_config *cfg, size_t *bytes)
{
    sa::g_last_error.clear();
    if (!bytes) return fail(SA_ERR_INVALID, "bytes must not be NULL");
    sa_status st = validate(prob, cfg);
    if (st != SA_OK) return st;
    Plan pl;
    st = plan(prob, cfg, kLdsPerWorkgroup, &pl);
    if (st != SA_OK) return st;
    *bytes = pl.lay.total;
    return SA_OK;
}

sa_status sa_create(const sa_problem *prob, const sa_config *cfg, void *stream, void *workspace, size_t ws_bytes,
                    sa_ctx **out)
{
    sa::g_last_error.clear();
    if (!out) return fail(SA_ERR_INVALID, "out must not be NULL");
    *out = nullptr;
    sa_status st = validate(prob, cfg);
    if (st != SA_OK) return st;
    if (!workspace) SA_FAULT_CHECK(sa::kFaultAlloc);

    int dev = 0;
    SA_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    SA_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SA_ERR_UNSUPPORTED, "device %d is %s; this library is built for gfx950 only", dev,
                    prop.gcnArchName);
    const size_t lds_limit = std::min<size_t>(kLdsPerWorkgroup, prop.sharedMemPerBlock);

    sa_ctx *c = new (std::nothrow) sa_ctx;
    if (!c) return fail(SA_ERR_NOMEM, "host allocation failed");
    c->device = dev;
    if (hipDeviceGetAttribute(&c->clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) c->clock_khz = 0;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    c->cfg = *cfg;
    c->seed = cfg->seed;
    c->fp64 = cfg->precision == SA_FP64;
    c->lower.assign(prob->lower, prob->lower + prob->n);
    c->upper.assign(prob->upper, prob->upper + prob->n);
    if (prob->shift) c->shift.assign(prob->shift, prob->shift + prob->n);
    c->prob = *prob;
    c->prob.lower = c->lower.data();
    c->prob.upper = c->upper.data();
    c->prob.shift = prob->shift ? c->shift.data() : nullptr;
    if (!c->fp64) {
        for (uint32_t i = 0; i < prob->n; ++i) {
            if (!(sa::round_up_f(prob->lower[i]) < sa::round_down_f(prob->upper[i]))) {
                delete c;
                return fail(SA_ERR_INVALID, "box %u is empty after rounding inward to FP32", i);
            }
        }
    }
    st = plan(&c->prob, &c->cfg, lds_limit, &c->pl);
    if (st != SA_OK) {
        delete c;
        return st;
    }
    if (workspace) {
        if (ws_bytes < c->pl.lay.total) {
            delete c;
            return fail(SA_ERR_INVALID, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes,
                        c->pl.lay.total);
        }
        if (reinterpret_cast<uintptr_t>(workspace) % kAlign) {
            delete c;
            return fail(SA_ERR_INVALID, "workspace must be %zu-byte aligned", kAlign);
        }
        c->ws = static_cast<unsigned char *>(workspace);
    } else {
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&c->ws), c->pl.lay.total);
        if (e != hipSuccess) {
            delete c;
            return fail(SA_ERR_NOMEM, "hipMalloc(%zu): %s", c->pl.lay.total, hipGetErrorString(e));
        }
        c->own_ws = true;
    }
    if (c->fp64)
        fill_args<double>(c, c->a64);
    else
        fill_args<float>(c, c->a32);
    c->a32.num_cus = c->a64.num_cus = (uint32_t)prop.multiProcessorCount;
    st = upload_tables(c);
    if (st == SA_OK) st = enqueue_reset(c);
    if (st != SA_OK) {
        sa_destroy(c);
        return st;
    }
    *out = c;
    return SA_OK;
}

sa_status sa_run(sa_ctx *c, uint32_t levels)
{
    sa::g_last_error.clear();
    if (!c) return fail(SA_ERR_INVALID, "null context");
    const uint32_t L = c->cfg.levels;
    if (c->next_level >= L) return fail(SA_ERR_STATE, "all %u levels have run", L);
    const uint32_t count = levels ? levels : L - c->next_level;
    if (count > L - c->next_level)
        return fail(SA_ERR_STATE, "%u levels requested, %u remain", count, L - c->next_level);
    SA_FAULT_CHECK(sa::kFaultLaunch);
    const uint32_t first = c->next_level;
    if (c->cfg.flags & SA_FLAG_GRAPH) {
        const auto key = std::make_tuple(first, count, c->groups);
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            if (!c->capture) SA_HIP(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
            SA_HIP(hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
            uint32_t groups = c->groups;
            sa_status st = enqueue_levels(c, first, count, c->capture, &groups);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(c->capture, &g);
            if (st != SA_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) return fail(SA_ERR_DEVICE, "graph capture: %s", hipGetErrorString(e));
            hipGraphExec_t ge = nullptr;
            e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                return fail(SA_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
            }
            sa_ctx::Graph gr;
            gr.g = g;
            gr.exec = ge;
            gr.groups = groups;
            it = c->graphs.emplace(key, gr).first;
        }
        SA_HIP(hipGraphLaunch(it->second.exec, c->stream));
        c->groups = it->second.groups;
    } else {
        sa_status st = enqueue_levels(c, first, count, c->stream, &c->groups);
        if (st != SA_OK) return st;
    }
    c->next_level = first + count;
    return SA_OK;
}

sa_status sa_reset(sa_ctx *c, uint64_t seed)
{
    sa::g_last_error.clear();
    if (!c) return fail(SA_ERR_INVALID, "null context");
    SA_FAULT_CHECK(sa::kFaultLaunch);
    if (seed != c->seed) {
        // Captured graphs hold the seed in their kernel arguments.
        drop_graphs(c);
        c->seed = seed;
        c->a32.seed_lo = c->a64.seed_lo = (uint32_t)seed;
        c->a32.seed_hi = c->a64.seed_hi = (uint32_t)(seed >> 32);
    }
    return enqueue_reset(c);
}

sa_status sa_levels_done(const sa_ctx *c, uint32_t *levels)
{
    if (!c || !levels) return fail(SA_ERR_INVALID, "null argument");
    *levels = c->next_level;
    return SA_OK;
}

sa_status sa_best(sa_ctx *c, double *x_out, double *f_out, uint32_t *level_found)
{
    sa::g_last_error.clear();
    if (!c) return fail(SA_ERR_INVALID, "null context");
    if (c->next_level == 0) return fail(SA_ERR_STATE, "no level has run");
    SA_HIP(hipStreamSynchronize(c->stream));
    const Layout &l = c->pl.lay;
    const uint32_t n = c->prob.n;
    double rec[2];
    uint32_t lvl = 0;
    SA_HIP(hipMemcpy(rec, c->ws + l.rec, sizeof rec, hipMemcpyDeviceToHost));
    SA_HIP(hipMemcpy(&lvl, c->ws + l.rec_level, sizeof lvl, hipMemcpyDeviceToHost));
    if (lvl == 0xFFFFFFFFu) return fail(SA_ERR_STATE, "no record yet");
    if (x_out) {
        if (c->fp64) {
            SA_HIP(hipMemcpy(x_out, c->ws + l.x_rec, n * sizeof(double), hipMemcpyDeviceToHost));
        } else {
            std::vector<float> x(n);
            SA_HIP(hipMemcpy(x.data(), c->ws + l.x_rec, n * sizeof(float), hipMemcpyDeviceToHost));
            for (uint32_t i = 0; i < n; ++i) x_out[i] = x[i];
        }
    }
    if (f_out) *f_out = rec[0];
    if (level_found) *level_found = lvl;
    return SA_OK;
}

sa_status sa_trace(sa_ctx *c, uint32_t first, uint32_t count, sa_level *out, double *x_best)
{
    sa::g_last_error.clear();
    if (!c) return fail(SA_ERR_INVALID, "null context");
    if (count == 0) return SA_OK;
    if (first >= c->next_level || count > c->next_level - first)
        return fail(SA_ERR_STATE, "levels [%u, %u) have not all run (%u done)", first, first + count,
                    c->next_level);
    if (first < c->first_level)
        return fail(SA_ERR_STATE, "the run started at level %u; level %u has no trace", c->first_level, first);
    if (x_best && !(c->cfg.flags & SA_FLAG_TRACE_X))
        return fail(SA_ERR_STATE, "x_best trace needs SA_FLAG_TRACE_X");
    SA_HIP(hipStreamSynchronize(c->stream));
    const Layout &l = c->pl.lay;
    if (out) {
        SA_HIP(hipMemcpy(out, c->ws + l.trace + (size_t)first * sizeof(sa_level), count * sizeof(sa_level),
                         hipMemcpyDeviceToHost));
        sa::stamps_to_ns(out, count, c->clock_khz);
    }
    if (x_best) {
        const size_t n = c->prob.n, m = n * count;
        if (c->fp64) {
            SA_HIP(hipMemcpy(x_best, c->ws + l.trace_x + first * n * sizeof(double), m * sizeof(double),
                             hipMemcpyDeviceToHost));
        } else {
            std::vector<float> x(m);
            SA_HIP(hipMemcpy(x.data(), c->ws + l.trace_x + first * n * sizeof(float), m * sizeof(float),
                             hipMemcpyDeviceToHost));
            for (size_t i = 0; i < m; ++i) x_best[i] = x[i];
        }
    }
    return SA_OK;
}

sa_status sa_move_log(sa_ctx *c, sa_move_rec *moves, double *final_f)
{
    sa::g_last_error.clear();
    if (!c) return fail(SA_ERR_INVALID, "null context");
    if (!c->cfg.log_chains) return fail(SA_ERR_STATE, "the context was created without a move log");
    SA_HIP(hipStreamSynchronize(c->stream));
    const Layout &l = c->pl.lay;
    if (moves)
        SA_HIP(hipMemcpy(moves, c->ws + l.log,
                         (size_t)c->cfg.log_levels * c->cfg.log_chains * c->cfg.steps * sizeof(sa_move_rec),
                         hipMemcpyDeviceToHost));
    if (final_f)
        SA_HIP(hipMemcpy(final_f, c->ws + l.log_final, (size_t)c->cfg.log_levels * c->cfg.chains * sizeof(double),
                         hipMemcpyDeviceToHost));
    return SA_OK;
}

sa_status sa_layout(const sa_ctx *c, uint32_t *workgroup, uint32_t *overlay_slots, uint32_t *tiles)
{
    if (!c) return fail(SA_ERR_INVALID, "null context");
    if (workgroup) *workgroup = c->pl.wg;
    if (overlay_slots) *overlay_slots = c->pl.overlay ? c->pl.ov_slots : 0;
    if (tiles) *tiles = c->pl.groups;
    return SA_OK;
}

sa_status sa_set_start(sa_ctx *c, uint32_t level, const double *x)
{
    sa::g_last_error.clear();
    if (!c || !x) return fail(SA_ERR_INVALID, "null argument");
    if (c->next_level != 0) return fail(SA_ERR_STATE, "a start state is set before the first level (after sa_reset)");
    if (level == 0 || level >= c->cfg.levels)
        return fail(SA_ERR_INVALID, "start level must be in [1, %u)", c->cfg.levels);
    const uint32_t n = c->prob.n;
    for (uint32_t i = 0; i < n; ++i)
        if (!(x[i] >= c->lower[i] && x[i] <= c->upper[i]))
            return fail(SA_ERR_INVALID, "start coordinate %u lies outside the box", i);
    const Layout &l = c->pl.lay;
    if (c->fp64) {
        SA_HIP(hipMemcpyAsync(c->ws + l.x_start, x, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    } else {
        std::vector<float> xf(n);
        for (uint32_t i = 0; i < n; ++i) {
            // the FP32 box is the FP64 box rounded inward
            const float lo = sa::round_up_f(c->lower[i]), hi = sa::round_down_f(c->upper[i]);
            xf[i] = std::min(std::max((float)x[i], lo), hi);
        }
        SA_HIP(hipMemcpyAsync(c->ws + l.x_start, xf.data(), n * sizeof(float), hipMemcpyHostToDevice, c->stream));
    }
    SA_HIP(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->a32.start_level = c->a64.start_level = level;
    c->next_level = c->first_level = level;
    c->groups = 0;
    return SA_OK;
}

sa_status sa_set_proposal(sa_ctx *c, const float *params, float eps)
{
    sa::g_last_error.clear();
    if (!c) return fail(SA_ERR_INVALID, "null context");
    if (!(c->cfg.flags & SA_FLAG_LEARNED)) return fail(SA_ERR_STATE, "the context was created without SA_FLAG_LEARNED");
    if (!params) {
        if (c->learned) drop_graphs(c);
        c->learned = false;
        return SA_OK;
    }
    if (!(eps >= 0.0f && eps <= 1.0f)) return fail(SA_ERR_INVALID, "eps must lie in [0, 1]");
    if (c->capturing) return fail(SA_ERR_STATE, "capture records plain runs; stop it (sa_capture(NULL)) first");
    SA_FAULT_CHECK(sa::kFaultLaunch);
    for (uint32_t i = 0; i < sa::mlp::kNumParams; ++i)
        if (!std::isfinite(params[i])) return fail(SA_ERR_INVALID, "parameter %u is not finite", i);
    const Layout &l = c->pl.lay;
    float *theta = reinterpret_cast<float *>(c->ws + l.theta);
    SA_HIP(hipMemcpyAsync(theta, params, sa::mlp::kNumParams * sizeof(float), hipMemcpyHostToDevice, c->stream));
    hipError_t e = sa::launch_pack_net(theta, c->ws + l.net, c->stream);
    if (e != hipSuccess) return fail(SA_ERR_DEVICE, "pack launch: %s", hipGetErrorString(e));
    SA_HIP(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->a32.eps = eps;
    c->learned = true;
    return SA_OK;
}

sa_status sa_set_network_kind(sa_ctx *c, int kind)
{
    sa::g_last_error.clear();
    if (!c) return fail(SA_ERR_INVALID, "null context");
    if (kind != SA_NET_RELU_CAUCHY && kind != SA_NET_GELU_GAUSS) return fail(SA_ERR_INVALID, "unknown network kind %d", kind);
    if (c->capturing) return fail(SA_ERR_STATE, "the network kind fixes the captured features; stop the capture first");
    if (kind == c->net_kind) return SA_OK;
    c->net_kind = kind;
    c->a32.net_kind = c->a64.net_kind = kind;
    const uint32_t L = c->cfg.levels;
    const double tau = feature_temperature_scale(c);
    std::vector<float> featT(L);
    double t = c->cfg.T0;
    for (uint32_t k = 0; k < L; ++k) {
        featT[k] = (float)std::log(tau * t);
        t = t * c->cfg.alpha;
    }
    SA_HIP(hipMemcpyAsync(c->ws + c->pl.lay.featT, featT.data(), L * sizeof(float), hipMemcpyHostToDevice, c->stream));
    SA_HIP(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    return SA_OK;
}

sa_status sa_capture(sa_ctx *c, float *records, uint64_t capacity)
{
    sa::g_last_error.clear();
    if (!c) return fail(SA_ERR_INVALID, "null context");
    if (records && capacity == 0) return fail(SA_ERR_INVALID, "capacity must be positive");
    if (records && reinterpret_cast<uintptr_t>(records) % sizeof(float))
        return fail(SA_ERR_INVALID, "records must be float-aligned");
    if (records && c->learned) return fail(SA_ERR_STATE, "capture records plain runs; clear the proposal first");
    if (records && c->pl.overlay) return fail(SA_ERR_UNSUPPORTED, "capture runs on the dense state layout");
    if (records && full_eval(&c->prob, &c->cfg))
        return fail(SA_ERR_UNSUPPORTED, "capture records incremental moves of the separable families");
    if (records && variant_of(&c->cfg)) return fail(SA_ERR_UNSUPPORTED, "capture records plain-exchange runs");
    drop_graphs(c);
    c->a32.cap_rec = records;
    c->a64.cap_rec = records;
    c->a32.cap_capacity = c->a64.cap_capacity = records ? capacity : 0;
    c->capturing = records != nullptr;
    SA_HIP(hipMemsetAsync(c->ws + c->pl.lay.cap_count, 0, sizeof(unsigned long long), c->stream));
    return SA_OK;
}

sa_status sa_capture_count(sa_ctx *c, uint64_t *count)
{
    sa::g_last_error.clear();
    if (!c || !count) return fail(SA_ERR_INVALID, "null argument");
    SA_HIP(hipStreamSynchronize(c->stream));
    unsigned long long v = 0;
    SA_HIP(hipMemcpy(&v, c->ws + c->pl.lay.cap_count, sizeof v, hipMemcpyDeviceToHost));
    *count = v;
    return SA_OK;
}

sa_status sa_candidates(sa_ctx *c, uint32_t k, double *x_out, double *f_out, uint32_t *chains_out,
                        uint32_t *available)
{
    sa::g_last_error.clear();
    if (!c) return fail(SA_ERR_INVALID, "null context");
    if (c->next_level == 0 || c->next_level == c->first_level) return fail(SA_ERR_STATE, "no level has run");
    if (available) *available = c->groups;
    if (k > c->groups) return fail(SA_ERR_INVALID, "k = %u exceeds the %u candidates of the last level", k, c->groups);
    if (k == 0) return SA_OK;
    SA_HIP(hipStreamSynchronize(c->stream));
    return c->fp64 ? read_candidates<double>(c, k, x_out, f_out, chains_out)
                   : read_candidates<float>(c, k, x_out, f_out, chains_out);
}

void sa_destroy(sa_ctx *c)
{
    if (!c) return;
    if (c->stream || c->ws) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->capture) (void)hipStreamDestroy(c->capture);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    delete c;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free run (sa_run_static): the workspace of sa_create lives in a
// file-scope device array, one copy per GPU, instead of hipMalloc'd memory.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kStaticScratchBytes = SA_STATIC_SCRATCH_BYTES;
constexpr uint32_t kStaticMaxLevels = SA_STATIC_MAX_LEVELS;
constexpr uint32_t kStaticMaxN = SA_STATIC_MAX_N;
constexpr int kStaticMaxDevices = 64;

// Device scratch: one copy per GPU the library's code object is loaded on.
// Host code never passes this name to a kernel or a copy: it reaches the
// memory through the per-device address hipGetSymbolAddress returns.
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Host staging of the tables and of the record's read-back (sized for the
// largest level count and dimension sa_run_static accepts).
alignas(64) double g_static_T[kStaticMaxLevels];
alignas(64) float g_static_inv_T[kStaticMaxLevels];
alignas(64) float g_static_featT[kStaticMaxLevels];
alignas(64) double g_static_tab[4 * (size_t)kStaticMaxN];
alignas(64) float g_static_gco[kStaticMaxN];
alignas(64) float g_static_x[kStaticMaxN];

// Serialises sa_run_static within the process (the host staging above and the
// device scratch are shared by every call).
std::mutex g_static_mu;
unsigned char *g_static_ptr[kStaticMaxDevices];  // device address of `scratch`, per device

}  // namespace

extern "C" sa_status sa_run_static(const sa_problem *prob, const sa_config *cfg, void *stream, double *x_out,
                                   double *f_out, uint32_t *level_found)
{
    std::lock_guard<std::mutex> lock(g_static_mu);
    sa::g_last_error.clear();
    sa_status st = validate(prob, cfg);
    if (st != SA_OK) return st;
    if (cfg->flags & ~SA_FLAG_OVERLAY)
        return fail(SA_ERR_UNSUPPORTED, "sa_run_static takes SA_FLAG_OVERLAY only (no trace, graph or learned runs)");
    if (cfg->log_chains) return fail(SA_ERR_UNSUPPORTED, "sa_run_static keeps no move log");
    if (prob->n > kStaticMaxN) return fail(SA_ERR_UNSUPPORTED, "sa_run_static: n = %u exceeds %u", prob->n, kStaticMaxN);
    if (cfg->levels > kStaticMaxLevels)
        return fail(SA_ERR_UNSUPPORTED, "sa_run_static: %u levels exceed %u", cfg->levels, kStaticMaxLevels);
    SA_FAULT_CHECK(sa::kFaultLaunch);

    int dev = 0;
    SA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticMaxDevices) return fail(SA_ERR_UNSUPPORTED, "device index %d out of range", dev);
    if (!g_static_ptr[dev]) {
        hipDeviceProp_t prop;
        SA_HIP(hipGetDeviceProperties(&prop, dev));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(SA_ERR_UNSUPPORTED, "device %d is %s; this library is built for gfx950 only", dev,
                        prop.gcnArchName);
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SA_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_static_ptr[dev] = static_cast<unsigned char *>(ptr);
    }
    int lds = 0, cus = 0;
    SA_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    SA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));

    // The context lives on the stack and reads the caller's arrays in place
    // (they are valid for the duration of the call): no host or device
    // allocation.
    sa_ctx c;
    c.device = dev;
    c.stream = reinterpret_cast<hipStream_t>(stream);
    c.cfg = *cfg;
    c.seed = cfg->seed;
    c.fp64 = cfg->precision == SA_FP64;
    c.prob = *prob;
    if (!c.fp64) {
        for (uint32_t i = 0; i < prob->n; ++i)
            if (!(sa::round_up_f(prob->lower[i]) < sa::round_down_f(prob->upper[i])))
                return fail(SA_ERR_INVALID, "box %u is empty after rounding inward to FP32", i);
    }
    st = plan(&c.prob, &c.cfg, std::min<size_t>(kLdsPerWorkgroup, (size_t)lds), &c.pl);
    if (st != SA_OK) return st;
    if (c.pl.lay.total > kStaticScratchBytes)
        return fail(SA_ERR_UNSUPPORTED, "the run needs %zu bytes of workspace; the static scratch holds %zu",
                    c.pl.lay.total, kStaticScratchBytes);
    c.ws = g_static_ptr[dev];
    if (c.fp64)
        fill_args<double>(&c, c.a64);
    else
        fill_args<float>(&c, c.a32);
    c.a32.num_cus = c.a64.num_cus = (uint32_t)cus;
    st = upload_tables(&c, Staging{g_static_T, g_static_inv_T, g_static_featT, g_static_tab, g_static_gco});
    // The record starts empty (a kernel clears it: the scratch keeps the
    // previous call's contents); every other word a run reads is written by
    // the level that precedes the read.
    if (st == SA_OK) st = enqueue_reset(&c);
    if (st == SA_OK) st = enqueue_levels(&c, 0, cfg->levels, c.stream, &c.groups);
    if (st != SA_OK) {
        (void)hipStreamSynchronize(c.stream);
        return st;
    }
    SA_HIP(hipStreamSynchronize(c.stream));
    const Layout &l = c.pl.lay;
    double rec[2];
    uint32_t lvl = 0;
    SA_HIP(hipMemcpy(rec, c.ws + l.rec, sizeof rec, hipMemcpyDeviceToHost));
    SA_HIP(hipMemcpy(&lvl, c.ws + l.rec_level, sizeof lvl, hipMemcpyDeviceToHost));
    if (lvl == 0xFFFFFFFFu) return fail(SA_ERR_STATE, "no record after %u levels", cfg->levels);
    if (x_out) {
        const uint32_t n = prob->n;
        if (c.fp64) {
            SA_HIP(hipMemcpy(x_out, c.ws + l.x_rec, n * sizeof(double), hipMemcpyDeviceToHost));
        } else {
            SA_HIP(hipMemcpy(g_static_x, c.ws + l.x_rec, n * sizeof(float), hipMemcpyDeviceToHost));
            for (uint32_t i = 0; i < n; ++i) x_out[i] = g_static_x[i];
        }
    }
    if (f_out) *f_out = rec[0];
    if (level_found) *level_found = lvl;
    return SA_OK;
}
