// Host runtime of batched runs (sa_batch_* in include/sa.h) and the
// autotuner that picks chains per problem and tiles per workgroup.
//
// The host splits every problem's chains into 64-chain tiles, packs tiles of
// different problems into workgroups (first fit, largest LDS region first)
// so that each CU's 160 KiB of LDS is filled, lays out one workspace, and
// enqueues one launch per level plus one finalising launch per sa_batch_run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <utility>
#include <vector>

#include "sa_host.hpp"
#include "sa_internal.hpp"

using sa::align_up;
using sa::fail;
using sa::kAlign;
using sa::kLdsPerWorkgroup;

namespace {

constexpr uint32_t kMaxChainsPerProblem = 1u << 20;

struct BatchLayout {
    size_t probs, tile_prob, tile_xoff, wg_tile, wg_lds, table, T, inv_T, slots, slot_x, x_best, x_rec, rec, rec_level,
        trace, trace_x, log, log_final, total;
};

struct BatchPlan {
    uint32_t nprob = 0, ntiles = 0, groups = 0, wpg = 4, max_n = 0;
    size_t real = 0, lds = 0, sum_n = 0, slot_x_stride = 0;
    std::vector<sa::BatchProblem> probs;
    std::vector<uint32_t> tile_prob, tile_xoff, wg_tile, wg_lds;
    BatchLayout lay{};
};

sa_status validate_batch(const sa_problem *probs, uint32_t nprob, const uint32_t *chains, const sa_batch_config *c)
{
    if (!probs || !chains || !c) return fail(SA_ERR_INVALID, "null problems, chains or config");
    if (nprob == 0) return fail(SA_ERR_INVALID, "nprob must be >= 1");
    if (nprob >= (1u << 24)) return fail(SA_ERR_INVALID, "nprob must be < 2^24 (problem ids share a counter word)");
    for (uint32_t p = 0; p < nprob; ++p) {
        if (sa_status st = sa::validate_problem(&probs[p], p); st != SA_OK) return st;
        if (!sa::separable(probs[p].func))
            return fail(SA_ERR_UNSUPPORTED, "problem %u: batches hold the separable families (Schwefel, Rastrigin, "
                        "Ackley)", p);
        if (chains[p] == 0 || chains[p] % 64 || chains[p] > kMaxChainsPerProblem)
            return fail(SA_ERR_INVALID, "problem %u: chains must be a multiple of 64 in [64, 2^20]", p);
    }
    if (sa_status st = sa::validate_schedule(c->levels, c->steps, c->precision, c->move, c->T0, c->alpha,
                                             c->radius_frac);
        st != SA_OK)
        return st;
    if (c->flags & ~(SA_FLAG_GRAPH | SA_FLAG_TRACE_X)) return fail(SA_ERR_INVALID, "unknown flag bits");
    if (c->waves_per_group != 0 && c->waves_per_group != 1 && c->waves_per_group != 2 && c->waves_per_group != 4)
        return fail(SA_ERR_INVALID, "waves_per_group must be 0, 1, 2 or 4");
    if (c->log_chains) {
        if (c->log_problem >= nprob) return fail(SA_ERR_INVALID, "log_problem out of range");
        if (c->log_chains > chains[c->log_problem]) return fail(SA_ERR_INVALID, "log_chains exceeds the chains");
        if (c->log_levels == 0 || c->log_level >= c->levels || c->log_levels > c->levels - c->log_level)
            return fail(SA_ERR_INVALID, "logged level range outside [0, levels)");
    }
    return SA_OK;
}

sa_status plan_batch(const sa_problem *probs, uint32_t nprob, const uint32_t *chains, const sa_batch_config *c,
                     size_t lds_limit, BatchPlan *out)
{
    BatchPlan pl;
    pl.nprob = nprob;
    pl.real = c->precision == SA_FP64 ? sizeof(double) : sizeof(float);
    pl.wpg = c->waves_per_group ? c->waves_per_group : 4;
    pl.probs.resize(nprob);
    size_t tab = 0;
    uint64_t tiles = 0;
    for (uint32_t p = 0; p < nprob; ++p) {
        sa::BatchProblem &P = pl.probs[p];
        P.func = probs[p].func;
        P.n = probs[p].n;
        P.chains = chains[p];
        P.first_tile = (uint32_t)tiles;
        P.tab_off = (uint32_t)tab;
        P.x_off = (uint32_t)tab;
        P.inv_n = (float)(1.0 / (double)P.n);
        P.pad = 0;
        tab += P.n;
        tiles += chains[p] / 64;
        pl.max_n = std::max(pl.max_n, P.n);
        if (sa::batch_wave_lds_bytes(P.n, pl.real) > lds_limit)
            return fail(SA_ERR_UNSUPPORTED, "problem %u: n=%u does not fit one wave's LDS region", p, P.n);
    }
    if (tiles >= 0xFFFFFFFFull || tab >= 0xFFFFFFFFull) return fail(SA_ERR_INVALID, "batch too large");
    pl.ntiles = (uint32_t)tiles;
    pl.sum_n = tab;
    pl.tile_prob.resize(pl.ntiles);
    pl.tile_xoff.resize(pl.ntiles);
    size_t xo = 0;
    for (uint32_t p = 0; p < nprob; ++p) {
        for (uint32_t t = 0; t < chains[p] / 64; ++t) {
            const uint32_t tile = pl.probs[p].first_tile + t;
            pl.tile_prob[tile] = p;
            pl.tile_xoff[tile] = (uint32_t)xo;
            xo += pl.probs[p].n;
        }
    }
    if (xo >= 0xFFFFFFFFull) return fail(SA_ERR_INVALID, "batch too large");
    pl.slot_x_stride = xo;

    // Pack tiles into workgroups of up to wpg waves; budget per workgroup so
    // that 4 / wpg workgroups share a CU's LDS (one wave per SIMD), raised to
    // the largest single region when one tile needs more.
    std::vector<uint32_t> order(pl.ntiles);
    std::iota(order.begin(), order.end(), 0u);
    auto region = [&](uint32_t tile) {
        return (sa::batch_wave_lds_bytes(pl.probs[pl.tile_prob[tile]].n, pl.real) + 15) / 16 * 16;
    };
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return region(x) > region(y); });
    size_t budget = lds_limit / (4 / pl.wpg);
    if (!order.empty()) budget = std::max(budget, region(order[0]));
    budget = std::min(budget, lds_limit);
    struct Group {
        uint32_t count = 0;
        size_t bytes = 0;
    };
    std::vector<Group> groups;
    std::vector<uint32_t> slot_tile, slot_lds;
    size_t open_from = 0;  // groups before this index are full (count == wpg)
    for (uint32_t tile : order) {
        const size_t r = region(tile);
        size_t g = open_from;
        for (; g < groups.size(); ++g)
            if (groups[g].count < pl.wpg && groups[g].bytes + r <= budget) break;
        if (g == groups.size()) {
            groups.push_back(Group{});
            slot_tile.insert(slot_tile.end(), pl.wpg, 0xFFFFFFFFu);
            slot_lds.insert(slot_lds.end(), pl.wpg, 0u);
        }
        Group &G = groups[g];
        slot_tile[g * pl.wpg + G.count] = tile;
        slot_lds[g * pl.wpg + G.count] = (uint32_t)G.bytes;
        G.bytes += r;
        G.count += 1;
        pl.lds = std::max(pl.lds, G.bytes);
        while (open_from < groups.size() && groups[open_from].count == pl.wpg) ++open_from;
    }
    pl.groups = (uint32_t)groups.size();
    pl.wg_tile = std::move(slot_tile);
    pl.wg_lds = std::move(slot_lds);

    const size_t R = pl.real, L = c->levels;
    BatchLayout &l = pl.lay;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + (bytes ? bytes : 1));
        return at;
    };
    l.probs = take(nprob * sizeof(sa::BatchProblem));
    l.tile_prob = take(pl.ntiles * sizeof(uint32_t));
    l.tile_xoff = take(pl.ntiles * sizeof(uint32_t));
    l.wg_tile = take(pl.wg_tile.size() * sizeof(uint32_t));
    l.wg_lds = take(pl.wg_lds.size() * sizeof(uint32_t));
    l.table = take(4 * pl.sum_n * R);
    l.T = take(L * sizeof(double));
    l.inv_T = take(L * sizeof(float));
    l.slots = take(2 * (size_t)pl.ntiles * sizeof(sa::Slot<double>));
    l.slot_x = take(2 * pl.slot_x_stride * R);
    l.x_best = take(pl.sum_n * R);
    l.x_rec = take(pl.sum_n * R);
    l.rec = take(nprob * sizeof(double));
    l.rec_level = take(nprob * sizeof(uint32_t));
    l.trace = take((size_t)nprob * L * sizeof(sa_level));
    l.trace_x = take((c->flags & SA_FLAG_TRACE_X) ? L * pl.sum_n * R : 0);
    const size_t log_moves = c->log_chains ? (size_t)c->log_levels * c->log_chains * c->steps : 0;
    l.log = take(log_moves * sizeof(sa_move_rec));
    l.log_final = take(c->log_chains ? (size_t)c->log_levels * chains[c->log_problem] * sizeof(double) : 0);
    l.total = off;
    *out = std::move(pl);
    return SA_OK;
}

}  // namespace

struct sa_batch {
    int device = 0;
    int clock_khz = 0;  // rate of the device's constant clock
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    sa_batch_config cfg{};
    BatchPlan pl;
    std::vector<std::vector<double>> lower, upper, shift;
    unsigned char *ws = nullptr;
    bool own_ws = false;
    bool fp64 = false;
    uint32_t next_level = 0;
    uint64_t seed = 0;
    uint64_t *clock = nullptr;  // caller's tile clock log (sa_batch_clock)
    uint32_t clock_level = 0, clock_levels = 0;
    sa::BatchArgs<float> a32{};
    sa::BatchArgs<double> a64{};
    struct Graph {
        hipGraph_t g = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::map<std::pair<uint32_t, uint32_t>, Graph> graphs;
};

namespace {

template <typename R> void fill_batch_args(sa_batch *b, sa::BatchArgs<R> &a)
{
    const BatchLayout &l = b->pl.lay;
    unsigned char *w = b->ws;
    a.nprob = b->pl.nprob;
    a.ntiles = b->pl.ntiles;
    a.steps = b->cfg.steps;
    a.move = b->cfg.move;
    a.seed_lo = (uint32_t)b->seed;
    a.seed_hi = (uint32_t)(b->seed >> 32);
    a.waves_per_group = b->pl.wpg;
    a.levels = b->cfg.levels;
    a.probs = reinterpret_cast<const sa::BatchProblem *>(w + l.probs);
    a.tile_prob = reinterpret_cast<const uint32_t *>(w + l.tile_prob);
    a.tile_xoff = reinterpret_cast<const uint32_t *>(w + l.tile_xoff);
    a.wg_tile = reinterpret_cast<const uint32_t *>(w + l.wg_tile);
    a.wg_lds = reinterpret_cast<const uint32_t *>(w + l.wg_lds);
    a.table = reinterpret_cast<const R *>(w + l.table);
    a.T = reinterpret_cast<const double *>(w + l.T);
    a.inv_T = reinterpret_cast<const float *>(w + l.inv_T);
    a.slots = reinterpret_cast<sa::Slot<R> *>(w + l.slots);
    a.slot_x = reinterpret_cast<R *>(w + l.slot_x);
    a.slot_x_stride = (uint32_t)b->pl.slot_x_stride;
    a.x_best = reinterpret_cast<R *>(w + l.x_best);
    a.x_rec = reinterpret_cast<R *>(w + l.x_rec);
    a.rec = reinterpret_cast<double *>(w + l.rec);
    a.rec_level = reinterpret_cast<uint32_t *>(w + l.rec_level);
    a.trace = reinterpret_cast<sa_level *>(w + l.trace);
    a.trace_x = (b->cfg.flags & SA_FLAG_TRACE_X) ? reinterpret_cast<R *>(w + l.trace_x) : nullptr;
    a.log = b->cfg.log_chains ? reinterpret_cast<sa_move_rec *>(w + l.log) : nullptr;
    a.log_final = b->cfg.log_chains ? reinterpret_cast<double *>(w + l.log_final) : nullptr;
    a.log_problem = b->cfg.log_problem;
    a.log_chains = b->cfg.log_chains;
    a.log_level = b->cfg.log_level;
    a.log_levels = b->cfg.log_chains ? b->cfg.log_levels : 0;
    a.clock = b->clock;
    a.clock_level = b->clock_level;
    a.clock_levels = b->clock ? b->clock_levels : 0;
}

template <typename R> sa_status upload_table(sa_batch *b)
{
    const BatchPlan &pl = b->pl;
    std::vector<R> tab(4 * pl.sum_n);
    double v[4];
    for (uint32_t p = 0; p < pl.nprob; ++p) {
        const auto &lo = b->lower[p], &hi = b->upper[p], &sh = b->shift[p];
        for (uint32_t i = 0; i < pl.probs[p].n; ++i) {
            sa::coord_values(lo[i], hi[i], sh.empty() ? 0.0 : sh[i], b->fp64, b->cfg.move, b->cfg.radius_frac, v);
            for (int k = 0; k < 4; ++k) tab[4 * ((size_t)pl.probs[p].tab_off + i) + k] = (R)v[k];
        }
    }
    SA_HIP(hipMemcpy(b->ws + pl.lay.table, tab.data(), tab.size() * sizeof(R), hipMemcpyHostToDevice));
    return SA_OK;
}

sa_status upload_batch(sa_batch *b)
{
    const BatchPlan &pl = b->pl;
    const BatchLayout &l = pl.lay;
    SA_HIP(hipMemcpy(b->ws + l.probs, pl.probs.data(), pl.probs.size() * sizeof(sa::BatchProblem),
                     hipMemcpyHostToDevice));
    SA_HIP(hipMemcpy(b->ws + l.tile_prob, pl.tile_prob.data(), pl.tile_prob.size() * sizeof(uint32_t),
                     hipMemcpyHostToDevice));
    SA_HIP(hipMemcpy(b->ws + l.tile_xoff, pl.tile_xoff.data(), pl.tile_xoff.size() * sizeof(uint32_t),
                     hipMemcpyHostToDevice));
    SA_HIP(hipMemcpy(b->ws + l.wg_tile, pl.wg_tile.data(), pl.wg_tile.size() * sizeof(uint32_t),
                     hipMemcpyHostToDevice));
    SA_HIP(hipMemcpy(b->ws + l.wg_lds, pl.wg_lds.data(), pl.wg_lds.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    const uint32_t L = b->cfg.levels;
    std::vector<double> T(L);
    std::vector<float> inv_T(L);
    double t = b->cfg.T0;
    for (uint32_t k = 0; k < L; ++k) {
        T[k] = t;
        inv_T[k] = (float)(1.0 / t);
        t = t * b->cfg.alpha;
    }
    SA_HIP(hipMemcpy(b->ws + l.T, T.data(), L * sizeof(double), hipMemcpyHostToDevice));
    SA_HIP(hipMemcpy(b->ws + l.inv_T, inv_T.data(), L * sizeof(float), hipMemcpyHostToDevice));
    return b->fp64 ? upload_table<double>(b) : upload_table<float>(b);
}

sa_status enqueue_batch_levels(sa_batch *b, uint32_t first, uint32_t count, hipStream_t s)
{
    const uint32_t lg0 = b->cfg.log_level, lg1 = b->cfg.log_chains ? b->cfg.log_level + b->cfg.log_levels : 0;
    for (uint32_t k = first; k < first + count; ++k) {
        const bool log = k >= lg0 && k < lg1;
        hipError_t e = b->fp64 ? sa::launch_batch_level_f64(b->a64, b->pl.groups, b->pl.lds, log, k, s)
                               : sa::launch_batch_level_f32(b->a32, b->pl.groups, b->pl.lds, log, k, s);
        if (e != hipSuccess) return fail(SA_ERR_DEVICE, "batch level %u launch: %s", k, hipGetErrorString(e));
    }
    const uint32_t last = first + count - 1;
    hipError_t e = b->fp64 ? sa::launch_batch_finalize_f64(b->a64, last, b->pl.max_n, s)
                           : sa::launch_batch_finalize_f32(b->a32, last, b->pl.max_n, s);
    if (e != hipSuccess) return fail(SA_ERR_DEVICE, "batch finalise launch: %s", hipGetErrorString(e));
    return SA_OK;
}

void drop_batch_graphs(sa_batch *b)
{
    for (auto &g : b->graphs) {
        if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
        if (g.second.g) (void)hipGraphDestroy(g.second.g);
    }
    b->graphs.clear();
}

sa_status enqueue_batch_reset(sa_batch *b)
{
    hipError_t e = sa::launch_batch_reset(reinterpret_cast<double *>(b->ws + b->pl.lay.rec),
                                          reinterpret_cast<uint32_t *>(b->ws + b->pl.lay.rec_level), b->pl.nprob,
                                          b->stream);
    if (e != hipSuccess) return fail(SA_ERR_DEVICE, "batch reset launch: %s", hipGetErrorString(e));
    b->next_level = 0;
    return SA_OK;
}

}  // namespace

extern "C" {

sa_status sa_batch_workspace_bytes(const sa_problem *probs, uint32_t nprob, const uint32_t *chains,
                                   const sa_batch_config *cfg, size_t *bytes)
{
    sa::g_last_error.clear();
    if (!bytes) return fail(SA_ERR_INVALID, "bytes must not be NULL");
    if (sa_status st = validate_batch(probs, nprob, chains, cfg); st != SA_OK) return st;
    BatchPlan pl;
    if (sa_status st = plan_batch(probs, nprob, chains, cfg, kLdsPerWorkgroup, &pl); st != SA_OK) return st;
    *bytes = pl.lay.total;
    return SA_OK;
}

sa_status sa_batch_create(const sa_problem *probs, uint32_t nprob, const uint32_t *chains,
                          const sa_batch_config *cfg, void *stream, void *workspace, size_t ws_bytes,
                          sa_batch **out)
{
    sa::g_last_error.clear();
    if (!out) return fail(SA_ERR_INVALID, "out must not be NULL");
    *out = nullptr;
    if (sa_status st = validate_batch(probs, nprob, chains, cfg); st != SA_OK) return st;
    if (!workspace) SA_FAULT_CHECK(sa::kFaultAlloc);
    int dev = 0;
    SA_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    SA_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SA_ERR_UNSUPPORTED, "device %d is %s; this library is built for gfx950 only", dev,
                    prop.gcnArchName);
    const size_t lds_limit = std::min<size_t>(kLdsPerWorkgroup, prop.sharedMemPerBlock);
    sa_batch *b = new (std::nothrow) sa_batch;
    if (!b) return fail(SA_ERR_NOMEM, "host allocation failed");
    b->device = dev;
    if (hipDeviceGetAttribute(&b->clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) b->clock_khz = 0;
    b->stream = reinterpret_cast<hipStream_t>(stream);
    b->cfg = *cfg;
    b->seed = cfg->seed;
    b->fp64 = cfg->precision == SA_FP64;
    b->lower.resize(nprob);
    b->upper.resize(nprob);
    b->shift.resize(nprob);
    for (uint32_t p = 0; p < nprob; ++p) {
        const sa_problem &P = probs[p];
        b->lower[p].assign(P.lower, P.lower + P.n);
        b->upper[p].assign(P.upper, P.upper + P.n);
        if (P.shift) b->shift[p].assign(P.shift, P.shift + P.n);
        if (!b->fp64) {
            for (uint32_t i = 0; i < P.n; ++i) {
                if (!(sa::round_up_f(P.lower[i]) < sa::round_down_f(P.upper[i]))) {
                    delete b;
                    return fail(SA_ERR_INVALID, "problem %u: box %u is empty after rounding inward to FP32", p, i);
                }
            }
        }
    }
    if (sa_status st = plan_batch(probs, nprob, chains, cfg, lds_limit, &b->pl); st != SA_OK) {
        delete b;
        return st;
    }
    if (workspace) {
        if (ws_bytes < b->pl.lay.total || reinterpret_cast<uintptr_t>(workspace) % kAlign) {
            const size_t need = b->pl.lay.total;
            delete b;
            return fail(SA_ERR_INVALID, "workspace must be %zu-byte aligned and at least %zu bytes", kAlign, need);
        }
        b->ws = static_cast<unsigned char *>(workspace);
    } else {
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&b->ws), b->pl.lay.total);
        if (e != hipSuccess) {
            const size_t need = b->pl.lay.total;
            delete b;
            return fail(SA_ERR_NOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
        }
        b->own_ws = true;
    }
    if (b->fp64)
        fill_batch_args<double>(b, b->a64);
    else
        fill_batch_args<float>(b, b->a32);
    sa_status st = upload_batch(b);
    if (st == SA_OK) st = enqueue_batch_reset(b);
    if (st != SA_OK) {
        sa_batch_destroy(b);
        return st;
    }
    *out = b;
    return SA_OK;
}

sa_status sa_batch_run(sa_batch *b, uint32_t levels)
{
    sa::g_last_error.clear();
    if (!b) return fail(SA_ERR_INVALID, "null batch");
    const uint32_t L = b->cfg.levels;
    if (b->next_level >= L) return fail(SA_ERR_STATE, "all %u levels have run", L);
    const uint32_t count = levels ? levels : L - b->next_level;
    if (count > L - b->next_level)
        return fail(SA_ERR_STATE, "%u levels requested, %u remain", count, L - b->next_level);
    SA_FAULT_CHECK(sa::kFaultLaunch);
    const uint32_t first = b->next_level;
    if (b->cfg.flags & SA_FLAG_GRAPH) {
        const auto key = std::make_pair(first, count);
        auto it = b->graphs.find(key);
        if (it == b->graphs.end()) {
            if (!b->capture) SA_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
            SA_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
            sa_status st = enqueue_batch_levels(b, first, count, b->capture);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->capture, &g);
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
            it = b->graphs.emplace(key, sa_batch::Graph{g, ge}).first;
        }
        SA_HIP(hipGraphLaunch(it->second.exec, b->stream));
    } else {
        if (sa_status st = enqueue_batch_levels(b, first, count, b->stream); st != SA_OK) return st;
    }
    b->next_level = first + count;
    return SA_OK;
}

sa_status sa_batch_reset(sa_batch *b, uint64_t seed)
{
    sa::g_last_error.clear();
    if (!b) return fail(SA_ERR_INVALID, "null batch");
    SA_FAULT_CHECK(sa::kFaultLaunch);
    if (seed != b->seed) {
        drop_batch_graphs(b);
        b->seed = seed;
        b->a32.seed_lo = b->a64.seed_lo = (uint32_t)seed;
        b->a32.seed_hi = b->a64.seed_hi = (uint32_t)(seed >> 32);
    }
    return enqueue_batch_reset(b);
}

sa_status sa_batch_best(sa_batch *b, uint32_t prob, double *x_out, double *f_out, uint32_t *level_found)
{
    sa::g_last_error.clear();
    if (!b) return fail(SA_ERR_INVALID, "null batch");
    if (prob >= b->pl.nprob) return fail(SA_ERR_INVALID, "problem %u out of range", prob);
    if (b->next_level == 0) return fail(SA_ERR_STATE, "no level has run");
    SA_HIP(hipStreamSynchronize(b->stream));
    const BatchLayout &l = b->pl.lay;
    const sa::BatchProblem &P = b->pl.probs[prob];
    double f = 0.0;
    uint32_t lvl = 0;
    SA_HIP(hipMemcpy(&f, b->ws + l.rec + prob * sizeof(double), sizeof f, hipMemcpyDeviceToHost));
    SA_HIP(hipMemcpy(&lvl, b->ws + l.rec_level + prob * sizeof(uint32_t), sizeof lvl, hipMemcpyDeviceToHost));
    if (lvl == 0xFFFFFFFFu) return fail(SA_ERR_STATE, "no record yet");
    if (x_out) {
        if (b->fp64) {
            SA_HIP(hipMemcpy(x_out, b->ws + l.x_rec + (size_t)P.x_off * sizeof(double), P.n * sizeof(double),
                             hipMemcpyDeviceToHost));
        } else {
            std::vector<float> x(P.n);
            SA_HIP(hipMemcpy(x.data(), b->ws + l.x_rec + (size_t)P.x_off * sizeof(float), P.n * sizeof(float),
                             hipMemcpyDeviceToHost));
            for (uint32_t i = 0; i < P.n; ++i) x_out[i] = x[i];
        }
    }
    if (f_out) *f_out = f;
    if (level_found) *level_found = lvl;
    return SA_OK;
}

sa_status sa_batch_trace(sa_batch *b, uint32_t prob, uint32_t first, uint32_t count, sa_level *out,
                         double *x_best)
{
    sa::g_last_error.clear();
    if (!b) return fail(SA_ERR_INVALID, "null batch");
    if (prob >= b->pl.nprob) return fail(SA_ERR_INVALID, "problem %u out of range", prob);
    if (count == 0) return SA_OK;
    if (first >= b->next_level || count > b->next_level - first)
        return fail(SA_ERR_STATE, "levels [%u, %u) have not all run (%u done)", first, first + count,
                    b->next_level);
    if (x_best && !(b->cfg.flags & SA_FLAG_TRACE_X))
        return fail(SA_ERR_STATE, "x_best trace needs SA_FLAG_TRACE_X");
    SA_HIP(hipStreamSynchronize(b->stream));
    if (out) {
        SA_HIP(hipMemcpy(out, b->ws + b->pl.lay.trace + ((size_t)prob * b->cfg.levels + first) * sizeof(sa_level),
                         count * sizeof(sa_level), hipMemcpyDeviceToHost));
        sa::stamps_to_ns(out, count, b->clock_khz);
    }
    if (x_best) {
        const sa::BatchProblem &P = b->pl.probs[prob];
        const size_t base = (size_t)b->cfg.levels * P.x_off + (size_t)first * P.n, m = (size_t)count * P.n;
        if (b->fp64) {
            SA_HIP(hipMemcpy(x_best, b->ws + b->pl.lay.trace_x + base * sizeof(double), m * sizeof(double),
                             hipMemcpyDeviceToHost));
        } else {
            std::vector<float> x(m);
            SA_HIP(hipMemcpy(x.data(), b->ws + b->pl.lay.trace_x + base * sizeof(float), m * sizeof(float),
                             hipMemcpyDeviceToHost));
            for (size_t i = 0; i < m; ++i) x_best[i] = x[i];
        }
    }
    return SA_OK;
}

sa_status sa_batch_move_log(sa_batch *b, sa_move_rec *moves, double *final_f)
{
    sa::g_last_error.clear();
    if (!b) return fail(SA_ERR_INVALID, "null batch");
    if (!b->cfg.log_chains) return fail(SA_ERR_STATE, "the batch was created without a move log");
    SA_HIP(hipStreamSynchronize(b->stream));
    const BatchLayout &l = b->pl.lay;
    if (moves)
        SA_HIP(hipMemcpy(moves, b->ws + l.log,
                         (size_t)b->cfg.log_levels * b->cfg.log_chains * b->cfg.steps * sizeof(sa_move_rec),
                         hipMemcpyDeviceToHost));
    if (final_f)
        SA_HIP(hipMemcpy(final_f, b->ws + l.log_final,
                         (size_t)b->cfg.log_levels * b->pl.probs[b->cfg.log_problem].chains * sizeof(double),
                         hipMemcpyDeviceToHost));
    return SA_OK;
}

sa_status sa_batch_layout(const sa_batch *b, uint32_t *tiles, uint32_t *groups, uint32_t *waves_per_group,
                          uint32_t *lds_bytes)
{
    if (!b) return fail(SA_ERR_INVALID, "null batch");
    if (tiles) *tiles = b->pl.ntiles;
    if (groups) *groups = b->pl.groups;
    if (waves_per_group) *waves_per_group = b->pl.wpg;
    if (lds_bytes) *lds_bytes = (uint32_t)b->pl.lds;
    return SA_OK;
}

sa_status sa_batch_clock(sa_batch *b, uint64_t *ticks, uint32_t first_level, uint32_t levels,
                         uint64_t *ticks_per_s)
{
    sa::g_last_error.clear();
    if (!b) return fail(SA_ERR_INVALID, "null batch");
    if (ticks && (levels == 0 || first_level >= b->cfg.levels || levels > b->cfg.levels - first_level))
        return fail(SA_ERR_INVALID, "clocked levels [%u, %u + %u) must lie inside the %u levels", first_level,
                    first_level, levels, b->cfg.levels);
    if (ticks && reinterpret_cast<uintptr_t>(ticks) % sizeof(uint64_t))
        return fail(SA_ERR_INVALID, "ticks must be 8-byte aligned");
    if (ticks_per_s) {
        int khz = 0;
        SA_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device));
        *ticks_per_s = (uint64_t)khz * 1000u;
    }
    drop_batch_graphs(b);  // captured launches hold the arguments
    b->clock = ticks;
    b->clock_level = ticks ? first_level : 0;
    b->clock_levels = ticks ? levels : 0;
    if (b->fp64)
        fill_batch_args<double>(b, b->a64);
    else
        fill_batch_args<float>(b, b->a32);
    return SA_OK;
}

void sa_batch_destroy(sa_batch *b)
{
    if (!b) return;
    if (b->ws) (void)hipStreamSynchronize(b->stream);
    drop_batch_graphs(b);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->own_ws && b->ws) (void)hipFree(b->ws);
    delete b;
}

sa_status sa_batch_autotune(const sa_problem *probs, uint32_t nprob, const sa_batch_config *cfg, void *stream,
                            uint32_t trial_levels, uint32_t *chains_out, uint32_t *waves_per_group_out,
                            double *moves_per_s_out)
{
    sa::g_last_error.clear();
    if (!probs || !cfg || !chains_out || nprob == 0) return fail(SA_ERR_INVALID, "null or empty arguments");
    if (trial_levels == 0) return fail(SA_ERR_INVALID, "trial_levels must be >= 1");
    std::vector<uint32_t> ones(nprob, 64u);
    if (sa_status st = validate_batch(probs, nprob, ones.data(), cfg); st != SA_OK) return st;

    // Candidate chain assignments: uniform, and proportional to n.
    std::vector<std::vector<uint32_t>> cands;
    for (uint32_t c = 64; c <= 1024; c *= 2) cands.emplace_back(nprob, c);
    double sum_n = 0.0;
    for (uint32_t p = 0; p < nprob; ++p) sum_n += probs[p].n;
    for (double per_problem : {128.0, 256.0, 512.0}) {
        std::vector<uint32_t> v(nprob);
        const double k = per_problem * nprob / sum_n;
        for (uint32_t p = 0; p < nprob; ++p) {
            const double c = k * probs[p].n;
            v[p] = (uint32_t)std::min(1024.0, std::max(64.0, 64.0 * std::round(c / 64.0)));
        }
        cands.push_back(std::move(v));
    }
    // Candidates run as production runs do (graph-replayed levels); the timed
    // window leaves out level 0, whose random starts cost a full evaluation
    // per chain, and each candidate's graphs are captured in an untimed pass
    // over the same chunks first.
    sa_batch_config tc = *cfg;
    tc.levels = std::min(trial_levels, cfg->levels);
    tc.flags = SA_FLAG_GRAPH;
    tc.log_chains = 0;
    const uint32_t head = tc.levels > 1 ? 1u : 0u;  // untimed leading levels of each pass
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    SA_HIP(hipEventCreate(&e0));
    SA_HIP(hipEventCreate(&e1));
    struct Result {
        size_t cand;
        uint32_t wpg;
        double rate;
        uint64_t chains;
    };
    std::vector<Result> res;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        for (uint32_t wpg : {1u, 2u, 4u}) {
            tc.waves_per_group = wpg;
            sa_batch *b = nullptr;
            sa_status st = sa_batch_create(probs, nprob, cands[ci].data(), &tc, stream, nullptr, 0, &b);
            if (st == SA_ERR_UNSUPPORTED) continue;
            if (st != SA_OK) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return st;
            }
            for (int pass = 0; pass < 2 && st == SA_OK; ++pass) {
                if (pass) st = sa_batch_reset(b, tc.seed);
                if (st == SA_OK && head) st = sa_batch_run(b, head);
                if (st == SA_OK && pass && hipEventRecord(e0, s) != hipSuccess) st = fail(SA_ERR_DEVICE, "event record");
                if (st == SA_OK) st = sa_batch_run(b, 0);
                if (st == SA_OK && pass && hipEventRecord(e1, s) != hipSuccess) st = fail(SA_ERR_DEVICE, "event record");
            }
            if (st == SA_OK && hipEventSynchronize(e1) != hipSuccess) st = fail(SA_ERR_DEVICE, "event sync");
            float ms = 0.0f;
            if (st == SA_OK) (void)hipEventElapsedTime(&ms, e0, e1);
            sa_batch_destroy(b);
            if (st != SA_OK) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return st;
            }
            uint64_t chains = 0;
            for (uint32_t c : cands[ci]) chains += c;
            const double moves = (double)chains * tc.steps * (tc.levels - head);
            res.push_back(Result{ci, wpg, ms > 0.0f ? moves / (ms * 1e-3) : 0.0, chains});
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (res.empty()) return fail(SA_ERR_UNSUPPORTED, "no candidate configuration fits this device");
    double best = 0.0;
    for (const Result &r : res) best = std::max(best, r.rate);
    const Result *pick = nullptr;
    for (const Result &r : res) {
        if (r.rate < 0.95 * best) continue;
        if (!pick || r.chains < pick->chains || (r.chains == pick->chains && r.rate > pick->rate)) pick = &r;
    }
    std::copy(cands[pick->cand].begin(), cands[pick->cand].end(), chains_out);
    if (waves_per_group_out) *waves_per_group_out = pick->wpg;
    if (moves_per_s_out) *moves_per_s_out = pick->rate;
    return SA_OK;
}

}  // extern "C"
