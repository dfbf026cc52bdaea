// Internal interface between the host runtime (sa_api.hip) and the kernels
// (sa_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sa.h"

namespace sa {

constexpr int kSchwefel = SA_SCHWEFEL;
constexpr int kRastrigin = SA_RASTRIGIN;
constexpr int kAckley = SA_ACKLEY;
constexpr int kGriewank = SA_GRIEWANK;
constexpr int kLevyMontalvo = SA_LEVY_MONTALVO;
constexpr int kRosenbrock = SA_ROSENBROCK;

// Full evaluation of a state in FP64 arithmetic: the cost and, for Ackley,
// the two sums under its exponentials.
struct Full {
    double f, s1, s2;
};

// A workgroup's candidate at the end of a level: its best chain's carried
// cost and index, the workgroup's accepted moves, and the candidate state's
// full re-evaluation (cost and Ackley's two sums, FP64 arithmetic).
template <typename R> struct Slot {
    R f;
    uint32_t chain;
    uint32_t accepts;
    uint32_t pad;
    double ff, s1, s2;
};

// Arguments of one level launch.  Device pointers point into the context's
// workspace.  R is the state precision (float or double).
// Words of a chain's carried cost state between levels (the most any Cost keeps).
constexpr uint32_t kCostWords = 6;

template <typename R> struct LevelArgs {
    uint32_t n, chains, steps, move;
    uint32_t problem, seed_lo, seed_hi, wg;
    // Box and shift: either one value for every coordinate (table == nullptr)
    // or a table of n entries {l, u, rho, s} (rho = u - l for resampling).
    R lo, hi, rho, sh;
    const R *table;
    float inv_n;
    const double *T;     // T_k, FP64
    const float *inv_T;  // 1 / T_k rounded to FP32
    uint32_t tiles;      // chains / wg
    uint32_t num_cus;    // compute units of the device (grid sizing)
    uint32_t ov_slots;   // overlay layout: table slots per chain (0: dense layout)
    R *x_best;           // n: winner of the last finished level
    Slot<R> *slots;      // 2 x tiles candidates (double-buffered by level parity)
    R *slot_x;           // 2 x tiles x n candidate states
    R *x_rec;            // n
    double *rec;         // {f_rec}
    uint32_t *rec_level;
    // Elitist exchange: the broadcast state is the record.  The record after
    // level m is mirrored in elite_x[(m & 1) n ..] and elite_f[3 (m & 1) ..]
    // (f, s1, s2 of its full evaluation), so that every workgroup of the next
    // launch reads the one the launch before wrote while workgroup 0 writes
    // the other.
    uint32_t elitist;
    R *elite_x;          // 2 x n
    double *elite_f;     // 2 x 3
    // Exchange period (Sec. 2.2): level L > 0 starts from the broadcast winner
    // when exchange > 0 and L % exchange == 0 (exchange = 1: every level);
    // otherwise every chain continues from its own state and carried cost.
    uint32_t exchange;
    R *chain_x;     // n x chains, coordinate-major: chain c's x_i at [i * chains + c]
    R *chain_cost;  // kCostWords x chains: the carried cost state (Cost::save)
    sa_level *trace;     // one per level
    R *trace_x;          // n per level, or nullptr
    sa_move_rec *log;    // move log, or nullptr
    double *log_final;   // per-chain final cost at logged levels
    uint32_t log_chains, log_level, log_levels;
    // Start state: at level start_level (>= 1; ~0 = none) every chain starts
    // from x_start instead of the previous level's winner.
    const R *x_start;
    uint32_t start_level;
    // Learned proposal and capture of accepted moves.
    const float *featT;         // per level: ln(tau T_k), the network's temperature feature
    const unsigned char *net;   // packed network (global memory), learned modes
    float eps;                  // probability of a plain move in the learned mixture
    int net_kind;               // mlp::NetKind of the proposal network (capture: its history features)
    float *cap_rec;             // captured records, 7 floats each
    unsigned long long *cap_count;  // accepted moves seen by the capture
    uint64_t cap_capacity;      // records cap_rec holds
    // Full-evaluation kernel, FP32 runs: Griewank's c_i = 1/(2 pi sqrt(i+1))
    // (n values) and the family's scale (Levy-Montalvo pi/n, Schwefel -1/n,
    // Ackley 1/n).
    const float *gcoef;
    float cscale;
};

// What a level launch does besides the plain steps.
enum LevelMode : int {
    kModePlain = 0,
    kModeLog = 1,       // log every move of the logged chains
    kModeCapture = 2,   // record every accepted move (features, scaled displacement)
    kModeLearn = 3,     // learned-proposal mixture (FP32, radius moves)
    kModeLearnLog = 4,  // learned mixture with the move log
    kModeLearnG = 5,    // learned mixture, Gaussian network kind (GELU)
    kModeLearnLogG = 6, // the same with the move log
};

// Host-side launchers.  A level launch runs one level and publishes one
// candidate per workgroup; *groups returns how many (the next level's launch,
// or the finalising launch, reduces them).
hipError_t launch_level_f32(int func, bool table, int mode, const LevelArgs<float> &a, uint32_t level,
                            uint32_t prev_groups, uint32_t *groups, hipStream_t s);
hipError_t launch_level_f64(int func, bool table, int mode, const LevelArgs<double> &a, uint32_t level,
                            uint32_t prev_groups, uint32_t *groups, hipStream_t s);
// Publish level `level` (trace entry, record, broadcast state) from its candidates.
hipError_t launch_finalize_f32(const LevelArgs<float> &a, uint32_t level, uint32_t groups, hipStream_t s);
hipError_t launch_finalize_f64(const LevelArgs<double> &a, uint32_t level, uint32_t groups, hipStream_t s);
// Reset the record (a kernel, so it can be captured in a graph).
hipError_t launch_reset(double *rec, uint32_t *rec_level, double *elite_f, hipStream_t s);

// Dynamic LDS bytes of a level launch (learn: the packed network as well).
size_t level_lds_bytes(uint32_t n, uint32_t wg, size_t real_size, bool table, bool learn);

// Level launches on the base-plus-overlay state (plain and logged moves).
hipError_t launch_overlay_level_f32(int func, bool table, bool log, const LevelArgs<float> &a, uint32_t level,
                                    uint32_t prev_groups, uint32_t *groups, hipStream_t s);
hipError_t launch_overlay_level_f64(int func, bool table, bool log, const LevelArgs<double> &a, uint32_t level,
                                    uint32_t prev_groups, uint32_t *groups, hipStream_t s);
size_t overlay_lds_bytes(uint32_t n, uint32_t wg, uint32_t slots, size_t real_size, bool table);

// Exchange variants of the level kernel (bit set): the stochastic exchange
// and the best-seen reduction.  Plain or logged moves, dense layout,
// separable families.
constexpr int kVarSos = 1;
constexpr int kVarBest = 2;
hipError_t launch_variant_level_f32(int func, bool table, int var, bool log, const LevelArgs<float> &a,
                                    uint32_t level, uint32_t prev_groups, uint32_t *groups, hipStream_t s);
hipError_t launch_variant_level_f64(int func, bool table, int var, bool log, const LevelArgs<double> &a,
                                    uint32_t level, uint32_t prev_groups, uint32_t *groups, hipStream_t s);
// Dynamic LDS bytes of a variant launch (best_seen: the accept bits and the
// replay lists as well).
size_t variant_lds_bytes(uint32_t n, uint32_t wg, size_t real_size, bool table, bool best_seen, uint32_t steps);

// Level launches with a full re-evaluation per move: the non-separable
// families, and the separable ones when a run asks for it (dense state
// layout; plain and logged moves).
hipError_t launch_coupled_level_f32(int func, bool table, bool log, const LevelArgs<float> &a, uint32_t level,
                                    uint32_t prev_groups, uint32_t *groups, hipStream_t s);
hipError_t launch_coupled_level_f64(int func, bool table, bool log, const LevelArgs<double> &a, uint32_t level,
                                    uint32_t prev_groups, uint32_t *groups, hipStream_t s);

}  // namespace sa

namespace sa {

// ---------------------------------------------------------------------------
// Batched runs: many independent problems, one wave (64 chains) per tile.
// ---------------------------------------------------------------------------
struct BatchProblem {
    uint32_t func, n, chains, first_tile;  // tiles [first_tile, first_tile + chains / 64)
    uint32_t tab_off;                      // first entry of this problem's {l,u,rho,s} table (entries)
    uint32_t x_off;                        // first element of this problem's n-vectors
    float inv_n;
    uint32_t pad;
};

template <typename R> struct BatchArgs {
    uint32_t nprob, ntiles, steps, move;
    uint32_t seed_lo, seed_hi, waves_per_group, levels;
    const BatchProblem *probs;  // nprob
    const uint32_t *tile_prob;  // ntiles: owning problem
    const uint32_t *tile_xoff;  // ntiles: first element of the tile's candidate state
    const uint32_t *wg_tile;    // groups x waves_per_group: tile of each wave (~0 = idle)
    const uint32_t *wg_lds;     // groups x waves_per_group: byte offset of each wave's LDS region
    const R *table;             // sum_p 4 n_p entries {l, u, rho, s}
    const double *T;            // levels
    const float *inv_T;         // levels
    Slot<R> *slots;             // 2 x ntiles
    R *slot_x;                  // 2 x sum over tiles of n
    uint32_t slot_x_stride;     // sum over tiles of n (elements per parity)
    R *x_best;                  // sum_p n_p
    R *x_rec;                   // sum_p n_p
    double *rec;                // nprob
    uint32_t *rec_level;        // nprob
    sa_level *trace;            // nprob x levels
    R *trace_x;                 // levels x n_p per problem (at levels * x_off), or nullptr
    sa_move_rec *log;           // move log of one problem, or nullptr
    double *log_final;          // per-chain final cost of that problem at logged levels
    uint32_t log_problem, log_chains, log_level, log_levels;
    uint64_t *clock;            // per tile and clocked level: start and end wall-clock ticks, or nullptr
    uint32_t clock_level, clock_levels;
};

// Bytes of LDS one wave of a batched launch needs for dimension n.
size_t batch_wave_lds_bytes(uint32_t n, size_t real_size);

hipError_t launch_batch_level_f32(const BatchArgs<float> &a, uint32_t groups, size_t lds, bool log, uint32_t level,
                                  hipStream_t s);
hipError_t launch_batch_level_f64(const BatchArgs<double> &a, uint32_t groups, size_t lds, bool log, uint32_t level,
                                  hipStream_t s);
// max_n: the largest problem dimension (sizes the finalising launch's LDS).
hipError_t launch_batch_finalize_f32(const BatchArgs<float> &a, uint32_t level, uint32_t max_n, hipStream_t s);
hipError_t launch_batch_finalize_f64(const BatchArgs<double> &a, uint32_t level, uint32_t max_n, hipStream_t s);
hipError_t launch_batch_reset(double *rec, uint32_t *rec_level, uint32_t nprob, hipStream_t s);

}  // namespace sa
