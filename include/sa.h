/*
 * sa.h -- C ABI of the MI355X (gfx950) synchronous parallel simulated
 * annealing library (libsa_hip.so).
 *
 * Method: Ferreiro, Garcia, Lopez-Salas, Vazquez, "An efficient implementation
 * of parallel simulated annealing algorithm in GPUs".
 *   - Problem: minimise f over the box I = [l_1,u_1] x ... x [l_n,u_n]
 *     (Sec. 1, eq. (1)).
 *   - Each of `chains` Markov chains runs `steps` Metropolis moves at a fixed
 *     temperature T_k (Sec. 2.1, Steps 2-4; Sec. 2.2.2).  A move changes one
 *     random coordinate (Step 2) and is accepted when dE <= 0 or
 *     U < exp(-dE/T) (eq. (5), Step 3).
 *   - After every level the chain with the lowest final cost is found and its
 *     state starts every chain at the next level (Sec. 2.2.2, synchronous
 *     kernel listing of Sec. 3.3).  T_{k+1} = alpha T_k (Sec. 2.1, Step 5).
 *
 * Fixed readings (the paper leaves them open):
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = (seed low
 *     word, seed high word).  A chain's move stream at a level is the word
 *     sequence of the blocks (b, level, chain, 0 | problem<<8), b = 0, 1, ...
 *     (word i is word i mod 4 of block i/4); move `step` takes words 3 step,
 *     3 step + 1, 3 step + 2 (coordinate, change, acceptance), so four moves
 *     use three blocks.  Start counter = (i/4, 0xFFFFFFFF, chain,
 *     1 | problem<<8), word i mod 4, for coordinate i.
 *     Uniform U = (r >> 8) * 2^-24; coordinate d = (r * n) >> 32.
 *   - Move: x'_d = clamp(x_d + rho_d (2 U1 - 1), l_d, u_d) with
 *     rho_d = radius_frac (u_d - l_d) (SA_MOVE_RADIUS), or
 *     x'_d = l_d + (u_d - l_d) U1 (SA_MOVE_RESAMPLE).
 *   - Level 0 starts every chain at its own uniform random point in the box.
 *   - Winner: lowest final cost, ties to the lowest chain index.  Its state is
 *     re-evaluated in full (in FP64 arithmetic) and that value starts the next
 *     level; the record (x_rec, f_rec) keeps the lowest re-evaluated winner.
 *   - T_k = T0 * alpha * ... * alpha (k products in FP64).
 *   - FP32 runs keep the box rounded inward to FP32, so every state lies in
 *     the true box.
 *
 * Functions (evaluated at y = x - s, s = shift or 0):
 *   SA_SCHWEFEL   f = -(1/n) sum y_i sin(sqrt|y_i|)          (Sec. 4.1, eq. (6))
 *   SA_RASTRIGIN  f = 10 n + sum (y_i^2 - 10 cos(2 pi y_i))  (Appendix, Test 13)
 *   SA_ACKLEY     f = -20 exp(-0.2 sqrt(sum y^2 / n)) - exp(sum cos(2 pi y)/n)
 *                     + 20 + e                                (Appendix, Test 1)
 *   SA_GRIEWANK   f = 1 + sum y_i^2 / 4000 - prod_i cos(y_i / sqrt(i))
 *                                                             (Appendix, Test 8)
 *   SA_LEVY_MONTALVO  f = (pi/n) [10 sin^2(pi w_1) + sum_{i<n} (w_i - 1)^2
 *                     (1 + 10 sin^2(pi w_{i+1})) + (w_n - 1)^2],
 *                     w_i = 1 + (y_i + 1)/4                   (Appendix, Test 10)
 *   SA_ROSENBROCK f = sum_{i<n} [100 (y_{i+1} - y_i^2)^2 + (1 - y_i)^2]
 *                                                             (Appendix, Test 14)
 *   Centre families, d_i = sum_j (y_j - a_ij)^2 over the appendix's tables of
 *   centres a_i and constants c_i, centres in table order:
 *   SA_SHEKEL5, SA_SHEKEL7, SA_SHEKEL10  f = -sum_{i<m} 1 / (d_i + c_i),
 *                     m = 5, 7, 10; n = 4                     (Appendix, Test 18)
 *   SA_FOXHOLES   f = -sum_{i<30} 1 / (d_i + c_i), n <= 10  (Appendix, Test 19)
 *   SA_LANGERMAN  f = -sum_{i<5} c_i exp(-d_i / pi) cos(pi d_i), n <= 10, the
 *                     first five centres and constants of the foxholes
 *                     tables                                  (Appendix, Test 11)
 *   Other n for these: SA_ERR_INVALID.
 * The first three are sums of per-coordinate terms (Ackley through its two
 * sums), so a move updates the cost by the changed coordinate's terms; the
 * others are not, and every move evaluates f(x') in full, as the paper's
 * kernel does for every function (Sec. 3.3).  The printed Griewank form puts
 * the product inside the sum and the printed Rosenbrock form squares
 * (y_{i+1} - y_i); the forms above are the named functions, with the stated
 * minima 0 at y = 0 and 0 at y = (1, ..., 1).  The non-separable families
 * run on the dense state layout with plain or logged moves (not with
 * SA_FLAG_OVERLAY, SA_FLAG_LEARNED, sa_capture or in batches).
 *
 * Conventions for every call:
 *   - Host pointers are read during the call only; the library copies what it
 *     keeps.  Output pointers are caller-owned host memory.
 *   - A context is used from one host thread at a time.
 *   - sa_run only enqueues work on the context's HIP stream.  sa_best,
 *     sa_trace and sa_move_log synchronise that stream.
 *   - Errors: a negative sa_status; sa_last_error() describes the last error
 *     of the calling thread.  No call aborts the process.
 *   - Fault injection, for tests of callers' error paths: with the
 *     environment variable SA_FAULT=alloc every call that would allocate
 *     device memory (sa_create, sa_batch_create without a workspace,
 *     sa_mlp_create, sa_nm_polish without a workspace) returns SA_ERR_NOMEM
 *     once its arguments are validated, before it touches the device; with
 *     SA_FAULT=launch every call that would enqueue kernels (sa_run, sa_reset,
 *     sa_set_proposal, sa_run_static, sa_nm_polish, sa_batch_run,
 *     sa_batch_reset, sa_mlp_grad, sa_mlp_train, sa_mlp_infer) returns
 *     SA_ERR_DEVICE before enqueuing anything and leaves its context as it
 *     was.  The variable is read at every call; other values do nothing.
 *   - Execution: sa_run enqueues one kernel launch per level and one that
 *     publishes the last level; each level's launch reduces the previous
 *     level's per-workgroup candidates to the winner on the device.  There is
 *     no host work and no grid-wide barrier inside a launch.
 *
 * Beyond the paper's single problem with plain moves:
 *   - sa_batch_*: many independent problems of uneven dimension advanced
 *     together, one launch per level, with a measuring autotuner;
 *   - sa_set_proposal / sa_capture / sa_mlp_*: a learned proposal (a small
 *     network trained on the accepted moves the method generates) mixed with
 *     the plain move and corrected by Metropolis-Hastings;
 *   - sa_set_start: a run that starts from a given state at a given level.
 */
#ifndef SA_H
#define SA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SA_ABI_VERSION 1

typedef enum {
    SA_OK = 0,
    SA_ERR_INVALID = -1,     /* bad argument */
    SA_ERR_NOMEM = -2,       /* device or host allocation failed */
    SA_ERR_DEVICE = -3,      /* a HIP call failed */
    SA_ERR_STATE = -4,       /* call not valid in the context's state */
    SA_ERR_UNSUPPORTED = -5  /* valid request the library does not support */
} sa_status;

typedef enum {
    SA_SCHWEFEL = 0,
    SA_RASTRIGIN = 1,
    SA_ACKLEY = 2,
    SA_GRIEWANK = 3,      /* non-separable: every move re-evaluates f in full */
    SA_LEVY_MONTALVO = 4, /* non-separable */
    SA_ROSENBROCK = 5,    /* non-separable */
    SA_SHEKEL5 = 6,       /* non-separable centre families */
    SA_SHEKEL7 = 7,
    SA_SHEKEL10 = 8,
    SA_FOXHOLES = 9,
    SA_LANGERMAN = 10
} sa_func;
typedef enum { SA_FP32 = 0, SA_FP64 = 1 } sa_precision;
typedef enum { SA_MOVE_RADIUS = 0, SA_MOVE_RESAMPLE = 1 } sa_move;

/* One box-constrained problem.  lower/upper: n host doubles each, finite,
 * lower[i] < upper[i].  shift: n host doubles or NULL (zero shift). */
typedef struct {
    uint32_t func; /* sa_func */
    uint32_t n;    /* dimension, >= 1 */
    const double *lower;
    const double *upper;
    const double *shift;
} sa_problem;

/* Annealing schedule and run options. */
typedef struct {
    uint64_t seed;      /* Philox key */
    uint32_t chains;    /* Markov chains, a multiple of 64 */
    uint32_t levels;    /* temperature levels L */
    uint32_t steps;     /* Metropolis steps per chain per level (N) */
    uint32_t precision; /* sa_precision */
    uint32_t move;      /* sa_move */
    uint32_t flags;     /* SA_FLAG_* */
    double T0;          /* T of level 0, > 0 */
    double alpha;       /* cooling factor, 0 < alpha <= 1 */
    double radius_frac; /* move radius as a fraction of u_d - l_d, > 0 */
    /* Move log (verification): moves of chains [0, log_chains) at levels
     * [log_level, log_level + log_levels) are recorded, together with the
     * final cost of every chain at those levels.  log_chains = 0: no log. */
    uint32_t log_chains;
    uint32_t log_level;
    uint32_t log_levels;
    /* Levels between broadcasts of the level winner (Sec. 2.2).  0 or 1: at
     * every level (the synchronous scheme of Sec. 2.2.2); k >= 2: at levels
     * k, 2k, ... (periodic exchange); SA_EXCHANGE_NEVER: never, only the
     * reduction of each level's best for the trace and record (the
     * asynchronous scheme of Sec. 2.2.1).  A level that starts without a
     * broadcast continues every chain from its own state and carried cost,
     * kept in the workspace (chains x (n + 6) reals).  Values other than 0/1
     * need the dense state layout (not SA_FLAG_OVERLAY, not an n that only
     * fits the overlay) and plain or logged moves (not SA_FLAG_LEARNED). */
    uint32_t exchange;
} sa_config;

#define SA_EXCHANGE_NEVER 0xFFFFFFFFu

/* Keep the winner state of every level (sa_trace x_best output). */
#define SA_FLAG_TRACE_X 0x1u
/* Capture the launches of each distinct sa_run (same first level and level
 * count) into a HIP graph once and replay it. */
#define SA_FLAG_GRAPH 0x2u
/* Reserve room for the learned proposal (sa_set_proposal): FP32 and the
 * radius move only; workgroups are sized so the packed network fits in LDS
 * beside the chains' states. */
#define SA_FLAG_LEARNED 0x4u
/* Keep chain states as one shared level-start state per workgroup plus a
 * per-chain table of the coordinates changed this level (chosen anyway when
 * the dense per-chain state does not fit in LDS, e.g. n = 1024 in FP32, or
 * when the tables keep at least twice as many waves in flight on the device,
 * e.g. n = 512 with 131072 chains).  Plain and logged moves only (not with
 * SA_FLAG_LEARNED or sa_capture); results are identical to the dense
 * layout. */
#define SA_FLAG_OVERLAY 0x8u
/* Exchange variants (Sec. 2.2 reads the minimum operator of the synchronous
 * scheme as a deterministic crossover and names a stochastic one without
 * defining it).  Dense state layout, separable families, plain or logged
 * moves (not with SA_FLAG_OVERLAY, SA_FLAG_LEARNED or sa_capture).
 * SA_FLAG_SOS: stochastic exchange.  At a level L > 0 that starts with an
 *   exchange (every level for exchange 0/1, every k-th for k >= 2), chain p
 *   keeps its own final state and carried cost of level L-1 iff
 *   f_p - f_w <= 0 or U < exp(-(f_p - f_w) / T_{L-1}) -- f_w the winner's
 *   carried (reduced) cost, U from word 0 of the Philox block
 *   (0, L, p, 5 | problem<<8) -- and otherwise starts from the winner's state
 *   with its full re-evaluation.  Every chain's state is kept in the
 *   workspace (chains x (n + 6) reals).  The start level of sa_set_start
 *   starts every chain from its state.
 * SA_FLAG_BEST_SEEN: each chain's best-seen state of a level -- the first
 *   state of lowest carried cost among its start state and its states after
 *   each accepted move -- stands in for its final state in the level's
 *   argmin, broadcast and record (sa_trace f_win is its cost; sa_move_log's
 *   final_f holds it).  A chain that continues on its own state continues
 *   from its final state. */
#define SA_FLAG_SOS 0x10u
#define SA_FLAG_BEST_SEEN 0x20u

/* SA_FLAG_ELITIST: an exchange broadcasts the record -- the lowest full
 * re-evaluation of a level winner so far, the first of equal ones, with that
 * full evaluation as the chains' start cost -- instead of the last level's
 * winner (the paper's exchange broadcasts the winner, Sec. 2.2.2; keeping the
 * best point found as the next start is its elitist reading).  The trace's
 * winner fields and x_best still describe each level's winner.  Any state
 * layout and family; not with SA_FLAG_SOS (whose keep test compares a chain
 * with the winner): SA_ERR_UNSUPPORTED; not a flag of sa_batch_config. */
#define SA_FLAG_ELITIST 0x40u

/* SA_FLAG_FULL_EVAL: every move of a separable family (Schwefel, Rastrigin,
 * Ackley) takes its cost increment as f(x') - f(x) with f(x') evaluated in
 * full -- the paper's kernel evaluates f at every neighbour (Sec. 3.3, the
 * synchronous kernel) -- instead of the O(1) increment of the one changed
 * term; each move then reads all n coordinates.  FP64 runs give the same
 * trajectory up to rounding; FP32 runs evaluate the cancellation-free forms
 * (Rastrigin as sum y^2 + 20 sin^2(pi y), Ackley through expm1) on the
 * hardware transcendentals.  The non-separable families always evaluate in
 * full, so the flag changes nothing for them.  Dense state layout, plain or
 * logged moves: not with SA_FLAG_LEARNED, SA_FLAG_OVERLAY, SA_FLAG_SOS,
 * SA_FLAG_BEST_SEEN or sa_capture (SA_ERR_UNSUPPORTED); not a flag of
 * sa_batch_config. */
#define SA_FLAG_FULL_EVAL 0x80u

/* Per-level record returned by sa_trace. */
typedef struct {
    uint32_t win_chain; /* chain index of the level winner */
    uint32_t reserved;
    double f_win;       /* winner's final cost as carried by its chain */
    double f_best;      /* full re-evaluation of the winner (FP64 arithmetic) */
    double f_rec;       /* lowest f_best so far */
    uint64_t accepts;   /* accepted moves over all chains */
    uint64_t t_ns;      /* when the level's record was written, in ns of the device's constant clock */
} sa_level;

/* One logged move (sa_move_log).  In FP32 runs the values are the FP32
 * quantities the device used, widened to double. */
typedef struct {
    uint32_t d;      /* coordinate */
    uint32_t accept; /* 1 if taken */
    double x_old;    /* x_d before the move */
    double x_new;    /* proposed x'_d (after clamping; a learned proposal
                        outside the box is logged as drawn, with accept 0
                        and df 0) */
    double df;       /* cost increment the device computed */
} sa_move_rec;

typedef struct sa_ctx sa_ctx;

/* Bytes of device workspace sa_create needs for this problem and config:
 * the states of the parallel chains of Sec. 2.2, their per-level
 * candidates and records (Sec. 2.2.2), and the level tables. */
sa_status sa_workspace_bytes(const sa_problem *prob, const sa_config *cfg, size_t *bytes);

/*
 * Create a context for one problem on the current HIP device: the
 * box-constrained minimisation of Sec. 1 with the schedule parameters of the
 * algorithm of Sec. 2.1 (T0, rho, N steps per level) and the chain count of
 * the parallel versions (Sec. 2.2).
 *   stream:    hipStream_t to enqueue on (NULL = the null stream); not owned.
 *   workspace: device memory of at least sa_workspace_bytes bytes, 256-byte
 *              aligned, owned by the caller and kept alive until sa_destroy;
 *              NULL = the library allocates and frees its own.
 * The run starts at level 0 with an empty record.  *out is set on success.
 */
sa_status sa_create(const sa_problem *prob, const sa_config *cfg, void *stream, void *workspace,
                    size_t ws_bytes, sa_ctx **out);

/* Enqueue the next `levels` levels (0 = all remaining): at each, every
 * chain runs N steps of Sec. 2.1 (Steps 2-4) at T_k = T0 rho^k, then the
 * level's best state is exchanged per cfg->exchange (Sec. 2.2.2; 1 = the
 * synchronous scheme, never = the asynchronous one of Sec. 2.2.1).
 * SA_ERR_STATE if the run already finished or `levels` passes cfg->levels. */
sa_status sa_run(sa_ctx *ctx, uint32_t levels);

/* Restart at level 0 (Sec. 2.1 Step 1: new random starts) with an empty
 * record and a new seed (enqueued). */
sa_status sa_reset(sa_ctx *ctx, uint64_t seed);

/* Levels enqueued so far. */
sa_status sa_levels_done(const sa_ctx *ctx, uint32_t *levels);

/* Record after the enqueued levels: the best point found, the method's
 * result (Sec. 2.1, Sec. 2.2.2) (synchronises).  x_out: n doubles;
 * f_out: f(x_rec) in FP64 arithmetic; level_found: level that set it.
 * SA_ERR_STATE before the first level has run.  Any output may be NULL. */
sa_status sa_best(sa_ctx *ctx, double *x_out, double *f_out, uint32_t *level_found);

/* Per-level records of levels [first, first + count): each level's
 * exchanged state and the record so far, the data of the convergence curves
 * of Sec. 4.1 (synchronises).  x_best: count * n doubles or NULL; needs
 * SA_FLAG_TRACE_X. */
sa_status sa_trace(sa_ctx *ctx, uint32_t first, uint32_t count, sa_level *out, double *x_best);

/* Logged moves, every step of Sec. 2.1 Steps 2-3 of the logged chains (for
 * verification; synchronises).  moves: log_levels * log_chains * steps
 * records, index ((level - log_level) * log_chains + chain) * steps + step;
 * final_f: log_levels * chains doubles, index (level - log_level) * chains +
 * chain.  Either may be NULL. */
sa_status sa_move_log(sa_ctx *ctx, sa_move_rec *moves, double *final_f);

/* Start the run at `level` (1 <= level < cfg->levels) with every chain at x
 * -- the state the exchange of Sec. 2.2.2 broadcasts at a level's start --
 * (n doubles inside the box; FP32 runs round them to FP32, kept inside the
 * inward-rounded box), instead of the random starts of level 0: the levels
 * before `level` are skipped and the record starts empty.  With an exchange
 * period other than 1, `level` starts every chain from x and the later
 * levels follow the period (chains keep their own states until its next
 * multiple).  Only before the first sa_run (or after sa_reset, which clears
 * it).  Synchronises. */
sa_status sa_set_start(sa_ctx *ctx, uint32_t level, const double *x);

/*
 * Learned proposal (an extension of the method, not in the paper).  With
 * params (SA_MLP_PARAMS host floats, the network of sa_mlp_*) every later
 * move is, with probability eps, the plain radius move with the Metropolis
 * test, and otherwise a draw from the network's Cauchy distribution over the
 * chosen coordinate's scaled displacement, dl = mu + exp(s) t (t standard
 * Cauchy, tan(pi (U - 1/2)) with U from word 0 of the Philox block
 * (step, level, chain, 3 | problem << 8)),
 * x'_d = x_d + dl (u_d - l_d); a proposal outside [l_d, u_d] is rejected, and
 * otherwise it is taken iff U < exp(-df/T + ln q(x | x') - ln q(x' | x))
 * (Metropolis-Hastings with the network evaluated at x_d and at x'_d, both
 * with the chain's current history: exact for a network that ignores the
 * history features; with them the chain is adaptive, since an accepted move
 * changes the history the next proposal sees, and exp(-f/T) is invariant only
 * approximately); the change and acceptance uniforms of
 * either component are the move's words of the plain move stream.  The
 * plain/learned choice is U < eps with U from word 1 of the learned block.
 * The history (last four accepted scaled displacements,
 * most recent first) restarts at zero at every level.  params = NULL returns
 * to plain moves.  Needs SA_FLAG_LEARNED; SA_ERR_STATE while capturing.
 * Synchronises.
 */
sa_status sa_set_proposal(sa_ctx *ctx, const float *params, float eps);

/* Kinds of proposal network (the learned-proposal configuration that names
 * GELU and a Gaussian output beside the relu/Cauchy network above):
 *   SA_NET_RELU_CAUCHY  as described above (the default);
 *   SA_NET_GELU_GAUSS   GELU hidden activations, x Phi(x) (Phi the standard
 *                       normal distribution function; FP32 on the device, by
 *                       the rational approximation 26.2.17 of Abramowitz and
 *                       Stegun, then rounded to BF16), a Gaussian over the
 *                       scaled displacement with mean mu and standard
 *                       deviation exp(s) (t = sqrt(-2 ln(1 - U0)) cos(2 pi U2)
 *                       from words 0 and 2 of the learned block, Box-Muller),
 *                       the history's scaled displacements entered as they
 *                       are, and the temperature feature ln T (tau = 1). */
#define SA_NET_RELU_CAUCHY 0
#define SA_NET_GELU_GAUSS 1

/* Select the kind of network the context's learned levels evaluate and the
 * features its captures record (history form, temperature feature); the
 * parameters set by sa_set_proposal are read under the kind in force when a
 * level runs.  SA_ERR_INVALID for an unknown kind; SA_ERR_STATE while
 * capturing.  Synchronises. */
sa_status sa_set_network_kind(sa_ctx *ctx, int kind);

/* Record every accepted move of the following plain levels into `records`
 * (device memory, capacity x 7 floats: the six network features at the old
 * state -- (x_d - l_d)/(u_d - l_d), ln(tau T), the history features of the
 * chain's last four accepted scaled displacements -- and the accepted scaled
 * displacement
 * (x'_d - x_d)/(u_d - l_d)).  Records go to slots in the order the device
 * reserves them; once `capacity` are taken, later ones are counted but not
 * stored.  Resets the count.  records = NULL stops capturing.  SA_ERR_STATE
 * while a proposal network is set. */
sa_status sa_capture(sa_ctx *ctx, float *records, uint64_t capacity);

/* Accepted moves the capture has seen since sa_capture (synchronises); the
 * records stored are min(count, capacity). */
sa_status sa_capture_count(sa_ctx *ctx, uint64_t *count);

/* Layout the context launches with (the blocks and threads of Sec. 3.3 on
 * this device): lanes per workgroup, overlay table slots
 * per chain (0 = dense per-chain state), and chain tiles (chains / workgroup).
 * Any output may be NULL. */
sa_status sa_layout(const sa_ctx *ctx, uint32_t *workgroup, uint32_t *overlay_slots, uint32_t *tiles);

/* Release the context and any memory the library allocated (no passage of
 * the paper: resource ownership). */
void sa_destroy(sa_ctx *ctx);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one whole
 * run -- sa_create, sa_run of every level, sa_best and sa_destroy in one call
 * -- with the workspace in a file-scope device array of
 * SA_STATIC_SCRATCH_BYTES per GPU (held by each GPU the library runs on
 * until the process ends) instead of allocated memory.  The call makes no
 * hipMalloc/hipFree and no host heap allocation; it enqueues on `stream`
 * (NULL = the null stream), synchronises it, and writes the record as
 * sa_best does: x_out (n doubles), f_out, level_found (any may be NULL).
 * Results equal those of sa_create + sa_run(ctx, 0) + sa_best on the same
 * problem and config (the same kernels and launches).
 * Limits: n <= SA_STATIC_MAX_N, levels <= SA_STATIC_MAX_LEVELS, a workspace
 * (sa_workspace_bytes) of at most SA_STATIC_SCRATCH_BYTES, flags 0 or
 * SA_FLAG_OVERLAY, log_chains = 0; otherwise SA_ERR_UNSUPPORTED with the
 * reason in sa_last_error().  Every call on a GPU shares that GPU's array,
 * which keeps the last call's contents (each call clears what it reads
 * before writing it).  Calls are serialised within a process; calls from
 * different processes on one GPU use different arrays.
 */
#define SA_STATIC_SCRATCH_BYTES ((size_t)8 << 20)
#define SA_STATIC_MAX_N 4096u
#define SA_STATIC_MAX_LEVELS 16384u
sa_status sa_run_static(const sa_problem *prob, const sa_config *cfg, void *stream, double *x_out, double *f_out,
                        uint32_t *level_found);

/* ------------------------------------------------------------------------
 * Batched runs: nprob independent problems (each with its own function,
 * dimension, box, shift and chain count) advance together, one launch per
 * level.  Problem p draws its randoms with `problem` = p in the counters
 * above, so problem p of a batch follows the same trajectory as a
 * single-problem run of it with problem id p.  Chains of problem p are
 * numbered 0 .. chains[p]-1.
 * ------------------------------------------------------------------------ */
typedef struct {
    uint64_t seed;
    uint32_t levels, steps;
    uint32_t precision; /* sa_precision */
    uint32_t move;      /* sa_move */
    uint32_t flags;     /* SA_FLAG_GRAPH, SA_FLAG_TRACE_X */
    uint32_t waves_per_group; /* 64-chain tiles per workgroup: 1, 2 or 4 (0 = 4) */
    double T0, alpha, radius_frac;
    /* Move log of one problem (verification), as in sa_config. */
    uint32_t log_problem, log_chains, log_level, log_levels;
} sa_batch_config;

typedef struct sa_batch sa_batch;

/* Workspace bytes for these problems with chains[p] chains each
 * (multiples of 64, >= 64). */
sa_status sa_batch_workspace_bytes(const sa_problem *probs, uint32_t nprob, const uint32_t *chains,
                                   const sa_batch_config *cfg, size_t *bytes);

/* Create a batch of independent problems of Sec. 1, each annealed by the
 * synchronous scheme of Sec. 2.2.2 (same stream/workspace conventions as
 * sa_create).  probs: nprob host problems; chains: nprob chain counts (see
 * sa_batch_autotune). */
sa_status sa_batch_create(const sa_problem *probs, uint32_t nprob, const uint32_t *chains,
                          const sa_batch_config *cfg, void *stream, void *workspace, size_t ws_bytes,
                          sa_batch **out);

/* Enqueue the next `levels` levels of every problem (0 = all remaining), as
 * sa_run for each. */
sa_status sa_batch_run(sa_batch *b, uint32_t levels);

/* Restart every problem at level 0 with a new seed (enqueued), as sa_reset. */
sa_status sa_batch_reset(sa_batch *b, uint64_t seed);

/* Record of problem p (synchronises), as sa_best. */
sa_status sa_batch_best(sa_batch *b, uint32_t prob, double *x_out, double *f_out, uint32_t *level_found);

/* Per-level records of problem p, levels [first, first + count) (synchronises).
 * x_best: count * n_p doubles or NULL; needs SA_FLAG_TRACE_X. */
sa_status sa_batch_trace(sa_batch *b, uint32_t prob, uint32_t first, uint32_t count, sa_level *out,
                         double *x_best);

/* Logged moves of cfg->log_problem (synchronises), layout as sa_move_log with
 * chains = chains[log_problem]. */
sa_status sa_batch_move_log(sa_batch *b, sa_move_rec *moves, double *final_f);

/* Layout the batch runs with: 64-chain tiles, workgroups per launch, tiles
 * per workgroup, dynamic LDS bytes per workgroup.  Any output may be NULL. */
sa_status sa_batch_layout(const sa_batch *b, uint32_t *tiles, uint32_t *groups, uint32_t *waves_per_group,
                          uint32_t *lds_bytes);

/* Clock of the batched levels (measurement of how long each problem's
 * tiles wait for the level's slowest problem; no passage of the paper: the
 * batch has no counterpart there).  For levels [first_level, first_level +
 * levels) of later runs, every 64-chain tile records the device wall clock
 * when its wave starts the level and when it has published its candidate:
 * ticks (device memory, 8-byte aligned, levels x tiles x 2 uint64, index
 * ((level - first_level) * tiles + tile) * 2 + {0 = start, 1 = end}; tiles
 * as sa_batch_layout reports, tile t of problem p being the t - (first tile
 * of p)-th 64-chain group of p, tiles numbered problem by problem).
 * *ticks_per_s (may be NULL) returns the clock's rate.  ticks = NULL stops
 * recording.  Drops captured graphs (their launches hold the arguments).
 * SA_ERR_INVALID for levels outside the schedule. */
sa_status sa_batch_clock(sa_batch *b, uint64_t *ticks, uint32_t first_level, uint32_t levels, uint64_t *ticks_per_s);

void sa_batch_destroy(sa_batch *b);

/*
 * Autotuner: pick chains per problem and tiles per workgroup by measurement
 * on the current device (the chain-count question the paper studies by
 * sweeping the number of launched threads, Sec. 4.1, answered per problem).  Candidates: uniform chain counts 64..1024 and
 * counts proportional to each problem's dimension (64..1024, multiples of
 * 64), each with 1, 2 and 4 tiles per workgroup.  Each candidate runs
 * `trial_levels` levels of cfg's schedule twice with graph-replayed levels
 * (SA_FLAG_GRAPH; the first pass captures the graphs); the second pass is
 * timed with HIP events from level 1 on (level 0's random starts cost a full
 * evaluation per chain, which later levels do not pay; with trial_levels = 1
 * level 0 is timed).  The choice is the candidate with the fewest total chains whose
 * moves/s is within 5% of the best measured.  Writes nprob chain counts to
 * chains_out, the tiles per workgroup to *waves_per_group_out and the chosen
 * candidate's moves/s to *moves_per_s_out (any may be NULL except
 * chains_out).  Allocates and frees its own device memory.
 */
sa_status sa_batch_autotune(const sa_problem *probs, uint32_t nprob, const sa_batch_config *cfg, void *stream,
                            uint32_t trial_levels, uint32_t *chains_out, uint32_t *waves_per_group_out,
                            double *moves_per_s_out);

/* ------------------------------------------------------------------------
 * Nelder-Mead polish (the paper's hybrid strategy: a local minimizer started
 * where the annealing stopped, Sec. 4.2, hybrid results table).  The paper
 * names the method only; the steps are the standard simplex method with
 * reflection 1, expansion 2, contraction 1/2 and shrink 1/2 (Lagarias, Reeds,
 * Wright, Wright, SIAM J. Optim. 9, 1998), each trial point projected onto
 * the box.  Start simplex: x0 and x0 + h_i e_i, h_i = x0_i / 20 (0.00025 if
 * x0_i = 0), reflected to x0 - h_i e_i where that leaves the box.  Per
 * iteration b = lowest cost, w = highest among the others, s = highest among
 * all but w (ties to the lowest vertex); stop when f_w - f_b <= ftol and every
 * vertex is within xtol of x_b in every coordinate, or after maxiter
 * iterations.  FP64 arithmetic, costs summed in coordinate order.
 * ------------------------------------------------------------------------ */
typedef struct {
    uint32_t maxiter;   /* iteration cap */
    uint32_t log_steps; /* nonzero: record each iteration's step code */
    double ftol, xtol;  /* termination tolerances, >= 0 */
} sa_nm_config;

/* Nelder-Mead step codes in the step log. */
#define SA_NM_REFLECT 0
#define SA_NM_EXPAND 1
#define SA_NM_OUTSIDE 2
#define SA_NM_INSIDE 3
#define SA_NM_SHRINK 4

/* Bytes of device workspace sa_nm_polish needs. */
sa_status sa_nm_workspace_bytes(const sa_problem *prob, uint32_t starts, const sa_nm_config *cfg, size_t *bytes);

/* Polish `starts` start points at once (one wave each) on the current HIP
 * device.  x0: starts x n host doubles inside the box.  workspace: device
 * memory of sa_nm_workspace_bytes bytes, 256-byte aligned (NULL = the
 * library allocates and frees it).  Outputs (host, any may be NULL): x_out
 * starts x n (each start's lowest vertex at the end), f_out (its cost),
 * iters_out, evals_out (iterations and cost evaluations), step_log (starts x
 * maxiter codes, needs cfg->log_steps; entries past iters_out are unset).
 * n <= 2048.  Synchronises `stream`. */
sa_status sa_nm_polish(const sa_problem *prob, const double *x0, uint32_t starts, const sa_nm_config *cfg,
                       void *stream, void *workspace, size_t ws_bytes, double *x_out, double *f_out,
                       uint32_t *iters_out, uint32_t *evals_out, uint8_t *step_log);

/* The k lowest-cost candidates of the last level enqueued, lowest first
 * (each the best chain of one workgroup's tiles, by the cost its chain
 * carried; ties to the lower chain): the start points of a polish from the
 * top k chains (synchronises).  x_out: k x n doubles; f_out: k full FP64
 * re-evaluations; chains_out: k chain indices.  k must not exceed the number
 * of candidates the level published (*available, which may be NULL, returns
 * it; k = 0 only queries).  Any output may be NULL. */
sa_status sa_candidates(sa_ctx *ctx, uint32_t k, double *x_out, double *f_out, uint32_t *chains_out,
                        uint32_t *available);

/* Description of the calling thread's last error ("" if none). */
const char *sa_last_error(void);

/* ------------------------------------------------------------------------
 * Learned proposal network (an extension of the method; not in the paper):
 * per chosen coordinate, features z = ((x_d - l_d)/(u_d - l_d), ln(tau T),
 * the chain's last four accepted scaled displacements h, most recent first,
 * each as sign(h) ln(1 + 2^24 |h|) / 16; tau = n for Schwefel and Ackley, 1
 * for Rastrigin) -> 128 (relu) -> 128
 * (relu) -> (mu, s): a Cauchy distribution with location mu and scale
 * exp(s) over the coordinate's scaled displacement (x'_d - x_d)/(u_d - l_d).
 * Parameters: SA_MLP_PARAMS floats, W1[6][128], b1[128], W2[128][128],
 * b2[128], W3[128][2], b3[2].  Training minimises the mean Cauchy negative
 * log-likelihood s + ln pi + ln(1 + ((d - mu)/exp(s))^2) of captured accepted
 * displacements d with Adam (FP32 master
 * weights, BF16 weight matrices, BF16 MFMA with FP32 accumulate).
 * Captured records: 7 floats each, (z[0..5], d).
 * ------------------------------------------------------------------------ */
#define SA_MLP_PARAMS 17666

typedef struct sa_mlp sa_mlp;

/* Trainer for minibatches of up to max_batch records (a multiple of 32);
 * allocates its own device memory; parameters start at zero. */
sa_status sa_mlp_create(uint32_t max_batch, void *stream, sa_mlp **out);

/* Load host parameters (SA_MLP_PARAMS floats) and reset the optimiser. */
sa_status sa_mlp_set_params(sa_mlp *m, const float *params);

/* Copy the FP32 master parameters to the host (synchronises). */
sa_status sa_mlp_get_params(sa_mlp *m, float *params);

/* Gradient of the mean loss over records[idx[0..batch)] (records: device
 * pointer to nrec x 7 floats; idx: host indices < nrec; batch a multiple of
 * 32).  Writes SA_MLP_PARAMS floats to the host array grad and the mean loss
 * to *loss (either may be NULL).  Synchronises. */
sa_status sa_mlp_grad(sa_mlp *m, const float *records, uint64_t nrec, const uint32_t *idx, uint32_t batch,
                      float *grad, float *loss);

/* `steps` Adam steps (lr; beta1 0.9, beta2 0.999, eps 1e-8) on minibatches of
 * `batch` records drawn with replacement by Philox counters under `seed`.
 * loss_trace: `steps` host floats (each minibatch's mean loss) or NULL. */
sa_status sa_mlp_train(sa_mlp *m, const float *records, uint64_t nrec, uint32_t batch, uint32_t steps, float lr,
                       uint64_t seed, float *loss_trace);

/* Network kind (SA_NET_*) the trainer's forward pass, loss and inference use:
 * SA_NET_GELU_GAUSS trains GELU activations under the mean Gaussian negative
 * log-likelihood s + ln sqrt(2 pi) + ((d - mu)/exp(s))^2 / 2.  Default
 * SA_NET_RELU_CAUCHY.  SA_ERR_INVALID for an unknown kind. */
sa_status sa_mlp_set_kind(sa_mlp *m, int kind);

/* Evaluate the network at the current parameters for `rows` feature vectors
 * Z (device, rows x 6 floats) into out (device, rows x 2 floats: mu, s),
 * asynchronously on the trainer's stream, with the same BF16-MFMA wave
 * routine the annealing kernels run: weight matrices and hidden activations
 * in BF16, features to about 16 bits (BF16 high part plus BF16 remainder),
 * biases and accumulation in FP32. */
sa_status sa_mlp_infer(sa_mlp *m, const float *Z, uint32_t rows, float *out);

void sa_mlp_destroy(sa_mlp *m);

#ifdef __cplusplus
}
#endif

#endif /* SA_H */
