/*
 * FP64 CPU oracle for synchronous parallel simulated annealing.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header or constant table with the GPU library, and the GPU library
 * never calls it.
 *
 * What it follows (Ferreiro, Garcia, Lopez-Salas, Vazquez, "An efficient
 * implementation of parallel simulated annealing algorithm in GPUs"):
 *   - the box-constrained problem min f(x), x in I = [l_1,u_1] x ... x [l_n,u_n]
 *     (Sec. 1, eq. (1));
 *   - Metropolis acceptance with k_b = 1: a move with energy increment dE is
 *     taken when dE < 0, otherwise with probability exp(-dE/T)
 *     (Sec. 2.1, eqs. (4)-(5) and Steps 1-5);
 *   - geometric cooling T_{k+1} = rho * T_k (Sec. 2.1, Step 5);
 *   - a neighbour that changes one randomly chosen coordinate, three uniforms
 *     per move (Sec. 2.1, Step 2 and Step 3);
 *   - the synchronous multiple-Markov-chain scheme: every chain runs N
 *     Metropolis steps at a fixed T, the chain with the lowest final cost is
 *     selected and its state is the start of every chain at the next level
 *     (Sec. 2.2.2 and the synchronous kernel listing of Sec. 3.3);
 *   - the asynchronous scheme (no exchange; Sec. 2.2.1) as a switch;
 *   - the test functions: normalized Schwefel (Sec. 4.1, eq. (6)), Ackley
 *     (Appendix, Test 1) and Rastrigin (Appendix, Test 13).
 *
 * Readings where the paper is silent (all are stated again, with reasons, in
 * the project design notes):
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
 *     (seed_lo, seed_hi); the move stream of a chain at a level is the word
 *     sequence of the blocks (b, level, chain, tag | problem<<8), b = 0, 1, ...
 *     (word i of the stream is word i mod 4 of block i / 4), and move `step`
 *     takes its words 3 step, 3 step + 1, 3 step + 2 (coordinate, change,
 *     acceptance); uniform U = (r >> 8) * 2^-24; coordinate d = (r * n) >> 32;
 *   - neighbour: x'_d = clamp(x_d + rho_d (2U - 1), l_d, u_d),
 *     rho_d = radius_frac (u_d - l_d); or resampling x'_d = l_d + (u_d - l_d) U;
 *   - accept iff dE <= 0 or U2 < exp(-dE/T);
 *   - the level winner is the lowest final cost, ties to the lowest chain;
 *   - the winner is re-evaluated in full; the record keeps the lowest such
 *     value (strictly lower replaces);
 *   - temperatures: T_0 = T0, T_{k+1} = T_k * alpha, repeated FP64 products.
 *
 * Cost increments: for a separable cost only the changed coordinate's term is
 * re-evaluated (the increment is mathematically f(x') - f(x)); for Ackley the
 * two sums under the exponentials are updated and f is re-formed from them.
 *
 * Build: gcc -O2 -shared -fPIC -fno-fast-math -ffp-contract=off -lm -lpthread
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SCHWEFEL 0
#define ORC_RASTRIGIN 1
#define ORC_ACKLEY 2
#define ORC_GRIEWANK 3
#define ORC_LEVY_MONTALVO 4
#define ORC_ROSENBROCK 5
#define ORC_SHEKEL5 6
#define ORC_SHEKEL7 7
#define ORC_SHEKEL10 8
#define ORC_FOXHOLES 9
#define ORC_LANGERMAN 10

#define ORC_TAG_MOVE 0u
#define ORC_TAG_INIT 1u
#define ORC_TAG_SOS 5u

/* Variants of the multi-chain run (orc_sa_run_v).
 *   ORC_VARIANT_SOS: stochastic exchange.  The paper's synchronous scheme
 *     reads its minimum operator as a deterministic crossover and names a
 *     stochastic crossover (the SOS scheme of its reference) without defining
 *     it (Sec. 2.2).  Reading taken: at a level that starts with an exchange,
 *     chain p keeps its own state and carried cost with the Metropolis
 *     probability exp(-(f_p - f_w) / T_prev) -- f_p its final cost, f_w the
 *     winner's reduced cost, T_prev the temperature of the level that ended --
 *     and otherwise starts from the winner's state with its full
 *     re-evaluation; the uniform is word 0 of the Philox block (0, level,
 *     chain, 5 | problem << 8) and the test is orc_accept's.  T_prev -> 0
 *     gives the minimum operator for every chain worse than the winner,
 *     T_prev -> infinity the asynchronous scheme.
 *   ORC_VARIANT_BEST_SEEN: each chain's best-seen state of the level (the
 *     first state of lowest carried cost among its start state and its states
 *     after each accepted move) stands in for its final state in the level's
 *     argmin, broadcast and record; a chain that continues on its own state
 *     continues from its final state.
 *   ORC_VARIANT_ELITIST: the state broadcast at an exchange is the record
 *     (the lowest fully re-evaluated level winner so far, the first of equal
 *     ones) instead of the last level's winner (Sec. 2.2.2 broadcasts the
 *     winner; keeping the best point found as the next start is the elitist
 *     reading of the same exchange).  Not defined together with
 *     ORC_VARIANT_SOS, whose keep test compares against the winner. */
#define ORC_VARIANT_SOS 1u
#define ORC_VARIANT_BEST_SEEN 2u
#define ORC_VARIANT_ELITIST 4u
/*   ORC_VARIANT_FULL: every move's cost is f evaluated in full at the moved
 *     state (Sec. 2.1 Step 3 compares f(x1) with f(x0); the paper's kernel
 *     evaluates f(x1) whole), not the separable families' increment of the
 *     changed term.  Non-separable families are evaluated in full anyway. */
#define ORC_VARIANT_FULL 8u

#define ORC_MOVE_RADIUS 0
#define ORC_MOVE_RESAMPLE 1

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 3 and Table 2).                  */
/* Round: (hi0,lo0) = M0*c0, (hi1,lo1) = M1*c2,                              */
/*        c' = (hi1^c1^k0, lo1, hi0^c3^k1, lo0); key += (W0, W1) between      */
/*        rounds.                                                            */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in [0,1) from the top 24 bits of a 32-bit word. */
double orc_uniform(uint32_t r) { return (double)(r >> 8) * 0x1p-24; }

/* Coordinate index in [0,n). */
uint32_t orc_pick(uint32_t r, uint32_t n) { return (uint32_t)(((uint64_t)r * (uint64_t)n) >> 32); }

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Word i of the move stream of one chain at one level: word i mod 4 of the
 * block with counter (i / 4, level, chain, MOVE | problem << 8). */
/* Uniform of the stochastic exchange decision of `chain` at the start of `level`. */
double orc_sos_uniform(uint64_t seed, uint32_t problem, uint32_t level, uint32_t chain)
{
    uint32_t r[4];
    draw(seed, 0u, level, chain, ORC_TAG_SOS | (problem << 8), r);
    return orc_uniform(r[0]);
}

static uint32_t move_word(uint64_t seed, uint32_t problem, uint32_t level, uint32_t chain, uint64_t i)
{
    uint32_t r[4];
    draw(seed, (uint32_t)(i >> 2), level, chain, ORC_TAG_MOVE | (problem << 8), r);
    return r[i & 3u];
}

/* The three random numbers of one move (Sec. 2.1, Step 3): coordinate,
 * change, acceptance -- words 3 step, 3 step + 1 and 3 step + 2 of the move
 * stream (so four moves take three blocks). */
void orc_move_draw(uint64_t seed, uint32_t problem, uint32_t level, uint32_t chain, uint32_t step,
                   uint32_t n, uint32_t *d, double *u1, double *u2)
{
    const uint64_t i = 3u * (uint64_t)step;
    *d = orc_pick(move_word(seed, problem, level, chain, i), n);
    *u1 = orc_uniform(move_word(seed, problem, level, chain, i + 1u));
    *u2 = orc_uniform(move_word(seed, problem, level, chain, i + 2u));
}

/* Random start of one chain (Sec. 2.2.2: threads start from a random initial
 * solution): x_i = l_i + (u_i - l_i) U_i, U_i from counter
 * (i/4, 0xFFFFFFFF, chain, INIT | problem<<8), word i%4. */
void orc_init_point(uint64_t seed, uint32_t problem, uint32_t chain, uint32_t n,
                    const double *lower, const double *upper, double *x)
{
    uint32_t r[4];
    for (uint32_t i = 0; i < n; ++i) {
        if ((i & 3u) == 0) draw(seed, i >> 2, 0xFFFFFFFFu, chain, ORC_TAG_INIT | (problem << 8), r);
        double u = orc_uniform(r[i & 3u]);
        double xi = lower[i] + (upper[i] - lower[i]) * u;
        if (xi > upper[i]) xi = upper[i];
        if (xi < lower[i]) xi = lower[i];
        x[i] = xi;
    }
}

/* ------------------------------------------------------------------------ */
/* Test functions, evaluated at y = x - s (s = 0 when no shift is given).     */
/* ------------------------------------------------------------------------ */
static const double ORC_PI = 3.14159265358979323846;
static const double ORC_E = 2.71828182845904523536;

/* One term of the normalized Schwefel function (Sec. 4.1, eq. (6)) before
 * the -1/n factor is applied: y sin(sqrt|y|). */
double orc_schwefel_term(double y) { return y * sin(sqrt(fabs(y))); }

/* One term of the Rastrigin sum (Appendix, Test 13): y^2 - 10 cos(2 pi y). */
double orc_rastrigin_term(double y) { return y * y - 10.0 * cos(2.0 * ORC_PI * y); }

/* Ackley (Appendix, Test 1) from its two sums S1 = sum y^2, S2 = sum cos(2 pi y). */
double orc_ackley_from_sums(double s1, double s2, uint32_t n)
{
    double dn = (double)n;
    return -20.0 * exp(-0.2 * sqrt(s1 / dn)) - exp(s2 / dn) + 20.0 + ORC_E;
}

static double shifted(const double *x, const double *s, uint32_t i) { return s ? x[i] - s[i] : x[i]; }

/* Coordinate i of y = x - s, with coordinate d replaced by xdn when d < n. */
static double y_at(const double *x, const double *s, uint32_t i, uint32_t d, double xdn)
{
    const double v = i == d ? xdn : x[i];
    return s ? v - s[i] : v;
}

/*
 * Tables of the centre families (Appendix: Test 18 Shekel, Test 19 modified
 * Shekel foxholes, Test 11 modified Langerman), as printed there: row i is
 * centre a_i, c_i its offset (Shekel, foxholes) or weight (Langerman).  The
 * Langerman problem takes the first five rows of the foxholes tables, as its
 * own printed tables are.  Parity unpinned for columns 6-10 of the foxholes
 * table: the appendix prints minima at n = 2 and 5 only.
 */
static const double orc_shekel_c[10] = {0.1, 0.2, 0.2, 0.4, 0.4, 0.6, 0.3, 0.7, 0.5, 0.5};
static const double orc_shekel_a[10][4] = {{4.0, 4.0, 4.0, 4.0}, {1.0, 1.0, 1.0, 1.0}, {8.0, 8.0, 8.0, 8.0}, {6.0, 6.0, 6.0, 6.0}, {3.0, 7.0, 3.0, 7.0}, {2.0, 9.0, 2.0, 9.0}, {5.0, 5.0, 3.0, 3.0}, {8.0, 1.0, 8.0, 1.0}, {6.0, 2.0, 6.0, 2.0}, {7.0, 3.6, 7.0, 3.6}};
static const double orc_fox_c[30] = {0.806, 0.517, 0.1, 0.908, 0.965, 0.669, 0.524, 0.902, 0.531, 0.876, 0.462, 0.491, 0.463, 0.714, 0.352, 0.869, 0.813, 0.811, 0.828, 0.964, 0.789, 0.36, 0.369, 0.992, 0.332, 0.817, 0.632, 0.883, 0.608, 0.326};
static const double orc_fox_a[30][10] = {
    {9.681, 0.667, 4.783, 9.095, 3.517, 9.325, 6.544, 0.211, 5.122, 2.02},
    {9.4, 2.041, 3.788, 7.931, 2.882, 2.672, 3.568, 1.284, 7.033, 7.374},
    {8.025, 9.152, 5.114, 7.621, 4.564, 4.711, 2.996, 6.126, 0.734, 4.982},
    {2.196, 0.415, 5.649, 6.979, 9.51, 9.166, 6.304, 6.054, 9.377, 1.426},
    {8.074, 8.777, 3.467, 1.863, 6.708, 6.349, 4.534, 0.276, 7.633, 1.567},
    {7.65, 5.658, 0.72, 2.764, 3.278, 5.283, 7.474, 6.274, 1.409, 8.208},
    {1.256, 3.605, 8.623, 6.905, 4.584, 8.133, 6.071, 6.888, 4.187, 5.448},
    {8.314, 2.261, 4.224, 1.781, 4.124, 0.932, 8.129, 8.658, 1.208, 5.762},
    {0.226, 8.858, 1.42, 0.945, 1.622, 4.698, 6.228, 9.096, 0.972, 7.637},
    {7.305, 2.228, 1.242, 5.928, 9.133, 1.826, 4.06, 5.204, 8.713, 8.247},
    {0.652, 7.027, 0.508, 4.876, 8.807, 4.632, 5.808, 6.937, 3.291, 7.016},
    {2.699, 3.516, 5.874, 4.119, 4.461, 7.496, 8.817, 0.69, 6.593, 9.789},
    {8.327, 3.897, 2.017, 9.57, 9.825, 1.15, 1.395, 3.885, 6.354, 0.109},
    {2.132, 7.006, 7.136, 2.641, 1.882, 5.943, 7.273, 7.691, 2.88, 0.564},
    {4.707, 5.579, 4.08, 0.581, 9.698, 8.542, 8.077, 8.515, 9.231, 4.67},
    {8.304, 7.559, 8.567, 0.322, 7.128, 8.392, 1.472, 8.524, 2.277, 7.826},
    {8.632, 4.409, 4.832, 5.768, 7.05, 6.715, 1.711, 4.323, 4.405, 4.591},
    {4.887, 9.112, 0.17, 8.967, 9.693, 9.867, 7.508, 7.77, 8.382, 6.74},
    {2.44, 6.686, 4.299, 1.007, 7.008, 1.427, 9.398, 8.48, 9.95, 1.675},
    {6.306, 8.583, 6.084, 1.138, 4.35, 3.134, 7.853, 6.061, 7.457, 2.258},
    {0.652, 2.343, 1.37, 0.821, 1.31, 1.063, 0.689, 8.819, 8.833, 9.07},
    {5.558, 1.272, 5.756, 9.857, 2.279, 2.764, 1.284, 1.677, 1.244, 1.234},
    {3.352, 7.549, 9.817, 9.437, 8.687, 4.167, 2.57, 6.54, 0.228, 0.027},
    {8.798, 0.88, 2.37, 0.168, 1.701, 3.68, 1.231, 2.39, 2.499, 0.064},
    {1.46, 8.057, 1.336, 7.217, 7.914, 3.615, 9.981, 9.198, 5.292, 1.224},
    {0.432, 8.645, 8.774, 0.249, 8.081, 7.461, 4.416, 0.652, 4.002, 4.644},
    {0.679, 2.8, 5.523, 3.049, 2.968, 7.225, 6.73, 4.199, 9.614, 9.229},
    {4.263, 1.074, 7.286, 5.599, 8.291, 5.2, 9.214, 8.272, 4.398, 4.506},
    {9.496, 4.83, 3.15, 8.27, 5.079, 1.231, 5.731, 9.494, 1.883, 9.732},
    {4.138, 2.562, 2.532, 9.661, 5.611, 5.5, 6.886, 2.341, 9.699, 6.5},
};

/*
 * The non-separable families, evaluated in full (the paper's move evaluates
 * f(x1) in full, Sec. 3.3).  Coordinate d may be replaced by xdn (d >= n:
 * none).  Sums and products run over the coordinates in order 1..n.
 *   Griewank (Appendix, Test 8): 1 + sum y_i^2 / 4000 - prod cos(y_i / sqrt(i)).
 *     The printed form puts the product inside the sum; with it f(0) = 1 - n,
 *     not the stated minimum 0, so the sum and the product are read as
 *     separate terms (Griewank's own definition).
 *   Levy and Montalvo (Appendix, Test 10), w_i = 1 + (y_i + 1) / 4:
 *     (pi / n) [10 sin^2(pi w_1) + sum_{i<n} (w_i - 1)^2 (1 + 10 sin^2(pi w_{i+1}))
 *     + (w_n - 1)^2].
 *   Generalized Rosenbrock (Appendix, Test 14):
 *     sum_{i<n} [100 (y_{i+1} - y_i^2)^2 + (1 - y_i)^2].  The printed form has
 *     (y_{i+1} - y_i)^2; the named function (De Jong's second) squares y_i,
 *     and both have the stated minimum 0 at (1, ..., 1).
 *   The centre families, n = 4 for Shekel and n <= 10 otherwise (the tables'
 *   width), centres in table order, coordinates in order:
 *     Shekel with m = 5, 7, 10 (Test 18) and the modified foxholes (Test 19,
 *     m = 30): -sum_{i<m} 1 / (sum_j (y_j - a_ij)^2 + c_i);
 *     modified Langerman (Test 11, m = 5):
 *     -sum_{i<m} c_i exp(-(1/pi) sum_j (y_j - a_ij)^2) cos(pi sum_j (y_j - a_ij)^2).
 *   Other n: NaN.
 */
static double f_coupled(int func, uint32_t n, const double *x, const double *s, uint32_t d, double xdn)
{
    if (func == ORC_GRIEWANK) {
        double sum = 0.0, prod = 1.0;
        for (uint32_t i = 0; i < n; ++i) {
            const double y = y_at(x, s, i, d, xdn);
            sum += y * y / 4000.0;
            prod *= cos(y / sqrt((double)(i + 1)));
        }
        return 1.0 + sum - prod;
    }
    if (func == ORC_LEVY_MONTALVO) {
        double w0 = 1.0 + (y_at(x, s, 0, d, xdn) + 1.0) / 4.0;
        const double sp = sin(ORC_PI * w0);
        double acc = 10.0 * sp * sp;
        for (uint32_t i = 0; i + 1 < n; ++i) {
            const double w1 = 1.0 + (y_at(x, s, i + 1, d, xdn) + 1.0) / 4.0;
            const double sn = sin(ORC_PI * w1);
            acc += (w0 - 1.0) * (w0 - 1.0) * (1.0 + 10.0 * sn * sn);
            w0 = w1;
        }
        acc += (w0 - 1.0) * (w0 - 1.0);
        return ORC_PI / (double)n * acc;
    }
    if (func == ORC_ROSENBROCK) {
        double acc = 0.0;
        for (uint32_t i = 0; i + 1 < n; ++i) {
            const double a = y_at(x, s, i, d, xdn), b = y_at(x, s, i + 1, d, xdn);
            acc += 100.0 * (b - a * a) * (b - a * a) + (1.0 - a) * (1.0 - a);
        }
        return acc;
    }
    if (func >= ORC_SHEKEL5 && func <= ORC_LANGERMAN) {
        /* squared distance to each centre a_i over the n coordinates, then
         * Shekel / foxholes: -sum_i 1 / (|y - a_i|^2 + c_i);
         * Langerman:         -sum_i c_i exp(-|y - a_i|^2 / pi) cos(pi |y - a_i|^2). */
        const int shekel = func <= ORC_SHEKEL10;
        const uint32_t m = func == ORC_SHEKEL5 ? 5 : func == ORC_SHEKEL7 ? 7 : func == ORC_SHEKEL10 ? 10
                         : func == ORC_FOXHOLES ? 30 : 5;
        if (shekel ? n != 4 : n > 10) return NAN;
        double acc = 0.0;
        for (uint32_t i = 0; i < m; ++i) {
            const double *a = shekel ? orc_shekel_a[i] : orc_fox_a[i];
            const double c = shekel ? orc_shekel_c[i] : orc_fox_c[i];
            double dd = 0.0;
            for (uint32_t j = 0; j < n; ++j) {
                const double t = y_at(x, s, j, d, xdn) - a[j];
                dd += t * t;
            }
            acc += func == ORC_LANGERMAN ? c * exp(-dd / ORC_PI) * cos(ORC_PI * dd) : 1.0 / (dd + c);
        }
        return -acc;
    }
    return NAN;
}

/* Table of a centre family: writes its m centres (10 coordinates each,
 * Shekel's last six zero) to a[m][10] and constants to c[m] when they are
 * not NULL; returns m, or 0 for another function id. */
uint32_t orc_centres(int func, double *a, double *c)
{
    if (func < ORC_SHEKEL5 || func > ORC_LANGERMAN) return 0;
    const int shekel = func <= ORC_SHEKEL10;
    const uint32_t m = func == ORC_SHEKEL5 ? 5 : func == ORC_SHEKEL7 ? 7 : func == ORC_SHEKEL10 ? 10
                     : func == ORC_FOXHOLES ? 30 : 5;
    for (uint32_t i = 0; i < m; ++i) {
        for (uint32_t j = 0; j < 10; ++j)
            if (a) a[i * 10 + j] = shekel ? (j < 4 ? orc_shekel_a[i][j] : 0.0) : orc_fox_a[i][j];
        if (c) c[i] = shekel ? orc_shekel_c[i] : orc_fox_c[i];
    }
    return m;
}

/* Full evaluation, summing the coordinates in order 0..n-1. */
double orc_f(int func, uint32_t n, const double *x, const double *s)
{
    if (func >= ORC_GRIEWANK) return f_coupled(func, n, x, s, n, 0.0);
    if (func == ORC_SCHWEFEL) {
        double acc = 0.0;
        for (uint32_t i = 0; i < n; ++i) acc += orc_schwefel_term(shifted(x, s, i));
        return -acc / (double)n;
    }
    if (func == ORC_RASTRIGIN) {
        double acc = 0.0;
        for (uint32_t i = 0; i < n; ++i) acc += orc_rastrigin_term(shifted(x, s, i));
        return 10.0 * (double)n + acc;
    }
    if (func == ORC_ACKLEY) {
        double s1 = 0.0, s2 = 0.0;
        for (uint32_t i = 0; i < n; ++i) {
            double y = shifted(x, s, i);
            s1 += y * y;
            s2 += cos(2.0 * ORC_PI * y);
        }
        return orc_ackley_from_sums(s1, s2, n);
    }
    return NAN;
}

/* Per-chain cost state: the current cost and, for Ackley, its two sums. */
typedef struct {
    double f, s1, s2;
} orc_cost;

static void cost_full(int func, uint32_t n, const double *x, const double *s, orc_cost *c)
{
    c->s1 = 0.0;
    c->s2 = 0.0;
    if (func == ORC_ACKLEY) {
        for (uint32_t i = 0; i < n; ++i) {
            double y = shifted(x, s, i);
            c->s1 += y * y;
            c->s2 += cos(2.0 * ORC_PI * y);
        }
        c->f = orc_ackley_from_sums(c->s1, c->s2, n);
    } else {
        c->f = orc_f(func, n, x, s);
    }
}

/* Cost increment of changing coordinate d of x (shift s) to xn, and the new
 * cost state.  Separable costs: only coordinate d's term is re-evaluated;
 * the other families: f(x') evaluated in full. */
static double cost_delta(int func, uint32_t n, const orc_cost *c, const double *x, const double *s, uint32_t d,
                         double xn, orc_cost *out)
{
    const double sd = s ? s[d] : 0.0;
    double y = x[d] - sd, yn = xn - sd;
    *out = *c;
    if (func >= ORC_GRIEWANK) {
        out->f = f_coupled(func, n, x, s, d, xn);
        return out->f - c->f;
    }
    if (func == ORC_SCHWEFEL) {
        double df = -(orc_schwefel_term(yn) - orc_schwefel_term(y)) / (double)n;
        out->f = c->f + df;
        return df;
    }
    if (func == ORC_RASTRIGIN) {
        double df = orc_rastrigin_term(yn) - orc_rastrigin_term(y);
        out->f = c->f + df;
        return df;
    }
    /* Ackley */
    out->s1 = c->s1 + (yn * yn - y * y);
    out->s2 = c->s2 + (cos(2.0 * ORC_PI * yn) - cos(2.0 * ORC_PI * y));
    out->f = orc_ackley_from_sums(out->s1, out->s2, n);
    return out->f - c->f;
}

/* Metropolis criterion, eq. (5) with k_b = 1. */
int orc_accept(double df, double T, double u2)
{
    if (df <= 0.0) return 1;
    return u2 < exp(-df / T);
}

/* Neighbour of coordinate value xd (Sec. 2.1, Step 2). */
double orc_neighbour(int move_rule, double xd, double lo, double hi, double radius_frac, double u1)
{
    double xn;
    if (move_rule == ORC_MOVE_RESAMPLE) {
        xn = lo + (hi - lo) * u1;
    } else {
        double rho = radius_frac * (hi - lo);
        xn = xd + rho * (2.0 * u1 - 1.0);
    }
    if (xn > hi) xn = hi;
    if (xn < lo) xn = lo;
    return xn;
}

/* Temperature of level k: T0 multiplied by alpha k times, in order. */
double orc_temperature(double T0, double alpha, uint32_t level)
{
    double T = T0;
    for (uint32_t k = 0; k < level; ++k) T = T * alpha;
    return T;
}

/* ------------------------------------------------------------------------ */
/* One Markov chain at a fixed temperature (Sec. 2.2.2: each thread runs a    */
/* Metropolis process of length N).  x is updated in place.                   */
/* Returns the number of accepted moves.                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int func;
    uint32_t n;
    const double *lower, *upper, *shift;
    uint64_t seed;
    uint32_t problem;
    uint32_t steps;
    double radius_frac;
    int move_rule;
    int full_eval; /* re-evaluate f in full at every move (ORC_VARIANT_FULL) */
} orc_problem;

/* Capture sink: while set (orc_sa_run_capture), every accepted move appends
 * one record -- the learned proposal's features at the old state and the
 * accepted scaled displacement -- in chain order, then step order. */
static struct {
    float *rec;
    uint64_t capacity, count;
    double tau;
} capture_sink;

/* Kind of the proposal network (orc_set_net_kind):
 *   ORC_NET_RELU_CAUCHY  relu hidden activations, a Cauchy distribution over
 *                        the scaled displacement, history features entered as
 *                        sign(h) ln(1 + 2^24 |h|) / 16;
 *   ORC_NET_GELU_GAUSS   the written learned-proposal configuration: GELU
 *                        (exact erf form), a Gaussian distribution (mean, log
 *                        standard deviation), the last accepted scaled
 *                        displacements entered as they are. */
#define ORC_NET_RELU_CAUCHY 0
#define ORC_NET_GELU_GAUSS 1
static int orc_net_kind = ORC_NET_RELU_CAUCHY;

void orc_set_net_kind(int kind) { orc_net_kind = kind == ORC_NET_GELU_GAUSS ? kind : ORC_NET_RELU_CAUCHY; }

/* History feature of the learned proposal's input: sign(h) ln(1 + 2^24 |h|) / 16
 * (ORC_NET_RELU_CAUCHY), or h itself (ORC_NET_GELU_GAUSS). */
double orc_hist_feature(double h)
{
    if (orc_net_kind == ORC_NET_GELU_GAUSS) return h;
    return copysign(log(1.0 + ldexp(fabs(h), 24)) / 16.0, h);
}

static void capture_move(const orc_problem *p, double T, uint32_t d, double xd, double xn, double hist[4])
{
    const double w = p->upper[d] - p->lower[d];
    const double dl = (xn - xd) / w;
    if (capture_sink.count < capture_sink.capacity) {
        float *r = capture_sink.rec + capture_sink.count * 7;
        r[0] = (float)((xd - p->lower[d]) / w);
        r[1] = (float)log(capture_sink.tau * T);
        for (int k = 0; k < 4; ++k) r[2 + k] = (float)orc_hist_feature(hist[k]);
        r[6] = (float)dl;
    }
    capture_sink.count += 1;
    hist[3] = hist[2];
    hist[2] = hist[1];
    hist[1] = hist[0];
    hist[0] = dl;
}

/* bs_x/bs_f (optional): the chain's best-seen state of the level -- the
 * first state of lowest carried cost among its start state (set by the
 * caller) and its states after each accepted move. */
static uint64_t run_chain(const orc_problem *p, uint32_t level, uint32_t chain, double T, double *x,
                          orc_cost *c, double *bs_x, double *bs_f)
{
    uint64_t accepted = 0;
    double hist[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t step = 0; step < p->steps; ++step) {
        uint32_t d;
        double u1, u2;
        orc_move_draw(p->seed, p->problem, level, chain, step, p->n, &d, &u1, &u2);
        double xd = x[d];
        double xn = orc_neighbour(p->move_rule, xd, p->lower[d], p->upper[d], p->radius_frac, u1);
        orc_cost cn;
        double df;
        if (p->full_eval) {
            /* the move's cost from scratch: f at x with x_d replaced */
            x[d] = xn;
            cost_full(p->func, p->n, x, p->shift, &cn);
            x[d] = xd;
            df = cn.f - c->f;
        } else {
            df = cost_delta(p->func, p->n, c, x, p->shift, d, xn, &cn);
        }
        if (orc_accept(df, T, u2)) {
            if (capture_sink.rec) capture_move(p, T, d, xd, xn, hist);
            x[d] = xn;
            *c = cn;
            ++accepted;
            if (bs_x && c->f < *bs_f) {
                *bs_f = c->f;
                memcpy(bs_x, x, sizeof(double) * p->n);
            }
        }
    }
    return accepted;
}

/*
 * Multi-chain SA over levels [level_begin, level_begin + count), with the
 * level winner broadcast to every chain every `exchange` levels (Sec. 2.2):
 * exchange = 1 is the synchronous scheme with an exchange at each level
 * (Sec. 2.2.2), k > 1 the periodic exchange every k levels, 0 the
 * asynchronous scheme (Sec. 2.2.1: no exchange, only the final reduction).
 *
 * Level start: at level 0 every chain starts from its own random point.  At a
 * later level L with exchange > 0 and L % exchange == 0 every chain starts
 * from x_start (the previous level's winner) with its cost evaluated in full.
 * At any other level chain p continues from its own state and carried cost,
 * as the asynchronous kernel carries f(x0) through every temperature level:
 * `chain_x` (chains * n) and `chain_cost` (chains * 3: f, s1, s2), in/out,
 * required when exchange != 1.
 *
 * Per level k (index k - level_begin into the per-level outputs):
 *   win_chain[k]  chain with the lowest final cost (ties: lowest index)
 *   f_win[k]      that chain's final cost as carried incrementally
 *   f_best[k]     full re-evaluation of the winner's state
 *   f_rec[k]      lowest f_best so far (record), including rec_in
 *   x_best[k*n..] winner's state (optional)
 *   accepts[k]    accepted moves over all chains (optional)
 * x_rec/f_rec_io/rec_level_io carry the record in and out (f_rec_io = +inf
 * for a fresh run).  x_start is in/out: the last winner on return.
 */
/* Threads orc_sa_run spreads a level's chains over (1 = the plain sequential
 * loop).  Chains are independent within a level; the winner is reduced in
 * chain order afterwards, so every thread count gives the same bits. */
static int orc_threads = 1;

void orc_set_threads(int threads) { orc_threads = threads < 1 ? 1 : threads; }

/* One level's work on chains [ch0, ch1): each chain from its start, its
 * final cost into final_f, and the chunk's candidate for the level winner
 * (the first chain of lowest non-NaN final cost; none if every cost is NaN)
 * with its state. */
typedef struct {
    const orc_problem *p;
    uint32_t level, ch0, ch1, exchange, variant;
    int broadcast;
    double T;
    double T_prev, f_win_prev; /* SOS: the previous level's T and winner cost */
    uint8_t *kept;             /* SOS: per chain, 1 if it kept its own state (optional) */
    double *bsx;               /* best-seen: n doubles, owned by the caller */
    const double *x_start;
    orc_cost start_cost;
    double *chain_x, *chain_cost, *fin;
    /* outputs */
    uint64_t acc;
    int has_best;
    double best_f;
    uint32_t best_chain;
    double *bx, *x; /* n each, owned by the caller */
    double *x0;     /* chain 0's final state (the chunk holding chain 0) */
} level_chunk;

static void *run_level_chunk(void *arg)
{
    level_chunk *w = (level_chunk *)arg;
    const orc_problem *p = w->p;
    const uint32_t n = p->n;
    w->acc = 0;
    w->has_best = 0;
    for (uint32_t ch = w->ch0; ch < w->ch1; ++ch) {
        orc_cost c;
        int own = !w->broadcast;
        if (w->level > 0 && w->broadcast && (w->variant & ORC_VARIANT_SOS)) {
            /* stochastic exchange: keep the own state with probability
             * exp(-(f_own - f_win) / T_prev) */
            const double f_own = w->chain_cost[3 * (size_t)ch];
            own = orc_accept(f_own - w->f_win_prev, w->T_prev, orc_sos_uniform(p->seed, p->problem, w->level, ch));
        }
        if (w->kept) w->kept[ch] = (uint8_t)(w->level > 0 && own);
        if (w->level == 0) {
            orc_init_point(p->seed, p->problem, ch, n, p->lower, p->upper, w->x);
            cost_full(p->func, n, w->x, p->shift, &c);
        } else if (!own) {
            memcpy(w->x, w->x_start, sizeof(double) * n);
            c = w->start_cost;
        } else {
            memcpy(w->x, w->chain_x + (size_t)ch * n, sizeof(double) * n);
            c.f = w->chain_cost[3 * (size_t)ch];
            c.s1 = w->chain_cost[3 * (size_t)ch + 1];
            c.s2 = w->chain_cost[3 * (size_t)ch + 2];
        }
        const int bs = (w->variant & ORC_VARIANT_BEST_SEEN) != 0;
        double bsf = c.f;
        if (bs) memcpy(w->bsx, w->x, sizeof(double) * n);
        w->acc += run_chain(p, w->level, ch, w->T, w->x, &c, bs ? w->bsx : NULL, &bsf);
        if (w->exchange != 1 || (w->variant & ORC_VARIANT_SOS)) {
            memcpy(w->chain_x + (size_t)ch * n, w->x, sizeof(double) * n);
            w->chain_cost[3 * (size_t)ch] = c.f;
            w->chain_cost[3 * (size_t)ch + 1] = c.s1;
            w->chain_cost[3 * (size_t)ch + 2] = c.s2;
        }
        /* the value the level's argmin runs over, and the state it stands for */
        const double rf = bs ? bsf : c.f;
        const double *rx = bs ? w->bsx : w->x;
        w->fin[ch] = rf;
        if (ch == 0) memcpy(w->x0, rx, sizeof(double) * n);
        if (!isnan(rf) && (!w->has_best || rf < w->best_f)) {
            w->has_best = 1;
            w->best_f = rf;
            w->best_chain = ch;
            memcpy(w->bx, rx, sizeof(double) * n);
        }
    }
    return NULL;
}

/* orc_sa_run with a variant (ORC_VARIANT_*).  f_win_io carries the last
 * level's winner cost in and out (needed in by the stochastic exchange when
 * level_begin > 0).  kept (optional, chains bytes): at the last level, 1 for
 * each chain that continued from its own state. */
int orc_sa_run_v(int func, uint32_t n, const double *lower, const double *upper, const double *shift,
                 uint64_t seed, uint32_t problem, uint32_t chains, uint32_t steps, double T0, double alpha,
                 double radius_frac, int move_rule, uint32_t exchange, uint32_t variant, uint32_t level_begin,
                 uint32_t count, double *x_start, double *chain_x, double *chain_cost, double *f_win_io,
                 double *x_rec, double *f_rec_io, uint32_t *rec_level_io, uint32_t *win_chain, double *f_win,
                 double *f_best, double *f_rec, double *x_best, uint64_t *accepts, double *final_f, uint8_t *kept)
{
    if (n == 0 || chains == 0) return -1;
    if ((exchange != 1 || (variant & ORC_VARIANT_SOS)) && (!chain_x || !chain_cost)) return -1;
    if ((variant & ORC_VARIANT_SOS) && level_begin > 0 && !f_win_io) return -1;
    if ((variant & ORC_VARIANT_SOS) && (variant & ORC_VARIANT_ELITIST)) return -1;
    if (exchange && level_begin > 0 && !x_start) return -1;
    if ((variant & ORC_VARIANT_ELITIST) && !x_rec) return -1;
    orc_problem p = {func, n, lower, upper, shift, seed, problem, steps, radius_frac, move_rule,
                     (variant & ORC_VARIANT_FULL) != 0};
    /* the capture sink appends in chain order: one thread while it is set */
    uint32_t nt = capture_sink.rec ? 1u : (uint32_t)orc_threads;
    if (nt > chains) nt = chains;
    level_chunk *w = (level_chunk *)calloc(nt, sizeof(level_chunk));
    pthread_t *tid = (pthread_t *)calloc(nt, sizeof(pthread_t));
    double *bufs = (double *)malloc(sizeof(double) * n * (3 * (size_t)nt + 1));
    double *fin = (double *)malloc(sizeof(double) * chains);
    if (!w || !tid || !bufs || !fin) {
        free(w); free(tid); free(bufs); free(fin);
        return -2;
    }

    double f_win_prev = f_win_io ? *f_win_io : 0.0;
    for (uint32_t k = 0; k < count; ++k) {
        uint32_t level = level_begin + k;
        double T = orc_temperature(T0, alpha, level);
        const double T_prev = level > 0 ? orc_temperature(T0, alpha, level - 1) : T;
        const int broadcast = level > 0 && exchange > 0 && level % exchange == 0;
        orc_cost start_cost = {0.0, 0.0, 0.0};
        if (broadcast) cost_full(func, n, x_start, shift, &start_cost);
        for (uint32_t t = 0; t < nt; ++t) {
            level_chunk *c = &w[t];
            c->p = &p;
            c->level = level;
            c->ch0 = (uint32_t)((uint64_t)chains * t / nt);
            c->ch1 = (uint32_t)((uint64_t)chains * (t + 1) / nt);
            c->exchange = exchange;
            c->variant = variant;
            c->broadcast = broadcast;
            c->T = T;
            c->T_prev = T_prev;
            c->f_win_prev = f_win_prev;
            c->kept = k + 1 == count ? kept : NULL;
            c->bsx = bufs + (size_t)n * (2 * (size_t)nt + 1) + (size_t)n * t;
            c->x_start = x_start;
            c->start_cost = start_cost;
            c->chain_x = chain_x;
            c->chain_cost = chain_cost;
            c->fin = fin;
            c->bx = bufs + (size_t)2 * n * t;
            c->x = c->bx + n;
            c->x0 = bufs + (size_t)2 * n * nt;
        }
        if (nt == 1) {
            run_level_chunk(&w[0]);
        } else {
            uint32_t started = 0;
            for (; started < nt; ++started)
                if (pthread_create(&tid[started], NULL, run_level_chunk, &w[started]) != 0) break;
            for (uint32_t t = started; t < nt; ++t) run_level_chunk(&w[t]); /* could not start: run here */
            for (uint32_t t = 0; t < started; ++t) pthread_join(tid[t], NULL);
        }
        /* Winner in chain order: chain 0 if its cost is NaN (nothing compares
         * below it), else the first chain of lowest cost; accepted moves summed. */
        uint64_t acc_total = 0;
        double best_f = fin[0];
        uint32_t best_chain = 0;
        const double *bx = NULL;
        for (uint32_t t = 0; t < nt; ++t) acc_total += w[t].acc;
        if (!isnan(fin[0])) {
            for (uint32_t t = 0; t < nt; ++t) {
                if (w[t].has_best && (bx == NULL || w[t].best_f < best_f)) {
                    best_f = w[t].best_f;
                    best_chain = w[t].best_chain;
                    bx = w[t].bx;
                }
            }
        }
        if (!bx) bx = w[0].x0;
        if (final_f && k + 1 == count) memcpy(final_f, fin, sizeof(double) * chains);
        double fresh = orc_f(func, n, bx, shift);
        if (fresh < *f_rec_io) {
            *f_rec_io = fresh;
            *rec_level_io = level;
            memcpy(x_rec, bx, sizeof(double) * n);
        }
        /* the next exchange broadcasts the winner, or the record (elitist) */
        if (x_start) memmove(x_start, (variant & ORC_VARIANT_ELITIST) && isfinite(*f_rec_io) ? x_rec : bx,
                             sizeof(double) * n);
        if (win_chain) win_chain[k] = best_chain;
        if (f_win) f_win[k] = best_f;
        f_win_prev = best_f;
        if (f_best) f_best[k] = fresh;
        if (f_rec) f_rec[k] = *f_rec_io;
        if (x_best) memcpy(x_best + (size_t)k * n, bx, sizeof(double) * n);
        if (accepts) accepts[k] = acc_total;
    }
    if (f_win_io) *f_win_io = f_win_prev;
    free(w);
    free(tid);
    free(bufs);
    free(fin);
    return 0;
}

int orc_sa_run(int func, uint32_t n, const double *lower, const double *upper, const double *shift,
               uint64_t seed, uint32_t problem, uint32_t chains, uint32_t steps, double T0, double alpha,
               double radius_frac, int move_rule, uint32_t exchange, uint32_t level_begin, uint32_t count,
               double *x_start, double *chain_x, double *chain_cost, double *x_rec, double *f_rec_io,
               uint32_t *rec_level_io, uint32_t *win_chain, double *f_win, double *f_best, double *f_rec,
               double *x_best, uint64_t *accepts, double *final_f)
{
    return orc_sa_run_v(func, n, lower, upper, shift, seed, problem, chains, steps, T0, alpha, radius_frac, move_rule,
                        exchange, 0u, level_begin, count, x_start, chain_x, chain_cost, NULL, x_rec, f_rec_io,
                        rec_level_io, win_chain, f_win, f_best, f_rec, x_best, accepts, final_f, NULL);
}

/*
 * orc_sa_run that also records every accepted move into rec (capacity x 7
 * floats: (x_d - l_d)/(u_d - l_d), ln(tau T), the chain's last four accepted
 * scaled displacements (most recent first, zero at each level start), and
 * the accepted scaled displacement (x'_d - x_d)/(u_d - l_d)); *count gets the
 * number of accepted moves (records beyond capacity are dropped).
 */
int orc_sa_run_capture(int func, uint32_t n, const double *lower, const double *upper, const double *shift,
                       uint64_t seed, uint32_t problem, uint32_t chains, uint32_t steps, double T0, double alpha,
                       double radius_frac, int move_rule, uint32_t level_begin, uint32_t count, double *x_start,
                       double tau, float *rec, uint64_t capacity, uint64_t *n_captured)
{
    double *x_rec = (double *)malloc(sizeof(double) * n);
    double f_rec = INFINITY;
    uint32_t rec_level = 0;
    if (!x_rec) return -2;
    capture_sink.rec = rec;
    capture_sink.capacity = capacity;
    capture_sink.count = 0;
    capture_sink.tau = tau;
    int rc = orc_sa_run(func, n, lower, upper, shift, seed, problem, chains, steps, T0, alpha, radius_frac, move_rule,
                        1, level_begin, count, x_start, NULL, NULL, x_rec, &f_rec, &rec_level, NULL, NULL, NULL, NULL,
                        NULL, NULL, NULL);
    *n_captured = capture_sink.count;
    capture_sink.rec = NULL;
    free(x_rec);
    return rc;
}

/*
 * Replay one level for chains [chain0, chain0 + nchains) starting from x_start
 * (cost state recomputed in full), and log every move:
 *   log_d[m], log_xold[m], log_xnew[m], log_df[m], log_acc[m]
 * with m = (chain - chain0) * steps + step.  Final states are written to
 * x_final (nchains * n) when given.
 */
int orc_replay_level(int func, uint32_t n, const double *lower, const double *upper, const double *shift,
                     uint64_t seed, uint32_t problem, uint32_t steps, double T, double radius_frac,
                     int move_rule, uint32_t level, const double *x_start, uint32_t chain0, uint32_t nchains,
                     uint32_t *log_d, double *log_xold, double *log_xnew, double *log_df, uint8_t *log_acc,
                     double *x_final, double *f_final)
{
    double *x = (double *)malloc(sizeof(double) * n);
    if (!x) return -2;
    for (uint32_t j = 0; j < nchains; ++j) {
        uint32_t ch = chain0 + j;
        memcpy(x, x_start, sizeof(double) * n);
        orc_cost c;
        cost_full(func, n, x, shift, &c);
        for (uint32_t step = 0; step < steps; ++step) {
            uint32_t d;
            double u1, u2;
            orc_move_draw(seed, problem, level, ch, step, n, &d, &u1, &u2);
            double xd = x[d];
            double xn = orc_neighbour(move_rule, xd, lower[d], upper[d], radius_frac, u1);
            orc_cost cn;
            double df = cost_delta(func, n, &c, x, shift, d, xn, &cn);
            int a = orc_accept(df, T, u2);
            size_t m = (size_t)j * steps + step;
            if (log_d) log_d[m] = d;
            if (log_xold) log_xold[m] = xd;
            if (log_xnew) log_xnew[m] = xn;
            if (log_df) log_df[m] = df;
            if (log_acc) log_acc[m] = (uint8_t)a;
            if (a) {
                x[d] = xn;
                c = cn;
            }
        }
        if (x_final) memcpy(x_final + (size_t)j * n, x, sizeof(double) * n);
        if (f_final) f_final[j] = c.f;
    }
    free(x);
    return 0;
}

/* ======================================================================== */
/* Learned proposal (an extension of the method, not in the paper): a small  */
/* per-coordinate network maps the features of the chosen coordinate to a   */
/* Cauchy distribution over its scaled displacement.  FP64 reference of its */
/* forward pass,                                                            */
/* pass, negative log-likelihood loss, gradient and Adam step.               */
/*                                                                          */
/* Features z (6): z0 = (x_d - l_d)/(u_d - l_d); z1 = ln(tau T), tau = n    */
/* for the objectives normalised by n (Schwefel, Ackley: a one-coordinate    */
/* change moves f by O(1/n)) and 1 for Rastrigin; z2..z5 = the chain's last  */
/* four accepted scaled displacements h, most recent first, each as          */
/* sign(h) ln(1 + 2^24 |h|) / 16 (orc_hist_feature).                         */
/* Network: a1 = z W1 + b1 (6x128), h1 = relu(a1); a2 = h1 W2 + b2 (128x128), */
/* h2 = relu(a2); o = h2 W3 + b3 (128x2); mu = o0, s = o1 = ln sigma: the    */
/* location and log scale of a Cauchy distribution over the scaled           */
/* displacement (heavy tails: a likelihood fit follows the typical accepted  */
/* step rather than the rare long jumps, and proposals still make some).     */
/* Loss of a record (z, delta): the Cauchy negative log-likelihood           */
/* s + ln pi + ln(1 + ((delta - mu) / e^s)^2).                               */
/* Parameter vector order: W1 (row-major, [in][out]), b1, W2, b2, W3, b3.    */
/* ======================================================================== */
#define ORC_H 128
#define ORC_LN_PI 1.14472988584940017414
#define ORC_NIN 6
#define ORC_NPARAM (ORC_NIN * ORC_H + ORC_H + ORC_H * ORC_H + ORC_H + ORC_H * 2 + 2)

uint32_t orc_mlp_nparam(void) { return ORC_NPARAM; }

#define ORC_SQRT1_2 0.70710678118654752440
#define ORC_INV_SQRT_2PI 0.39894228040143267794
#define ORC_LN_SQRT_2PI 0.91893853320467274178

/* Hidden activation: relu, or GELU a Phi(a) = a (1 + erf(a / sqrt 2)) / 2. */
double orc_act(double a)
{
    if (orc_net_kind == ORC_NET_GELU_GAUSS) return 0.5 * a * (1.0 + erf(a * ORC_SQRT1_2));
    return a > 0.0 ? a : 0.0;
}

/* Derivative of the activation: relu's taken as 0 at a = 0; GELU's
 * Phi(a) + a phi(a). */
double orc_act_grad(double a)
{
    if (orc_net_kind == ORC_NET_GELU_GAUSS)
        return 0.5 * (1.0 + erf(a * ORC_SQRT1_2)) + a * ORC_INV_SQRT_2PI * exp(-0.5 * a * a);
    return a > 0.0 ? 1.0 : 0.0;
}

typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3;
} orc_mlp;

static orc_mlp mlp_view(const double *p)
{
    orc_mlp m;
    m.W1 = p;
    m.b1 = m.W1 + ORC_NIN * ORC_H;
    m.W2 = m.b1 + ORC_H;
    m.b2 = m.W2 + ORC_H * ORC_H;
    m.W3 = m.b2 + ORC_H;
    m.b3 = m.W3 + ORC_H * 2;
    return m;
}

/* Forward pass of one feature vector; a1, a2 (pre-activations) optional. */
void orc_mlp_forward(const double *params, const double *z, double *out2, double *a1_out, double *a2_out)
{
    orc_mlp m = mlp_view(params);
    double a1[ORC_H], h1[ORC_H], a2[ORC_H], h2[ORC_H];
    for (int j = 0; j < ORC_H; ++j) {
        double s = m.b1[j];
        for (int i = 0; i < ORC_NIN; ++i) s += z[i] * m.W1[i * ORC_H + j];
        a1[j] = s;
        h1[j] = orc_act(s);
    }
    for (int j = 0; j < ORC_H; ++j) {
        double s = m.b2[j];
        for (int i = 0; i < ORC_H; ++i) s += h1[i] * m.W2[i * ORC_H + j];
        a2[j] = s;
        h2[j] = orc_act(s);
    }
    for (int k = 0; k < 2; ++k) {
        double s = m.b3[k];
        for (int i = 0; i < ORC_H; ++i) s += h2[i] * m.W3[i * 2 + k];
        out2[k] = s;
    }
    if (a1_out) memcpy(a1_out, a1, sizeof a1);
    if (a2_out) memcpy(a2_out, a2, sizeof a2);
}

/* Mean loss over a batch and its gradient (grad may be NULL). */
double orc_mlp_loss_grad(const double *params, uint32_t batch, const double *Z, const double *delta, double *grad)
{
    orc_mlp m = mlp_view(params);
    double loss = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * ORC_NPARAM);
    double *gW1 = grad, *gb1 = grad ? gW1 + ORC_NIN * ORC_H : NULL, *gW2 = grad ? gb1 + ORC_H : NULL;
    double *gb2 = grad ? gW2 + ORC_H * ORC_H : NULL, *gW3 = grad ? gb2 + ORC_H : NULL;
    double *gb3 = grad ? gW3 + ORC_H * 2 : NULL;
    const double inv_b = 1.0 / (double)batch;
    for (uint32_t r = 0; r < batch; ++r) {
        const double *z = Z + (size_t)r * ORC_NIN;
        double a1[ORC_H], a2[ORC_H], h1[ORC_H], h2[ORC_H], o[2];
        orc_mlp_forward(params, z, o, a1, a2);
        for (int j = 0; j < ORC_H; ++j) {
            h1[j] = orc_act(a1[j]);
            h2[j] = orc_act(a2[j]);
        }
        const double mu = o[0], s = o[1];
        const double e = delta[r] - mu;
        const double r = e * exp(-s); /* standardised residual */
        double dmu, ds;
        if (orc_net_kind == ORC_NET_GELU_GAUSS) {
            /* Gaussian NLL: s + ln sqrt(2 pi) + r^2 / 2 */
            loss += (s + ORC_LN_SQRT_2PI + 0.5 * r * r) * inv_b;
            dmu = -r * exp(-s) * inv_b;
            ds = (1.0 - r * r) * inv_b;
        } else {
            const double q = 1.0 + r * r;
            loss += (s + ORC_LN_PI + log(q)) * inv_b;
            dmu = -2.0 * r * exp(-s) / q * inv_b;
            ds = (1.0 - 2.0 * r * r / q) * inv_b;
        }
        if (!grad) continue;
        double dh2[ORC_H], da2[ORC_H], dh1[ORC_H], da1[ORC_H];
        gb3[0] += dmu;
        gb3[1] += ds;
        for (int i = 0; i < ORC_H; ++i) {
            gW3[i * 2 + 0] += h2[i] * dmu;
            gW3[i * 2 + 1] += h2[i] * ds;
            dh2[i] = m.W3[i * 2 + 0] * dmu + m.W3[i * 2 + 1] * ds;
            da2[i] = dh2[i] * orc_act_grad(a2[i]);
        }
        for (int j = 0; j < ORC_H; ++j) gb2[j] += da2[j];
        for (int i = 0; i < ORC_H; ++i) {
            double acc = 0.0;
            for (int j = 0; j < ORC_H; ++j) {
                gW2[i * ORC_H + j] += h1[i] * da2[j];
                acc += m.W2[i * ORC_H + j] * da2[j];
            }
            dh1[i] = acc;
            da1[i] = dh1[i] * orc_act_grad(a1[i]);
        }
        for (int j = 0; j < ORC_H; ++j) gb1[j] += da1[j];
        for (int i = 0; i < ORC_NIN; ++i)
            for (int j = 0; j < ORC_H; ++j) gW1[i * ORC_H + j] += z[i] * da1[j];
    }
    return loss;
}

/* One Adam step (Kingma & Ba): m, v moments, t = step number (1-based). */
void orc_adam_step(double *params, const double *grad, double *m, double *v, uint32_t nparam, uint32_t t, double lr,
                   double beta1, double beta2, double eps)
{
    const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (uint32_t i = 0; i < nparam; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
        const double mh = m[i] / c1, vh = v[i] / c2;
        params[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* Forward pass plus, per output, a first-order bound on how far an
 * evaluation may land from it when it rounds each hidden activation to BF16
 * (relative error at most u = 2^-9) and computes everything else in FP32:
 * relu is 1-Lipschitz, so a rounding of h1_i moves a2_j by at most
 * u |W2_ij h1_i|, and o_k moves by at most
 *   u sum_j |W3_jk| (|h2_j| + sum_i |W2_ij| |h1_i|),
 * doubled here to cover second-order terms, FP32 accumulation and the
 * ~2^-17 rounding of the features. */
void orc_mlp_forward_bound(const double *params, const double *z, double *out2, double *bound2)
{
    orc_mlp m = mlp_view(params);
    double a1[ORC_H], a2[ORC_H];
    orc_mlp_forward(params, z, out2, a1, a2);
    double prop[ORC_H]; /* sum_i |W2_ij| |h1_i| */
    for (int j = 0; j < ORC_H; ++j) {
        double t = 0.0;
        for (int i = 0; i < ORC_H; ++i) t += fabs(m.W2[i * ORC_H + j]) * fabs(orc_act(a1[i]));
        prop[j] = t;
    }
    /* GELU's slope stays below 1.13 (relu's below 1) */
    const double u = ldexp(1.0, -9) * (orc_net_kind == ORC_NET_GELU_GAUSS ? 1.13 : 1.0);
    for (int k = 0; k < 2; ++k) {
        double t = 0.0;
        for (int j = 0; j < ORC_H; ++j) t += fabs(m.W3[j * 2 + k]) * (fabs(orc_act(a2[j])) + prop[j]);
        bound2[k] = 2.0 * u * t;
    }
}

/* The learned block of a move: counter (step, level, chain, 3 | problem << 8).
 * Its first word U0 gives the standard Cauchy draw, by inversion of the
 * distribution function: t = tan(pi (U0 - 1/2)); its second word U1 chooses
 * the component of the mixture (the plain move iff U1 < eps). */
static void learn_block(uint64_t seed, uint32_t problem, uint32_t level, uint32_t chain, uint32_t step,
                        uint32_t r[4])
{
    const uint32_t ctr[4] = {step, level, chain, 3u | (problem << 8)};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, r);
}

double orc_learn_draw(uint64_t seed, uint32_t problem, uint32_t level, uint32_t chain, uint32_t step)
{
    uint32_t r[4];
    learn_block(seed, problem, level, chain, step, r);
    if (orc_net_kind == ORC_NET_GELU_GAUSS) {
        /* standard normal by Box-Muller on words 0 and 2: the radius from
         * U = 1 - U0 in (0, 1], the angle from U2 */
        const double u = 1.0 - orc_uniform(r[0]);
        return sqrt(-2.0 * log(u)) * cos(2.0 * ORC_PI * orc_uniform(r[2]));
    }
    return tan(ORC_PI * (orc_uniform(r[0]) - 0.5));
}

double orc_learn_mix(uint64_t seed, uint32_t problem, uint32_t level, uint32_t chain, uint32_t step)
{
    uint32_t r[4];
    learn_block(seed, problem, level, chain, step, r);
    return orc_uniform(r[1]);
}

/* Log density of the proposal, in scaled units: the Cauchy density with
 * location mu and scale e^s at delta, or the Gaussian one with mean mu and
 * standard deviation e^s. */
double orc_proposal_logpdf(double delta, double mu, double s)
{
    const double r = (delta - mu) * exp(-s);
    if (orc_net_kind == ORC_NET_GELU_GAUSS) return -s - ORC_LN_SQRT_2PI - 0.5 * r * r;
    return -s - ORC_LN_PI - log(1.0 + r * r);
}

/* ------------------------------------------------------------------------ */
/* The network under the device's stated precision: weight matrices in BF16  */
/* (the caller passes them already rounded), features represented as a BF16 */
/* high part plus a BF16 remainder, hidden activations rounded to BF16       */
/* (round to nearest even, after the FP32 accumulator) before each product,  */
/* biases and accumulation in FP32.  The values below are that arithmetic    */
/* carried out in FP64, with a bound on how far an FP32 accumulation in any  */
/* order (and feature errors up to ez[i]) can move the outputs: an           */
/* activation whose pre-activation interval rounds to one BF16 value is      */
/* exact; one whose interval straddles a rounding boundary may land on       */
/* either neighbour.  Rounding to BF16 decides values the way a quantised     */
/* code does, so both sides take that decision in the same precision.       */
/* ------------------------------------------------------------------------ */
static float bf16_round(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return f;
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

/* BF16 value of relu(a) for the FP32 accumulator holding a. */
static double bf16_relu(double a) { return a > 0.0 ? (double)bf16_round((float)a) : 0.0; }

/* Largest |v - value| over FP32 accumulators v within [a - e, a + e], for
 * the BF16 activation value = bf16_relu(a). */
static double bf16_relu_err(double a, double e)
{
    const double v = bf16_relu(a), lo = bf16_relu(a - e), hi = bf16_relu(a + e);
    if (lo == v && hi == v) return 0.0;
    return fmax(fabs(hi - v), fabs(v - lo));
}

/* GELU kind: the device evaluates a (1 + erf(a / sqrt 2)) / 2 in FP32 (erf to
 * a few ulps, three roundings): its deviation from the exact value, below. */
static double gelu_dev_err(double a) { return fabs(orc_act(a)) * ldexp(1.0, -20) + fabs(a) * ldexp(1.0, -22); }

/* BF16 value of the activation of the FP32 accumulator holding a. */
static double bf16_act(double a)
{
    if (orc_net_kind == ORC_NET_GELU_GAUSS) return (double)bf16_round((float)orc_act(a));
    return bf16_relu(a);
}

/* FP32 value at or below (dir < 0) / at or above (dir > 0) v. */
static float f32_dir(double v, int dir)
{
    float f = (float)v;
    if (dir < 0 && (double)f > v) f = nextafterf(f, -INFINITY);
    if (dir > 0 && (double)f < v) f = nextafterf(f, INFINITY);
    return f;
}

/* Largest |w - bf16_act(a)| over the BF16 activations w the device can
 * produce from an accumulator within [a - e, a + e]: GELU falls to its
 * minimum at a = -0.7518 and rises after it, and the device's GELU adds its
 * own FP32 error before the rounding to BF16 (which keeps order). */
static double bf16_act_err(double a, double e)
{
    if (orc_net_kind != ORC_NET_GELU_GAUSS) return bf16_relu_err(a, e);
    const double c = -0.751791524693564457;
    const double lo = a - e, hi = a + e, g1 = orc_act(lo), g2 = orc_act(hi);
    double gmin = fmin(g1, g2), gmax = fmax(g1, g2);
    if (lo < c && c < hi) gmin = fmin(gmin, orc_act(c));
    const double eg = fmax(gelu_dev_err(lo), gelu_dev_err(hi));
    const double v = bf16_act(a);
    const double wlo = bf16_round(f32_dir(gmin - eg, -1)), whi = bf16_round(f32_dir(gmax + eg, 1));
    return fmax(fabs(whi - v), fabs(v - wlo));
}

/* FP32 accumulation of k terms in any order: |error| <= gamma_k * sum |terms|,
 * gamma_k = k u / (1 - k u), u = 2^-24; doubled for the MFMA's internal
 * summation order. */
static double acc_bound(int k, double sum_abs)
{
    const double ku = (double)k * ldexp(1.0, -24);
    return 2.0 * ku / (1.0 - ku) * sum_abs;
}

void orc_mlp_forward_device(const double *params, const double *z, const double *ez, double *out2, double *bound2)
{
    orc_mlp m = mlp_view(params);
    double zin[ORC_NIN], ezin[ORC_NIN];
    for (int i = 0; i < ORC_NIN; ++i) {
        const float zf = (float)z[i];
        const float hi = bf16_round(zf);
        const float lo = bf16_round(zf - hi);
        zin[i] = (double)hi + (double)lo;
        /* split of the FP32 feature, plus the feature's own error and the
         * FP32 rounding of z */
        ezin[i] = fabs((double)zf - zin[i]) + ldexp(fabs(z[i]), -18) + (ez ? ez[i] : 0.0) +
                  ldexp(fabs(z[i]), -24);
    }
    double h1[ORC_H], e1[ORC_H], h2[ORC_H], e2[ORC_H];
    for (int j = 0; j < ORC_H; ++j) {
        const double b = (double)(float)m.b1[j];
        double a = b, sa = fabs(b), prop = 0.0;
        int k = 1; /* terms the accumulator adds (a zero product adds exactly nothing) */
        for (int i = 0; i < ORC_NIN; ++i) {
            const double t = zin[i] * m.W1[i * ORC_H + j];
            a += t;
            sa += 2.0 * fabs(t);
            prop += fabs(m.W1[i * ORC_H + j]) * ezin[i];
            k += t != 0.0 ? 2 : 0;
        }
        const double e = prop + acc_bound(k, sa);
        h1[j] = bf16_act(a);
        e1[j] = bf16_act_err(a, e);
    }
    for (int j = 0; j < ORC_H; ++j) {
        const double b = (double)(float)m.b2[j];
        double a = b, sa = fabs(b), prop = 0.0;
        int k = 1;
        for (int i = 0; i < ORC_H; ++i) {
            const double t = h1[i] * m.W2[i * ORC_H + j];
            a += t;
            sa += fabs(t);
            prop += fabs(m.W2[i * ORC_H + j]) * e1[i];
            k += (t != 0.0 || (e1[i] != 0.0 && m.W2[i * ORC_H + j] != 0.0)) ? 1 : 0;
        }
        /* activations that may differ enlarge the accumulated magnitudes too */
        const double e = prop + acc_bound(k, sa + prop);
        h2[j] = bf16_act(a);
        e2[j] = bf16_act_err(a, e);
    }
    for (int k = 0; k < 2; ++k) {
        const double b = (double)(float)m.b3[k];
        double a = b, sa = fabs(b), prop = 0.0;
        int terms = 1;
        for (int i = 0; i < ORC_H; ++i) {
            const double t = h2[i] * m.W3[i * 2 + k];
            a += t;
            sa += fabs(t);
            prop += fabs(m.W3[i * 2 + k]) * e2[i];
            terms += (t != 0.0 || (e2[i] != 0.0 && m.W3[i * 2 + k] != 0.0)) ? 1 : 0;
        }
        out2[k] = a;
        if (bound2) bound2[k] = prop + acc_bound(terms, sa + prop);
    }
}

/* ------------------------------------------------------------------------ */
/* The learned-proposal mixture move (an extension of the method, not in the */
/* paper; Metropolis-Hastings form of the acceptance of Sec. 2.1, eq. (5)).  */
/* Per move, with the move's plain words (coordinate, change, acceptance)    */
/* and the learned block of the move:                                        */
/*   - the coordinate d from the plain stream;                               */
/*   - with probability eps (U1 of the learned block < eps): the plain radius */
/*     move and the plain Metropolis test;                                   */
/*   - otherwise the network at the features of x_d gives (mu, s); the      */
/*     scaled displacement is dl = mu + e^s t with t the standard Cauchy draw */
/*     by inversion of U0; x'_d = x_d + dl (u_d - l_d); a proposal outside   */
/*     [l_d, u_d] is rejected (no clamp, which would change the proposal     */
/*     density); otherwise the network is evaluated again at x'_d with the   */
/*     same history and the move is taken iff                               */
/*        U2 < exp(-df/T + ln q(x | x') - ln q(x' | x)),                    */
/*     q the Cauchy densities, U2 the plain acceptance uniform;              */
/*   - an accepted move (either component) pushes its scaled displacement    */
/*     onto the chain's history of the last four (most recent first).        */
/* With the history features the proposal depends on the chain's past, so    */
/* the chain is adaptive: exp(-f/T) is left exactly invariant for a fixed    */
/* history (a network that ignores the history features), and approximately */
/* otherwise.                                                                */
/* mode 0 evaluates the network in FP64 (its definition); mode 1 under the   */
/* device's stated precision (orc_mlp_forward_device), with bounds.          */
/* ------------------------------------------------------------------------ */
static void learned_features(double xd, double lo, double hi, double featT, const double hist[4], double z[ORC_NIN])
{
    z[0] = (xd - lo) / (hi - lo);
    z[1] = featT;
    for (int k = 0; k < 4; ++k) z[2 + k] = orc_hist_feature(hist[k]);
}

/* Feature error the device's FP32 evaluation of the features may add. */
static void feature_errors(const double z[ORC_NIN], double ez[ORC_NIN])
{
    for (int i = 0; i < ORC_NIN; ++i) ez[i] = i == 1 ? 0.0 : ldexp(fabs(z[i]), -21) + ldexp(1.0, -22);
}

static void net_eval(const double *params, int mode, const double z[ORC_NIN], double out[2], double bound[2])
{
    if (mode == 1) {
        double ez[ORC_NIN];
        feature_errors(z, ez);
        orc_mlp_forward_device(params, z, ez, out, bound);
    } else {
        orc_mlp_forward(params, z, out, NULL, NULL);
        bound[0] = bound[1] = 0.0;
    }
}

/*
 * Proposal of move `step` of one chain from state x with history hist.
 * out_u[0] = d, out_u[1] = 1 if the plain component was chosen;
 * out_d[0] = x_d, out_d[1] = proposed x'_d (plain: clamped; learned: as
 * drawn, possibly outside the box), out_d[2..3] = mu, s of the network at
 * x_d (learned), out_d[4] = t, out_d[5..6] = bounds on mu, s (mode 1).
 */
void orc_learned_propose(const double *params, int mode, uint64_t seed, uint32_t problem, uint32_t level,
                         uint32_t chain, uint32_t step, uint32_t n, const double *x, const double *lower,
                         const double *upper, double radius_frac, double featT, double eps, const double hist[4],
                         uint32_t *out_u, double *out_d)
{
    uint32_t d;
    double u1, u2;
    orc_move_draw(seed, problem, level, chain, step, n, &d, &u1, &u2);
    const int plain = orc_learn_mix(seed, problem, level, chain, step) < eps;
    const double xd = x[d], lo = lower[d], hi = upper[d];
    out_u[0] = d;
    out_u[1] = (uint32_t)plain;
    out_d[0] = xd;
    for (int k = 2; k < 7; ++k) out_d[k] = 0.0;
    if (plain) {
        out_d[1] = orc_neighbour(ORC_MOVE_RADIUS, xd, lo, hi, radius_frac, u1);
        return;
    }
    double z[ORC_NIN], o[2], b[2];
    learned_features(xd, lo, hi, featT, hist, z);
    net_eval(params, mode, z, o, b);
    const double t = orc_learn_draw(seed, problem, level, chain, step);
    const double dl = o[0] + exp(o[1]) * t;
    out_d[1] = xd + dl * (hi - lo);
    out_d[2] = o[0];
    out_d[3] = o[1];
    out_d[4] = t;
    out_d[5] = b[0];
    out_d[6] = b[1];
}

/* Decision on the proposal x_new for coordinate d, given the chain's cost
 * state c at x.  out[0] = df (0 for an outside learned proposal),
 * out[1] = ln q(x | x') - ln q(x' | x) (learned, inside), out[2] = the log
 * acceptance ratio -df/T + out[1], out[3] = U2, out[4..5] = mu', s' of the
 * network at x'_d, out[6..7] = their bounds (mode 1).  *cn gets the cost
 * state after the move.  Returns 1 if the move is taken. */
static int learned_decide(const double *params, int mode, int func, uint32_t n, const double *lower,
                          const double *upper, const double *shift, uint64_t seed, uint32_t problem, uint32_t level,
                          uint32_t chain, uint32_t step, double T, double featT, int plain, const double *x,
                          const orc_cost *c, uint32_t d, double x_new, double mu, double s, const double hist[4],
                          double *out, orc_cost *cn)
{
    uint32_t dd;
    double u1, u2;
    orc_move_draw(seed, problem, level, chain, step, n, &dd, &u1, &u2);
    const double xd = x[d], lo = lower[d], hi = upper[d];
    for (int k = 0; k < 8; ++k) out[k] = 0.0;
    out[3] = u2;
    if (plain) {
        const double df = cost_delta(func, n, c, x, shift, d, x_new, cn);
        out[0] = df;
        out[2] = -df / T;
        return orc_accept(df, T, u2);
    }
    if (!(x_new >= lo && x_new <= hi)) {
        *cn = *c;
        return 0;
    }
    const double df = cost_delta(func, n, c, x, shift, d, x_new, cn);
    double z[ORC_NIN], o[2], b[2];
    learned_features(x_new, lo, hi, featT, hist, z);
    net_eval(params, mode, z, o, b);
    const double dl = (x_new - xd) / (hi - lo);
    const double lq = orc_proposal_logpdf(-dl, o[0], o[1]) - orc_proposal_logpdf(dl, mu, s);
    out[0] = df;
    out[1] = lq;
    out[2] = -df / T + lq;
    out[4] = o[0];
    out[5] = o[1];
    out[6] = b[0];
    out[7] = b[1];
    return u2 < exp(out[2]);
}

/* The decision of learned_decide for a chain at state x (its cost evaluated
 * in full), for checking a given proposal; returns 1 if taken. */
int orc_learned_accept(const double *params, int mode, int func, uint32_t n, const double *lower, const double *upper,
                       const double *shift, uint64_t seed, uint32_t problem, uint32_t level, uint32_t chain,
                       uint32_t step, double T, double featT, int plain, const double *x, uint32_t d, double x_new,
                       double mu, double s, const double hist[4], double *out)
{
    orc_cost c, cn;
    cost_full(func, n, x, shift, &c);
    return learned_decide(params, mode, func, n, lower, upper, shift, seed, problem, level, chain, step, T, featT,
                          plain, x, &c, d, x_new, mu, s, hist, out, &cn);
}

/*
 * One level of the learned mixture for chains [chain0, chain0 + nchains),
 * each starting from x_start with its cost evaluated in full and an empty
 * history, `steps` moves at temperature T (ln(tau T) = featT).  Per move m =
 * (chain - chain0) * steps + step, optional logs: coordinate, plain flag,
 * x_d, proposal, df, accept.  x_final (nchains x n), f_final (nchains) and
 * accepts (nchains) optional; trace0 (nchains x steps) gets x[0] after every
 * move (a one-coordinate chain's path).  With eps = 1 every move is the
 * plain move, in the same arithmetic as orc_replay_level.
 */
int orc_learned_run(const double *params, int mode, int func, uint32_t n, const double *lower, const double *upper,
                    const double *shift, uint64_t seed, uint32_t problem, uint32_t level, uint32_t chain0,
                    uint32_t nchains, uint32_t steps, double T, double featT, double eps, double radius_frac,
                    const double *x_start, uint32_t *log_d, uint8_t *log_plain, double *log_xold, double *log_xnew,
                    double *log_df, uint8_t *log_acc, double *x_final, double *f_final, uint64_t *accepts,
                    double *trace0)
{
    double *x = (double *)malloc(sizeof(double) * n);
    if (!x) return -2;
    for (uint32_t j = 0; j < nchains; ++j) {
        const uint32_t ch = chain0 + j;
        memcpy(x, x_start, sizeof(double) * n);
        orc_cost c;
        cost_full(func, n, x, shift, &c);
        double hist[4] = {0.0, 0.0, 0.0, 0.0};
        uint64_t acc = 0;
        for (uint32_t step = 0; step < steps; ++step) {
            uint32_t pu[2];
            double pd[7], dd[8];
            orc_learned_propose(params, mode, seed, problem, level, ch, step, n, x, lower, upper, radius_frac, featT,
                                eps, hist, pu, pd);
            const uint32_t d = pu[0];
            orc_cost cn;
            const int take = learned_decide(params, mode, func, n, lower, upper, shift, seed, problem, level, ch, step,
                                            T, featT, (int)pu[1], x, &c, d, pd[1], pd[2], pd[3], hist, dd, &cn);
            const size_t m = (size_t)j * steps + step;
            if (log_d) log_d[m] = d;
            if (log_plain) log_plain[m] = (uint8_t)pu[1];
            if (log_xold) log_xold[m] = x[d];
            if (log_xnew) log_xnew[m] = pd[1];
            if (log_df) log_df[m] = dd[0];
            if (log_acc) log_acc[m] = (uint8_t)take;
            if (take) {
                const double dl = (pd[1] - x[d]) / (upper[d] - lower[d]);
                hist[3] = hist[2];
                hist[2] = hist[1];
                hist[1] = hist[0];
                hist[0] = dl;
                x[d] = pd[1];
                c = cn;
                ++acc;
            }
            if (trace0) trace0[m] = x[0];
        }
        if (x_final) memcpy(x_final + (size_t)j * n, x, sizeof(double) * n);
        if (f_final) f_final[j] = c.f;
        if (accepts) accepts[j] = acc;
    }
    free(x);
    return 0;
}

/* ======================================================================== */
/* Nelder-Mead polish of an annealing result (the paper's hybrid strategy:   */
/* a local minimizer started where the annealing stopped, Sec. 4.2 and its   */
/* hybrid results table).  The paper names the method, not its details; the */
/* steps below are the standard simplex method with the coefficients of     */
/* Lagarias, Reeds, Wright and Wright (SIAM J. Optim. 9, 1998): reflection   */
/* 1, expansion 2, contraction 1/2, shrink 1/2.                              */
/*   Vertices live in slots 0..n.  Per iteration: b = lowest f (ties: lowest */
/*   slot), w = highest f among the other slots (ties: lowest slot), s =     */
/*   highest f among slots other than w (ties: lowest slot); stop when       */
/*   f[w] - f[b] <= ftol and every vertex is within xtol of x_b in every     */
/*   coordinate, or after maxiter iterations.  xm = mean of the slots other  */
/*   than w; xr = xm + (xm - x_w).                                          */
/*   - f[b] <= fr < f[s]: take xr (reflect);                                */
/*   - fr < f[b]: xe = xm + 2 (xm - x_w); take xe if fe < fr, else xr        */
/*     (expand);                                                            */
/*   - f[s] <= fr < f[w]: xc = xm + (xr - xm)/2; take xc if fc <= fr         */
/*     (outside contraction), else shrink;                                  */
/*   - fr >= f[w]: xc = xm - (xm - x_w)/2; take xc if fc < f[w] (inside     */
/*     contraction), else shrink;                                           */
/*   - shrink: every slot v other than b becomes x_b + (v - x_b)/2.         */
/*   A taken point replaces slot w.  The problem is box-constrained and the  */
/*   method is not: every trial point is projected onto the box (clamped)    */
/*   before it is evaluated, and the projected point is the one taken.       */
/*   Start: slot 0 = x0, slot i = x0 + h_i e_i, h_i = x0_i / 20 (0.00025 if   */
/*   x0_i = 0), reflected to x0 - h_i e_i when x0 + h_i e_i leaves the box.  */
/* Step codes logged per iteration: 0 reflect, 1 expand, 2 outside          */
/* contraction, 3 inside contraction, 4 shrink.  gap_log (optional) gets     */
/* f[w] - f[b] at the start of each iteration.                               */
/* ======================================================================== */
static void nm_point(uint32_t n, const double *lower, const double *upper, const double *xm, const double *xw,
                     double t, double *out)
{
    /* out = xm + t (xm - xw), projected onto the box */
    for (uint32_t j = 0; j < n; ++j) {
        double v = xm[j] + t * (xm[j] - xw[j]);
        if (v > upper[j]) v = upper[j];
        if (v < lower[j]) v = lower[j];
        out[j] = v;
    }
}

int orc_nelder_mead(int func, uint32_t n, const double *lower, const double *upper, const double *shift,
                    const double *x0, uint32_t maxiter, double ftol, double xtol, double *x_out, double *f_out,
                    uint32_t *iters_out, uint32_t *evals_out, uint8_t *step_log, double *gap_log)
{
    const uint32_t m = n + 1;
    double *V = (double *)malloc(sizeof(double) * (size_t)m * n);
    double *F = (double *)malloc(sizeof(double) * m);
    double *xm = (double *)malloc(sizeof(double) * n);
    double *xr = (double *)malloc(sizeof(double) * n);
    double *xt = (double *)malloc(sizeof(double) * n);
    if (!V || !F || !xm || !xr || !xt) {
        free(V); free(F); free(xm); free(xr); free(xt);
        return -2;
    }
    uint32_t evals = 0;
    for (uint32_t i = 0; i < m; ++i) {
        double *v = V + (size_t)i * n;
        memcpy(v, x0, sizeof(double) * n);
        if (i > 0) {
            const uint32_t j = i - 1;
            const double h = x0[j] != 0.0 ? x0[j] / 20.0 : 0.00025;
            v[j] = x0[j] + h;
            if (v[j] > upper[j] || v[j] < lower[j]) v[j] = x0[j] - h;
            if (v[j] > upper[j]) v[j] = upper[j];
            if (v[j] < lower[j]) v[j] = lower[j];
        }
        F[i] = orc_f(func, n, v, shift);
        ++evals;
    }
    uint32_t it = 0;
    for (; it < maxiter; ++it) {
        uint32_t b = 0;
        for (uint32_t i = 1; i < m; ++i)
            if (F[i] < F[b]) b = i;
        uint32_t w = b == 0 ? 1 : 0;
        for (uint32_t i = 0; i < m; ++i)
            if (i != b && F[i] > F[w]) w = i;
        uint32_t s = w == 0 ? 1 : 0;
        for (uint32_t i = 0; i < m; ++i)
            if (i != w && F[i] > F[s]) s = i;
        if (gap_log) gap_log[it] = F[w] - F[b];
        /* convergence */
        double spread = 0.0;
        const double *xb = V + (size_t)b * n;
        for (uint32_t i = 0; i < m; ++i)
            for (uint32_t j = 0; j < n; ++j) spread = fmax(spread, fabs(V[(size_t)i * n + j] - xb[j]));
        if (F[w] - F[b] <= ftol && spread <= xtol) break;
        /* centroid of every slot but w */
        for (uint32_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (uint32_t i = 0; i < m; ++i)
                if (i != w) acc += V[(size_t)i * n + j];
            xm[j] = acc / (double)n;
        }
        const double *xw = V + (size_t)w * n;
        nm_point(n, lower, upper, xm, xw, 1.0, xr);
        const double fr = orc_f(func, n, xr, shift);
        ++evals;
        int code;
        const double *take = NULL;
        double ftake = 0.0;
        if (fr < F[b]) {
            nm_point(n, lower, upper, xm, xw, 2.0, xt);
            const double fe = orc_f(func, n, xt, shift);
            ++evals;
            code = 1;
            if (fe < fr) { take = xt; ftake = fe; }
            else { take = xr; ftake = fr; }
        } else if (fr < F[s]) {
            code = 0;
            take = xr;
            ftake = fr;
        } else if (fr < F[w]) {
            nm_point(n, lower, upper, xm, xw, 0.5, xt);
            const double fc = orc_f(func, n, xt, shift);
            ++evals;
            code = 2;
            if (fc <= fr) { take = xt; ftake = fc; }
        } else {
            nm_point(n, lower, upper, xm, xw, -0.5, xt);
            const double fc = orc_f(func, n, xt, shift);
            ++evals;
            code = 3;
            if (fc < F[w]) { take = xt; ftake = fc; }
        }
        if (take) {
            memcpy(V + (size_t)w * n, take, sizeof(double) * n);
            F[w] = ftake;
        } else {
            code = 4;
            for (uint32_t i = 0; i < m; ++i) {
                if (i == b) continue;
                double *v = V + (size_t)i * n;
                for (uint32_t j = 0; j < n; ++j) v[j] = xb[j] + 0.5 * (v[j] - xb[j]);
                F[i] = orc_f(func, n, v, shift);
                ++evals;
            }
        }
        if (step_log) step_log[it] = (uint8_t)code;
    }
    uint32_t b = 0;
    for (uint32_t i = 1; i < m; ++i)
        if (F[i] < F[b]) b = i;
    memcpy(x_out, V + (size_t)b * n, sizeof(double) * n);
    *f_out = F[b];
    if (iters_out) *iters_out = it;
    if (evals_out) *evals_out = evals;
    free(V); free(F); free(xm); free(xr); free(xt);
    return 0;
}
