/*
 * Drives every entry point of the FP64 oracle on small inputs, for a build
 * of the oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
 * code only; tests/test_oracle_sanitize.py compiles and runs it).  Any
 * out-of-bounds access, use after free, leak or undefined operation aborts
 * the run with the sanitizer's report; a clean run prints "ok".
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_f(int func, uint32_t n, const double *x, const double *s);
void orc_set_threads(int threads);
int orc_sa_run_v(int func, uint32_t n, const double *lower, const double *upper, const double *shift, uint64_t seed,
                 uint32_t problem, uint32_t chains, uint32_t steps, double T0, double alpha, double radius_frac,
                 int move_rule, uint32_t exchange, uint32_t variant, uint32_t level_begin, uint32_t count,
                 double *x_start, double *chain_x, double *chain_cost, double *f_win_io, double *x_rec,
                 double *f_rec_io, uint32_t *rec_level_io, uint32_t *win_chain, double *f_win, double *f_best,
                 double *f_rec, double *x_best, uint64_t *accepts, double *final_f, uint8_t *kept);
int orc_sa_run_capture(int func, uint32_t n, const double *lower, const double *upper, const double *shift,
                       uint64_t seed, uint32_t problem, uint32_t chains, uint32_t steps, double T0, double alpha,
                       double radius_frac, int move_rule, uint32_t level_begin, uint32_t count, double *x_start,
                       double tau, float *rec, uint64_t capacity, uint64_t *n_captured);
int orc_replay_level(int func, uint32_t n, const double *lower, const double *upper, const double *shift,
                     uint64_t seed, uint32_t problem, uint32_t steps, double T, double radius_frac, int move_rule,
                     uint32_t level, const double *x_start, uint32_t chain0, uint32_t nchains, uint32_t *log_d,
                     double *log_xold, double *log_xnew, double *log_df, uint8_t *log_acc, double *x_final,
                     double *f_final);
uint32_t orc_mlp_nparam(void);
uint32_t orc_centres(int func, double *a, double *c);
void orc_set_net_kind(int kind);
void orc_mlp_forward(const double *params, const double *z, double *out2, double *a1_out, double *a2_out);
double orc_mlp_loss_grad(const double *params, uint32_t batch, const double *Z, const double *delta, double *grad);
void orc_adam_step(double *params, const double *grad, double *m, double *v, uint32_t nparam, uint32_t t, double lr,
                   double beta1, double beta2, double eps);
void orc_mlp_forward_bound(const double *params, const double *z, double *out2, double *bound2);
void orc_mlp_forward_device(const double *params, const double *z, const double *ez, double *out2, double *bound2);
int orc_learned_run(const double *params, int mode, int func, uint32_t n, const double *lower, const double *upper,
                    const double *shift, uint64_t seed, uint32_t problem, uint32_t level, uint32_t chain0,
                    uint32_t nchains, uint32_t steps, double T, double featT, double eps, double radius_frac,
                    const double *x_start, uint32_t *log_d, uint8_t *log_plain, double *log_xold, double *log_xnew,
                    double *log_df, uint8_t *log_acc, double *x_final, double *f_final, uint64_t *accepts,
                    double *trace0);
int orc_nelder_mead(int func, uint32_t n, const double *lower, const double *upper, const double *shift,
                    const double *x0, uint32_t maxiter, double ftol, double xtol, double *x_out, double *f_out,
                    uint32_t *iters_out, uint32_t *evals_out, uint8_t *step_log, double *gap_log);

static const double half_box[11] = {500.0, 5.12, 32.768, 600.0, 10.0, 2.048, 10.0, 10.0, 10.0, 15.0, 10.0};

static void fail(const char *what, int rc)
{
    fprintf(stderr, "%s failed: %d\n", what, rc);
    exit(1);
}

static double *vec(uint32_t n, double v)
{
    double *p = (double *)malloc(sizeof(double) * n);
    for (uint32_t i = 0; i < n; ++i) p[i] = v;
    return p;
}

static void runs(int func, uint32_t n)
{
    const uint32_t chains = 64, steps = 9, levels = 4;
    double *lo = vec(n, -half_box[func]), *hi = vec(n, half_box[func]), *sh = vec(n, 0.3);
    double *xs = vec(n, 0.0), *cx = vec(chains * n, 0.0), *cc = vec(chains * 3, 0.0), *xr = vec(n, 0.0);
    double *xb = vec(levels * n, 0.0), *fw = vec(levels, 0.0), *fb = vec(levels, 0.0), *fr = vec(levels, 0.0);
    double *ff = vec(chains, 0.0);
    uint32_t win[4];
    uint64_t acc[4];
    uint8_t kept[64];
    for (uint32_t variant = 0; variant < 4; ++variant) {
        for (uint32_t ex = 0; ex < 4; ex += 3) {
            const uint32_t exchange = ex == 0 ? 0u : ex == 3 ? 3u : 1u;
            for (int threads = 1; threads <= 3; threads += 2) {
                orc_set_threads(threads);
                double f_rec = INFINITY, fwin = 0.0;
                uint32_t rec_level = 0;
                int rc = orc_sa_run_v(func, n, lo, hi, (variant & 1) ? sh : NULL, 7, 1, chains, steps, 5.0, 0.8, 0.1,
                                      (int)(variant >> 1), exchange, variant, 0, levels, xs, cx, cc, &fwin, xr,
                                      &f_rec, &rec_level, win, fw, fb, fr, xb, acc, ff, kept);
                if (rc) fail("orc_sa_run_v", rc);
            }
        }
    }
    orc_set_threads(1);
    {
        double f_rec = INFINITY, fwin = fw[levels - 1];
        uint32_t rec_level = 0;
        int rc = orc_sa_run_v(func, n, lo, hi, NULL, 7, 0, chains, steps, 5.0, 0.8, 0.1, 0, 1, 1, levels, 2, xs, cx,
                              cc, &fwin, xr, &f_rec, &rec_level, win, fw, fb, fr, xb, acc, ff, kept);
        if (rc) fail("orc_sa_run_v (resumed)", rc);
    }
    if (func <= 2) {
        float rec[7 * 40];
        uint64_t got = 0;
        int rc = orc_sa_run_capture(func, n, lo, hi, sh, 3, 0, chains, steps, 5.0, 0.8, 0.1, 0, 0, 2, xs, 4.0, rec, 40,
                                    &got);
        if (rc) fail("orc_sa_run_capture", rc);
    }
    {
        const uint32_t nch = 3, m = nch * steps;
        uint32_t *d = (uint32_t *)malloc(sizeof(uint32_t) * m);
        uint8_t *a = (uint8_t *)malloc(m);
        double *xo = vec(m, 0.0), *xn = vec(m, 0.0), *df = vec(m, 0.0), *xf = vec(nch * n, 0.0), *fff = vec(nch, 0.0);
        int rc = orc_replay_level(func, n, lo, hi, sh, 5, 0, steps, 1.5, 0.1, 1, 2, xs, 4, nch, d, xo, xn, df, a, xf,
                                  fff);
        if (rc) fail("orc_replay_level", rc);
        free(d); free(a); free(xo); free(xn); free(df); free(xf); free(fff);
    }
    {
        double x[3 * 8], xo[8], f;
        uint32_t it, ev;
        uint8_t steps_log[300];
        double gaps[300];
        for (uint32_t i = 0; i < n && i < 8; ++i) x[i] = 0.37 * half_box[func] * (i % 2 ? -1.0 : 1.0);
        if (n <= 8) {
            int rc = orc_nelder_mead(func, n, lo, hi, sh, x, 300, 1e-12, 1e-10, xo, &f, &it, &ev, steps_log, gaps);
            if (rc) fail("orc_nelder_mead", rc);
        }
    }
    double *xv = vec(n, 0.11 * half_box[func]);
    (void)orc_f(func, n, xv, sh);
    (void)orc_f(func, n, xv, NULL);
    free(lo); free(hi); free(sh); free(xs); free(cx); free(cc); free(xr); free(xb); free(fw); free(fb); free(fr);
    free(ff); free(xv);
}

static void network(void)
{
    const uint32_t np = orc_mlp_nparam(), batch = 5;
    double *p = vec(np, 0.0), *g = vec(np, 0.0), *m = vec(np, 0.0), *v = vec(np, 0.0);
    for (uint32_t i = 0; i < np; ++i) p[i] = 0.01 * (double)((i * 2654435761u) % 997) / 997.0 - 0.005;
    double z[6] = {0.3, -1.0, 0.1, -0.2, 0.0, 0.05}, ez[6] = {1e-7, 0, 1e-7, 1e-7, 1e-7, 1e-7};
    double out[2], bound[2], a1[128], a2[128];
    orc_mlp_forward(p, z, out, a1, a2);
    orc_mlp_forward_bound(p, z, out, bound);
    orc_mlp_forward_device(p, z, ez, out, bound);
    double Z[6 * 5], dl[5];
    for (uint32_t r = 0; r < batch; ++r) {
        for (int k = 0; k < 6; ++k) Z[6 * r + k] = z[k] * (1.0 + 0.1 * r);
        dl[r] = 0.001 * (r + 1);
    }
    (void)orc_mlp_loss_grad(p, batch, Z, dl, g);
    orc_adam_step(p, g, m, v, np, 1, 1e-3, 0.9, 0.999, 1e-8);
    const uint32_t n = 4, nch = 2, steps = 11, mm = nch * steps;
    double *lo = vec(n, -500.0), *hi = vec(n, 500.0), *xs = vec(n, 100.0);
    uint32_t d[22];
    uint8_t pl[22], acc8[22];
    double xo[22], xn[22], df[22], xf[8], ff[2], tr[22];
    uint64_t accepts[2];
    for (int mode = 0; mode < 2; ++mode) {
        int rc = orc_learned_run(p, mode, 0, n, lo, hi, NULL, 9, 0, 3, 0, nch, steps, 2.0, 0.5, 0.3, 0.1, xs, d, pl,
                                 xo, xn, df, acc8, xf, ff, accepts, tr);
        if (rc) fail("orc_learned_run", rc);
    }
    (void)mm;
    free(p); free(g); free(m); free(v); free(lo); free(hi); free(xs);
}

int main(void)
{
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x32_10(ctr, key, out);
    const uint32_t dims[3] = {1, 2, 7};
    for (int func = 0; func < 11; ++func) {
        if (func >= 6 && func <= 8) {
            runs(func, 4); /* Shekel: n = 4 only */
            continue;
        }
        for (int k = 0; k < 3; ++k) runs(func, dims[k]);
    }
    {
        double a[30 * 10], c[30];
        for (int func = 0; func < 12; ++func) (void)orc_centres(func, a, c);
        (void)orc_centres(9, NULL, NULL);
    }
    for (int kind = 0; kind < 2; ++kind) {
        orc_set_net_kind(kind);
        network();
    }
    orc_set_net_kind(0);
    printf("ok\n");
    return 0;
}
