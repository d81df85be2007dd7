/* The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: every entry
 * point on small systems (n = 1, 2, 37, with partial and full active lists, with
 * and without softening), its argument checks, and a short integration. Prints "ok"
 * and returns 0 when every call returns the expected code and every output is
 * finite. The prototypes restate those of oracle/nbody_oracle.c. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int nbo_evaluate(int64_t n, const double *m, const double *xp, const double *vp,
                 const double *ap, double eps, int64_t n_act, const int32_t *idx,
                 double *out, int nthreads);
int nbo_evaluate_crackle(int64_t n, const double *m, const double *xp, const double *vp,
                         const double *ap, const double *jp, double eps, int64_t n_act,
                         const int32_t *idx, double *out, int nthreads);
int nbo_predict(int64_t n, const int64_t *tick, int64_t tick_next, int dt_min_log2,
                const double *x, const double *v, const double *a, const double *jk,
                const double *s, const double *c, double *xp, double *vp, double *ap);
int nbo_correct(int64_t n, int64_t n_act, const int32_t *idx, int64_t tick_next,
                int dt_min_log2, const double *anew, int64_t *tick, double *x,
                double *v, double *a, double *jk, double *s, double *c,
                double *a4n, double *a5n);
int nbo_timesteps(int64_t n, int64_t n_act, const int32_t *idx, int init,
                  const int64_t *tick, int32_t *level, const double *a,
                  const double *jk, const double *s, const double *c,
                  const double *a4n, const double *a5n, double eta, double eta_init,
                  int dt_max_log2, int dt_min_log2);
int64_t nbo_active(int64_t n, const int64_t *tick, const int32_t *level, int L,
                   int32_t *idx_out, int64_t *tick_next);
int nbo_energy(int64_t n, const double *m, const double *x, const double *v,
               double eps, double *ekin, double *epot, int nthreads);
int64_t nbo_integrate(int64_t n, const double *m, double *x, double *v, double *a,
                      double *jk, double *s, double *c, double *a4n, double *a5n,
                      int64_t *tick, int32_t *level, double eps, double eta,
                      double eta_init, int dt_max_log2, int dt_min_log2,
                      int64_t tick_end, int64_t max_steps, int64_t *step_tick,
                      int64_t *step_nact, double *interactions, int start_crackle,
                      int nthreads);

static int fails = 0;
#define EXPECT(cond)                                                             \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond);  \
            ++fails;                                                             \
        }                                                                        \
    } while (0)

static double *vec(int64_t k)
{
    double *p = (double *)calloc((size_t)(k > 0 ? k : 1), sizeof(double));
    if (!p)
        abort();
    return p;
}

static int all_finite(const double *p, int64_t k)
{
    for (int64_t i = 0; i < k; ++i)
        if (!isfinite(p[i]))
            return 0;
    return 1;
}

static void check_system(int64_t n, double eps)
{
    const int L = 37, dmax = -3, dmin = -40;
    double *m = vec(n), *x = vec(3 * n), *v = vec(3 * n), *a = vec(3 * n), *jk = vec(3 * n),
           *s = vec(3 * n), *c = vec(3 * n), *a4 = vec(n), *a5 = vec(n);
    double *xp = vec(3 * n), *vp = vec(3 * n), *ap = vec(3 * n), *out = vec(13 * n);
    int64_t *tick = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int32_t *level = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int32_t *idx = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    srand(1234 + (unsigned)n);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = 1.0 / (double)n;
        for (int k = 0; k < 3; ++k) {
            x[k * n + i] = (double)rand() / RAND_MAX - 0.5 + 0.01 * (double)i;
            v[k * n + i] = 0.1 * ((double)rand() / RAND_MAX - 0.5);
            a[k * n + i] = 0.01 * ((double)rand() / RAND_MAX - 0.5);
        }
        idx[i] = (int32_t)i;
    }
    /* full and partial evaluations, both kernels of the oracle */
    EXPECT(nbo_evaluate(n, m, x, v, a, eps, n, idx, out, 2) == 0);
    EXPECT(all_finite(out, 10 * n));
    const int64_t half = n / 2;
    for (int64_t q = 0; q < half; ++q)
        idx[q] = (int32_t)(2 * q + (n & 1));
    EXPECT(nbo_evaluate(n, m, x, v, a, eps, half, idx, out, 1) == 0);
    EXPECT(all_finite(out, 10 * half));
    EXPECT(nbo_evaluate_crackle(n, m, x, v, a, jk, eps, half, idx, out, 2) == 0);
    EXPECT(all_finite(out, 13 * half));
    for (int64_t i = 0; i < n; ++i)
        idx[i] = (int32_t)i;
    /* one hand-made block step: predict, evaluate, correct, levels, active set */
    EXPECT(nbo_timesteps(n, n, idx, 1, tick, level, a, jk, s, c, a4, a5, 0.45, 0.01, dmax, dmin) == 0);
    int64_t tn = 0;
    const int64_t na = nbo_active(n, tick, level, L, idx, &tn);
    EXPECT(na >= 1 && na <= n && tn > 0);
    EXPECT(nbo_predict(n, tick, tn, dmin, x, v, a, jk, s, c, xp, vp, ap) == 0);
    EXPECT(nbo_evaluate(n, m, xp, vp, ap, eps, na, idx, out, 2) == 0);
    EXPECT(nbo_correct(n, na, idx, tn, dmin, out, tick, x, v, a, jk, s, c, a4, a5) == 0);
    /* the state was not started like a real run: a body may need a step below the
     * smallest (code 2); the call must still complete */
    const int ts = nbo_timesteps(n, na, idx, 0, tick, level, a, jk, s, c, a4, a5, 0.45, 0.01, dmax, dmin);
    EXPECT(ts == 0 || ts == 2);
    EXPECT(all_finite(x, 3 * n) && all_finite(v, 3 * n));
    double ek = 0.0, ep = 0.0;
    EXPECT(nbo_energy(n, m, x, v, eps, &ek, &ep, 2) == 0);
    EXPECT(isfinite(ek) && isfinite(ep));
    free(m); free(x); free(v); free(a); free(jk); free(s); free(c); free(a4); free(a5);
    free(xp); free(vp); free(ap); free(out); free(tick); free(level); free(idx);
}

static void check_integrate(int64_t n)
{
    double *m = vec(n), *x = vec(3 * n), *v = vec(3 * n), *a = vec(3 * n), *jk = vec(3 * n),
           *s = vec(3 * n), *c = vec(3 * n), *a4 = vec(n), *a5 = vec(n);
    int64_t *tick = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int32_t *level = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    srand(99);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = 1.0 / (double)n;
        for (int k = 0; k < 3; ++k) {
            x[k * n + i] = (double)rand() / RAND_MAX - 0.5;
            v[k * n + i] = 0.2 * ((double)rand() / RAND_MAX - 0.5);
        }
    }
    int64_t st[64], sn[64];
    double inter = 0.0;
    const int64_t steps = nbo_integrate(n, m, x, v, a, jk, s, c, a4, a5, tick, level, 0.05, 0.45, 0.01,
                                        -3, -40, (int64_t)1 << 37, 64, st, sn, &inter, 1, 2);
    if (steps < 1)
        fprintf(stderr, "integrate returned %lld\n", (long long)steps);
    EXPECT(steps >= 1);  /* more than 64 steps are counted, only 64 recorded */
    EXPECT(all_finite(x, 3 * n) && inter > 0.0);
    free(m); free(x); free(v); free(a); free(jk); free(s); free(c); free(a4); free(a5);
    free(tick); free(level);
}

int main(void)
{
    check_system(1, 0.0);
    check_system(2, 0.01);
    check_system(37, 0.0);
    check_system(37, 1e-4);
    check_integrate(24);
    /* argument checks return codes, not crashes */
    double d = 0.0, e = 0.0;
    int32_t i0 = 0;
    int64_t t0 = 0, tn = 0;
    EXPECT(nbo_evaluate(-1, &d, &d, &d, &d, 0.0, 0, &i0, &d, 1) != 0);
    EXPECT(nbo_evaluate(1, &d, &d, &d, &d, -1.0, 1, &i0, &d, 1) != 0);
    EXPECT(nbo_evaluate(1, &d, &d, &d, &d, 0.0, 2, &i0, &d, 1) != 0);
    EXPECT(nbo_evaluate(1, &d, &d, &d, &d, 0.0, 1, &i0, &d, 0) != 0);
    EXPECT(nbo_active(0, &t0, &i0, 5, &i0, &tn) == -1);
    EXPECT(nbo_active(1, &t0, &i0, 63, &i0, &tn) == -1);
    EXPECT(nbo_energy(-1, &d, &d, &d, 0.0, &d, &e, 1) != 0);
    EXPECT(nbo_integrate(0, &d, &d, &d, &d, &d, &d, &d, &d, &d, &t0, &i0, 0.0, 0.45, 0.01, -3, -40,
                         1, 1, NULL, NULL, &d, 0, 1) < 0);
    if (fails)
        return 1;
    printf("ok\n");
    return 0;
}
