/*
 * nbody_oracle.c -- plain, slow, FP64 CPU reference of the Hermite 6th-order
 * block-time-step direct N-body method.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the GPU library includes, links or calls
 * this file; it shares no header, helper or constant with it. Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * The paper (Goz et al., "Astrophysical code migration into Exascale Era",
 * section "Code implementation") names the integrator -- Hermite 6th order,
 * derived from HiGPUs -- and requires double precision for inter-particle
 * distances and accelerations; section "Performance results" names the O(N^2)
 * evaluation as the dominant kernel. It prints no formula, so every formula below
 * is the standard one for that scheme (Nitadori & Makino 2008, New Astronomy 13,
 * 498: 6th-order Hermite predictor/corrector and its generalised Aarseth step
 * criterion; Makino 1991 / Aarseth 2003: power-of-two block steps). The readings
 * taken where the paper is silent are listed with each function.
 *
 * Conventions
 *   - vectors are structure-of-arrays, component-major: x[k*n + i], k = 0..2;
 *   - evaluation output is out[c*n_act + q], c = 0..9 = ax ay az jx jy jz sx sy sz phi;
 *   - time is an int64 tick count, one tick = 2^dt_min_log2; a body on level k
 *     has step dt = 2^(dt_max_log2 - k), i.e. 2^(L - k) ticks, L = dt_max_log2 - dt_min_log2;
 *   - all arithmetic is IEEE binary64 with no contraction (built -ffp-contract=off);
 *     every sum over bodies is a Neumaier-compensated sum in ascending index order.
 *
 * Return codes: 0 ok, 1 bad argument, 2 numeric failure (non-finite value or a
 * step below the smallest level).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_NUMERIC 2

/* ---------------------------------------------------------------- sums ---- */
/* Neumaier's improvement of Kahan summation: s + c carries the running sum with
 * the low-order part of every addition kept in c. */
typedef struct { double s, c; } csum;

static void cs_add(csum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double cs_val(const csum *a) { return a->s + a->c; }

/* ------------------------------------------------------ pairwise terms ---- */
/*
 * Evaluation of acceleration, jerk, snap and potential for the active bodies
 * (the O(N^2) kernel of section "Performance results").
 *
 * For an active body i and every j != i, with predicted positions, velocities and
 * accelerations, r = x_j - x_i, v = v_j - v_i, a = a_j - a_i and the Plummer-
 * softened squared distance R = r.r + eps^2:
 *     A = m_j r / R^(3/2)                       (acceleration term)
 *     J = dA/dt = m_j v / R^(3/2) - 3 alpha A,  alpha = (r.v) / R
 *     S = dJ/dt = m_j a / R^(3/2) - 6 alpha J - 3 beta A,
 *                                 beta = (v.v + r.a) / R + alpha^2
 *     phi_i -= m_j / R^(1/2)
 * J and S are the first and second time derivatives of A along the relative
 * motion r' = v, v' = a. Readings: softening enters only through R; the self pair
 * is excluded from every sum, the potential included. Sums run over j in
 * ascending order.
 */
int nbo_evaluate(int64_t n, const double *m, const double *xp, const double *vp,
                 const double *ap, double eps, int64_t n_act, const int32_t *idx,
                 double *out, int nthreads)
{
    if (n < 0 || n_act < 0 || n_act > n || eps < 0.0 || nthreads < 1)
        return ORC_ERR_ARG;
    for (int64_t q = 0; q < n_act; ++q)
        if (idx[q] < 0 || idx[q] >= n)
            return ORC_ERR_ARG;
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t q = 0; q < n_act; ++q) {
        const int64_t i = idx[q];
        csum acc[10];
        memset(acc, 0, sizeof acc);
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double r[3], v[3], a[3];
            for (int k = 0; k < 3; ++k) {
                r[k] = xp[k * n + j] - xp[k * n + i];
                v[k] = vp[k * n + j] - vp[k * n + i];
                a[k] = ap[k * n + j] - ap[k * n + i];
            }
            const double R = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
            const double sqR = sqrt(R);
            const double m3 = m[j] / (R * sqR);          /* m_j R^(-3/2) */
            const double alpha = (r[0] * v[0] + r[1] * v[1] + r[2] * v[2]) / R;
            const double beta = (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]
                                 + r[0] * a[0] + r[1] * a[1] + r[2] * a[2]) / R
                                + alpha * alpha;
            double A[3], J[3], S[3];
            for (int k = 0; k < 3; ++k) {
                A[k] = m3 * r[k];
                J[k] = m3 * v[k] - 3.0 * alpha * A[k];
                S[k] = m3 * a[k] - 6.0 * alpha * J[k] - 3.0 * beta * A[k];
            }
            for (int k = 0; k < 3; ++k) {
                cs_add(&acc[k], A[k]);
                cs_add(&acc[3 + k], J[k]);
                cs_add(&acc[6 + k], S[k]);
            }
            cs_add(&acc[9], -(m[j] / sqR));
        }
        for (int c = 0; c < 10; ++c)
            out[c * n_act + q] = cs_val(&acc[c]);
    }
    return ORC_OK;
}

/*
 * The same evaluation extended by one derivative: crackle, the third time
 * derivative of the acceleration (the term an 8th-order Hermite scheme, or an
 * exact initial third derivative for the 6th-order one, needs; Nitadori & Makino
 * 2008). With j = j_j - j_i the relative predicted jerk, along r' = v, v' = a,
 * a' = j:
 *     C = dS/dt = m_j j / R^(3/2) - 9 alpha S - 9 beta J - 3 gamma A,
 *     gamma = (3 v.a + r.j) / R + alpha (3 beta - 4 alpha^2)
 * (alpha' = beta - 3 alpha^2 and beta' = (3 v.a + r.j) / R - 4 alpha^3 give it).
 * Output out[c*n_act + q], c = 0..12 = a(3) j(3) s(3) c(3) phi.
 */
int nbo_evaluate_crackle(int64_t n, const double *m, const double *xp, const double *vp,
                         const double *ap, const double *jp, double eps, int64_t n_act,
                         const int32_t *idx, double *out, int nthreads)
{
    if (n < 0 || n_act < 0 || n_act > n || eps < 0.0 || nthreads < 1)
        return ORC_ERR_ARG;
    for (int64_t q = 0; q < n_act; ++q)
        if (idx[q] < 0 || idx[q] >= n)
            return ORC_ERR_ARG;
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t q = 0; q < n_act; ++q) {
        const int64_t i = idx[q];
        csum acc[13];
        memset(acc, 0, sizeof acc);
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double r[3], v[3], a[3], jj[3];
            for (int k = 0; k < 3; ++k) {
                r[k] = xp[k * n + j] - xp[k * n + i];
                v[k] = vp[k * n + j] - vp[k * n + i];
                a[k] = ap[k * n + j] - ap[k * n + i];
                jj[k] = jp[k * n + j] - jp[k * n + i];
            }
            const double R = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
            const double sqR = sqrt(R);
            const double m3 = m[j] / (R * sqR);
            const double va = v[0] * a[0] + v[1] * a[1] + v[2] * a[2];
            const double rj = r[0] * jj[0] + r[1] * jj[1] + r[2] * jj[2];
            const double alpha = (r[0] * v[0] + r[1] * v[1] + r[2] * v[2]) / R;
            const double beta = (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]
                                 + r[0] * a[0] + r[1] * a[1] + r[2] * a[2]) / R
                                + alpha * alpha;
            const double gamma = (3.0 * va + rj) / R + alpha * (3.0 * beta - 4.0 * alpha * alpha);
            double A[3], J[3], S[3], C[3];
            for (int k = 0; k < 3; ++k) {
                A[k] = m3 * r[k];
                J[k] = m3 * v[k] - 3.0 * alpha * A[k];
                S[k] = m3 * a[k] - 6.0 * alpha * J[k] - 3.0 * beta * A[k];
                C[k] = m3 * jj[k] - 9.0 * alpha * S[k] - 9.0 * beta * J[k] - 3.0 * gamma * A[k];
            }
            for (int k = 0; k < 3; ++k) {
                cs_add(&acc[k], A[k]);
                cs_add(&acc[3 + k], J[k]);
                cs_add(&acc[6 + k], S[k]);
                cs_add(&acc[9 + k], C[k]);
            }
            cs_add(&acc[12], -(m[j] / sqR));
        }
        for (int c = 0; c < 13; ++c)
            out[c * n_act + q] = cs_val(&acc[c]);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------ predictor ---- */
/*
 * Taylor prediction of every body to the block time t_next, h = t_next - t_i:
 *     xp = x + h v + h^2/2 a + h^3/6 j + h^4/24 s + h^5/120 c
 *     vp = v + h a + h^2/2 j + h^3/6 s + h^4/24 c
 *     ap = a + h j + h^2/2 s + h^3/6 c
 * where c is the third derivative of a interpolated by the previous corrector
 * (zero before the first step). Reading: the series stops at that term.
 */
int nbo_predict(int64_t n, const int64_t *tick, int64_t tick_next, int dt_min_log2,
                const double *x, const double *v, const double *a, const double *jk,
                const double *s, const double *c, double *xp, double *vp, double *ap)
{
    if (n < 0)
        return ORC_ERR_ARG;
    const double tick_size = ldexp(1.0, dt_min_log2);
    for (int64_t i = 0; i < n; ++i) {
        if (tick[i] > tick_next)
            return ORC_ERR_ARG;
        const double h = (double)(tick_next - tick[i]) * tick_size;
        const double f2 = h * h / 2.0;
        const double f3 = h * h * h / 6.0;
        const double f4 = h * h * h * h / 24.0;
        const double f5 = h * h * h * h * h / 120.0;
        for (int k = 0; k < 3; ++k) {
            const int64_t e = k * n + i;
            xp[e] = x[e] + h * v[e] + f2 * a[e] + f3 * jk[e] + f4 * s[e] + f5 * c[e];
            vp[e] = v[e] + h * a[e] + f2 * jk[e] + f3 * s[e] + f4 * c[e];
            ap[e] = a[e] + h * jk[e] + f2 * s[e] + f3 * c[e];
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------ corrector ---- */
/*
 * Sixth-order Hermite corrector for the active bodies over h = t_next - t_i, from
 * the old (a0, j0, s0) and the new evaluation (a1, j1, s1):
 *     v1 = v0 + h/2 (a0 + a1) - h^2/10 (j1 - j0) + h^3/120 (s0 + s1)
 *     x1 = x0 + h/2 (v0 + v1) - h^2/10 (a1 - a0) + h^3/120 (j0 + j1)
 * Then the third, fourth and fifth derivatives of a at t_next, from the unique
 * quintic through (a, j, s) at both ends of the step:
 *     a3 = [ 60 (a1-a0) - h (36 j1 + 24 j0) + h^2 ( 9 s1 -  3 s0)] / h^3
 *     a4 = [360 (a1-a0) - h(192 j1 + 168 j0) + h^2 (36 s1 - 24 s0)] / h^4
 *     a5 = [720 (a1-a0) - 360 h (j1 + j0)    + 60 h^2 (s1 - s0)]    / h^5
 * The new a, j, s are kept as the body's derivatives (one evaluation per step);
 * a3 becomes the crackle c used by the next prediction; |a4| and |a5| feed the
 * step criterion. Finally t_i = t_next.
 * anew is an evaluation output, anew[c*n_act + q] for the q-th active body.
 */
int nbo_correct(int64_t n, int64_t n_act, const int32_t *idx, int64_t tick_next,
                int dt_min_log2, const double *anew, int64_t *tick, double *x,
                double *v, double *a, double *jk, double *s, double *c,
                double *a4n, double *a5n)
{
    if (n < 0 || n_act < 0 || n_act > n)
        return ORC_ERR_ARG;
    const double tick_size = ldexp(1.0, dt_min_log2);
    int status = ORC_OK;
    for (int64_t q = 0; q < n_act; ++q) {
        const int64_t i = idx[q];
        if (i < 0 || i >= n || tick[i] >= tick_next)
            return ORC_ERR_ARG;
        const double h = (double)(tick_next - tick[i]) * tick_size;
        const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
        double a4sq = 0.0, a5sq = 0.0;
        for (int k = 0; k < 3; ++k) {
            const int64_t e = k * n + i;
            const double a0 = a[e], j0 = jk[e], s0 = s[e];
            const double a1 = anew[(0 + k) * n_act + q];
            const double j1 = anew[(3 + k) * n_act + q];
            const double s1 = anew[(6 + k) * n_act + q];
            const double v0 = v[e], x0 = x[e];
            const double v1 = v0 + h / 2.0 * (a0 + a1) - h2 / 10.0 * (j1 - j0)
                              + h3 / 120.0 * (s0 + s1);
            const double x1 = x0 + h / 2.0 * (v0 + v1) - h2 / 10.0 * (a1 - a0)
                              + h3 / 120.0 * (j0 + j1);
            const double d3 = (60.0 * (a1 - a0) - h * (36.0 * j1 + 24.0 * j0)
                               + h2 * (9.0 * s1 - 3.0 * s0)) / h3;
            const double d4 = (360.0 * (a1 - a0) - h * (192.0 * j1 + 168.0 * j0)
                               + h2 * (36.0 * s1 - 24.0 * s0)) / h4;
            const double d5 = (720.0 * (a1 - a0) - 360.0 * h * (j1 + j0)
                               + 60.0 * h2 * (s1 - s0)) / h5;
            x[e] = x1;
            v[e] = v1;
            a[e] = a1;
            jk[e] = j1;
            s[e] = s1;
            c[e] = d3;
            a4sq += d4 * d4;
            a5sq += d5 * d5;
            if (!isfinite(x1) || !isfinite(v1) || !isfinite(d3) || !isfinite(d4)
                || !isfinite(d5))
                status = ORC_ERR_NUMERIC;
        }
        a4n[i] = sqrt(a4sq);
        a5n[i] = sqrt(a5sq);
        tick[i] = tick_next;
    }
    return status;
}

/* ----------------------------------------------------------- time steps ---- */
static double norm3(const double *p, int64_t n, int64_t i)
{
    const double x = p[i], y = p[n + i], z = p[2 * n + i];
    return sqrt(x * x + y * y + z * z);
}

/*
 * Block time steps for the active bodies, at their (new) time tick[i].
 *
 * Regular step (generalised Aarseth criterion of order p = 6, exponent
 * 1/(p - 3) = 1/3):
 *     Delta = eta * [ (sqrt(|a| |s|) + |j|) / (sqrt(|a3| |a5|) + |a4|) ]^(1/3)
 * Initial step (init != 0): Delta = eta_init * min(|a|/|j|, sqrt(|a|/|s|)).
 * Quantisation: dt is a power of two 2^(dt_max_log2 - k), k >= 0; the candidate
 * is the largest such dt <= min(Delta, dt_max). Without taking a cube root, a
 * level fits the regular criterion when dt^3 <= eta^3 * ratio.
 * Block rules for a regular step: shrinking is allowed to any fitting level;
 * growing is by one level (x2) only, and only when the body's time is a multiple
 * of the doubled step and the doubled step fits. Otherwise the level stays. At
 * init the level must also divide the body's time.
 * A body that fits no level up to L (dt_min) is a numeric failure; its level is
 * clamped to L. Zero or non-finite denominators mean "no constraint" (level 0).
 * Readings: exponent form and eta_init start as stated above; the paper gives
 * neither formula. Pins: on a circular orbit (|a^(k)| = |a| omega^k) the criterion
 * is eta / omega and the start rule eta_init / omega, whatever the radius; the block
 * rules, the power-of-two quantisation and the time divisibility by hand cases.
 */
int nbo_timesteps(int64_t n, int64_t n_act, const int32_t *idx, int init,
                  const int64_t *tick, int32_t *level, const double *a,
                  const double *jk, const double *s, const double *c,
                  const double *a4n, const double *a5n, double eta, double eta_init,
                  int dt_max_log2, int dt_min_log2)
{
    const int L = dt_max_log2 - dt_min_log2;
    if (n < 0 || n_act < 0 || n_act > n || L < 0 || L > 62 || !(eta > 0.0)
        || !(eta_init > 0.0))
        return ORC_ERR_ARG;
    int status = ORC_OK;
    for (int64_t q = 0; q < n_act; ++q) {
        const int64_t i = idx[q];
        if (i < 0 || i >= n)
            return ORC_ERR_ARG;
        const double an = norm3(a, n, i), jn = norm3(jk, n, i), sn = norm3(s, n, i);
        int kc = -1;
        if (init) {
            double d0;
            const double ra = (jn > 0.0) ? an / jn : INFINITY;
            const double rs = (sn > 0.0) ? sqrt(an / sn) : INFINITY;
            d0 = eta_init * (ra < rs ? ra : rs);
            if (isnan(d0))
                d0 = INFINITY;
            for (int k = 0; k <= L; ++k)
                if (ldexp(1.0, dt_max_log2 - k) <= d0) { kc = k; break; }
        } else {
            const double cn = norm3(c, n, i);
            const double num = sqrt(an * sn) + jn;
            const double den = sqrt(cn * a5n[i]) + a4n[i];
            double qv = INFINITY;
            if (den > 0.0)
                qv = (eta * eta * eta) * (num / den);
            if (isnan(qv) || !(den > 0.0) || isinf(den))
                qv = INFINITY;
            for (int k = 0; k <= L; ++k)
                if (ldexp(1.0, 3 * (dt_max_log2 - k)) <= qv) { kc = k; break; }
        }
        if (kc < 0) {
            kc = L;
            status = ORC_ERR_NUMERIC;
        }
        const int64_t t = tick[i];
        int knew;
        if (init) {
            knew = kc;
            while (knew < L && (t % ((int64_t)1 << (L - knew))) != 0)
                ++knew;
        } else {
            const int kold = level[i];
            if (kc > kold)
                knew = kc;
            else if (kold >= 1 && kc <= kold - 1
                     && (t % ((int64_t)1 << (L - kold + 1))) == 0)
                knew = kold - 1;
            else
                knew = kold;
        }
        level[i] = knew;
    }
    return status;
}

/* ----------------------------------------------------------- active set ---- */
/*
 * Next block time t_next = min_i (t_i + dt_i) and the active set
 * {i : t_i + dt_i == t_next}, in ascending index order. Returns its size (or -1
 * on a bad argument) and writes t_next.
 */
int64_t nbo_active(int64_t n, const int64_t *tick, const int32_t *level, int L,
                   int32_t *idx_out, int64_t *tick_next)
{
    if (n < 1 || L < 0 || L > 62)
        return -1;
    int64_t tn = INT64_MAX;
    for (int64_t i = 0; i < n; ++i) {
        if (level[i] < 0 || level[i] > L)
            return -1;
        const int64_t e = tick[i] + ((int64_t)1 << (L - level[i]));
        if (e < tn)
            tn = e;
    }
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i)
        if (tick[i] + ((int64_t)1 << (L - level[i])) == tn)
            idx_out[cnt++] = (int32_t)i;
    *tick_next = tn;
    return cnt;
}

/* --------------------------------------------------------------- energy ---- */
/*
 * Total energy of a (synchronised or predicted) state with Plummer softening:
 *     E_kin = sum_i m_i |v_i|^2 / 2
 *     E_pot = -1/2 sum_i sum_{j != i} m_i m_j / sqrt(|x_j - x_i|^2 + eps^2)
 */
int nbo_energy(int64_t n, const double *m, const double *x, const double *v,
               double eps, double *ekin, double *epot, int nthreads)
{
    if (n < 0 || eps < 0.0 || nthreads < 1)
        return ORC_ERR_ARG;
    const double eps2 = eps * eps;
    double *phi = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!phi)
        return ORC_ERR_ARG;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t i = 0; i < n; ++i) {
        csum p = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            const double dx = x[j] - x[i], dy = x[n + j] - x[n + i],
                         dz = x[2 * n + j] - x[2 * n + i];
            cs_add(&p, m[j] / sqrt(dx * dx + dy * dy + dz * dz + eps2));
        }
        phi[i] = cs_val(&p);
    }
    csum ek = {0.0, 0.0}, ep = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        const double vx = v[i], vy = v[n + i], vz = v[2 * n + i];
        cs_add(&ek, 0.5 * m[i] * (vx * vx + vy * vy + vz * vz));
        cs_add(&ep, -0.5 * m[i] * phi[i]);
    }
    free(phi);
    *ekin = cs_val(&ek);
    *epot = cs_val(&ep);
    return ORC_OK;
}

/* ------------------------------------------------------------ integrate ---- */
/*
 * Full block-step integration from a synchronised state at tick t0 to tick_end
 * (tick_end - t0 must be a multiple of dt_max so every body lands on it).
 *
 * Start: predicted state = state; pass 1 evaluates a and j (they do not depend on
 * the predicted accelerations), pass 2 evaluates s with the predicted
 * accelerations set to the pass-1 a; c = 0, or with start_crackle a third pass
 * that evaluates the crackle with the predicted jerks set to the pass-2 j and
 * stores it as c; initial levels from the init rule.
 * Step: active set and t_next; predict every body to t_next; evaluate the active
 * bodies; correct them; new levels for them. Repeat until t_next > tick_end.
 *
 * State arrays are updated in place (x, v, a, jk, s, c, a4n, a5n [3][n] or [n],
 * tick, level). step_tick/step_nact (capacity max_steps, may be NULL) record
 * each block step. Returns the number of steps, or a negative code.
 */
int64_t nbo_integrate(int64_t n, const double *m, double *x, double *v, double *a,
                      double *jk, double *s, double *c, double *a4n, double *a5n,
                      int64_t *tick, int32_t *level, double eps, double eta,
                      double eta_init, int dt_max_log2, int dt_min_log2,
                      int64_t tick_end, int64_t max_steps, int64_t *step_tick,
                      int64_t *step_nact, double *interactions, int start_crackle,
                      int nthreads)
{
    const int L = dt_max_log2 - dt_min_log2;
    if (n < 1 || L < 0 || L > 62 || max_steps < 0)
        return -ORC_ERR_ARG;
    const size_t n3 = 3 * (size_t)n;
    double *xp = (double *)malloc(sizeof(double) * n3);
    double *vp = (double *)malloc(sizeof(double) * n3);
    double *ap = (double *)malloc(sizeof(double) * n3);
    double *out = (double *)malloc(sizeof(double) * 10 * (size_t)n);
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t steps = 0;
    int rc = ORC_OK;
    double inter = 0.0;
    if (!xp || !vp || !ap || !out || !idx) {
        rc = ORC_ERR_ARG;
        goto done;
    }
    const int64_t t0 = tick[0];
    for (int64_t i = 0; i < n; ++i)
        if (tick[i] != t0) { rc = ORC_ERR_ARG; goto done; }
    if (((tick_end - t0) % ((int64_t)1 << L)) != 0 || tick_end < t0) {
        rc = ORC_ERR_ARG;
        goto done;
    }
    /* start-up: two evaluation passes on the synchronised state */
    for (int64_t i = 0; i < n; ++i)
        idx[i] = (int32_t)i;
    memcpy(xp, x, sizeof(double) * n3);
    memcpy(vp, v, sizeof(double) * n3);
    memset(ap, 0, sizeof(double) * n3);
    rc = nbo_evaluate(n, m, xp, vp, ap, eps, n, idx, out, nthreads);
    if (rc) goto done;
    for (int k = 0; k < 3; ++k)
        for (int64_t i = 0; i < n; ++i)
            ap[k * n + i] = out[k * n + i];
    rc = nbo_evaluate(n, m, xp, vp, ap, eps, n, idx, out, nthreads);
    if (rc) goto done;
    inter += 2.0 * (double)n * (double)n;
    for (int k = 0; k < 3; ++k)
        for (int64_t i = 0; i < n; ++i) {
            a[k * n + i] = out[(0 + k) * n + i];
            jk[k * n + i] = out[(3 + k) * n + i];
            s[k * n + i] = out[(6 + k) * n + i];
            c[k * n + i] = 0.0;
        }
    for (int64_t i = 0; i < n; ++i)
        a4n[i] = a5n[i] = 0.0;
    if (start_crackle) {
        double *out13 = (double *)malloc(sizeof(double) * 13 * (size_t)n);
        if (!out13) { rc = ORC_ERR_ARG; goto done; }
        rc = nbo_evaluate_crackle(n, m, xp, vp, ap, jk, eps, n, idx, out13, nthreads);
        if (!rc)
            for (int k = 0; k < 3; ++k)
                for (int64_t i = 0; i < n; ++i)
                    c[k * n + i] = out13[(9 + k) * n + i];
        free(out13);
        if (rc) goto done;
        inter += (double)n * (double)n;
    }
    rc = nbo_timesteps(n, n, idx, 1, tick, level, a, jk, s, c, a4n, a5n, eta, eta_init,
                       dt_max_log2, dt_min_log2);
    if (rc) goto done;
    for (;;) {
        int64_t tn;
        const int64_t na = nbo_active(n, tick, level, L, idx, &tn);
        if (na < 0) { rc = ORC_ERR_ARG; goto done; }
        if (tn > tick_end)
            break;
        if (step_tick && steps < max_steps) step_tick[steps] = tn;
        if (step_nact && steps < max_steps) step_nact[steps] = na;
        rc = nbo_predict(n, tick, tn, dt_min_log2, x, v, a, jk, s, c, xp, vp, ap);
        if (rc) goto done;
        rc = nbo_evaluate(n, m, xp, vp, ap, eps, na, idx, out, nthreads);
        if (rc) goto done;
        inter += (double)na * (double)n;
        rc = nbo_correct(n, na, idx, tn, dt_min_log2, out, tick, x, v, a, jk, s, c,
                         a4n, a5n);
        if (rc) goto done;
        rc = nbo_timesteps(n, na, idx, 0, tick, level, a, jk, s, c, a4n, a5n, eta,
                           eta_init, dt_max_log2, dt_min_log2);
        if (rc) goto done;
        ++steps;
    }
done:
    free(xp); free(vp); free(ap); free(out); free(idx);
    if (interactions)
        *interactions = inter;
    return rc ? -rc : steps;
}
