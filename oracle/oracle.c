/*
 * oracle.c -- plain FP64 CPU oracle of the greedy-selection hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled and called by the test
 * suite, by the package's smoke check and by the benchmark's CPU-baseline leg,
 * never by the product path.  It shares no code, header or table with the HIP
 * library: it is written from the paper's equations in their own order, in
 * plain loops, in FP64, with no blocking or fusion.
 *
 * Conventions (readings of points the paper leaves open):
 *  - Matern kernel, half-integer nu, Euclidean distance r, length scale ell:
 *      nu=1/2: s2*exp(-r/ell)
 *      nu=3/2: s2*(1+a)exp(-a),          a = sqrt(3) r/ell
 *      nu=5/2: s2*(1+a+a^2/3)exp(-a),    a = sqrt(5) r/ell
 *    plus a nugget on the diagonal by index.
 *  - A candidate is valid while its tracked conditional variance exceeds
 *    1e-12 times its prior variance and it is not yet selected.
 *  - Argmax ties go to the smallest pool slot (pools are sorted by distance).
 *  - gap_t = (s1 - s2) / s1 over the two best valid scores (1 if one valid
 *    candidate, 0 if s1 == 0).
 *  - status: 0 ok, 1 stopped early (no valid candidate), 2 Theta_ss not PD.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    const double *x; /* [n][d] */
    int d;
    int two_nu;
    double ell, s2, nugget;
} orc_cov;

/* Matern covariance of two points (the kernel is never printed in the paper;
 * these are the textbook half-integer forms). */
double orc_matern(int two_nu, double ell, double s2, double r) {
    if (two_nu == 1) return s2 * exp(-r / ell);
    if (two_nu == 3) {
        double a = sqrt(3.0) * r / ell;
        return s2 * (1.0 + a) * exp(-a);
    }
    if (two_nu == 5) {
        double a = sqrt(5.0) * r / ell;
        return s2 * (1.0 + a + a * a / 3.0) * exp(-a);
    }
    return NAN;
}

static double theta(const orc_cov *c, int32_t i, int32_t j) {
    double s = 0.0;
    for (int k = 0; k < c->d; ++k) {
        double e = c->x[(int64_t)i * c->d + k] - c->x[(int64_t)j * c->d + k];
        s += e * e;
    }
    double v = orc_matern(c->two_nu, c->ell, c->s2, sqrt(s));
    if (i == j) v += c->nugget;
    return v;
}

/* Dense Cholesky in place (lower, row-major m x m).  Returns 0 or the 1-based
 * index of the first non-positive pivot. */
static int chol(double *A, int m) {
    for (int j = 0; j < m; ++j) {
        double p = A[j * m + j];
        for (int q = 0; q < j; ++q) p -= A[j * m + q] * A[j * m + q];
        if (!(p > 0.0)) return j + 1;
        double dj = sqrt(p);
        A[j * m + j] = dj;
        for (int r = j + 1; r < m; ++r) {
            double s = A[r * m + j];
            for (int q = 0; q < j; ++q) s -= A[r * m + q] * A[j * m + q];
            A[r * m + j] = s / dj;
        }
    }
    return 0;
}

/* Column of eq. L_col for the ordered index set s (s[0] is the column's own
 * index): x = Theta_ss^{-1} e_1, values = x / sqrt(x_1).  Returns the status
 * (0 or 2) and writes -log x_1 = log Theta_{ii | s \ i} to *logcv. */
static int lcol(const orc_cov *c, const int32_t *s, int m, double *vals, double *logcv) {
    double *A = (double *)malloc(sizeof(double) * m * m);
    double *y = (double *)malloc(sizeof(double) * m);
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) A[a * m + b] = theta(c, s[a], s[b]);
    int bad = chol(A, m);
    if (bad) {
        for (int a = 0; a < m; ++a) vals[a] = NAN;
        *logcv = NAN;
        free(A); free(y);
        return 2;
    }
    /* forward: R y = e_1 */
    for (int a = 0; a < m; ++a) {
        double r = (a == 0) ? 1.0 : 0.0;
        for (int q = 0; q < a; ++q) r -= A[a * m + q] * y[q];
        y[a] = r / A[a * m + a];
    }
    /* back: R^T x = y */
    for (int a = m - 1; a >= 0; --a) {
        double r = y[a];
        for (int q = a + 1; q < m; ++q) r -= A[q * m + a] * vals[q];
        vals[a] = r / A[a * m + a];
    }
    double x1 = vals[0];
    double sc = 1.0 / sqrt(x1);
    for (int a = 0; a < m; ++a) vals[a] *= sc;
    *logcv = -log(x1);
    free(A); free(y);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Single-target greedy selection by the Cholesky approach (Sec. 3.1,        */
/* eq. cond_select and eq. obj_gp; App. C.1), then eq. L_col.                */
/* ------------------------------------------------------------------------ */
/* Rows 0..C-1 are the pool, row C the target.  Outputs:
 *   sel[k]        selected ids in selection order, -1 padded
 *   gap[k]        top-two relative score gap per step (NaN padded)
 *   factor[k+1]   [0] = L_ii, [1+t] = entry of sel[t] (0 padded)
 *   logcv         log Theta_{ii | s_i \ i}
 *   var_out[C]    (optional) conditional variances of the pool after selection
 * Returns status. */
/* When `forced` is given, step t takes forced[t] (a pool id; -1 ends the
 * run) instead of the argmax and records, in FP64, the best score over valid
 * candidates (best_out[t]) and the forced pick's score (pick_out[t]): a replay
 * of another run's selection under exact arithmetic. */
/* When `diag` is given, step t records the tracked state before the pick:
 * diag[5t..5t+4] = var and cov of the best candidate, var and cov of the
 * second best (NaN when there is none), and the target's own conditional
 * variance. */
static int select_column_impl(const orc_cov *c, int32_t i, const int32_t *pool, int32_t C, int32_t k, int32_t *sel,
                              double *gap, double *factor, double *logcv, double *var_out, double *cov_out,
                              const int32_t *forced, double *best_out, double *pick_out, double *diag) {
    int32_t R = C + 1;
    int32_t kk = k < C ? k : C;
    double *L = (double *)calloc((size_t)R * (kk > 0 ? kk : 1), sizeof(double));
    double *var = (double *)malloc(sizeof(double) * R);
    double *prior = (double *)malloc(sizeof(double) * R);
    double *cov = (double *)malloc(sizeof(double) * R);
    double *u = (double *)malloc(sizeof(double) * R);
    char *taken = (char *)calloc(R, 1);
    int32_t *row_id = (int32_t *)malloc(sizeof(int32_t) * R);
    for (int32_t j = 0; j < C; ++j) row_id[j] = pool[j];
    row_id[C] = i;
    for (int32_t r = 0; r < R; ++r) {
        prior[r] = theta(c, row_id[r], row_id[r]);
        var[r] = prior[r];
        cov[r] = theta(c, i, row_id[r]);
    }
    double v = theta(c, i, i);
    (void)v;
    for (int32_t t = 0; t < k; ++t) { sel[t] = -1; gap[t] = NAN; }
    int status = 0;
    int32_t t;
    for (t = 0; t < kk; ++t) {
        /* score every valid candidate: cov^2 / var (eq. obj_gp) */
        int32_t best = -1, second = -1, nvalid = 0;
        double s1 = -INFINITY, s2 = -INFINITY;
        for (int32_t j = 0; j < C; ++j) {
            if (taken[j] || !(var[j] > 1e-12 * prior[j])) continue;
            ++nvalid;
            double sc = cov[j] * cov[j] / var[j];
            if (sc > s1) { s2 = s1; second = best; s1 = sc; best = j; }
            else if (sc > s2) { s2 = sc; second = j; }
        }
        if (diag) {
            diag[5 * t + 0] = best >= 0 ? var[best] : NAN;
            diag[5 * t + 1] = best >= 0 ? cov[best] : NAN;
            diag[5 * t + 2] = second >= 0 ? var[second] : NAN;
            diag[5 * t + 3] = second >= 0 ? cov[second] : NAN;
            diag[5 * t + 4] = var[C];
        }
        if (forced) {
            /* replay: take the given pick if it is a valid candidate */
            int32_t f = forced[t], fj = -1;
            if (f < 0) break;
            for (int32_t j = 0; j < C; ++j)
                if (pool[j] == f && !taken[j] && var[j] > 1e-12 * prior[j]) fj = j;
            if (fj < 0) { status = 5; break; }
            best_out[t] = s1;
            pick_out[t] = cov[fj] * cov[fj] / var[fj];
            best_out[k + t] = var[C]; /* the target's conditional variance before this step */
            best = fj;
        }
        if (nvalid == 0) { status = 1; break; }
        gap[t] = (nvalid == 1) ? 1.0 : (s1 == 0.0 ? 0.0 : (s1 - s2) / s1);
        /* new column of the partial Cholesky factor by left-looking (eq. cond_select) */
        double sd = sqrt(var[best]);
        for (int32_t r = 0; r < R; ++r) {
            double dot = 0.0;
            for (int32_t q = 0; q < t; ++q) dot += L[(int64_t)r * kk + q] * L[(int64_t)best * kk + q];
            u[r] = (theta(c, row_id[r], row_id[best]) - dot) / sd;
        }
        for (int32_t r = 0; r < R; ++r) L[(int64_t)r * kk + t] = u[r];
        /* rank-one downdate of variances and covariances with the target */
        double ui = u[C];
        for (int32_t r = 0; r < R; ++r) {
            var[r] -= u[r] * u[r];
            cov[r] -= u[r] * ui;
        }
        taken[best] = 1;
        sel[t] = pool[best];
    }
    int32_t nsel = t;
    if (var_out) for (int32_t j = 0; j < C; ++j) var_out[j] = var[j];
    if (cov_out) for (int32_t j = 0; j < C; ++j) cov_out[j] = cov[j];
    /* eq. L_col on s = [i, sel...] */
    int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (nsel + 1));
    s[0] = i;
    for (int32_t q = 0; q < nsel; ++q) s[q + 1] = sel[q];
    for (int32_t q = 0; q <= k; ++q) factor[q] = 0.0;
    int st = lcol(c, s, nsel + 1, factor, logcv);
    if (st) status = st;
    free(s); free(L); free(var); free(prior); free(cov); free(u); free(taken); free(row_id);
    return status;
}

int orc_select_column(const orc_cov *c, int32_t i, const int32_t *pool, int32_t C, int32_t k, int32_t *sel,
                      double *gap, double *factor, double *logcv, double *var_out, double *cov_out) {
    return select_column_impl(c, i, pool, C, k, sel, gap, factor, logcv, var_out, cov_out, NULL, NULL, NULL, NULL);
}

/* Replay of a given selection sequence (see select_column_impl); the factor
 * and log_condvar are eq. L_col on [i, forced...].  Status 5 marks a forced
 * pick that is not a valid candidate. */
int orc_replay_one(const double *x, int32_t d, int32_t two_nu, double ell, double s2, double nugget, int32_t target,
                   const int32_t *pool, int32_t C, int32_t k, const int32_t *forced, double *best_out,
                   double *pick_out, double *factor, double *logcv) {
    orc_cov c = {x, d, two_nu, ell, s2, nugget};
    int32_t *sel = (int32_t *)malloc(sizeof(int32_t) * (k > 0 ? k : 1));
    double *gap = (double *)malloc(sizeof(double) * (k > 0 ? k : 1));
    for (int32_t t = 0; t < k; ++t) { best_out[t] = NAN; best_out[k + t] = NAN; pick_out[t] = NAN; }
    int st = select_column_impl(&c, target, pool, C, k, sel, gap, factor, logcv, NULL, NULL, forced, best_out,
                                pick_out, NULL);
    free(sel); free(gap);
    return st;
}

void orc_select_and_factor(const double *x, int32_t d, int32_t two_nu, double ell, double s2, double nugget,
                           int64_t n_targets, const int32_t *targets, const int32_t *pool, const int32_t *pool_len,
                           int32_t stride, int32_t k, int32_t *sel, double *gap, double *factor, double *logcv,
                           uint8_t *status, int32_t nthreads) {
    orc_cov c = {x, d, two_nu, ell, s2, nugget};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_targets; ++t) {
        status[t] = (uint8_t)orc_select_column(&c, targets[t], pool + t * stride, pool_len[t], k, sel + t * k,
                                               gap + t * k, factor + t * (k + 1), logcv + t, NULL, NULL);
    }
}

/* Batched selection that also records, per step, the tracked state of the
 * two best candidates and of the target (diag [n_targets][k][5], see
 * select_column_impl). */
void orc_select_and_factor_diag(const double *x, int32_t d, int32_t two_nu, double ell, double s2, double nugget,
                                int64_t n_targets, const int32_t *targets, const int32_t *pool,
                                const int32_t *pool_len, int32_t stride, int32_t k, int32_t *sel, double *gap,
                                double *factor, double *logcv, uint8_t *status, double *diag, int32_t nthreads) {
    orc_cov c = {x, d, two_nu, ell, s2, nugget};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_targets; ++t) {
        double *dg = diag + t * 5 * (int64_t)k;
        for (int64_t e = 0; e < 5 * (int64_t)k; ++e) dg[e] = NAN;
        status[t] = (uint8_t)select_column_impl(&c, targets[t], pool + t * stride, pool_len[t], k, sel + t * k,
                                                gap + t * k, factor + t * (k + 1), logcv + t, NULL, NULL, NULL, NULL,
                                                NULL, dg);
    }
}

/* Single-column entry with extra diagnostics (tracked variances) for tests. */
int orc_select_one(const double *x, int32_t d, int32_t two_nu, double ell, double s2, double nugget, int32_t target,
                   const int32_t *pool, int32_t C, int32_t k, int32_t *sel, double *gap, double *factor,
                   double *logcv, double *var_out, double *cov_out) {
    orc_cov c = {x, d, two_nu, ell, s2, nugget};
    return orc_select_column(&c, target, pool, C, k, sel, gap, factor, logcv, var_out, cov_out);
}

/* ------------------------------------------------------------------------ */
/* Multi-target selection with two partial Cholesky factors (Sec. 5.2,       */
/* eq. greedy_mult; App. C.2) and aggregated entries (Sec. 5.1, eq. obj_mult; */
/* App. A.4, eq. L_precision).                                               */
/* ------------------------------------------------------------------------ */
/* Rows 0..C-1 pool, C..C+m-1 targets (ascending ids).  Factor B conditions on
 * the targets first, then on the selected points; factor A on the selected
 * points only.  score_j = 1 - var2_j / var1_j (the log-determinant decrease of
 * eq. greedy_mult, monotone).  Outputs:
 *   sel[k], gap[k]      as in the single-target case
 *   logdet              log det Theta_{TT | sel} = sum log pivots of the targets
 *                       plus sum_t (log var2 - log var1) at the picks
 *   post_var[m]         Theta_qq | sel by the direct formula of Alg. infer_select
 *   var1_tgt[m]         the factor-A target rows (same quantity, tracked)
 * Returns status (0, 1 early stop). */
static int multi_select_impl(const orc_cov *c, const int32_t *T, int32_t m, const int32_t *pool, int32_t C,
                             int32_t k, int32_t *sel, double *gap, double *logdet, double *post_var,
                             double *var1_tgt, const int32_t *forced, double *best_out, double *pick_out) {
    int32_t R = C + m;
    int32_t kk = k < C ? k : C;
    int32_t wa = kk > 0 ? kk : 1, wb = m + kk;
    double *A = (double *)calloc((size_t)R * wa, sizeof(double));
    double *B = (double *)calloc((size_t)R * wb, sizeof(double));
    double *var1 = (double *)malloc(sizeof(double) * R);
    double *var2 = (double *)malloc(sizeof(double) * R);
    double *prior = (double *)malloc(sizeof(double) * R);
    double *u1 = (double *)malloc(sizeof(double) * R);
    double *u2 = (double *)malloc(sizeof(double) * R);
    char *taken = (char *)calloc(R, 1);
    int32_t *row_id = (int32_t *)malloc(sizeof(int32_t) * R);
    for (int32_t j = 0; j < C; ++j) row_id[j] = pool[j];
    for (int32_t q = 0; q < m; ++q) row_id[C + q] = T[q];
    for (int32_t r = 0; r < R; ++r) {
        prior[r] = theta(c, row_id[r], row_id[r]);
        var1[r] = prior[r];
        var2[r] = prior[r];
    }
    /* factor B: condition on the targets, in order, by left-looking */
    double ldT = 0.0;
    for (int32_t q = 0; q < m; ++q) {
        int32_t piv = C + q;
        double pv = var2[piv];
        ldT += log(pv);
        double sd = sqrt(pv);
        for (int32_t r = 0; r < R; ++r) {
            double dot = 0.0;
            for (int32_t p = 0; p < q; ++p) dot += B[(int64_t)r * wb + p] * B[(int64_t)piv * wb + p];
            u2[r] = (theta(c, row_id[r], row_id[piv]) - dot) / sd;
        }
        for (int32_t r = 0; r < R; ++r) { B[(int64_t)r * wb + q] = u2[r]; var2[r] -= u2[r] * u2[r]; }
    }
    for (int32_t t = 0; t < k; ++t) { sel[t] = -1; gap[t] = NAN; }
    double ld = 0.0;
    int status = 0;
    int32_t t;
    for (t = 0; t < kk; ++t) {
        int32_t best = -1, nvalid = 0;
        double s1 = -INFINITY, s2 = -INFINITY;
        for (int32_t j = 0; j < C; ++j) {
            if (taken[j] || !(var1[j] > 1e-12 * prior[j]) || !(var2[j] > 1e-12 * prior[j])) continue;
            ++nvalid;
            /* conditioning on more points never raises a variance, so
             * var2 <= var1 and the score is >= 0 in exact arithmetic;
             * rounding below 0 is clamped (eq. greedy_mult) */
            double sc = 1.0 - var2[j] / var1[j];
            if (sc < 0.0) sc = 0.0;
            if (sc > s1) { s2 = s1; s1 = sc; best = j; }
            else if (sc > s2) s2 = sc;
        }
        if (forced) {
            /* replay: take the given pick if it is a valid candidate */
            int32_t f = forced[t], fj = -1;
            if (f < 0) break;
            for (int32_t j = 0; j < C; ++j)
                if (pool[j] == f && !taken[j] && var1[j] > 1e-12 * prior[j] && var2[j] > 1e-12 * prior[j]) fj = j;
            if (fj < 0) { status = 5; break; }
            best_out[t] = s1;
            pick_out[t] = fmax(0.0, 1.0 - var2[fj] / var1[fj]);
            best = fj;
        }
        if (nvalid == 0) { status = 1; break; }
        gap[t] = (nvalid == 1) ? 1.0 : (s1 == 0.0 ? 0.0 : (s1 - s2) / s1);
        double sd1 = sqrt(var1[best]), sd2 = sqrt(var2[best]);
        ld += log(var2[best]) - log(var1[best]);
        for (int32_t r = 0; r < R; ++r) {
            double th = theta(c, row_id[r], row_id[best]);
            double d1 = 0.0, d2 = 0.0;
            for (int32_t q = 0; q < t; ++q) d1 += A[(int64_t)r * wa + q] * A[(int64_t)best * wa + q];
            for (int32_t q = 0; q < m + t; ++q) d2 += B[(int64_t)r * wb + q] * B[(int64_t)best * wb + q];
            u1[r] = (th - d1) / sd1;
            u2[r] = (th - d2) / sd2;
        }
        for (int32_t r = 0; r < R; ++r) {
            A[(int64_t)r * wa + t] = u1[r];
            B[(int64_t)r * wb + m + t] = u2[r];
            var1[r] -= u1[r] * u1[r];
            var2[r] -= u2[r] * u2[r];
        }
        taken[best] = 1;
        sel[t] = pool[best];
    }
    int32_t nsel = t;
    if (logdet) *logdet = ldT + ld;
    if (var1_tgt) for (int32_t q = 0; q < m; ++q) var1_tgt[q] = var1[C + q];
    if (post_var) {
        /* Theta_qq - Theta_{q,I} Theta_{I,I}^{-1} Theta_{I,q}, directly */
        double *G = (double *)malloc(sizeof(double) * (nsel > 0 ? nsel * nsel : 1));
        double *w = (double *)malloc(sizeof(double) * (nsel > 0 ? nsel : 1));
        for (int32_t a = 0; a < nsel; ++a)
            for (int32_t b = 0; b < nsel; ++b) G[a * nsel + b] = theta(c, sel[a], sel[b]);
        int bad = chol(G, nsel);
        for (int32_t q = 0; q < m; ++q) {
            if (bad) { post_var[q] = NAN; continue; }
            for (int32_t a = 0; a < nsel; ++a) {
                double r = theta(c, sel[a], T[q]);
                for (int32_t p = 0; p < a; ++p) r -= G[a * nsel + p] * w[p];
                w[a] = r / G[a * nsel + a];
            }
            double qf = 0.0;
            for (int32_t a = 0; a < nsel; ++a) qf += w[a] * w[a];
            post_var[q] = theta(c, T[q], T[q]) - qf;
        }
        free(G); free(w);
    }
    free(A); free(B); free(var1); free(var2); free(prior); free(u1); free(u2); free(taken); free(row_id);
    return status;
}

int orc_multi_select(const orc_cov *c, const int32_t *T, int32_t m, const int32_t *pool, int32_t C, int32_t k,
                     int32_t *sel, double *gap, double *logdet, double *post_var, double *var1_tgt) {
    return multi_select_impl(c, T, m, pool, C, k, sel, gap, logdet, post_var, var1_tgt, NULL, NULL, NULL);
}

/* Replay of a given multi-target selection: per step the best valid score
 * and the forced pick's score (1 - var2/var1, FP64); logdet and post_var as
 * for the forced sequence.  Status 5: a forced pick was not valid. */
int orc_multi_replay_one(const double *x, int32_t d, int32_t two_nu, double ell, double s2, double nugget,
                         const int32_t *T, int32_t m, const int32_t *pool, int32_t C, int32_t k,
                         const int32_t *forced, double *best_out, double *pick_out, double *logdet,
                         double *post_var) {
    orc_cov c = {x, d, two_nu, ell, s2, nugget};
    int32_t *sel = (int32_t *)malloc(sizeof(int32_t) * (k > 0 ? k : 1));
    double *gap = (double *)malloc(sizeof(double) * (k > 0 ? k : 1));
    for (int32_t t = 0; t < k; ++t) { best_out[t] = NAN; pick_out[t] = NAN; }
    int st = multi_select_impl(&c, T, m, pool, C, k, sel, gap, logdet, post_var, NULL, forced, best_out, pick_out);
    free(sel); free(gap);
    return st;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Aggregated columns: s_g = sort(T u sel); member q gets s_q = {j in s_g : j >= q}
 * and the eq. L_col column on s_q, each solved independently.  Values for
 * member a (0-based within the group) start at vals + off[a], rows likewise;
 * off[a] = sum_{b<a} (m - b + nsel).  Returns the number of values written. */
int64_t orc_aggregated_columns(const orc_cov *c, const int32_t *T, int32_t m, const int32_t *sel, int32_t nsel,
                               int32_t *rows, double *vals, double *member_logcv, uint8_t *member_status) {
    int32_t ns = m + nsel;
    int32_t *sg = (int32_t *)malloc(sizeof(int32_t) * ns);
    for (int32_t q = 0; q < m; ++q) sg[q] = T[q];
    for (int32_t q = 0; q < nsel; ++q) sg[m + q] = sel[q];
    qsort(sg, ns, sizeof(int32_t), cmp_i32);
    int64_t off = 0;
    for (int32_t a = 0; a < m; ++a) {
        int32_t q = T[a];
        int32_t p0 = 0;
        while (sg[p0] != q) ++p0;
        int32_t len = ns - p0;
        for (int32_t b = 0; b < len; ++b) rows[off + b] = sg[p0 + b];
        member_status[a] = (uint8_t)lcol(c, sg + p0, len, vals + off, member_logcv + a);
        off += len;
    }
    free(sg);
    return off;
}

/* Batched aggregated selection over groups in CSR form.  For group g with
 * m_g members: sel at sel + g*k, logdet[g], and when rows/vals are given the
 * member columns at val_ptr[first member of g]. */
void orc_aggregated_select(const double *x, int32_t d, int32_t two_nu, double ell, double s2, double nugget,
                           int64_t n_groups, const int32_t *group_ptr, const int32_t *members, const int32_t *pool,
                           const int32_t *pool_len, int32_t stride, int32_t k, int32_t *sel, double *gap,
                           double *logdet, double *post_var, const int64_t *val_ptr, int32_t *rows, double *vals,
                           double *member_logcv, uint8_t *status, int32_t nthreads) {
    orc_cov c = {x, d, two_nu, ell, s2, nugget};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < n_groups; ++g) {
        int32_t b = group_ptr[g], m = group_ptr[g + 1] - b;
        int st = orc_multi_select(&c, members + b, m, pool + g * stride, pool_len[g], k, sel + g * k, gap + g * k,
                                  logdet ? logdet + g : NULL, post_var ? post_var + b : NULL, NULL);
        if (vals) {
            int32_t nsel = 0;
            while (nsel < k && sel[g * k + nsel] >= 0) ++nsel;
            uint8_t *mst = (uint8_t *)malloc(m);
            orc_aggregated_columns(&c, members + b, m, sel + g * k, nsel, rows + val_ptr[b], vals + val_ptr[b],
                                   member_logcv + b, mst);
            for (int32_t a = 0; a < m; ++a) if (mst[a]) st = mst[a];
            free(mst);
        }
        status[g] = (uint8_t)st;
    }
}

/* Single group with the tracked factor-A target variances (for tests). */
int orc_multi_one(const double *x, int32_t d, int32_t two_nu, double ell, double s2, double nugget, const int32_t *T,
                  int32_t m, const int32_t *pool, int32_t C, int32_t k, int32_t *sel, double *gap, double *logdet,
                  double *post_var, double *var1_tgt) {
    orc_cov c = {x, d, two_nu, ell, s2, nugget};
    return orc_multi_select(&c, T, m, pool, C, k, sel, gap, logdet, post_var, var1_tgt);
}

int64_t orc_aggregated_one(const double *x, int32_t d, int32_t two_nu, double ell, double s2, double nugget,
                           const int32_t *T, int32_t m, const int32_t *sel, int32_t nsel, int32_t *rows,
                           double *vals, double *member_logcv, uint8_t *member_status) {
    orc_cov c = {x, d, two_nu, ell, s2, nugget};
    return orc_aggregated_columns(&c, T, m, sel, nsel, rows, vals, member_logcv, member_status);
}

/* ------------------------------------------------------------------------ */
/* Sparse factor products (the factor is used through L^T x and L x, e.g.   */
/* as a preconditioner, Sec. 6.3).  CSC: column j holds rows                */
/* row_idx[col_ptr[j] .. col_ptr[j+1]) with values val[...].                */
/* ------------------------------------------------------------------------ */
void orc_apply_factor(int64_t n, const int64_t *col_ptr, const int32_t *row_idx, const double *val, int32_t transpose,
                      const double *xin, double *y) {
    /* entries whose row lies outside [0, n) are padding and are skipped */
    if (transpose) {
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; ++p)
                if (row_idx[p] >= 0 && row_idx[p] < n) s += val[p] * xin[row_idx[p]];
            y[j] = s;
        }
    } else {
        for (int64_t r = 0; r < n; ++r) y[r] = 0.0;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; ++p)
                if (row_idx[p] >= 0 && row_idx[p] < n) y[row_idx[p]] += val[p] * xin[j];
    }
}

/* Dense covariance matrix for small problems (tests). */
void orc_covariance(const double *x, int32_t n, int32_t d, int32_t two_nu, double ell, double s2, double nugget,
                    double *out) {
    orc_cov c = {x, d, two_nu, ell, s2, nugget};
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j) out[(int64_t)i * n + j] = theta(&c, i, j);
}
