/*
 * rapdhg_oracle.c -- plain FP64 CPU reference of rAPDHG.  TEST INFRASTRUCTURE
 * ONLY (tests, the smoke check and the CPU-baseline leg of the benchmark).
 *
 * Written from Lu & Yang, arXiv 2311.07710:
 *   - inner iteration: Algorithm 1 (restarted accelerated PDHG) with the
 *     parameters of Theorem 1 / eq. (param-choice) for beta_k and theta_k;
 *   - adaptive restart, step size and primal weight: Sec. 6 (PDQP.jl);
 *   - progress metric and termination: Sec. 5 (relative KKT error);
 *   - fixed-frequency and "halving" restarts: Algorithm 1 and Sec. 5;
 *   - the Sec. 5 baselines: PDHG without momentum (beta = theta = 1) with and
 *     without restarts.
 * Everything is unblocked: each row sum runs in CSR order, each dot product
 * runs from index 0 upward.  By default every loop is sequential.  For timing
 * on a multi-core host, orc_set_threads(t > 1) runs the row loops of the
 * matrix-vector products and the element-wise updates of the iteration on t
 * OpenMP threads; each output element is still computed by one thread with the
 * same operations in the same order (A'y then runs over a column-major copy of
 * A whose column lists hold the entries in increasing row order, the order in
 * which the sequential scatter adds them), so the results are bitwise those of
 * one thread.  The reductions (norms, dot products, relKKT terms) stay
 * sequential.
 */
#include "rapdhg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static int g_threads = 1;

void orc_set_threads(int32_t t) { g_threads = t < 1 ? 1 : t; }

int32_t orc_get_threads(void) { return g_threads; }

void orc_default_settings(orc_settings *s) {
    memset(s, 0, sizeof(*s));
    s->eps = 1e-6;               /* Sec. 5: high accuracy */
    s->max_iter = 200000;        /* Sec. 5 iteration limit */
    s->time_limit_s = 3600.0;    /* Sec. 6.1 time limit */
    s->check_every = 64;
    s->restart_mode = ORC_RESTART_ADAPTIVE;
    s->fixed_K = 100;
    s->beta_sufficient = 0.2;    /* Sec. 6, restart (i) */
    s->beta_necessary = 0.8;     /* Sec. 6, restart (ii) */
    s->beta_artificial = 0.36;   /* Sec. 6, restart (iii) */
    s->pw_smoothing = 0.2;       /* Sec. 6, primal weight theta */
    s->eps_zero = 1e-10;
    s->step_safety = 0.99;       /* Sec. 6 step-size rule */
    s->norm_A = 0.0;
    s->norm_Q = 0.0;
    s->power_iter_max = 1000;
    s->power_iter_rtol = 1e-7;
    s->warm_fallback = 1;
    s->momentum = 1;
    s->detect_infeasibility = 0;
    s->eps_infeasible = 1e-8;
}

/* ------------------------------------------------------------------ */
/* linear algebra                                                      */
/* ------------------------------------------------------------------ */
void orc_spmv(int64_t nrows, const int32_t *rowptr, const int32_t *col, const double *val,
              const double *x, double *y) {
#pragma omp parallel for num_threads(g_threads) if (g_threads > 1) schedule(static)
    for (int64_t i = 0; i < nrows; ++i) {
        double s = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            double prod = val[e] * x[col[e]];
            s = s + prod;
        }
        y[i] = s;
    }
}

void orc_spmv_t(int64_t nrows, int64_t ncols, const int32_t *rowptr, const int32_t *col,
                const double *val, const double *x, double *y) {
    for (int64_t j = 0; j < ncols; ++j) y[j] = 0.0;
    for (int64_t i = 0; i < nrows; ++i) {
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            double prod = val[e] * x[i];
            y[col[e]] = y[col[e]] + prod;
        }
    }
}

/* Column-major copy of an nrows x ncols CSR matrix: column j's entries in increasing
 * row order (and, within a row, in stored order), with their row indices. */
typedef struct {
    int32_t *colptr, *row;
    double *val;
} orc_csc;

static void csc_build(int64_t nrows, int64_t ncols, const int32_t *rowptr, const int32_t *col,
                      const double *val, orc_csc *t) {
    const int64_t nnz = rowptr[nrows];
    t->colptr = calloc((size_t)ncols + 1, sizeof(int32_t));
    t->row = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    t->val = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    for (int64_t e = 0; e < nnz; ++e) t->colptr[col[e] + 1]++;
    for (int64_t j = 0; j < ncols; ++j) t->colptr[j + 1] += t->colptr[j];
    int32_t *next = malloc(sizeof(int32_t) * (size_t)(ncols > 0 ? ncols : 1));
    for (int64_t j = 0; j < ncols; ++j) next[j] = t->colptr[j];
    for (int64_t i = 0; i < nrows; ++i)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int32_t q = next[col[e]]++;
            t->row[q] = (int32_t)i;
            t->val[q] = val[e];
        }
    free(next);
}

static void csc_free(orc_csc *t) {
    free(t->colptr); free(t->row); free(t->val);
}

/* y = A'x through the column-major copy: the same products, added to y[j] in the
 * same order as orc_spmv_t, one column per thread */
static void spmv_t_csc(int64_t ncols, const orc_csc *t, const double *x, double *y) {
#pragma omp parallel for num_threads(g_threads) if (g_threads > 1) schedule(static)
    for (int64_t j = 0; j < ncols; ++j) {
        double s = 0.0;
        for (int64_t q = t->colptr[j]; q < t->colptr[j + 1]; ++q) {
            double prod = t->val[q] * x[t->row[q]];
            s = s + prod;
        }
        y[j] = s;
    }
}

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double norm2(int64_t n, const double *a) { return sqrt(dot(n, a, a)); }

static double dist2(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = a[i] - b[i];
        s += d * d;
    }
    return sqrt(s);
}

/* projection onto X = [l, u] */
static double proj_box(double v, double lo, double hi) {
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

/* projection onto Y: y_i >= 0 on GE rows, free on EQ rows */
static double proj_dual(double v, uint8_t type) { return (type == 1 && v < 0.0) ? 0.0 : v; }

/* ------------------------------------------------------------------ */
/* relative KKT error (Sec. 5), generalised to EQ/GE rows and bounds   */
/* ------------------------------------------------------------------ */
void orc_rel_kkt(const orc_problem *p, const double *x, const double *y, orc_kkt *out) {
    const int64_t n = p->n, m = p->m;
    double *ax = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *qx = (double *)malloc(sizeof(double) * (size_t)n);
    double *aty = (double *)malloc(sizeof(double) * (size_t)n);
    orc_spmv(m, p->a_rowptr, p->a_col, p->a_val, x, ax);
    orc_spmv(n, p->q_rowptr, p->q_col, p->q_val, x, qx);
    orc_spmv_t(m, n, p->a_rowptr, p->a_col, p->a_val, y, aty);

    /* primal residual: EQ rows |A_i x - b_i|, GE rows [b_i - A_i x]_+ */
    double res_p = 0.0, ax_inf = 0.0, b_inf = 0.0, by = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double r = ax[i] - p->b[i];
        if (p->row_type[i] == 1) r = (r < 0.0) ? -r : 0.0;
        r = fabs(r);
        if (r > res_p || isnan(r)) res_p = r;
        if (fabs(ax[i]) > ax_inf || isnan(ax[i])) ax_inf = fabs(ax[i]);
        if (fabs(p->b[i]) > b_inf) b_inf = fabs(p->b[i]);
        by += p->b[i] * y[i];
    }
    /* reduced cost lambda = Qx + c - A'y; its admissible part lies in the
     * normal-cone directions allowed by the finite bounds */
    double res_d = 0.0, qx_inf = 0.0, aty_inf = 0.0, c_inf = 0.0;
    double xqx = 0.0, cx = 0.0, bound_term = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double lam = qx[j] + p->c[j] - aty[j];
        int lo_fin = isfinite(p->l[j]), hi_fin = isfinite(p->u[j]);
        double lam_hat;
        if (lo_fin && hi_fin) lam_hat = lam;
        else if (lo_fin) lam_hat = lam > 0.0 ? lam : 0.0;
        else if (hi_fin) lam_hat = lam < 0.0 ? lam : 0.0;
        else lam_hat = 0.0;
        double dres = fabs(lam - lam_hat);
        if (dres > res_d || isnan(dres)) res_d = dres;
        if (fabs(qx[j]) > qx_inf || isnan(qx[j])) qx_inf = fabs(qx[j]);
        if (fabs(aty[j]) > aty_inf || isnan(aty[j])) aty_inf = fabs(aty[j]);
        if (fabs(p->c[j]) > c_inf) c_inf = fabs(p->c[j]);
        xqx += x[j] * qx[j];
        cx += p->c[j] * x[j];
        if (lo_fin && lam_hat > 0.0) bound_term += p->l[j] * lam_hat;
        if (hi_fin && lam_hat < 0.0) bound_term += p->u[j] * lam_hat;
    }
    double P = 0.5 * xqx + cx;
    double D = -0.5 * xqx + by + bound_term;
    out->ax_inf = ax_inf; out->b_inf = b_inf; out->qx_inf = qx_inf; out->aty_inf = aty_inf;
    out->c_inf = c_inf; out->xqx = xqx; out->cx = cx; out->by = by;
    out->primal_obj = P;
    out->dual_obj = D;
    out->r_primal = res_p / (1.0 + fmax(ax_inf, b_inf));
    out->r_dual = res_d / (1.0 + fmax(fmax(qx_inf, aty_inf), c_inf));
    out->r_gap = fabs(P - D) / (1.0 + fmax(fabs(P), fabs(D)));
    double r = out->r_primal;
    if (out->r_dual > r) r = out->r_dual;
    if (out->r_gap > r) r = out->r_gap;
    if (isnan(out->r_primal) || isnan(out->r_dual) || isnan(out->r_gap)) r = NAN;
    out->rel_kkt = r;
    free(ax); free(qx); free(aty);
}

/* ------------------------------------------------------------------ */
/* operator norms by power iteration (the paper does not say how ||A|| */
/* and ||Q|| are obtained; the Rayleigh quotient is iterated until its */
/* relative change drops below rtol)                                   */
/* ------------------------------------------------------------------ */
double orc_norm_A(const orc_problem *p, int32_t maxit, double rtol, int32_t *iters_out) {
    const int64_t n = p->n, m = p->m;
    if (m == 0 || p->a_rowptr[m] == 0) { if (iters_out) *iters_out = 0; return 0.0; }
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)m);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) v[j] = 1.0 / sqrt((double)n);
    double lam = 0.0, lam_prev = 0.0;
    int32_t it = 0;
    for (it = 1; it <= maxit; ++it) {
        orc_spmv(m, p->a_rowptr, p->a_col, p->a_val, v, w);
        lam = dot(m, w, w);                      /* v'A'Av with ||v|| = 1 */
        orc_spmv_t(m, n, p->a_rowptr, p->a_col, p->a_val, w, z);
        double nz = norm2(n, z);
        if (nz == 0.0) break;
        for (int64_t j = 0; j < n; ++j) v[j] = z[j] / nz;
        if (it > 1 && fabs(lam - lam_prev) <= rtol * lam) break;
        lam_prev = lam;
    }
    if (iters_out) *iters_out = it > maxit ? maxit : it;
    free(v); free(w); free(z);
    return sqrt(lam);
}

double orc_norm_Q(const orc_problem *p, int32_t maxit, double rtol, int32_t *iters_out) {
    const int64_t n = p->n;
    if (p->q_rowptr[n] == 0) { if (iters_out) *iters_out = 0; return 0.0; }
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) v[j] = 1.0 / sqrt((double)n);
    double lam = 0.0, lam_prev = 0.0;
    int32_t it = 0;
    for (it = 1; it <= maxit; ++it) {
        orc_spmv(n, p->q_rowptr, p->q_col, p->q_val, v, w);
        lam = dot(n, v, w);                      /* Rayleigh quotient, Q PSD */
        double nw = norm2(n, w);
        if (nw == 0.0) break;
        for (int64_t j = 0; j < n; ++j) v[j] = w[j] / nw;
        if (it > 1 && fabs(lam - lam_prev) <= rtol * fabs(lam)) break;
        lam_prev = lam;
    }
    if (iters_out) *iters_out = it > maxit ? maxit : it;
    free(v); free(w);
    return fabs(lam);
}

/* ------------------------------------------------------------------ */
/* step scalars                                                        */
/* ------------------------------------------------------------------ */
/* Sec. 6: eta^{n,k} cap = 0.99 (k+2) / (||Q||/w + sqrt(||A||^2 (k+2)^2 + ||Q||^2/w^2));
 * at k = 0 this is the 1.98 / (...) start value.  Primal step eta/w, dual eta*w. */
static double pdqp_cap(const orc_settings *s, double nA, double nQ, double w, int64_t k) {
    double kk = (double)(k + 2);
    double qw = nQ / w;
    return s->step_safety * kk / (qw + sqrt(nA * nA * kk * kk + qw * qw));
}

/* Step scalars for inner index k of a cycle.  *s_last carries the PDQP scale
 * s_{k-1} of the same cycle (ignored at k = 0) and is updated to s_k. */
static void step_at(const orc_settings *s, double nA, double nQ, double omega, int64_t k,
                    double *s_last, double *p, double *d) {
    if (!s->momentum) {
        /* plain PDHG: beta = 1 in the step condition 1/p - ||Q||/beta - ||A||^2 d >= 0,
         * i.e. the Sec. 6 cap with (k+2) replaced by 2, held constant over the cycle */
        double qw = nQ / omega;
        double sk = s->step_safety * 2.0 / (qw + sqrt(4.0 * nA * nA + qw * qw));
        *s_last = sk;
        *p = sk / omega;
        *d = sk * omega;
        return;
    }
    if (s->restart_mode == ORC_RESTART_FIXED_K) {
        /* Theorem 1 / eq. (param-choice): eta_k = (k+1)/(2(||Q|| + K||A||)),
         * tau_k = (k+1)/(2 K ||A||) with K the restart frequency */
        double Kf = (double)s->fixed_K;
        *p = (double)(k + 1) / (2.0 * (nQ + Kf * nA));
        *d = nA > 0.0 ? (double)(k + 1) / (2.0 * Kf * nA) : 0.0;
        *s_last = 0.0;
        return;
    }
    double cap = pdqp_cap(s, nA, nQ, omega, k);
    double sk;
    if (k == 0) {
        sk = cap;
    } else {
        double grown = (1.0 + 1.0 / (double)k) * (*s_last);
        sk = grown < cap ? grown : cap;
    }
    *s_last = sk;
    *p = sk / omega;
    *d = sk * omega;
}

void orc_step_schedule(const orc_settings *s, double nA, double nQ, double omega, int64_t K,
                       double *p, double *d, double *scale) {
    double s_last = 0.0;
    for (int64_t k = 0; k < K; ++k) {
        step_at(s, nA, nQ, omega, k, &s_last, &p[k], &d[k]);
        if (scale) scale[k] = s_last;
    }
}

/* ------------------------------------------------------------------ */
/* the inner loop (Algorithm 1, mapped to the general form)            */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n, m;
    double *x, *x_prev, *xbar, *y, *ybar;
    double *xt, *xmd, *ax, *g, *aty;
    const orc_csc *at;  /* column-major copy of A for threaded runs, or NULL */
} orc_state;

static void state_alloc(orc_state *st, int64_t n, int64_t m) {
    st->n = n; st->m = m;
    size_t nn = (size_t)n * sizeof(double), mm = (size_t)(m > 0 ? m : 1) * sizeof(double);
    st->x = malloc(nn); st->x_prev = malloc(nn); st->xbar = malloc(nn);
    st->xt = malloc(nn); st->xmd = malloc(nn); st->g = malloc(nn); st->aty = malloc(nn);
    st->y = malloc(mm); st->ybar = malloc(mm); st->ax = malloc(mm);
    st->at = NULL;
}

static void state_free(orc_state *st) {
    free(st->x); free(st->x_prev); free(st->xbar); free(st->xt); free(st->xmd);
    free(st->g); free(st->aty); free(st->y); free(st->ybar); free(st->ax);
}

/* One iteration with inner index k, primal step pk, dual step dk.
 * Accelerated (Algorithm 1 with Theorem 1's weights): beta_k = (k+2)/2,
 * theta_k = k/(k+1); the running average z-bar takes weight 1/beta_k.
 * Plain PDHG (momentum = 0): beta = theta = 1, so Q is applied at x itself and
 * x~ = 2x - x_prev; z-bar is then the uniform average of the iterates of the
 * cycle (weight 1/(k+1)), the candidate of restarted PDHG. */
static void one_iteration(const orc_problem *p, orc_state *st, int momentum, int64_t k,
                          double pk, double dk) {
    const int64_t n = p->n, m = p->m;
    double w, theta, a;
    if (momentum) {
        w = 2.0 / (double)(k + 2);              /* 1/beta_k */
        theta = (double)k / (double)(k + 1);    /* theta_k */
        a = w;
    } else {
        w = 1.0;
        theta = 1.0;
        a = 1.0 / (double)(k + 1);
    }
    /* x_md = (1 - 1/beta) xbar + (1/beta) x ;  x~ = x + theta (x - x_prev) */
#pragma omp parallel for num_threads(g_threads) if (g_threads > 1) schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        st->xmd[j] = (1.0 - w) * st->xbar[j] + w * st->x[j];
        st->xt[j] = st->x[j] + theta * (st->x[j] - st->x_prev[j]);
    }
    /* dual step: y+ = proj_Y(y - d (A x~ - b)) */
    orc_spmv(m, p->a_rowptr, p->a_col, p->a_val, st->xt, st->ax);
#pragma omp parallel for num_threads(g_threads) if (g_threads > 1) schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double yn = st->y[i] - dk * (st->ax[i] - p->b[i]);
        st->y[i] = proj_dual(yn, p->row_type[i]);
    }
    /* primal step: x+ = proj_X(x - p (Q x_md + c - A' y+)) */
    orc_spmv(n, p->q_rowptr, p->q_col, p->q_val, st->xmd, st->g);
    if (st->at) spmv_t_csc(n, st->at, st->y, st->aty);
    else orc_spmv_t(m, n, p->a_rowptr, p->a_col, p->a_val, st->y, st->aty);
#pragma omp parallel for num_threads(g_threads) if (g_threads > 1) schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        double grad = st->g[j] + p->c[j] - st->aty[j];
        double xn = proj_box(st->x[j] - pk * grad, p->l[j], p->u[j]);
        st->x_prev[j] = st->x[j];
        st->x[j] = xn;
        st->xbar[j] = (1.0 - a) * st->xbar[j] + a * xn;
    }
#pragma omp parallel for num_threads(g_threads) if (g_threads > 1) schedule(static)
    for (int64_t i = 0; i < m; ++i) st->ybar[i] = (1.0 - a) * st->ybar[i] + a * st->y[i];
}

void orc_run_inner(const orc_problem *p, const orc_settings *s, double nA, double nQ,
                   double omega, int64_t iters, double *x, double *y, double *xbar, double *ybar) {
    orc_state st;
    state_alloc(&st, p->n, p->m);
    memcpy(st.x, x, sizeof(double) * (size_t)p->n);
    memcpy(st.x_prev, x, sizeof(double) * (size_t)p->n);
    memcpy(st.xbar, x, sizeof(double) * (size_t)p->n);
    if (p->m) {
        memcpy(st.y, y, sizeof(double) * (size_t)p->m);
        memcpy(st.ybar, y, sizeof(double) * (size_t)p->m);
    }
    double *pk = malloc(sizeof(double) * (size_t)(iters > 0 ? iters : 1));
    double *dk = malloc(sizeof(double) * (size_t)(iters > 0 ? iters : 1));
    orc_step_schedule(s, nA, nQ, omega, iters, pk, dk, NULL);
    for (int64_t k = 0; k < iters; ++k) one_iteration(p, &st, s->momentum, k, pk[k], dk[k]);
    memcpy(x, st.x, sizeof(double) * (size_t)p->n);
    memcpy(xbar, st.xbar, sizeof(double) * (size_t)p->n);
    if (p->m) {
        memcpy(y, st.y, sizeof(double) * (size_t)p->m);
        memcpy(ybar, st.ybar, sizeof(double) * (size_t)p->m);
    }
    free(pk); free(dk);
    state_free(&st);
}

/* ------------------------------------------------------------------ */
/* full solve: Algorithm 1 inner loop + Sec. 6 / Sec. 5 restart rules  */
/* ------------------------------------------------------------------ */
void orc_infeas_check(const orc_problem *p, const double *dx, const double *dy, orc_infeas *out) {
    const int64_t n = p->n, m = p->m;
    double *dyp = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *g = malloc(sizeof(double) * (size_t)n);
    double *dxp = malloc(sizeof(double) * (size_t)n);
    double *qd = malloc(sizeof(double) * (size_t)n);
    double *ad = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    /* primal infeasibility: Farkas direction dy projected onto the dual cone */
    dyp[0] = 0.0;
    for (int64_t i = 0; i < m; ++i) dyp[i] = (p->row_type[i] == 1 && dy[i] < 0.0) ? 0.0 : dy[i];
    orc_spmv_t(m, n, p->a_rowptr, p->a_col, p->a_val, dyp, g);
    double farkas = 0.0, viol = 0.0;
    for (int64_t i = 0; i < m; ++i) farkas = farkas + p->b[i] * dyp[i];
    for (int64_t j = 0; j < n; ++j) {
        double gj = g[j];
        if (gj > 0.0) {
            if (isfinite(p->u[j])) farkas = farkas - p->u[j] * gj;
            else if (gj > viol) viol = gj;
        } else if (gj < 0.0) {
            if (isfinite(p->l[j])) farkas = farkas - p->l[j] * gj;
            else if (-gj > viol) viol = -gj;
        }
    }
    out->primal_ratio = farkas > 0.0 ? viol / farkas : INFINITY;
    /* dual infeasibility: recession direction of X with c'dx < 0 */
    for (int64_t j = 0; j < n; ++j) {
        int lo = isfinite(p->l[j]), hi = isfinite(p->u[j]);
        double v = dx[j];
        if (lo && hi) v = 0.0;
        else if (lo && v < 0.0) v = 0.0;
        else if (hi && v > 0.0) v = 0.0;
        dxp[j] = v;
    }
    orc_spmv(n, p->q_rowptr, p->q_col, p->q_val, dxp, qd);
    orc_spmv(m, p->a_rowptr, p->a_col, p->a_val, dxp, ad);
    double cdx = 0.0, dv = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        cdx = cdx + p->c[j] * dxp[j];
        if (fabs(qd[j]) > dv) dv = fabs(qd[j]);
    }
    for (int64_t i = 0; i < m; ++i) {
        double r = p->row_type[i] == 1 ? (ad[i] < 0.0 ? -ad[i] : 0.0) : fabs(ad[i]);
        if (r > dv) dv = r;
    }
    out->dual_ratio = cdx < 0.0 ? dv / -cdx : INFINITY;
    free(dyp); free(g); free(dxp); free(qd); free(ad);
}

/* relKKT of (x, y).  Unscaled problem: directly.  Preconditioned problem: the point
 * is mapped back, x = D2 x~, y = D1 y~ (xu, yu are n- and m-sized work arrays), and
 * the error is that of the original problem (Sec. 5 measures the given instance). */
static void kkt_eval(const orc_problem *p, const orc_problem *orig, const double *dv,
                     const double *dr, const double *x, const double *y, double *xu, double *yu,
                     orc_kkt *out) {
    if (!orig) {
        orc_rel_kkt(p, x, y, out);
        return;
    }
    for (int64_t j = 0; j < p->n; ++j) xu[j] = x[j] * dv[j];
    for (int64_t i = 0; i < p->m; ++i) yu[i] = y[i] * dr[i];
    orc_rel_kkt(orig, xu, yu, out);
}

/* Certificates from the drift since the last restart, z - z_restart, measured on the
 * given problem (mapped back through D2, D1 when preconditioned). */
static int infeasible(const orc_problem *p, const orc_problem *orig, const double *dv,
                      const double *dr, const orc_state *st, const double *x_rs,
                      const double *y_rs, double *xu, double *yu, double tol, int *status) {
    const int64_t n = p->n, m = p->m;
    for (int64_t j = 0; j < n; ++j) {
        xu[j] = st->x[j] - x_rs[j];
        if (orig) xu[j] = xu[j] * dv[j];
    }
    for (int64_t i = 0; i < m; ++i) {
        yu[i] = st->y[i] - y_rs[i];
        if (orig) yu[i] = yu[i] * dr[i];
    }
    orc_infeas inf;
    orc_infeas_check(orig ? orig : p, xu, yu, &inf);
    if (inf.primal_ratio <= tol) {
        *status = ORC_PRIMAL_INFEASIBLE;
        return 1;
    }
    if (inf.dual_ratio <= tol) {
        *status = ORC_DUAL_INFEASIBLE;
        return 1;
    }
    return 0;
}

static int solve_impl(const orc_problem *p, const orc_problem *orig, const double *dv,
                      const double *dr, const orc_settings *s, const double *x0,
                      const double *y0, double omega0, double *x_out, double *y_out,
                      orc_result *res, orc_check_log *check_log, int64_t log_cap,
                      int64_t *log_len) {
    const int64_t n = p->n, m = p->m;
    const double t_start = now_s();
    memset(res, 0, sizeof(*res));
    if (log_len) *log_len = 0;

    double nA = s->norm_A > 0.0 ? s->norm_A
                                : orc_norm_A(p, s->power_iter_max, s->power_iter_rtol, NULL);
    double nQ = s->norm_Q > 0.0 ? s->norm_Q
                                : orc_norm_Q(p, s->power_iter_max, s->power_iter_rtol, NULL);
    res->norm_A = nA;
    res->norm_Q = nQ;
    if (!(nA > 0.0) && !(nQ > 0.0)) { res->status = ORC_NUMERICAL_ERROR; return -1; }

    const int fixed = s->restart_mode == ORC_RESTART_FIXED_K;
    const int64_t interval = fixed ? (int64_t)s->fixed_K : (int64_t)s->check_every;
    if (interval <= 0) return -1;

    orc_state st;
    state_alloc(&st, n, m);
    orc_csc at;
    if (g_threads > 1 && m > 0) {
        csc_build(m, n, p->a_rowptr, p->a_col, p->a_val, &at);
        st.at = &at;
    }
    double *xu = malloc(sizeof(double) * (size_t)n);
    double *yu = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *x_rs = malloc(sizeof(double) * (size_t)n);
    double *y_rs = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double s_last = 0.0; /* PDQP scale s_{k-1} of the current cycle */

    /* initial point: zeros (Sec. 5) or the warm start, projected onto X x Y */
    for (int64_t j = 0; j < n; ++j) st.x[j] = proj_box(0.0, p->l[j], p->u[j]);
    for (int64_t i = 0; i < m; ++i) st.y[i] = 0.0;
    orc_kkt kk;
    int64_t kkt_evals = 0;
    int used_warm = 0;
    if (x0 || y0) {
        double *xw = malloc(sizeof(double) * (size_t)n);
        double *yw = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
        for (int64_t j = 0; j < n; ++j) xw[j] = x0 ? proj_box(x0[j], p->l[j], p->u[j]) : st.x[j];
        for (int64_t i = 0; i < m; ++i) yw[i] = y0 ? proj_dual(y0[i], p->row_type[i]) : 0.0;
        int take = 1;
        if (s->warm_fallback) {
            orc_kkt kw, kc;
            kkt_eval(p, orig, dv, dr, xw, yw, xu, yu, &kw);
            kkt_eval(p, orig, dv, dr, st.x, st.y, xu, yu, &kc);
            kkt_evals += 2;
            take = kw.rel_kkt < kc.rel_kkt;
        }
        if (take) {
            memcpy(st.x, xw, sizeof(double) * (size_t)n);
            if (m) memcpy(st.y, yw, sizeof(double) * (size_t)m);
            used_warm = 1;
        }
        free(xw); free(yw);
    }
    memcpy(st.x_prev, st.x, sizeof(double) * (size_t)n);
    memcpy(st.xbar, st.x, sizeof(double) * (size_t)n);
    memcpy(x_rs, st.x, sizeof(double) * (size_t)n);
    if (m) {
        memcpy(st.ybar, st.y, sizeof(double) * (size_t)m);
        memcpy(y_rs, st.y, sizeof(double) * (size_t)m);
    }

    /* Sec. 6 InitializePrimalWeight */
    double omega = omega0;
    if (!(omega > 0.0)) {
        double nc = norm2(n, p->c), nb = norm2(m, p->b);
        omega = (nc > s->eps_zero && nb > s->eps_zero) ? nc / nb : 1.0;
    }

    kkt_eval(p, orig, dv, dr, st.x, st.y, xu, yu, &kk);
    kkt_evals += 1;
    double r0 = kk.rel_kkt;
    double prev_cand = INFINITY;
    int64_t total = 0, k = 0, restarts = 0, nlog = 0;
    int status = -1;
    int from_avg = 0; /* which point is returned */
    orc_kkt kc = kk;

    if (isnan(r0)) status = ORC_NUMERICAL_ERROR;
    else if (r0 <= s->eps) status = ORC_OPTIMAL;
    if (status < 0 && s->max_iter <= 0) status = ORC_ITERATION_LIMIT;

    while (status < 0) {
        int64_t len = interval;
        if (total + len > s->max_iter) len = s->max_iter - total;
        for (int64_t j = 0; j < len; ++j) {
            double pkj, dkj;
            step_at(s, nA, nQ, omega, k, &s_last, &pkj, &dkj);
            one_iteration(p, &st, s->momentum, k, pkj, dkj);
            ++k; ++total;
        }
        /* evaluation */
        orc_kkt kcur, kavg;
        kkt_eval(p, orig, dv, dr, st.x, st.y, xu, yu, &kcur);
        kkt_eval(p, orig, dv, dr, st.xbar, st.ybar, xu, yu, &kavg);
        kkt_evals += 2;
        double r = kcur.rel_kkt, rb = kavg.rel_kkt;
        int cand_avg;
        /* Algorithm 1 and the Sec. 5 methods (fixed-frequency, halving and no restart)
         * output and are measured at the average; choosing the better of the current
         * iterate and the average is the Sec. 6 rule (GetRestartCandidate) */
        if (s->restart_mode != ORC_RESTART_ADAPTIVE) cand_avg = 1;
        else cand_avg = !(r < rb);                    /* Sec. 6 GetRestartCandidate */
        double rc = cand_avg ? rb : r;
        kc = cand_avg ? kavg : kcur;
        from_avg = cand_avg;
        int restart = 0;
        if (isnan(r) || isnan(rb)) {
            status = ORC_NUMERICAL_ERROR;
        } else if (rc <= s->eps) {
            status = ORC_OPTIMAL;
        } else if (s->detect_infeasibility &&
                   infeasible(p, orig, dv, dr, &st, x_rs, y_rs, xu, yu, s->eps_infeasible,
                              &status)) {
            /* status set */
        } else if (total >= s->max_iter) {
            status = ORC_ITERATION_LIMIT;
        } else if (s->time_limit_s > 0.0 && now_s() - t_start >= s->time_limit_s) {
            status = ORC_TIME_LIMIT;
        } else {
            switch (s->restart_mode) {
            case ORC_RESTART_ADAPTIVE:
                restart = (rc <= s->beta_sufficient * r0) ||
                          (rc <= s->beta_necessary * r0 && rc > prev_cand) ||
                          ((double)k >= s->beta_artificial * (double)total);
                break;
            case ORC_RESTART_HALVING: /* Sec. 5: restart when relKKT(z-bar) <= r0 / 2 */
                restart = rb <= 0.5 * r0;
                break;
            case ORC_RESTART_FIXED_K:
                restart = 1;
                break;
            default:
                restart = 0;
            }
        }
        double omega_log = omega;
        if (restart) {
            const double *xc = cand_avg ? st.xbar : st.x;
            const double *yc = cand_avg ? st.ybar : st.y;
            if (!fixed) {
                /* Sec. 6 PrimalWeightUpdate */
                double dx = dist2(n, xc, x_rs), dy = dist2(m, yc, y_rs);
                if (dx > s->eps_zero && dy > s->eps_zero)
                    omega = exp(s->pw_smoothing * log(dy / dx) +
                                (1.0 - s->pw_smoothing) * log(omega));
            }
            if (cand_avg) {
                memcpy(st.x, st.xbar, sizeof(double) * (size_t)n);
                if (m) memcpy(st.y, st.ybar, sizeof(double) * (size_t)m);
            } else {
                memcpy(st.xbar, st.x, sizeof(double) * (size_t)n);
                if (m) memcpy(st.ybar, st.y, sizeof(double) * (size_t)m);
            }
            memcpy(st.x_prev, st.x, sizeof(double) * (size_t)n);
            memcpy(x_rs, st.x, sizeof(double) * (size_t)n);
            if (m) memcpy(y_rs, st.y, sizeof(double) * (size_t)m);
            k = 0;
            r0 = rc;
            prev_cand = INFINITY;
            ++restarts;
            omega_log = omega;
        } else if (status < 0) {
            prev_cand = rc;
        }
        if (check_log && nlog < log_cap) {
            check_log[nlog].total = total;
            check_log[nlog].k = restart ? 0 : k;
            check_log[nlog].r_cur = r;
            check_log[nlog].r_avg = rb;
            check_log[nlog].candidate = cand_avg;
            check_log[nlog].restarted = restart;
            check_log[nlog].omega = omega_log;
        }
        ++nlog;
    }

    const double *xs = from_avg ? st.xbar : st.x;
    const double *ys = from_avg ? st.ybar : st.y;
    for (int64_t j = 0; j < n; ++j) x_out[j] = orig ? xs[j] * dv[j] : xs[j];
    for (int64_t i = 0; i < m; ++i) y_out[i] = orig ? ys[i] * dr[i] : ys[i];
    res->status = status;
    res->iterations = total;
    res->restarts = restarts;
    res->kkt_evals = kkt_evals;
    res->rel_kkt = kc.rel_kkt;
    res->r_primal = kc.r_primal;
    res->r_dual = kc.r_dual;
    res->r_gap = kc.r_gap;
    res->primal_obj = kc.primal_obj;
    res->dual_obj = kc.dual_obj;
    res->omega = omega;
    res->used_warm_start = used_warm;
    if (log_len) *log_len = nlog < log_cap ? nlog : log_cap;
    free(x_rs); free(y_rs); free(xu); free(yu);
    if (st.at) csc_free(&at);
    state_free(&st);
    return 0;
}

int orc_solve(const orc_problem *p, const orc_settings *s, const double *x0, const double *y0,
              double omega0, double *x_out, double *y_out, orc_result *res,
              orc_check_log *check_log, int64_t log_cap, int64_t *log_len) {
    return solve_impl(p, NULL, NULL, NULL, s, x0, y0, omega0, x_out, y_out, res, check_log,
                      log_cap, log_len);
}

int orc_solve_scaled(const orc_problem *scaled, const orc_problem *orig, const double *d_var,
                     const double *d_row, const orc_settings *s, const double *x0,
                     const double *y0, double omega0, double *x_out, double *y_out,
                     orc_result *res, orc_check_log *check_log, int64_t log_cap,
                     int64_t *log_len) {
    const int64_t n = scaled->n, m = scaled->m;
    double *xs0 = NULL, *ys0 = NULL;
    if (x0) {
        xs0 = malloc(sizeof(double) * (size_t)n);
        for (int64_t j = 0; j < n; ++j) xs0[j] = x0[j] / d_var[j];
    }
    if (y0) {
        ys0 = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
        for (int64_t i = 0; i < m; ++i) ys0[i] = y0[i] / d_row[i];
    }
    int rc = solve_impl(scaled, orig, d_var, d_row, s, xs0, ys0, omega0, x_out, y_out, res,
                        check_log, log_cap, log_len);
    free(xs0);
    free(ys0);
    return rc;
}

/* ------------------------------------------------------------------ */
/* diagonal preconditioning (Sec. 5 "Preprocessing", also used by      */
/* Sec. 6): symmetric scaling of K = [[Q, A'], [A, 0]]                  */
/* ------------------------------------------------------------------ */
/* Row statistic of every row of K at the current values: kind 0 = max |k|,
 * 1 = sqrt(sum k^2), 2 = sum |k|.  Variable row j of K is Q's row j (stored
 * order) followed by A's column j (increasing row index); constraint row i of K is
 * A's row i (stored order). */
static void k_row_stat(const orc_problem *p, const double *qv, const double *av, int kind,
                       double *st) {
    const int64_t n = p->n, m = p->m;
    for (int64_t j = 0; j < n; ++j) {
        double a = 0.0;
        for (int64_t e = p->q_rowptr[j]; e < p->q_rowptr[j + 1]; ++e) {
            double v = fabs(qv[e]);
            if (kind == 0) a = v > a ? v : a;
            else if (kind == 1) a = a + v * v;
            else a = a + v;
        }
        st[j] = a;
    }
    for (int64_t i = 0; i < m; ++i) {
        double a = 0.0;
        for (int64_t e = p->a_rowptr[i]; e < p->a_rowptr[i + 1]; ++e) {
            double v = fabs(av[e]);
            int64_t j = p->a_col[e];
            if (kind == 0) {
                a = v > a ? v : a;
                st[j] = v > st[j] ? v : st[j];
            } else if (kind == 1) {
                a = a + v * v;
                st[j] = st[j] + v * v;
            } else {
                a = a + v;
                st[j] = st[j] + v;
            }
        }
        st[n + i] = a;
    }
    if (kind == 1)
        for (int64_t r = 0; r < n + m; ++r) st[r] = sqrt(st[r]);
}

/* One scaling step: f_r = 1/sqrt(stat_r) (1 for an empty row), K <- diag(f) K diag(f)
 * entry by entry as k * (f_r * f_c), d <- d * f. */
static void k_scale_step(const orc_problem *p, double *qv, double *av, const double *st,
                         double *f, double *d) {
    const int64_t n = p->n, m = p->m;
    for (int64_t r = 0; r < n + m; ++r) {
        f[r] = st[r] > 0.0 ? 1.0 / sqrt(st[r]) : 1.0;
        d[r] = d[r] * f[r];
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t e = p->q_rowptr[j]; e < p->q_rowptr[j + 1]; ++e)
            qv[e] = qv[e] * (f[j] * f[p->q_col[e]]);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t e = p->a_rowptr[i]; e < p->a_rowptr[i + 1]; ++e)
            av[e] = av[e] * (f[n + i] * f[p->a_col[e]]);
}

void orc_precondition(const orc_problem *p, int32_t ruiz_iters, int32_t l2, int32_t pc,
                      double *q_val, double *a_val, double *c, double *b, double *l, double *u,
                      double *d_var, double *d_row) {
    const int64_t n = p->n, m = p->m;
    const int64_t qn = p->q_rowptr[n], an = m > 0 ? p->a_rowptr[m] : 0;
    double *st = malloc(sizeof(double) * (size_t)(n + m));
    double *f = malloc(sizeof(double) * (size_t)(n + m));
    double *d = malloc(sizeof(double) * (size_t)(n + m));
    memcpy(q_val, p->q_val, sizeof(double) * (size_t)qn);
    if (an) memcpy(a_val, p->a_val, sizeof(double) * (size_t)an);
    for (int64_t r = 0; r < n + m; ++r) d[r] = 1.0;
    for (int32_t t = 0; t < ruiz_iters; ++t) {   /* Ruiz: infinity-norm equilibration */
        k_row_stat(p, q_val, a_val, 0, st);
        k_scale_step(p, q_val, a_val, st, f, d);
    }
    if (l2) {                                      /* l2-norm scaling */
        k_row_stat(p, q_val, a_val, 1, st);
        k_scale_step(p, q_val, a_val, st, f, d);
    }
    if (pc) {   /* Pock-Chambolle, alpha = 1: rows by sum |k|^alpha, columns by
                   sum |k|^(2-alpha); K is symmetric, so both are the row sums */
        k_row_stat(p, q_val, a_val, 2, st);
        k_scale_step(p, q_val, a_val, st, f, d);
    }
    /* x = D2 x~, y = D1 y~:  c~ = D2 c, b~ = D1 b, bounds l/D2, u/D2 */
    for (int64_t j = 0; j < n; ++j) {
        d_var[j] = d[j];
        c[j] = p->c[j] * d[j];
        l[j] = p->l[j] / d[j];
        u[j] = p->u[j] / d[j];
    }
    for (int64_t i = 0; i < m; ++i) {
        d_row[i] = d[n + i];
        b[i] = p->b[i] * d[n + i];
    }
    free(st); free(f); free(d);
}
