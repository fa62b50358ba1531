/* Drives every entry point of the CPU oracle (oracle/rapdhg_oracle.c) on small seeded
 * problems with edge cases (equality and >= rows, mixed bounds, an empty row, a row
 * longer than the variable count, m = 0, a log buffer shorter than the evaluations, warm
 * starts, every restart mode with and without momentum, preprocessing, infeasibility
 * detection, 1 and 3 threads).  Built by tests/test_host_sanitizers.py with
 * AddressSanitizer and UndefinedBehaviorSanitizer; it checks only that results are
 * well-formed (correctness is pinned elsewhere). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/rapdhg_oracle.h"

static uint64_t rs = 88172645463325252ull;
static double urand(void) { /* xorshift64, uniform in [0, 1) */
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (double)(rs >> 11) * (1.0 / 9007199254740992.0);
}

typedef struct {
    int64_t n, m;
    int32_t *qr, *qc, *ar, *ac;
    double *qv, *av, *c, *b, *l, *u;
    uint8_t *rt;
    orc_problem p;
} inst;

/* Q: diagonal plus a few symmetric pairs; A: random rows, row 1 empty, row 2 dense with
 * n + 3 entries (repeated columns); feasible b from x0 inside the bounds */
static void make(inst *I, int64_t n, int64_t m, int infeasible) {
    memset(I, 0, sizeof(*I));
    I->n = n;
    I->m = m;
    double *Qd = calloc((size_t)(n * n), sizeof(double));
    for (int64_t j = 0; j < n; ++j) Qd[j * n + j] = 1.0 + 3.0 * urand();
    for (int64_t k = 0; k < n; ++k) {
        int64_t i = (int64_t)(urand() * n), j = (int64_t)(urand() * n);
        if (i == j) continue;
        double v = 0.3 * (urand() - 0.5);
        Qd[i * n + j] += v;
        Qd[j * n + i] += v;
    }
    I->qr = malloc((size_t)(n + 1) * sizeof(int32_t));
    I->qc = malloc((size_t)(n * n) * sizeof(int32_t));
    I->qv = malloc((size_t)(n * n) * sizeof(double));
    int32_t nz = 0;
    I->qr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j)
            if (Qd[i * n + j] != 0.0) {
                I->qc[nz] = (int32_t)j;
                I->qv[nz++] = Qd[i * n + j];
            }
        I->qr[i + 1] = nz;
    }
    free(Qd);
    I->l = malloc((size_t)n * sizeof(double));
    I->u = malloc((size_t)n * sizeof(double));
    double *x0 = malloc((size_t)n * sizeof(double));
    I->c = malloc((size_t)n * sizeof(double));
    for (int64_t j = 0; j < n; ++j) {
        int kind = (int)(j % 4);
        I->l[j] = kind == 0 || kind == 1 ? -1.0 : -INFINITY;
        I->u[j] = kind == 0 || kind == 2 ? 2.0 : INFINITY;
        x0[j] = 0.5 * (urand() - 0.3);
        I->c[j] = urand() - 0.5;
    }
    int64_t cap = m * 8 + n + 8;
    I->ar = malloc((size_t)(m + 1) * sizeof(int32_t));
    I->ac = malloc((size_t)cap * sizeof(int32_t));
    I->av = malloc((size_t)cap * sizeof(double));
    I->b = malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    I->rt = malloc((size_t)(m > 0 ? m : 1));
    nz = 0;
    I->ar[0] = 0;
    for (int64_t i = 0; i < m; ++i) {
        int64_t len = i == 1 ? 0 : (i == 2 ? n + 3 : 1 + (int64_t)(urand() * 5));
        double ax = 0.0;
        for (int64_t k = 0; k < len; ++k) {
            int64_t j = i == 2 ? k % n : (int64_t)(urand() * n);
            double v = urand() - 0.5;
            I->ac[nz] = (int32_t)j;
            I->av[nz++] = v;
            ax += v * x0[j];
        }
        I->ar[i + 1] = nz;
        I->rt[i] = (uint8_t)(i % 3 == 0 ? 0 : 1);
        I->b[i] = I->rt[i] == 0 ? ax : ax - urand();
    }
    if (infeasible && m >= 4) { /* rows 3 and 4: a x >= 1 and -a x >= 0 with equal a */
        I->rt[3] = 1;
        I->rt[4] = 1;
        int32_t s3 = I->ar[3], e3 = I->ar[4], s4 = I->ar[4], e4 = I->ar[5];
        int32_t len = e3 - s3 < e4 - s4 ? e3 - s3 : e4 - s4;
        for (int32_t k = 0; k < len; ++k) {
            I->ac[s4 + k] = I->ac[s3 + k];
            I->av[s4 + k] = -I->av[s3 + k];
        }
        for (int32_t k = len; k < e4 - s4; ++k) I->av[s4 + k] = 0.0;
        for (int32_t k = len; k < e3 - s3; ++k) I->av[s3 + k] = 0.0;
        I->b[3] = 1.0;
        I->b[4] = 0.0;
    }
    free(x0);
    orc_problem p = {n, m, I->qr, I->qc, I->qv, I->ar, I->ac, I->av, I->c, I->b, I->l, I->u,
                     I->rt};
    I->p = p;
}

static void release(inst *I) {
    free(I->qr); free(I->qc); free(I->qv); free(I->ar); free(I->ac); free(I->av);
    free(I->c); free(I->b); free(I->l); free(I->u); free(I->rt);
}

static int failures = 0;
static void check(int cond, const char *what) {
    if (!cond) {
        printf("FAIL: %s\n", what);
        ++failures;
    }
}

static void check_result(const orc_result *r, int64_t n, int64_t m, const double *x,
                         const double *y) {
    check(r->status >= ORC_OPTIMAL && r->status <= ORC_DUAL_INFEASIBLE, "status range");
    check(r->iterations >= 0 && r->kkt_evals >= 1, "counters");
    int fin = isfinite(r->rel_kkt) && isfinite(r->omega);
    for (int64_t j = 0; j < n; ++j) fin = fin && isfinite(x[j]);
    for (int64_t i = 0; i < m; ++i) fin = fin && isfinite(y[i]);
    check(fin || r->status == ORC_NUMERICAL_ERROR, "finite results");
}

static void solves(inst *I) {
    const int64_t n = I->n, m = I->m, mm = m > 0 ? m : 1;
    double *x = malloc((size_t)n * sizeof(double)), *y = malloc((size_t)mm * sizeof(double));
    double *x0 = malloc((size_t)n * sizeof(double)), *y0 = malloc((size_t)mm * sizeof(double));
    for (int64_t j = 0; j < n; ++j) x0[j] = urand() - 0.5;
    for (int64_t i = 0; i < mm; ++i) y0[i] = urand() - 0.5;
    orc_check_log lg[3];
    int64_t nlog = 0;
    orc_result r;
    for (int mode = 0; mode < 4; ++mode)
        for (int mom = 0; mom < 2; ++mom)
            for (int warm = 0; warm < 2; ++warm) {
                orc_settings s;
                orc_default_settings(&s);
                s.eps = 1e-6;
                s.max_iter = 3000;
                s.check_every = 16;
                s.restart_mode = mode;
                s.fixed_K = 50;
                s.momentum = mom;
                orc_solve(&I->p, &s, warm ? x0 : NULL, warm ? y0 : NULL, 0.0, x, y, &r, lg, 3,
                          &nlog);
                check(nlog <= 3, "log truncated");
                check_result(&r, n, m, x, y);
            }
    /* norms, KKT, inner iterations, schedule */
    int32_t it = 0;
    double nA = orc_norm_A(&I->p, 500, 1e-9, &it), nQ = orc_norm_Q(&I->p, 500, 1e-9, &it);
    check(nA >= 0.0 && nQ > 0.0, "norms");
    orc_kkt k;
    orc_rel_kkt(&I->p, x, y, &k);
    check(isfinite(k.rel_kkt), "rel_kkt");
    double *xb = malloc((size_t)n * sizeof(double)), *yb = malloc((size_t)mm * sizeof(double));
    orc_settings s;
    orc_default_settings(&s);
    orc_run_inner(&I->p, &s, nA > 0 ? nA : 1.0, nQ, 1.0, 20, x, y, xb, yb);
    double pk[8], dk[8], sc[8];
    orc_step_schedule(&s, nA > 0 ? nA : 1.0, nQ, 1.3, 8, pk, dk, sc);
    check(pk[7] > 0.0 && dk[7] > 0.0, "schedule");
    /* preprocessing and the scaled solve */
    int64_t qn = I->qr[n], an = I->ar[m];
    double *qv = malloc((size_t)(qn > 0 ? qn : 1) * sizeof(double));
    double *av = malloc((size_t)(an > 0 ? an : 1) * sizeof(double));
    double *c = malloc((size_t)n * sizeof(double)), *b = malloc((size_t)mm * sizeof(double));
    double *l = malloc((size_t)n * sizeof(double)), *u = malloc((size_t)n * sizeof(double));
    double *dv = malloc((size_t)n * sizeof(double)), *dr = malloc((size_t)mm * sizeof(double));
    orc_precondition(&I->p, 10, 1, 1, qv, av, c, b, l, u, dv, dr);
    orc_problem sp = I->p;
    sp.q_val = qv;
    sp.a_val = av;
    sp.c = c;
    sp.b = b;
    sp.l = l;
    sp.u = u;
    s.eps = 1e-6;
    s.max_iter = 3000;
    s.detect_infeasibility = 1;
    orc_solve_scaled(&sp, &I->p, dv, dr, &s, x0, y0, 0.0, x, y, &r, lg, 3, &nlog);
    check_result(&r, n, m, x, y);
    orc_infeas inf;
    orc_infeas_check(&I->p, x, y, &inf);
    free(qv); free(av); free(c); free(b); free(l); free(u); free(dv); free(dr);
    free(xb); free(yb); free(x); free(y); free(x0); free(y0);
}

int main(void) {
    const int64_t shapes[][3] = {{40, 25, 0}, {7, 12, 0}, {30, 0, 0}, {25, 20, 1}};
    for (int th = 1; th <= 3; th += 2) {
        orc_set_threads(th);
        check(orc_get_threads() == th, "threads");
        for (size_t q = 0; q < sizeof(shapes) / sizeof(shapes[0]); ++q) {
            inst I;
            make(&I, shapes[q][0], shapes[q][1], (int)shapes[q][2]);
            solves(&I);
            release(&I);
        }
    }
    orc_set_threads(1);
    if (failures) return 1;
    printf("oracle sanitize run ok\n");
    return 0;
}
