/*
 * rapdhg_oracle.h -- plain, slow, FP64 CPU reference of restarted accelerated
 * PDHG (rAPDHG) for convex QP.  TEST INFRASTRUCTURE ONLY: nothing in the
 * product library may include, link or call this code.
 *
 * Paper: Lu & Yang, "A Practical and Optimal First-Order Method for
 * Large-Scale Convex Quadratic Programming" (arXiv 2311.07710).
 *
 * Problem (generalisation of Sec. 1 eq. (qp), per its footnote):
 *     min 1/2 x'Qx + c'x  s.t.  A_i x = b_i (EQ rows), A_i x >= b_i (GE rows),
 *                               l <= x <= u.
 * Saddle form (Sec. 1 eq. (minimax) with A_p = -A, b_p = -b):
 *     L(x,y) = 1/2 x'Qx + c'x - y'(Ax - b),  y_i >= 0 on GE rows, free on EQ rows.
 */
#ifndef RAPDHG_ORACLE_H
#define RAPDHG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* CSR: rowptr[nrows+1], col[nnz], val[nnz]; Q full symmetric. */
typedef struct {
    int64_t n, m;
    const int32_t *q_rowptr, *q_col;
    const double *q_val;
    const int32_t *a_rowptr, *a_col;
    const double *a_val;
    const double *c, *b, *l, *u; /* l, u hold -inf / +inf where unbounded */
    const uint8_t *row_type;     /* 0 = EQ, 1 = GE */
} orc_problem;

enum { ORC_RESTART_ADAPTIVE = 0, ORC_RESTART_FIXED_K = 1, ORC_RESTART_HALVING = 2,
       ORC_RESTART_NONE = 3 };
enum { ORC_OPTIMAL = 0, ORC_ITERATION_LIMIT = 1, ORC_TIME_LIMIT = 2, ORC_NUMERICAL_ERROR = 3,
       ORC_PRIMAL_INFEASIBLE = 4, ORC_DUAL_INFEASIBLE = 5 };

typedef struct {
    double eps;              /* relKKT tolerance (Sec. 5, eq. (terminate)) */
    int64_t max_iter;
    double time_limit_s;     /* <= 0: none */
    int32_t check_every;     /* evaluation cadence (ADAPTIVE / HALVING / NONE) */
    int32_t restart_mode;
    int32_t fixed_K;         /* FIXED_K: restart frequency K (Alg. 1) */
    double beta_sufficient, beta_necessary, beta_artificial; /* Sec. 6 restart (i)-(iii) */
    double pw_smoothing;     /* primal-weight smoothing theta (Sec. 6) */
    double eps_zero;
    double step_safety;      /* 0.99 of the Sec. 6 step-size rule */
    double norm_A, norm_Q;   /* > 0: use as ||A||_2, ||Q||_2 ; else power iteration */
    int32_t power_iter_max;
    double power_iter_rtol;
    int32_t warm_fallback;   /* 1: keep the warm start only if its relKKT beats the cold start's */
    int32_t detect_infeasibility; /* 1: test z - z_restart for infeasibility certificates
                                     at every evaluation (orc_infeas_check) */
    double eps_infeasible;   /* certificate tolerance (relative, see orc_infeas_check) */
    int32_t momentum;        /* 1: accelerated PDHG weights of Algorithm 1 (default);
                                0: plain PDHG, the Sec. 5 baseline (beta = theta = 1, constant
                                step, uniform average of the cycle as restart candidate) */
} orc_settings;

typedef struct {
    int32_t status;
    int64_t iterations, restarts, kkt_evals;
    double rel_kkt, r_primal, r_dual, r_gap, primal_obj, dual_obj;
    double omega, norm_A, norm_Q;
    int32_t used_warm_start;
} orc_result;

typedef struct {
    int64_t total, k;        /* iterations so far; inner index of the cycle */
    double r_cur, r_avg;     /* relKKT of z and of the average z-bar */
    int32_t candidate;       /* 0 = current iterate, 1 = average */
    int32_t restarted;
    double omega;            /* primal weight after this check */
} orc_check_log;

typedef struct {
    double r_primal, r_dual, r_gap, rel_kkt, primal_obj, dual_obj;
    double ax_inf, b_inf, qx_inf, aty_inf, c_inf, xqx, cx, by;
} orc_kkt;

void orc_default_settings(orc_settings *s);

/* y = M x for a CSR matrix, row sums accumulated in CSR order. */
void orc_spmv(int64_t nrows, const int32_t *rowptr, const int32_t *col, const double *val,
              const double *x, double *y);
/* y = M' x (transpose product) by scattering rows in increasing row order. */
void orc_spmv_t(int64_t nrows, int64_t ncols, const int32_t *rowptr, const int32_t *col,
                const double *val, const double *x, double *y);

/* Relative KKT error of Sec. 5, generalised to EQ/GE rows and bounds. */
void orc_rel_kkt(const orc_problem *p, const double *x, const double *y, orc_kkt *out);

/* Power iteration estimates; iters_out may be NULL. */
double orc_norm_A(const orc_problem *p, int32_t maxit, double rtol, int32_t *iters_out);
double orc_norm_Q(const orc_problem *p, int32_t maxit, double rtol, int32_t *iters_out);

/* Step scalars for inner indices k = 0..K-1 of one cycle:
 * primal step p[k], dual step d[k], PDQP scale s[k] (ADAPTIVE/HALVING/NONE only). */
void orc_step_schedule(const orc_settings *s, double norm_A, double norm_Q, double omega,
                       int64_t K, double *p, double *d, double *scale);

/* Run exactly `iters` inner iterations of (accelerated, unless s->momentum == 0) PDHG
 * (no restart, no check)
 * from (x,y) with the schedule of `s` at primal weight omega.  On return x,y hold
 * the last iterate and xbar,ybar the running averages. */
void orc_run_inner(const orc_problem *p, const orc_settings *s, double norm_A, double norm_Q,
                   double omega, int64_t iters, double *x, double *y, double *xbar, double *ybar);

/* Full solve.  x0/y0 nullable (cold start = zeros projected onto the sets).
 * omega0 <= 0 selects the initial primal weight rule.  log may be NULL. */
int orc_solve(const orc_problem *p, const orc_settings *s, const double *x0, const double *y0,
              double omega0, double *x_out, double *y_out, orc_result *res,
              orc_check_log *check_log, int64_t log_cap, int64_t *log_len);

/* Infeasibility certificates from a direction (dx, dy) (the paper is silent; the
 * drift of the iterates of an infeasible problem is such a direction).
 *  primal_ratio: dy is projected onto the dual cone (GE rows >= 0) giving dy+, g = A'dy+;
 *    farkas = b'dy+ - sum over finite bounds of the support of X in direction g
 *    (u_j g_j for g_j > 0, l_j g_j for g_j < 0); viol = max |g_j| over the components
 *    whose needed bound is infinite; ratio = viol / farkas if farkas > 0 else +inf.
 *    A ratio of 0 is an exact Farkas certificate: b'y > sup_{x in X} (A'y)'x.
 *  dual_ratio: dx is projected onto the recession cone of X giving dx+;
 *    cdx = c'dx+; viol = max(||Q dx+||_inf, ||(A dx+)_EQ||_inf, ||[-(A dx+)_GE]_+||_inf);
 *    ratio = viol / (-cdx) if cdx < 0 else +inf: a direction of unbounded descent. */
typedef struct {
    double primal_ratio, dual_ratio;
} orc_infeas;
void orc_infeas_check(const orc_problem *p, const double *dx, const double *dy, orc_infeas *out);

/* Diagonal preconditioning (Sec. 5 "Preprocessing"): ruiz_iters infinity-norm
 * (Ruiz) steps, then one l2-norm step if l2, then one Pock-Chambolle (alpha = 1)
 * step if pc, all on K = [[Q, A'], [A, 0]] with one symmetric diagonal scaling
 * d = (D2, D1).  Writes the scaled values (same sparsity as p): Q~ = D2 Q D2,
 * A~ = D1 A D2, c~ = D2 c, b~ = D1 b, l~ = l / D2, u~ = u / D2, and D2 (d_var, n),
 * D1 (d_row, m).  Solutions map back as x = D2 x~, y = D1 y~. */
void orc_precondition(const orc_problem *p, int32_t ruiz_iters, int32_t l2, int32_t pc,
                      double *q_val, double *a_val, double *c, double *b, double *l, double *u,
                      double *d_var, double *d_row);

/* Solve of a preconditioned problem: iterates live in the scaled space, every
 * relKKT is that of the original problem at (D2 x~, D1 y~); warm starts and
 * outputs are in the original space. */
int orc_solve_scaled(const orc_problem *scaled, const orc_problem *orig, const double *d_var,
                     const double *d_row, const orc_settings *s, const double *x0,
                     const double *y0, double omega0, double *x_out, double *y_out,
                     orc_result *res, orc_check_log *check_log, int64_t log_cap,
                     int64_t *log_len);

/* Host threads for the row loops of a solve (timing on multi-core hosts; default 1).
 * Results are bitwise those of one thread: every output element is computed by one
 * thread in the sequential order, and every reduction stays sequential. */
void orc_set_threads(int32_t t);
int32_t orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
