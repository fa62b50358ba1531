/*
 * qp.h -- C-ABI of the MI355X (gfx950) rAPDHG solver for convex quadratic programs.
 *
 * Method: restarted accelerated primal-dual hybrid gradient (rAPDHG) of
 * Lu & Yang, "A Practical and Optimal First-Order Method for Large-Scale Convex
 * Quadratic Programming" (arXiv 2311.07710):
 *   - inner iteration: Algorithm 1 (accelerated PDHG with momentum averaging);
 *   - step sizes, primal weight and adaptive restart: Sec. 6 (PDQP);
 *   - progress metric / termination: Sec. 5 (relative KKT error);
 *   - fixed-frequency restart: Algorithm 1 / Theorem 1; "halving" restart: Sec. 5.
 *
 * Problem (the paper's eq. (qp) generalised to equality rows and bounds):
 *     min  1/2 x'Qx + c'x
 *     s.t. A_i x  = b_i   for rows of type QP_ROW_EQ
 *          A_i x >= b_i   for rows of type QP_ROW_GE
 *          l <= x <= u    (entries may be -inf / +inf)
 * with Q symmetric positive semidefinite, stored as a FULL symmetric CSR matrix
 * (both triangles).  Saddle form: L(x,y) = 1/2 x'Qx + c'x - y'(Ax - b) with
 * y_i >= 0 on GE rows and y_i free on EQ rows (the paper's eq. (minimax) with
 * A replaced by -A and b by -b).
 *
 * Precision: everything is FP64.  Index type: int32 (row pointers and column
 * indices); nnz(Q) + nnz(A) and n + m must stay below 2^31.
 *
 * Errors: every int-returning function returns QP_OK (0) or a QP_ERR_* code;
 * qp_last_error() then returns a thread-local, human-readable message.  A solve
 * that does not converge is NOT an error: it returns QP_OK and reports the
 * outcome in qp_result.status.
 *
 * Threading: a handle may be used by one host thread at a time.  Different
 * handles are independent.  All calls are blocking with respect to the host.
 */
#ifndef QP_MI355X_H
#define QP_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QP_ABI_VERSION 2

/* return codes */
#define QP_OK 0
#define QP_ERR_INVALID_ARGUMENT 1
#define QP_ERR_OUT_OF_MEMORY 2
#define QP_ERR_DEVICE 3
#define QP_ERR_BATCH_MISMATCH 4
#define QP_ERR_UNSUPPORTED 5

/* qp_result.status */
#define QP_OPTIMAL 0          /* relKKT(candidate) <= eps (Sec. 5, eq. (terminate)) */
#define QP_ITERATION_LIMIT 1  /* max_iter reached */
#define QP_TIME_LIMIT 2       /* time_limit_s reached */
#define QP_NUMERICAL_ERROR 3  /* NaN met in the KKT evaluation */
#define QP_PRIMAL_INFEASIBLE 4 /* certificate found (settings.detect_infeasibility) */
#define QP_DUAL_INFEASIBLE 5   /* certificate of unbounded descent found (same setting) */

/* qp_settings.restart_mode */
#define QP_RESTART_ADAPTIVE 0 /* Sec. 6: candidate + criteria (i)-(iii) */
#define QP_RESTART_FIXED_K 1  /* Algorithm 1: restart at the average every K iterations,
                                 Theorem 1 step sizes */
#define QP_RESTART_HALVING 2  /* Sec. 5: restart at the average once relKKT halves */
#define QP_RESTART_NONE 3     /* accelerated PDHG without restarts */

/* qp_problem_desc.mem_space */
#define QP_MEM_HOST 0
#define QP_MEM_DEVICE 1

/* row types */
#define QP_ROW_EQ 0
#define QP_ROW_GE 1

/* Compressed sparse row matrix.  row_ptr has nrows+1 entries with row_ptr[0] = 0
 * and row_ptr[nrows] = nnz; col_idx are 0-based (sorted within a row is not
 * required).  For a batch (num_instances > 1) row_ptr runs over the concatenated
 * rows of all instances with GLOBAL offsets into col_idx/val, while col_idx
 * values are LOCAL to their instance (0 <= col < n_i): the segment-CSR layout. */
typedef struct {
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
    int64_t nnz;
} qp_csr;

typedef struct {
    int64_t n;               /* variables (sum over instances for a batch) */
    int64_t m;               /* constraint rows (sum over instances), may be 0 */
    int32_t num_instances;   /* 1 for a single QP; B > 1 for a batch of independent QPs */
    int32_t mem_space;       /* QP_MEM_HOST or QP_MEM_DEVICE: where every array below lives
                                (var_off/row_off are always host arrays) */
    qp_csr Q;                /* n x n, full symmetric */
    qp_csr A;                /* m x n */
    const double *c;         /* [n] */
    const double *b;         /* [m] (may be NULL when m == 0) */
    const double *l;         /* [n] lower bounds, NULL => all -inf */
    const double *u;         /* [n] upper bounds, NULL => all +inf */
    const uint8_t *row_type; /* [m] QP_ROW_EQ / QP_ROW_GE, NULL => all EQ */
    const int64_t *var_off;  /* batch only: [B+1] prefix sums of n_i (host array) */
    const int64_t *row_off;  /* batch only: [B+1] prefix sums of m_i (host array) */
    void *stream;            /* hipStream_t the caller's device arrays are ordered on, or
                                NULL; the library waits for it before reading them */
} qp_problem_desc;

/* One record per relKKT evaluation of a single-QP solve (settings.log_checks,
 * settings.log_cb): the restart test of Sec. 6 at that evaluation. */
typedef struct {
    int64_t total;           /* iterations done at this evaluation */
    int64_t k;               /* inner index after the evaluation (0 after a restart) */
    double r_cur, r_avg;     /* relKKT of the iterate z and of the average z-bar */
    int32_t candidate;       /* 0 = z, 1 = z-bar */
    int32_t restarted;
    double omega;            /* primal weight after the evaluation */
} qp_check_info;

/* Per-evaluation callback (settings.log_cb).  It runs on the host thread inside
 * qp_solve, once per evaluation and in order, as the host reads that evaluation's
 * state; the next check interval is enqueued only after it returns, so a slow
 * callback slows the solve.  It must not call the library with the same handle. */
typedef void (*qp_log_fn)(const qp_check_info *info, void *user);

typedef struct {
    double eps;              /* relKKT tolerance; default 1e-6 */
    int64_t max_iter;        /* default 200000 (Sec. 5) */
    double time_limit_s;     /* default 3600 (Sec. 6.1); <= 0 disables */
    int32_t check_every;     /* KKT evaluation cadence for ADAPTIVE/HALVING/NONE; default 64 */
    int32_t restart_mode;    /* QP_RESTART_*; default ADAPTIVE */
    int32_t fixed_K;         /* restart frequency for FIXED_K; default 100 */
    double beta_sufficient;  /* Sec. 6 restart (i); default 0.2; in (0, 1] */
    double beta_necessary;   /* Sec. 6 restart (ii); default 0.8; in (0, 1] */
    double beta_artificial;  /* Sec. 6 restart (iii); default 0.36; in (0, 1] */
    double pw_smoothing;     /* Sec. 6 primal-weight smoothing theta; default 0.2; in [0, 1] */
    double eps_zero;         /* Sec. 6 epsilon_zero; default 1e-10; >= 0 */
    double step_safety;      /* Sec. 6 step-size factor 0.99 */
    double norm_A;           /* > 0: use as ||A||_2 instead of power iteration */
    double norm_Q;           /* > 0: use as ||Q||_2 instead of power iteration */
    int32_t power_iter_max;  /* power-iteration steps at most; default 1000; >= 1 */
    double power_iter_rtol;  /* stop when the estimate moves by at most rtol (relative);
                                default 1e-7; >= 0 */
    int32_t warm_fallback;   /* 1 (default): a warm start is used only if its relKKT is
                                below that of the cold start */
    int32_t use_graph;       /* 1 (default): replay one captured hipGraph per check interval */
    int32_t profile;         /* k >= 1: time the dual and primal phases of every k-th
                                iteration with hipEvents (direct launches, no graph);
                                read with qp_get_profile; 0 (default): off */
    int32_t log_checks;      /* 1: record one qp_check_info per evaluation (qp_get_check_log) */
    int32_t device;          /* HIP device ordinal; default 0 */
    int32_t panels_dual;     /* column panels of A for the dual phase: 0 = automatic (4 when
                                the gathered vector exceeds 6 MB, or 1.75 MB with rows of
                                256 or more entries on average, else 1), 1 = unpanelled,
                                2/4/8 = panels pinned to groups of 8/np XCDs */
    int32_t panels_primal;   /* same for P = [Q | -A'] in the primal phase */
    int32_t momentum;        /* 1 (default): accelerated PDHG, Algorithm 1 with beta_k = (k+2)/2,
                                theta_k = k/(k+1) (Theorem 1); 0: plain PDHG, the Sec. 5
                                baseline: beta = theta = 1, the constant step of the Sec. 6 rule
                                at beta = 1, and the uniform average of the cycle's iterates as
                                the average candidate.  Combined with restart_mode this gives
                                the four methods of Sec. 5 (PDHG, restarted PDHG, accelerated
                                PDHG = momentum 1 + QP_RESTART_NONE, rAPDHG). */
    int32_t precondition;    /* 1: Sec. 5 preprocessing before the iteration: one symmetric
                                diagonal scaling of K = [[Q, A'], [A, 0]] from ruiz_iters
                                infinity-norm (Ruiz) steps, one l2-norm step and one
                                Pock-Chambolle step (alpha = 1); the solver iterates on
                                D2 Q D2, D1 A D2, D2 c, D1 b, l/D2, u/D2, while relKKT, warm
                                starts, outputs and the reported objective refer to the given
                                problem.  0 (default): off */
    int32_t ruiz_iters;      /* Ruiz steps of the preprocessing; default 10 (Sec. 5) */
    int32_t detect_infeasibility; /* 1: at every evaluation, test the drift since the last
                                restart, z - z_restart, for an infeasibility certificate on the
                                given problem (the paper is silent on infeasible inputs):
                                QP_PRIMAL_INFEASIBLE when its dual part, projected onto the
                                dual cone, is a Farkas ray (b'dy > support of X along A'dy,
                                with every component of A'dy that needs an infinite bound
                                below eps_infeasible times that margin); QP_DUAL_INFEASIBLE
                                when its primal part, projected onto the recession cone of X,
                                descends (c'dx < 0) with ||Q dx||_inf and the row violations
                                of A dx below eps_infeasible * |c'dx|.  Default 0 */
    double eps_infeasible;   /* certificate tolerance; default 1e-8 */
    int32_t check_symmetry;  /* 1: qp_create rejects a Q that differs from its transpose
                                (pattern or value, per instance); PSD is never checked.
                                Default 0 */
    qp_log_fn log_cb;        /* NULL (default) or called once per evaluation of a single-QP
                                solve with that evaluation's record (whether or not
                                log_checks is set); not called for a batch handle */
    void *log_user;          /* passed unchanged as log_cb's second argument */
} qp_settings;

typedef struct {
    const double *x0;        /* [n] or NULL; projected onto [l,u] */
    const double *y0;        /* [m] or NULL; projected onto the dual cone */
    double omega0;           /* > 0: initial primal weight; else the Sec. 6 rule */
} qp_warm_start;

typedef struct {
    int32_t status;          /* QP_OPTIMAL ... QP_NUMERICAL_ERROR */
    int32_t used_warm_start; /* 1 if the warm start was kept */
    int64_t iterations;
    int64_t restarts;
    int64_t kkt_evals;       /* number of points whose relKKT was evaluated */
    double rel_kkt, r_primal, r_dual, r_gap;
    double primal_obj, dual_obj;
    double omega;            /* final primal weight */
    double norm_A, norm_Q;   /* operator norms used */
    double solve_time_s;     /* host wall time of the solve (a batch: of the whole batch) */
    double start_s, end_s;   /* batch: when this instance's solve started and ended on the
                                device, in seconds after the batch began (device wall
                                clock); single solve: 0 and solve_time_s */
} qp_result;

typedef struct {
    int64_t dual_launches, primal_launches;  /* phases timed */
    double dual_ms, primal_ms;     /* summed hipEvent durations of the timed phases */
    double dual_bytes, primal_bytes; /* algorithmic HBM bytes of ONE launch */
} qp_profile;

typedef struct qp_handle qp_handle;

/* Fills *s with the defaults listed above. */
void qp_default_settings(qp_settings *s);

/* Sets up the problem of Sec. 1 eq. (qp) (generalised as above) for rAPDHG.
 * Validates the problem, copies it into library-owned device memory (the caller
 * keeps ownership of its arrays and may free them after the call), builds the
 * device layouts (A, and [Q | -A'] as one CSR matrix) and estimates ||A||_2 and
 * ||Q||_2 -- the operator norms the Sec. 6 step-size rule and Theorem 1's fixed-K
 * steps need -- by power iteration unless settings->norm_A / norm_Q > 0.  With
 * settings->precondition = 1 it applies the Sec. 5 diagonal preprocessing first.
 * settings may be NULL (defaults).  On success *out receives a handle to free with
 * qp_free.
 * Errors: QP_ERR_INVALID_ARGUMENT (malformed CSR, l > u, bad row type, index
 * overflow, both ||A|| and ||Q|| zero), QP_ERR_OUT_OF_MEMORY, QP_ERR_DEVICE. */
int qp_create(const qp_problem_desc *desc, const qp_settings *settings, qp_handle **out);

/* Solves a single QP (num_instances == 1) from zeros or from ws (nullable): the inner
 * loop of Algorithm 1 (accelerated PDHG with momentum averaging), restarted and stepped
 * by the Sec. 6 rules (adaptive restart criteria, step-size rule, primal weight) or, by
 * settings, by Algorithm 1's fixed frequency or the Sec. 5 halving rule, until the
 * Sec. 5 relative KKT error of the returned point is at most settings->eps.
 * x_out [n] and y_out [m] receive the returned point (Sec. 6 rule: the restart
 * candidate of the final evaluation; the Sec. 5 modes and fixed frequency: the
 * average); they live in the handle's mem_space and may be NULL.  Blocking with respect
 * to the handle's stream.  Returns QP_ERR_BATCH_MISMATCH for a batch handle; a solve
 * that does not converge returns QP_OK with res->status set. */
int qp_solve(qp_handle *h, const qp_warm_start *ws, qp_result *res, double *x_out,
             double *y_out);

/* Solves every instance of a batch handle (the same method as qp_solve: Algorithm 1 with
 * the Sec. 6 or Sec. 5 restart rules and the Sec. 5 termination test, applied to each
 * instance independently) in one persistent kernel launch per size class.
 * ws_array: NULL or B warm starts whose x0/y0 point into instance-local arrays;
 * res_array: B results; x_out/y_out: concatenated by var_off / row_off (nullable).
 * Every instance runs the same algorithm and settings as qp_solve and returns the
 * result qp_solve would return for it alone with the same norms.  Blocking.  Returns
 * QP_ERR_BATCH_MISMATCH for a single-QP handle. */
int qp_batch_solve(qp_handle *h, const qp_warm_start *ws_array, qp_result *res_array,
                   double *x_out, double *y_out);

/* Replaces the operator norms used for the step sizes (host arrays): one value each
 * for a single QP, one per instance for a batch.  NULL keeps the current values.
 * Errors: QP_ERR_INVALID_ARGUMENT for negative values or ||A|| = ||Q|| = 0. */
int qp_set_norms(qp_handle *h, const double *norm_A, const double *norm_Q);

/* Batch handles: instances are grouped in four size classes by n_i + m_i
 * (<= 256, <= 1024, <= 2048, larger), each solved by a team of 64, 128, 256, 512 or
 * 1024 threads (1-16 wavefronts) per instance (256, 1024, 1024, 1024 until changed).  qp_batch_autotune times every team size
 * on up to `sample` instances of each class for `iters` iterations and keeps the
 * fastest; threads_out[4] (nullable) receives the choice.  qp_batch_set_threads
 * sets the four team sizes directly.  Both return QP_ERR_BATCH_MISMATCH on a
 * single-QP handle. */
int qp_batch_autotune(qp_handle *h, int32_t sample, int32_t iters, int32_t *threads_out);
int qp_batch_set_threads(qp_handle *h, const int32_t *threads);

/* Copies up to cap records of the last solve's evaluation log (settings.log_checks). */
int qp_get_check_log(qp_handle *h, qp_check_info *buf, int64_t cap, int64_t *len);

/* Phase timings of the last solve run with settings.profile = k >= 1. */
int qp_get_profile(qp_handle *h, qp_profile *out);

/* Norms in use by the handle: one value each for a single QP, num_instances values
 * each for a batch (caller-sized host arrays, nullable). */
int qp_get_norms(qp_handle *h, double *norm_A, double *norm_Q);

/* The Sec. 5 preprocessing scaling in use (settings.precondition = 1): d_var receives
 * D2 (n values, all instances concatenated for a batch), d_row receives D1 (m values);
 * host arrays, nullable.  Without preprocessing both are filled with ones. */
int qp_get_scaling(qp_handle *h, double *d_var, double *d_row);

/* Changes c and/or b (same layout and mem_space as at create; NULL keeps the old
 * vector).  Norm estimates and matrices are unchanged. */
int qp_update_vectors(qp_handle *h, const double *c, const double *b);

/* Releases all device memory of the handle; NULL is a no-op. */
void qp_free(qp_handle *h);

/* Message of the last failed call on this host thread ("" if none). */
const char *qp_last_error(void);

/* QP_ABI_VERSION */
int qp_version(void);

#ifdef __cplusplus
}
#endif
#endif
