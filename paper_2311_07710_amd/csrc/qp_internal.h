// qp_internal.h -- device data layouts shared by the HIP kernels and the host
// orchestration of the rAPDHG solver.  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qpk {

// Row-kernel geometry: one workgroup of BS threads stages up to NNZ_BLK
// products in LDS; rows of a block never exceed BS; a row longer than NNZ_BLK
// is split into chunks whose partial sums are combined by the last chunk to
// arrive (deterministic: partials are summed in chunk order).
constexpr int BS = 256;
constexpr int NNZ_BLK = 2048;
constexpr int EPT = NNZ_BLK / BS;

struct Block {
    int32_t row0, row1;  // rows [row0, row1)
    int32_t e0, e1;      // nnz range [e0, e1) staged by this workgroup
};

// Row partition of one CSR matrix (device pointers).
struct Blocks {
    const Block *blk;
    const int32_t *lr;        // [nblk] long-row id of a chunk block, -1 otherwise
    const int32_t *lr_first;  // [nlr] first block of each long row
    const int32_t *lr_nchunk; // [nlr]
    int32_t *lr_count;        // [nlr] arrival counters, zero between launches
    double *lr_partial;       // [nblk * 4] chunk partial sums
    int32_t nblk, nlr;
};

// Column-panel layout of a matrix for the hot phases.  The columns are split
// into `np` ranges of equal nonzero count; panel k holds the entries of every
// row whose column falls in range k (original order within a row), as its own
// CSR (row pointers are global positions into col/val).  Panel k's row blocks
// run only on the XCDs k*(8/np) .. (k+1)*(8/np)-1 (workgroup w runs on XCD
// w % 8), so the slice of the gathered vector a panel touches stays in those
// XCDs' L2.  Each block writes one partial sum per row to part[k][row]; a
// combine kernel adds the np partials in panel order and runs the epilogue.
struct PBlock {
    int32_t row0, row1;  // rows [row0, row1)
    int32_t e0, e1;      // positions [e0, e1) in col/val
    int32_t panel;
    int32_t lr;          // long-row id (chunk of a row longer than NNZ_BLK) or -1
    int32_t pad0, pad1;
};

struct Panels {
    const PBlock *blk;
    const int32_t *map;       // [grid] block of workgroup w, -1 = idle slot
    const int32_t *rowptr;    // [np * (R + 1)]
    const int32_t *col;
    const double *val;
    const int32_t *lr_first, *lr_nchunk;
    int32_t *lr_count;
    double *lr_partial;       // [nblk * 4]
    double *part;             // [np * R]
    int32_t np, nblk, grid, nlr;
    int32_t nwg;              // persistent workgroups of the hot panel kernels (multiple of 8)
    int64_t R;
};

constexpr int PANEL_ROWS = 1024;  // rows per panel block
constexpr int FOLD_SLOTS = 64;    // spare partial slots for the two-stage KKT reduction

struct Csr {
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
    int64_t nrows;
};

// Per-iteration scalars of one inner index k, written by the decision kernel.
struct Step {
    double p;          // primal step  (Sec. 6: eta / omega; Thm 1: eta_k)
    double d;          // dual step    (Sec. 6: eta * omega; Thm 1: tau_k)
    double w;          // 1 / beta_k = 2 / (k + 2)
    double theta_next; // theta_{k+1} = (k + 1) / (k + 2)
    double w_next;     // 1 / beta_{k+1}
    double pad[3];
};

// Indices of the per-point KKT quantities in the block partials.
enum : int {
    RA_RES0 = 0, RA_RES1, RA_AX0, RA_AX1, RA_BY0, RA_BY1, RA_DY0, RA_DY1, RA_NV
};
enum : int {
    RP_DRES0 = 0, RP_DRES1, RP_QX0, RP_QX1, RP_ATY0, RP_ATY1, RP_XQX0, RP_XQX1, RP_CX0, RP_CX1,
    RP_BND0, RP_BND1, RP_DX0, RP_DX1, RP_NV
};

// Infeasibility certificate quantities of the direction (dx+, dy+) = projected
// z - z_restart, on the given problem: max violation of A dx+ (EQ |.|, GE [-.]+),
// b'dy+, ||Q dx+||_inf, max |A'dy+| over components whose needed bound is infinite,
// the support of X along A'dy+ over finite bounds, c'dx+.
enum : int { INF_AVIOL = 0, INF_BDY, INF_QDX, INF_GVIOL, INF_SUPP, INF_CDX, INF_NV };
// per-block partials: rows of A (maxima first) and rows of P (maxima first)
enum : int { IA_AVIOL = 0, IA_BDY, IA_NV };
enum : int { IP_QDX = 0, IP_GVIOL, IP_SUPP, IP_CDX, IP_NV };

struct State {
    double omega, r0, prev_cand, s_last;
    double r_cur, r_avg;
    double kkt[2][6];  // per point: r_primal, r_dual, r_gap, rel_kkt, primal_obj, dual_obj
    double inf[INF_NV];  // infeasibility quantities of the last evaluation
    int64_t total, k, restarts, kkt_evals;
    int32_t done, status, cand, restart_flag;
    int32_t used_warm, checks, pad0, pad1;
    int64_t t_start, t_end;  // batch: device wall-clock ticks after the launch began
};

struct DevSettings {
    double eps, beta_sufficient, beta_necessary, beta_artificial, pw_smoothing, eps_zero;
    double step_safety, norm_A, norm_Q, b_inf, c_inf;
    int64_t max_iter;
    int32_t restart_mode, fixed_K, interval;
    int32_t momentum;  // 1: Algorithm 1 weights; 0: plain PDHG (beta = theta = 1)
    int32_t detect_infeas;
    double eps_infeas;
};

enum : int { DECIDE_INIT = 0, DECIDE_CHECK = 1, DECIDE_FALLBACK = 2 };
enum : int { MODE_ADAPTIVE = 0, MODE_FIXED_K = 1, MODE_HALVING = 2, MODE_NONE = 3 };
enum : int { ST_OPTIMAL = 0, ST_ITER_LIMIT = 1, ST_TIME_LIMIT = 2, ST_NUMERICAL = 3,
             ST_PRIMAL_INFEASIBLE = 4, ST_DUAL_INFEASIBLE = 5 };

// Vectors of a single-instance solve (device pointers).
struct Vecs {
    double *x, *xbar, *xt, *xmd[2], *xrs;  // primal: iterate, average, extrapolated
                                          // point, x_md ping-pong, last restart point
    double *y, *ybar, *yrs;               // dual
    const double *c, *b, *l, *u;
    const uint8_t *rt;
    const double *dv, *dr;                // preconditioning D2 [n], D1 [m], or nullptr
    int32_t uniform_bounds;               // 1: l_j = lo_all and u_j = hi_all for every j
    double lo_all, hi_all;
    double2 *zz;                          // [n + m] pairs (x_j, x-bar_j), then (y_i, y-bar_i):
                                          // the gathers of the KKT panel kernels, or nullptr
};

// ---- infeasibility certificates (qp_kernels.hip) ----
// dxh [n], dyh [m]: scratch for the projected directions; part_a / part_p: per-block
// partials with FOLD_SLOTS spare slots; writes st->inf.
void launch_infeas(hipStream_t s, const Blocks &bkA, const Csr &A, const Blocks &bkP,
                   const Csr &P, const Vecs &v, double *dxh, double *dyh, double *part_a,
                   int32_t nslotA, double *part_p, int32_t nslotP, State *st, int64_t n,
                   int64_t m);

// ---- diagonal preconditioning (qp_scale.hip) ----
enum : int { SCALE_MAX = 0, SCALE_L2 = 1, SCALE_SUM = 2 };
struct ScaleInput {
    int64_t n, m;                       // variables / constraint rows (all instances)
    const int32_t *a_rowptr, *a_col;    // device CSR of A (batch: local columns)
    double *a_val;                      // scaled in place
    const int32_t *p_rowptr, *p_col;    // device CSR of P = [Q | -A']
    double *p_val;                      // scaled in place
    const int32_t *var_off, *row_off;   // device batch offsets [count+1], or nullptr
    int32_t count;
    int32_t ruiz_iters, l2, pc;
};
// d (device, n+m): receives the cumulative scaling (D2 for variables, then D1);
// work: 2(n+m) doubles.
int precondition_device(hipStream_t s, const ScaleInput &in, double *work, double *d);
// out = in * d (divide = 0) or in / d (divide = 1), elementwise
void launch_scale_pair(hipStream_t s, double *out, const double *in, const double *d,
                       int64_t len, int divide);

// ---- launchers (qp_kernels.hip) ----
void launch_dual(hipStream_t s, const Blocks &bk, const Csr &A, const Vecs &v, const Step *step,
                 const State *st);
void launch_primal(hipStream_t s, const Blocks &bk, const Csr &P, const Vecs &v, int md_in,
                   const Step *step, const State *st, int64_t n);
void launch_kkt_rows(hipStream_t s, const Blocks &bk, const Csr &A, const Vecs &v,
                     double *partials, const State *st);
void launch_kkt_cols(hipStream_t s, const Blocks &bk, const Csr &P, const Vecs &v,
                     double *partials, const State *st, int64_t n);
// KKT products through the column panels (kpart: 2 np m / 4 np n doubles); return the
// number of partial slots written for launch_decide
// fills v.zz from x, x-bar, y, y-bar (before the KKT panel kernels)
void launch_interleave(hipStream_t s, const Vecs &v, const State *st, int64_t n, int64_t m);
int32_t launch_kkt_rows_panels(hipStream_t s, const Panels &pn, const Vecs &v, double *kpart,
                               double *partials, const State *st, int64_t n, int64_t m);
int32_t launch_kkt_cols_panels(hipStream_t s, const Panels &pn, const Vecs &v, double *kpart,
                               double *partials, const State *st, int64_t n);
void launch_decide(hipStream_t s, int mode, double *partA, int32_t nslotA, double *partP,
                   int32_t nslotP, State *st, Step *table, const DevSettings &ds, int32_t len);
void launch_apply(hipStream_t s, const Vecs &v, int md_out, const State *st, int64_t n,
                  int64_t m);
void launch_init(hipStream_t s, const Vecs &v, const double *x0, const double *y0, int64_t n,
                 int64_t m, int pair_with_cold);
void launch_fallback_apply(hipStream_t s, const Vecs &v, const State *st, int64_t n, int64_t m);
void launch_state_reset(hipStream_t s, State *st, double omega, int64_t max_iter);

// column-panel phases (partials + combine); panel_resident_workgroups: workgroups of the
// persistent panel kernels resident at once on `device` (a multiple of 8; 0 on error)
int32_t panel_resident_workgroups(int device);
void launch_dual_panels(hipStream_t s, const Panels &pn, const Vecs &v, int64_t n,
                        const Step *step, const State *st);
void launch_primal_panels(hipStream_t s, const Panels &pn, const Vecs &v, int md_in, int64_t n,
                          const Step *step, const State *st);

// power iteration helpers: y = M_1 x + sign2 * M_2 x2 where M_1 holds the
// entries with col < split and M_2 those with col >= split (x or x2 may be null)
void launch_spmv_plain(hipStream_t s, const Blocks &bk, const Csr &M, const double *x,
                       const double *x2, int64_t split, double *y, double sign2);
// partials[i] = sum over the i-th contiguous chunk of a .* b (fixed order)
void launch_dot_partials(hipStream_t s, const double *a, const double *b, int64_t n,
                         double *partials, int32_t nparts);
void launch_div(hipStream_t s, double *dst, const double *src, int64_t n, double den);
void launch_fill(hipStream_t s, double *dst, int64_t n, double value);
int dot_nparts(int64_t n);

}  // namespace qpk
