// qp_batch.hip -- many independent small QPs solved by rAPDHG in one
// persistent launch per size class (segment-CSR layout).
//
// Layout: instances are concatenated; A's row pointers are global offsets into
// the concatenated nonzeros, column indices are local to the instance.  Each
// instance also gets its own P_i = [Q_i | -A_i'] (local columns < n_i address
// x, columns n_i + r address y_r), built on the host at create.
//
// Kernel: one workgroup (a "team" of NT threads = NT/64 wavefronts) per
// instance.  Workgroups pop instance ids from an atomic queue ordered by
// decreasing work, run the whole solve -- Algorithm 1 iterations, Sec. 5
// relKKT evaluation every `interval` iterations, Sec. 6 restart / primal
// weight / step sizes -- with workgroup barriers between the dual phase, the
// primal phase and the evaluation, write the returned point and their final
// state, and pop the next instance; every workgroup exits once the queue is
// empty.  Rows are handled one per thread with sums in CSR order, so each row
// sum is the same operation sequence as a sequential CSR product.  The team
// size per size class is chosen by timing (qp_batch_autotune).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "qp_batch.h"
#include "qp_decide.h"
#include "qp_host.h"
#include "qp_internal.h"

using qph::DevMem;
using qph::fail;

namespace qpb {

using namespace qpk;

constexpr int NCLASS = 4;
static const int32_t CLASS_LIMIT[NCLASS] = {256, 1024, 2048, 1 << 30};  // n_i + m_i upper bound
static const int32_t THREAD_CHOICES[] = {64, 128, 256, 512, 1024};
constexpr int NCHOICE = (int)(sizeof(THREAD_CHOICES) / sizeof(THREAD_CHOICES[0]));

struct BatchDev {
    int32_t count;
    const int32_t *var_off, *row_off;
    const int32_t *a_rowptr, *a_col;
    const double *a_val;
    const int32_t *p_rowptr, *p_col;
    const double *p_val;
    const double *c, *b, *l, *u;
    const uint8_t *rt;
    const double *normA, *normQ, *b_inf, *c_inf, *omega0;
    const uint8_t *has_x0, *has_y0;
    const double *x0, *y0;
    double *x, *xbar, *xt, *xmd0, *xmd1, *xrs, *y, *ybar, *yrs;
    double *x_out, *y_out;
    State *res;
    const int32_t *order;
    int32_t order_count;
    int32_t *head;
    const int64_t *clock0;
    int64_t deadline_ticks;  // 0: no time limit
    int32_t warm_fallback, any_warm;
    int32_t lds_doubles;     // dynamic LDS per team (doubles); 0: gathered vectors in HBM
    // rows longer than LONG_ROW nonzeros are reduced by the whole team
    const int32_t *lrA_off, *lrA;  // per instance [off[i], off[i+1]) into local A row ids
    const int32_t *lrP_off, *lrP;  // same for rows of P
    const double *dscale;          // preconditioning: D2 of all variables, then D1; or nullptr
    int64_t ntot;                  // variables of all instances
    // sliced copies of A and P for the iteration's row loops (see build_sliced)
    const int32_t *sa_inst, *sa_start, *sa_width, *sa_col;
    const double *sa_val;
    const int32_t *sp_inst, *sp_start, *sp_width, *sp_col;
    const double *sp_val;
};

constexpr int LONG_ROW = 128;
constexpr int SLICE = 64;  // rows per slice of the sliced layout: one per lane of a wavefront

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double bmax(double a, double b) { return (b > a || b != b) ? b : a; }

// Team-wide reduction of NV values, the first nmax_first by maximum and the rest by sum;
// result in thread 0's cv.  NV is a compile-time count so that cv, a local array of the
// caller, stays in registers (indexed at run time it would live in private memory, and
// every access would pay a memory round trip).
template <int NT, int NV>
__device__ __forceinline__ void team_reduce(double *cv, int nmax_first,
                                            double *red /*[32][NT/64]*/) {
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double x = cv[v];
        const bool mx = v < nmax_first;
        for (int off = 32; off >= 1; off >>= 1) {
            const double o = __shfl_xor(x, off, 64);
            x = mx ? bmax(x, o) : x + o;
        }
        if (lane == 0) red[v * (NT / 64) + wid] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const bool mx = v < nmax_first;
            double acc = red[v * (NT / 64)];
            for (int w = 1; w < NT / 64; ++w) {
                const double o = red[v * (NT / 64) + w];
                acc = mx ? bmax(acc, o) : acc + o;
            }
            cv[v] = acc;
        }
    }
    __syncthreads();
}

// sums of W values over the team, valid in thread 0 (fixed order)
template <int NT, int W>
__device__ void team_sum(double *v, double *red) {
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = 0; q < W; ++q) {
        double x = v[q];
        for (int off = 32; off >= 1; off >>= 1) x = x + __shfl_xor(x, off, 64);
        if (lane == 0) red[q * (NT / 64) + wid] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 0; q < W; ++q) {
            double acc = red[q * (NT / 64)];
            for (int w = 1; w < NT / 64; ++w) acc = acc + red[q * (NT / 64) + w];
            v[q] = acc;
        }
    __syncthreads();
}

// per-row KKT contributions (rows of A: primal residuals, |Ax|, b'y, restart distances)
// dr / dv: the instance's preconditioning D1 / D2 (nullptr: none); the infinity norms
// are those of the given problem, whose row i is the scaled row divided by D1_i and whose
// column j is the scaled one divided by D2_j (dot products are invariant).
__device__ __forceinline__ void kkt_row_contrib(int i, double s0, double s1, const double *b,
                                                const uint8_t *rt, const double *y,
                                                const double *ybar, const double *yrs,
                                                const double *dr, double *ra) {
    const double bi = b[i];
    double r0 = s0 - bi, r1 = s1 - bi;
    if (rt[i] == 1) {
        r0 = (r0 < 0.0) ? -r0 : 0.0;
        r1 = (r1 < 0.0) ? -r1 : 0.0;
    }
    const double sr = dr ? dr[i] : 1.0;
    ra[RA_RES0] = bmax(ra[RA_RES0], fabs(r0) / sr);
    ra[RA_RES1] = bmax(ra[RA_RES1], fabs(r1) / sr);
    ra[RA_AX0] = bmax(ra[RA_AX0], fabs(s0) / sr);
    ra[RA_AX1] = bmax(ra[RA_AX1], fabs(s1) / sr);
    const double yi = y[i], ybi = ybar[i], yr = yrs[i];
    ra[RA_BY0] += bi * yi;
    ra[RA_BY1] += bi * ybi;
    const double d0 = yi - yr, d1 = ybi - yr;
    ra[RA_DY0] += d0 * d0;
    ra[RA_DY1] += d1 * d1;
}

// per-column KKT contributions (rows of P: reduced costs, |Qx|, |A'y|, x'Qx, c'x, bound terms)
__device__ __forceinline__ void kkt_col_contrib(int j, const double *q, const double *na,
                                                const double *c, const double *l,
                                                const double *u, const double *x,
                                                const double *xbar, const double *xrs,
                                                const double *dv, double *rp) {
    const double cj = c[j], lj = l[j], uj = u[j];
    const bool lo_fin = isfinite(lj), hi_fin = isfinite(uj);
    const double sv = dv ? dv[j] : 1.0;
    for (int p = 0; p < 2; ++p) {
        const double xp = p == 0 ? x[j] : xbar[j];
        const double aty = -na[p];
        const double lam = q[p] + cj - aty;
        double lam_hat;
        if (lo_fin && hi_fin) lam_hat = lam;
        else if (lo_fin) lam_hat = lam > 0.0 ? lam : 0.0;
        else if (hi_fin) lam_hat = lam < 0.0 ? lam : 0.0;
        else lam_hat = 0.0;
        rp[RP_DRES0 + p] = bmax(rp[RP_DRES0 + p], fabs(lam - lam_hat) / sv);
        rp[RP_QX0 + p] = bmax(rp[RP_QX0 + p], fabs(q[p]) / sv);
        rp[RP_ATY0 + p] = bmax(rp[RP_ATY0 + p], fabs(aty) / sv);
        rp[RP_XQX0 + p] += xp * q[p];
        rp[RP_CX0 + p] += cj * xp;
        double bnd = 0.0;
        if (lo_fin && lam_hat > 0.0) bnd = lj * lam_hat;
        if (hi_fin && lam_hat < 0.0) bnd = uj * lam_hat;
        rp[RP_BND0 + p] += bnd;
        const double dx = xp - xrs[j];
        rp[RP_DX0 + p] += dx * dx;
    }
}

// Sum of val[e] * src(col[e]) over e in [e0, e1), added in CSR order; the loads of
// four entries are issued together so that their latencies overlap.
template <class F>
__device__ __forceinline__ double row_dot(const int32_t *__restrict__ col,
                                          const double *__restrict__ val, int e0, int e1, F src) {
    double s = 0.0;
    int e = e0;
    for (; e + 4 <= e1; e += 4) {
        const int c0 = col[e], c1 = col[e + 1], c2 = col[e + 2], c3 = col[e + 3];
        const double a0 = val[e], a1 = val[e + 1], a2 = val[e + 2], a3 = val[e + 3];
        const double g0 = src(c0), g1 = src(c1), g2 = src(c2), g3 = src(c3);
        s = s + a0 * g0;
        s = s + a1 * g1;
        s = s + a2 * g2;
        s = s + a3 * g3;
    }
    for (; e < e1; ++e) s = s + val[e] * src(col[e]);
    return s;
}

// The same sum over the sliced layout: entry k of this lane's row sits at e + 64 k.
// The slice width w (its longest row) is common to the wavefront, so the 64 lanes of
// each load read consecutive addresses; entries k >= len are padding and are skipped,
// so the row is added in CSR order exactly as row_dot does.  Entries go four at a time
// with their loads issued together; the last one to three as one more such group, whose
// missing entries repeat the first one (a valid column) and are never added.
template <class C, class F>
__device__ __forceinline__ double sliced_dot(const C *__restrict__ col,
                                             const double *__restrict__ val, int e, int w,
                                             int len, F src) {
    double s = 0.0;
    int k = 0;
    for (; k + 4 <= w; k += 4, e += 4 * SLICE) {
        const int c0 = col[e], c1 = col[e + SLICE], c2 = col[e + 2 * SLICE],
                  c3 = col[e + 3 * SLICE];
        const double a0 = val[e], a1 = val[e + SLICE], a2 = val[e + 2 * SLICE],
                     a3 = val[e + 3 * SLICE];
        const double g0 = src(c0), g1 = src(c1), g2 = src(c2), g3 = src(c3);
        if (k < len) s = s + a0 * g0;
        if (k + 1 < len) s = s + a1 * g1;
        if (k + 2 < len) s = s + a2 * g2;
        if (k + 3 < len) s = s + a3 * g3;
    }
    if (k < w) {
        const int r = w - k;
        const int e1 = r > 1 ? e + SLICE : e, e2 = r > 2 ? e + 2 * SLICE : e;
        const int c0 = col[e], c1 = col[e1], c2 = col[e2];
        const double a0 = val[e], a1 = val[e1], a2 = val[e2];
        const double g0 = src(c0), g1 = src(c1), g2 = src(c2);
        if (k < len) s = s + a0 * g0;
        if (k + 1 < len) s = s + a1 * g1;
        if (k + 2 < len) s = s + a2 * g2;
    }
    return s;
}

// Infeasibility quantities (State::inf order) of the drift z - z_restart of one instance,
// projected onto the dual cone (dy+) and the recession cone of X (dx+); result in
// thread 0's out.  Same row/column contributions as the single-instance kernels.
template <int NT>
__device__ __forceinline__ void team_infeas(int n, int m, const int32_t *arp, const int32_t *acol,
                                         const double *aval, const int32_t *prp,
                                         const int32_t *pcol, const double *pval,
                                         const double *c, const double *b, const double *l,
                                         const double *u, const uint8_t *rt, const double *x,
                                         const double *xrs, const double *y, const double *yrs,
                                         const double *dv, const double *dr, const int32_t *lra,
                                         int nlra, const int32_t *lrp, int nlrp, double *red,
                                         double *out) {
    auto dxh = [&](int j) {
        const bool lo = isfinite(l[j]), hi = isfinite(u[j]);
        double v = x[j] - xrs[j];
        if (lo && hi) v = 0.0;
        else if (lo && v < 0.0) v = 0.0;
        else if (hi && v > 0.0) v = 0.0;
        return v;
    };
    auto dyh = [&](int i) {
        const double v = y[i] - yrs[i];
        return (rt[i] == 1 && v < 0.0) ? 0.0 : v;
    };
    // cv: 0 A dx+ violation, 1 |Q dx+|, 2 |A'dy+| needing an infinite bound (maxima);
    //     3 b'dy+, 4 support of X along A'dy+, 5 c'dx+ (sums)
    double cv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    auto row = [&](int i, double sa) {
        const double viol = rt[i] == 1 ? (sa < 0.0 ? -sa : 0.0) : fabs(sa);
        cv[0] = bmax(cv[0], viol / (dr ? dr[i] : 1.0));
        cv[3] += b[i] * dyh(i);
    };
    auto col = [&](int j, double qd, double nat) {
        const double sv = dv ? dv[j] : 1.0;
        const double g = -nat;
        double viol = 0.0, supp = 0.0;
        if (g > 0.0) {
            if (isfinite(u[j])) supp = u[j] * g;
            else viol = g;
        } else if (g < 0.0) {
            if (isfinite(l[j])) supp = l[j] * g;
            else viol = -g;
        }
        cv[1] = bmax(cv[1], fabs(qd) / sv);
        cv[2] = bmax(cv[2], viol / sv);
        cv[4] += supp;
        cv[5] += c[j] * dxh(j);
    };
    for (int i = threadIdx.x; i < m; i += NT) {
        if (arp[i + 1] - arp[i] > LONG_ROW) continue;
        row(i, row_dot(acol, aval, arp[i], arp[i + 1], dxh));
    }
    for (int q = 0; q < nlra; ++q) {
        const int i = lra[q];
        double sv[1] = {0.0};
        for (int e = arp[i] + threadIdx.x; e < arp[i + 1]; e += NT)
            sv[0] = sv[0] + aval[e] * dxh(acol[e]);
        team_sum<NT, 1>(sv, red);
        if (threadIdx.x == 0) row(i, sv[0]);
    }
    for (int j = threadIdx.x; j < n; j += NT) {
        if (prp[j + 1] - prp[j] > LONG_ROW) continue;
        double qd = 0.0, na = 0.0;
        for (int e = prp[j]; e < prp[j + 1]; ++e) {
            const int cc = pcol[e];
            if (cc < n) qd = qd + pval[e] * dxh(cc);
            else na = na + pval[e] * dyh(cc - n);
        }
        col(j, qd, na);
    }
    for (int q = 0; q < nlrp; ++q) {
        const int j = lrp[q];
        double sv[2] = {0.0, 0.0};
        for (int e = prp[j] + threadIdx.x; e < prp[j + 1]; e += NT) {
            const int cc = pcol[e];
            if (cc < n) sv[0] = sv[0] + pval[e] * dxh(cc);
            else sv[1] = sv[1] + pval[e] * dyh(cc - n);
        }
        team_sum<NT, 2>(sv, red);
        if (threadIdx.x == 0) col(j, sv[0], sv[1]);
    }
    team_reduce<NT, 6>(cv, 3, red);
    if (threadIdx.x == 0) {
        out[INF_AVIOL] = cv[0];
        out[INF_QDX] = cv[1];
        out[INF_GVIOL] = cv[2];
        out[INF_BDY] = cv[3];
        out[INF_SUPP] = cv[4];
        out[INF_CDX] = cv[5];
    }
}

// KKT quantities of z = (x, y) and z-bar for one instance; results in thread 0's ra/rp.
// Rows up to LONG_ROW nonzeros: one thread each; longer rows: the whole team.
template <int NT>
__device__ void team_kkt(int n, int m, const int32_t *arp, const int32_t *acol, const double *aval,
                         const int32_t *prp, const int32_t *pcol, const double *pval,
                         const double *c, const double *b, const double *l, const double *u,
                         const uint8_t *rt, const double *x, const double *xbar,
                         const double *xrs, const double *y, const double *ybar,
                         const double *yrs, double *ra, double *rp, double *red,
                         const int32_t *lra, int nlra, const int32_t *lrp, int nlrp,
                         const double *dv, const double *dr) {
    // accumulators in registers (local arrays with constant indices); each set goes to
    // ra or rp, which the out-of-line decision reads from memory, right after its
    // reduction (so that only one set is live at a time)
    double la[RA_NV], lp[RP_NV];
    for (int v = 0; v < RA_NV; ++v) la[v] = 0.0;
    for (int i = threadIdx.x; i < m; i += NT) {
        if (arp[i + 1] - arp[i] > LONG_ROW) continue;
        double s0 = 0.0, s1 = 0.0;
        for (int e = arp[i]; e < arp[i + 1]; ++e) {
            const int cc = acol[e];
            const double a = aval[e];
            s0 = s0 + a * x[cc];
            s1 = s1 + a * xbar[cc];
        }
        kkt_row_contrib(i, s0, s1, b, rt, y, ybar, yrs, dr, la);
    }
    for (int q = 0; q < nlra; ++q) {
        const int i = lra[q];
        double sv[2] = {0.0, 0.0};
        for (int e = arp[i] + threadIdx.x; e < arp[i + 1]; e += NT) {
            const int cc = acol[e];
            const double a = aval[e];
            sv[0] = sv[0] + a * x[cc];
            sv[1] = sv[1] + a * xbar[cc];
        }
        team_sum<NT, 2>(sv, red);
        if (threadIdx.x == 0) kkt_row_contrib(i, sv[0], sv[1], b, rt, y, ybar, yrs, dr, la);
    }
    team_reduce<NT, RA_NV>(la, 4, red);
    if (threadIdx.x == 0)
        for (int v = 0; v < RA_NV; ++v) ra[v] = la[v];
    for (int v = 0; v < RP_NV; ++v) lp[v] = 0.0;
    for (int j = threadIdx.x; j < n; j += NT) {
        if (prp[j + 1] - prp[j] > LONG_ROW) continue;
        double q[2] = {0.0, 0.0}, na[2] = {0.0, 0.0};
        for (int e = prp[j]; e < prp[j + 1]; ++e) {
            const int cc = pcol[e];
            const double a = pval[e];
            if (cc < n) {
                q[0] = q[0] + a * x[cc];
                q[1] = q[1] + a * xbar[cc];
            } else {
                na[0] = na[0] + a * y[cc - n];
                na[1] = na[1] + a * ybar[cc - n];
            }
        }
        kkt_col_contrib(j, q, na, c, l, u, x, xbar, xrs, dv, lp);
    }
    for (int qq = 0; qq < nlrp; ++qq) {
        const int j = lrp[qq];
        double sv[4] = {0.0, 0.0, 0.0, 0.0};
        for (int e = prp[j] + threadIdx.x; e < prp[j + 1]; e += NT) {
            const int cc = pcol[e];
            const double a = pval[e];
            if (cc < n) {
                sv[0] = sv[0] + a * x[cc];
                sv[1] = sv[1] + a * xbar[cc];
            } else {
                sv[2] = sv[2] + a * y[cc - n];
                sv[3] = sv[3] + a * ybar[cc - n];
            }
        }
        team_sum<NT, 4>(sv, red);
        if (threadIdx.x == 0) {
            double q[2] = {sv[0], sv[1]}, na[2] = {sv[2], sv[3]};
            kkt_col_contrib(j, q, na, c, l, u, x, xbar, xrs, dv, lp);
        }
    }
    team_reduce<NT, RP_NV>(lp, 6, red);
    if (threadIdx.x == 0)
        for (int v = 0; v < RP_NV; ++v) rp[v] = lp[v];
}

// The evaluation logic is called out of line: inlined, its exp/log/sqrt code would
// set the register budget (and so the occupancy) of the whole iteration loop.
__device__ __attribute__((noinline)) void batch_decide(int mode, const double *ra,
                                                       const double *rp, State *S,
                                                       const DevSettings *ds, int32_t len) {
    decide_update(mode, ra, rp, *S, *ds, len);
}

// projected primal step and x-bar averaging of one row (row sum s, c_j, l_j, u_j,
// x_j, x-bar_j): the new x_j and x-bar_j
__device__ __forceinline__ void primal_update(double s, const Step &st, double cj, double lj,
                                              double uj, double xo, double xbo, double &xn,
                                              double &xb) {
    const double g = s + cj;
    xn = xo - st.p * g;
    if (xn < lj) xn = lj;
    if (xn > uj) xn = uj;
    xb = (1.0 - st.w) * xbo + st.w * xn;
}

// the row's outputs: x, x-bar and the next x~ / x_md
__device__ __forceinline__ void primal_store(int j, const Step &st, double xo, double xn,
                                             double xb, double *x, double *xbar, double *xt,
                                             double *xout) {
    x[j] = xn;
    xbar[j] = xb;
    xt[j] = xn + st.theta_next * (xn - xo);
    xout[j] = (1.0 - st.w_next) * xb + st.w_next * xn;
}

__device__ __forceinline__ void primal_row(int j, double s, const Step &st, const double *c,
                                           const double *l, const double *u, double *x,
                                           double *xbar, double *xt, double *xout) {
    const double xo = x[j];
    double xn, xb;
    primal_update(s, st, c[j], l[j], u[j], xo, xbar[j], xn, xb);
    primal_store(j, st, xo, xn, xb, x, xbar, xt, xout);
}

__device__ __forceinline__ double proj_box_b(double v, double lo, double hi) {
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

// LDS residency of an instance's vectors
enum LdsMode {
    LDS_NONE = 0,      // all vectors in HBM
    LDS_GATHERED = 1,  // x~ | x_md[0] | x_md[1] | y  (3 n + m doubles)
    LDS_ALL = 2,       // x~ | x_md[0] | x_md[1] | x | x-bar | y | y-bar  (5 n + 2 m doubles)
};

__host__ __device__ inline int lds_mode_of(int64_t n, int64_t m, int64_t lds_doubles) {
    if (5 * n + 2 * m <= lds_doubles) return LDS_ALL;
    if (3 * n + m <= lds_doubles) return LDS_GATHERED;
    return LDS_NONE;
}

// One instance, start to finish, by the whole team.  MODE says which vectors live in
// LDS.  As a compile-time parameter it lets every access to them compile to LDS
// instructions; chosen at run time through one pointer, they became generic (flat)
// accesses, which pay vector-memory latency even when the address is in LDS.
template <int NT, int MODE>
__device__ __forceinline__ void solve_instance(const BatchDev &a, const DevSettings &base,
                                               int id, double *smem, State &S, Step *stp,
                                               double *red, double &s_last) {
    const int t = threadIdx.x;
    {
        const int v0 = a.var_off[id], n = a.var_off[id + 1] - v0;
        const int r0 = a.row_off[id], m = a.row_off[id + 1] - r0;
        const int32_t *arp = a.a_rowptr + r0;
        const int32_t *prp = a.p_rowptr + v0;
        const double *c = a.c + v0, *l = a.l + v0, *u = a.u + v0, *b = a.b + r0;
        const uint8_t *rt = a.rt + r0;
        double *xrs = a.xrs + v0, *yrs = a.yrs + r0;
        // The vectors every iteration reads and writes live in LDS as far as the
        // instance fits: with all of them there (LDS_ALL) neither the gathers nor the
        // epilogues touch global memory and the barriers between the phases wait for
        // no global stores; LDS_GATHERED keeps only the gathered ones.
        // (named pointers, not an array indexed at run time, so LDS stays visible)
        constexpr bool G = MODE != LDS_NONE, ALL = MODE == LDS_ALL;
        double *xt = G ? smem : a.xt + v0;
        double *const xmd0 = G ? smem + n : a.xmd0 + v0;
        double *const xmd1 = G ? smem + 2 * n : a.xmd1 + v0;
        double *x = ALL ? smem + 3 * n : a.x + v0;
        double *xbar = ALL ? smem + 4 * n : a.xbar + v0;
        double *y = ALL ? smem + 5 * n : G ? smem + 3 * n : a.y + r0;
        double *ybar = ALL ? smem + 5 * n + m : a.ybar + r0;
        const double *dvi = a.dscale ? a.dscale + v0 : nullptr;
        const double *dri = a.dscale ? a.dscale + a.ntot + r0 : nullptr;
        const int32_t *sa_start = a.sa_start + a.sa_inst[id], *sa_width = a.sa_width + a.sa_inst[id];
        const int32_t *sp_start = a.sp_start + a.sp_inst[id], *sp_width = a.sp_width + a.sp_inst[id];
        const int32_t *lra = a.lrA + a.lrA_off[id];
        const int nlra = a.lrA_off[id + 1] - a.lrA_off[id];
        const int32_t *lrp = a.lrP + a.lrP_off[id];
        const int nlrp = a.lrP_off[id + 1] - a.lrP_off[id];
        // Matrix cache: with every vector in LDS (LDS_ALL), the rest of the team's LDS
        // holds the instance's leading slices of sliced A, then of sliced P (whole slices,
        // so the rows of a wavefront are all cached or all not), and those rows read their
        // entries from LDS.  A team streams its matrix through one CU's L1 every iteration;
        // the cached share leaves that path.  Columns are kept in 16 bits (with its vectors
        // in LDS an instance has n + m < 65536), 10 bytes an entry.  Values and order are
        // the global arrays': results are unchanged.
        int ca_sl = 0, cp_sl = 0;  // cached slices of A and of P
        int ca_n = 0, cp_n = 0;    // cached entries
        const int a_base = m > 0 ? sa_start[0] : 0, p_base = sp_start[0];
        double *cva = smem, *cvp = smem;
        uint16_t *cca = reinterpret_cast<uint16_t *>(smem), *ccp = cca;
        if (ALL && n + m <= 65535) {
            int64_t room = ((int64_t)a.lds_doubles - 5 * (int64_t)n - 2 * (int64_t)m) * 8;
            const int nsa = (m + SLICE - 1) / SLICE, nsp = (n + SLICE - 1) / SLICE;
            while (ca_sl < nsa && 10 * (int64_t)SLICE * sa_width[ca_sl] <= room) {
                room -= 10 * (int64_t)SLICE * sa_width[ca_sl];
                ca_n += SLICE * sa_width[ca_sl];
                ++ca_sl;
            }
            while (cp_sl < nsp && 10 * (int64_t)SLICE * sp_width[cp_sl] <= room) {
                room -= 10 * (int64_t)SLICE * sp_width[cp_sl];
                cp_n += SLICE * sp_width[cp_sl];
                ++cp_sl;
            }
            cva = smem + 5 * n + 2 * m;
            cvp = cva + ca_n;
            cca = reinterpret_cast<uint16_t *>(cvp + cp_n);
            ccp = cca + ca_n;
            for (int q = t; q < ca_n; q += NT) {
                cva[q] = a.sa_val[a_base + q];
                cca[q] = (uint16_t)a.sa_col[a_base + q];
            }
            for (int q = t; q < cp_n; q += NT) {
                cvp[q] = a.sp_val[p_base + q];
                ccp[q] = (uint16_t)a.sp_col[p_base + q];
            }
        }
        DevSettings ds = base;
        ds.norm_A = a.normA[id];
        ds.norm_Q = a.normQ[id];
        ds.b_inf = a.b_inf[id];
        ds.c_inf = a.c_inf[id];
        const bool warm = a.any_warm && (a.has_x0[id] || a.has_y0[id]);
        const bool pair = warm && a.warm_fallback;
        // initial point (zeros or the warm start, projected); with the fallback the
        // warm point sits in (x, y) and the cold one in (x-bar, y-bar)
        for (int j = t; j < n; j += NT) {
            const double xc = proj_box_b(0.0, l[j], u[j]);
            const double xw = (warm && a.has_x0[id]) ? proj_box_b(a.x0[v0 + j], l[j], u[j]) : xc;
            x[j] = xw;
            xbar[j] = pair ? xc : xw;
            xt[j] = xw;
            xmd0[j] = xw;
            xrs[j] = xw;
        }
        for (int i = t; i < m; i += NT) {
            double yw = (warm && a.has_y0[id]) ? a.y0[r0 + i] : 0.0;
            if (rt[i] == 1 && yw < 0.0) yw = 0.0;
            y[i] = yw;
            ybar[i] = pair ? 0.0 : yw;
            yrs[i] = yw;
        }
        if (t == 0) {
            S.omega = a.omega0[id];
            S.r0 = 0.0;
            S.prev_cand = INFINITY;
            S.s_last = 0.0;
            S.r_cur = S.r_avg = 0.0;
            S.total = S.k = S.restarts = S.kkt_evals = 0;
            S.done = 0;
            S.status = -1;
            S.cand = 0;
            S.restart_flag = 0;
            S.used_warm = (warm && !pair) ? 1 : 0;
            S.checks = 0;
            S.t_start = (int64_t)wall_clock64() - *a.clock0;
        }
        __syncthreads();
        double ra[RA_NV], rp[RP_NV];
        if (pair) {
            team_kkt<NT>(n, m, arp, a.a_col, a.a_val, prp, a.p_col, a.p_val, c, b, l, u, rt, x,
                         xbar, xrs, y, ybar, yrs, ra, rp, red, lra, nlra, lrp, nlrp, dvi, dri);
            if (t == 0) batch_decide(DECIDE_FALLBACK, ra, rp, &S, &ds, 0);
            __syncthreads();
            const int take = S.used_warm;
            for (int j = t; j < n; j += NT) {
                const double xv = take ? x[j] : xbar[j];
                x[j] = xbar[j] = xt[j] = xmd0[j] = xrs[j] = xv;
            }
            for (int i = t; i < m; i += NT) {
                const double yv = take ? y[i] : ybar[i];
                y[i] = ybar[i] = yrs[i] = yv;
            }
            __syncthreads();
        }
        team_kkt<NT>(n, m, arp, a.a_col, a.a_val, prp, a.p_col, a.p_val, c, b, l, u, rt, x, xbar,
                     xrs, y, ybar, yrs, ra, rp, red, lra, nlra, lrp, nlrp, dvi, dri);
        if (t == 0) {
            batch_decide(DECIDE_INIT, ra, rp, &S, &ds, 0);
            double sl = 0.0;
            stp[0] = make_step(ds, S.omega, 0, &sl);
            s_last = sl;
        }
        __syncthreads();
        int sp = 0, md = 0;
        // A thread's rows are the same in every iteration: the sliced position, width
        // (0 for a long row) and length of its first row of each phase are read once
        // here, so the common case (one row per thread and phase) starts every
        // iteration with the matrix loads themselves.
        int a_e = 0, a_w = 0, a_len = 0, p_e = 0, p_w = 0, p_len = 0;
        double a_b = 0.0, p_c = 0.0, p_l = 0.0, p_u = 0.0;
        uint8_t a_rt = 0;
        if (t < m) {
            a_len = arp[t + 1] - arp[t];
            a_e = sa_start[t / SLICE] + t % SLICE;
            a_w = a_len <= LONG_ROW ? sa_width[t / SLICE] : 0;
            a_b = b[t];
            a_rt = rt[t];
        }
        if (t < n) {
            p_len = prp[t + 1] - prp[t];
            p_e = sp_start[t / SLICE] + t % SLICE;
            p_w = p_len <= LONG_ROW ? sp_width[t / SLICE] : 0;
            p_c = c[t];
            p_l = l[t];
            p_u = u[t];
        }
        while (!S.done) {
            const int64_t left = ds.max_iter - S.total;
            const int len = (int)(left < ds.interval ? left : ds.interval);
            const int64_t k0 = S.k;
            for (int j = 0; j < len; ++j) {
                const Step st = stp[sp];
                // the next iteration's step depends only on omega and k: the team's last
                // thread (the one with the fewest rows) computes it while the others work,
                // into the slot nobody reads before the two barriers below
                if (t == NT - 1) {
                    double sl = s_last;
                    stp[sp ^ 1] = make_step(ds, S.omega, k0 + j + 1, &sl);
                    s_last = sl;
                }
                // dual phase: y+ = proj_Y(y - d (A x~ - b)), y-bar averaging
                for (int i = t; i < m; i += NT) {
                    // Every load the row needs is issued before any result is used:
                    // the slice's start and width (the slice is the wavefront's), the
                    // row pointers and the epilogue's operands; for the first row they
                    // were read before the loop.  The row's results are computed
                    // unconditionally and only the stores depend on the row being short
                    // (long rows: team loop).
                    int e = a_e, w = a_w, len = a_len;
                    double bi = a_b;
                    uint8_t ti = a_rt;
                    if (i != t) {
                        const int sl = __builtin_amdgcn_readfirstlane(i / SLICE);
                        len = arp[i + 1] - arp[i];
                        e = sa_start[sl] + i % SLICE;
                        w = len <= LONG_ROW ? sa_width[sl] : 0;
                        bi = b[i];
                        ti = rt[i];
                    }
                    const bool mine = len <= LONG_ROW;
                    const auto gx = [&](int cc) { return xt[cc]; };
                    const double s = ALL && i / SLICE < ca_sl
                                         ? sliced_dot(cca, cva, e - a_base, w, len, gx)
                                         : sliced_dot(a.sa_col, a.sa_val, e, w, len, gx);
                    double yn = y[i] - st.d * (s - bi);
                    if (ti == 1 && yn < 0.0) yn = 0.0;
                    const double ybn = (1.0 - st.w) * ybar[i] + st.w * yn;
                    if (mine) {
                        ybar[i] = ybn;
                        y[i] = yn;
                    }
                }
                for (int q = 0; q < nlra; ++q) {  // long rows: team-wide sum
                    const int i = lra[q];
                    double sv[1] = {0.0};
                    for (int e = arp[i] + t; e < arp[i + 1]; e += NT)
                        sv[0] = sv[0] + a.a_val[e] * xt[a.a_col[e]];
                    team_sum<NT, 1>(sv, red);
                    if (t == 0) {
                        double yn = y[i] - st.d * (sv[0] - b[i]);
                        if (rt[i] == 1 && yn < 0.0) yn = 0.0;
                        ybar[i] = (1.0 - st.w) * ybar[i] + st.w * yn;
                        y[i] = yn;
                    }
                }
                __syncthreads();
                // primal phase over P = [Q | -A'] gathering (x_md, y+)
                const double *xin = md ? xmd1 : xmd0;
                double *xout = md ? xmd0 : xmd1;
                for (int jj = t; jj < n; jj += NT) {
                    // loads first, stores predicated (as in the dual phase)
                    int e = p_e, w = p_w, len = p_len;
                    double cj = p_c, lj = p_l, uj = p_u;
                    if (jj != t) {
                        const int sl = __builtin_amdgcn_readfirstlane(jj / SLICE);
                        len = prp[jj + 1] - prp[jj];
                        e = sp_start[sl] + jj % SLICE;
                        w = len <= LONG_ROW ? sp_width[sl] : 0;
                        cj = c[jj];
                        lj = l[jj];
                        uj = u[jj];
                    }
                    const bool mine = len <= LONG_ROW;
                    const auto gz = [&](int cc) { return *(cc < n ? xin + cc : y + (cc - n)); };
                    const double s = ALL && jj / SLICE < cp_sl
                                         ? sliced_dot(ccp, cvp, e - p_base, w, len, gz)
                                         : sliced_dot(a.sp_col, a.sp_val, e, w, len, gz);
                    const double xo = x[jj];
                    double xn, xb;
                    primal_update(s, st, cj, lj, uj, xo, xbar[jj], xn, xb);
                    if (mine) primal_store(jj, st, xo, xn, xb, x, xbar, xt, xout);
                }
                for (int q = 0; q < nlrp; ++q) {  // long rows: team-wide sum
                    const int jj = lrp[q];
                    double sv[1] = {0.0};
                    for (int e = prp[jj] + t; e < prp[jj + 1]; e += NT) {
                        const int cc = a.p_col[e];
                        const double v = cc < n ? xin[cc] : y[cc - n];
                        sv[0] = sv[0] + a.p_val[e] * v;
                    }
                    team_sum<NT, 1>(sv, red);
                    if (t == 0) primal_row(jj, sv[0], st, c, l, u, x, xbar, xt, xout);
                }
                __syncthreads();
                sp ^= 1;
                md ^= 1;
            }
            team_kkt<NT>(n, m, arp, a.a_col, a.a_val, prp, a.p_col, a.p_val, c, b, l, u, rt, x,
                         xbar, xrs, y, ybar, yrs, ra, rp, red, lra, nlra, lrp, nlrp, dvi, dri);
            if (ds.detect_infeas)
                team_infeas<NT>(n, m, arp, a.a_col, a.a_val, prp, a.p_col, a.p_val, c, b, l, u,
                                rt, x, xrs, y, yrs, dvi, dri, lra, nlra, lrp, nlrp, red, S.inf);
            if (t == 0) {
                batch_decide(DECIDE_CHECK, ra, rp, &S, &ds, len);
                if (!S.done && a.deadline_ticks > 0 &&
                    (int64_t)wall_clock64() - *a.clock0 >= a.deadline_ticks) {
                    S.status = ST_TIME_LIMIT;
                    S.done = 1;
                    S.restart_flag = 0;
                }
                if (S.restart_flag) {
                    double sl = 0.0;
                    stp[sp] = make_step(ds, S.omega, 0, &sl);
                    s_last = sl;
                }
            }
            __syncthreads();
            if (S.restart_flag) {
                const int avg = S.cand;
                for (int j = t; j < n; j += NT) {
                    const double xc = avg ? xbar[j] : x[j];
                    double *xm = md ? xmd1 : xmd0;
                    x[j] = xbar[j] = xt[j] = xm[j] = xrs[j] = xc;
                }
                for (int i = t; i < m; i += NT) {
                    const double yc = avg ? ybar[i] : y[i];
                    y[i] = ybar[i] = yrs[i] = yc;
                }
                __syncthreads();
            }
        }
        // the returned point: the candidate of the last evaluation
        const int avg = S.cand;
        for (int j = t; j < n; j += NT) a.x_out[v0 + j] = avg ? xbar[j] : x[j];
        for (int i = t; i < m; i += NT) a.y_out[r0 + i] = avg ? ybar[i] : y[i];
        if (t == 0) {
            S.t_end = (int64_t)wall_clock64() - *a.clock0;
            a.res[id] = S;
        }
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_batch(BatchDev a, DevSettings base) {
    extern __shared__ double smem[];  // the LDS-resident vectors (LdsMode)
    __shared__ int s_q;
    __shared__ State S;
    __shared__ Step stp[2];
    __shared__ double red[32 * (NT / 64)];
    __shared__ double s_last;
    for (;;) {
        if (threadIdx.x == 0) s_q = atomicAdd(a.head, 1);
        __syncthreads();
        const int q = s_q;
        if (q >= a.order_count) break;
        const int id = a.order[q];
        const int n = a.var_off[id + 1] - a.var_off[id], m = a.row_off[id + 1] - a.row_off[id];
        const int mode = lds_mode_of(n, m, a.lds_doubles);
        if (mode == LDS_ALL)
            solve_instance<NT, LDS_ALL>(a, base, id, smem, S, stp, red, s_last);
        else if (mode == LDS_GATHERED)
            solve_instance<NT, LDS_GATHERED>(a, base, id, smem, S, stp, red, s_last);
        else
            solve_instance<NT, LDS_NONE>(a, base, id, smem, S, stp, red, s_last);
        __syncthreads();
    }
}

// power iteration per instance (same iteration as the single-instance path)
template <int NT>
__global__ __launch_bounds__(NT) void k_batch_norms(BatchDev a, int32_t maxit, double rtol,
                                                    double *outA, double *outQ) {
    __shared__ int s_q;
    __shared__ double red[32 * (NT / 64)];
    __shared__ double s_val[2];
    const int t = threadIdx.x;
    for (;;) {
        if (t == 0) s_q = atomicAdd(a.head, 1);
        __syncthreads();
        const int q = s_q;
        if (q >= a.order_count) break;
        const int id = a.order[q];
        const int v0 = a.var_off[id], n = a.var_off[id + 1] - v0;
        const int r0 = a.row_off[id], m = a.row_off[id + 1] - r0;
        const int32_t *arp = a.a_rowptr + r0;
        const int32_t *prp = a.p_rowptr + v0;
        const int32_t *lra = a.lrA + a.lrA_off[id];
        const int nlra = a.lrA_off[id + 1] - a.lrA_off[id];
        const int32_t *lrp = a.lrP + a.lrP_off[id];
        const int nlrp = a.lrP_off[id + 1] - a.lrP_off[id];
        double *v = a.xbar + v0, *z = a.xt + v0, *w = a.ybar + r0;
        double lam = 0.0;
        // ||A||_2: Rayleigh quotient of A'A
        if (m > 0 && arp[m] > arp[0]) {
            for (int j = t; j < n; j += NT) v[j] = 1.0 / sqrt((double)n);
            __syncthreads();
            double lam_prev = 0.0;
            for (int it = 1; it <= maxit; ++it) {
                double acc[2] = {0.0, 0.0};
                for (int i = t; i < m; i += NT) {
                    if (arp[i + 1] - arp[i] > LONG_ROW) continue;
                    double sacc = 0.0;
                    for (int e = arp[i]; e < arp[i + 1]; ++e) sacc = sacc + a.a_val[e] * v[a.a_col[e]];
                    w[i] = sacc;
                    acc[0] += sacc * sacc;
                }
                for (int qq = 0; qq < nlra; ++qq) {
                    const int i = lra[qq];
                    double sv[1] = {0.0};
                    for (int e = arp[i] + t; e < arp[i + 1]; e += NT)
                        sv[0] = sv[0] + a.a_val[e] * v[a.a_col[e]];
                    team_sum<NT, 1>(sv, red);
                    if (t == 0) {
                        w[i] = sv[0];
                        acc[0] += sv[0] * sv[0];
                    }
                }
                team_reduce<NT, 1>(acc, 0, red);
                if (t == 0) s_val[0] = acc[0];
                __syncthreads();
                lam = s_val[0];
                acc[0] = 0.0;
                for (int j = t; j < n; j += NT) {
                    if (prp[j + 1] - prp[j] > LONG_ROW) continue;
                    double sacc = 0.0;
                    for (int e = prp[j]; e < prp[j + 1]; ++e) {
                        const int cc = a.p_col[e];
                        if (cc >= n) sacc = sacc + (-1.0) * (a.p_val[e] * w[cc - n]);
                    }
                    z[j] = sacc;
                    acc[0] += sacc * sacc;
                }
                for (int qq = 0; qq < nlrp; ++qq) {
                    const int j = lrp[qq];
                    double sv[1] = {0.0};
                    for (int e = prp[j] + t; e < prp[j + 1]; e += NT) {
                        const int cc = a.p_col[e];
                        if (cc >= n) sv[0] = sv[0] + (-1.0) * (a.p_val[e] * w[cc - n]);
                    }
                    team_sum<NT, 1>(sv, red);
                    if (t == 0) {
                        z[j] = sv[0];
                        acc[0] += sv[0] * sv[0];
                    }
                }
                team_reduce<NT, 1>(acc, 0, red);
                if (t == 0) s_val[1] = sqrt(acc[0]);
                __syncthreads();
                const double nz = s_val[1];
                if (nz == 0.0) break;
                for (int j = t; j < n; j += NT) v[j] = z[j] / nz;
                __syncthreads();
                if (it > 1 && fabs(lam - lam_prev) <= rtol * lam) break;
                lam_prev = lam;
            }
        }
        if (t == 0) outA[id] = sqrt(lam);
        // ||Q||_2: Rayleigh quotient of Q
        lam = 0.0;
        for (int j = t; j < n; j += NT) v[j] = 1.0 / sqrt((double)n);
        __syncthreads();
        double lam_prev = 0.0;
        for (int it = 1; it <= maxit; ++it) {
            double acc[2] = {0.0, 0.0};
            for (int j = t; j < n; j += NT) {
                if (prp[j + 1] - prp[j] > LONG_ROW) continue;
                double sacc = 0.0;
                for (int e = prp[j]; e < prp[j + 1]; ++e) {
                    const int cc = a.p_col[e];
                    if (cc < n) sacc = sacc + a.p_val[e] * v[cc];
                }
                z[j] = sacc;
            }
            for (int qq = 0; qq < nlrp; ++qq) {
                const int j = lrp[qq];
                double sv[1] = {0.0};
                for (int e = prp[j] + t; e < prp[j + 1]; e += NT) {
                    const int cc = a.p_col[e];
                    if (cc < n) sv[0] = sv[0] + a.p_val[e] * v[cc];
                }
                team_sum<NT, 1>(sv, red);
                if (t == 0) z[j] = sv[0];
            }
            __syncthreads();
            for (int j = t; j < n; j += NT) {
                acc[0] += v[j] * z[j];
                acc[1] += z[j] * z[j];
            }
            team_reduce<NT, 2>(acc, 0, red);
            if (t == 0) {
                s_val[0] = acc[0];
                s_val[1] = sqrt(acc[1]);
            }
            __syncthreads();
            lam = s_val[0];
            const double nw = s_val[1];
            if (nw == 0.0) break;
            for (int j = t; j < n; j += NT) v[j] = z[j] / nw;
            __syncthreads();
            if (it > 1 && fabs(lam - lam_prev) <= rtol * fabs(lam)) break;
            lam_prev = lam;
        }
        if (t == 0) outQ[id] = fabs(lam);
        __syncthreads();
    }
}

// resets the queue heads of all size classes and the solve's start clock
__global__ void k_queue_reset(int32_t *head, int nhead, int64_t *clock0) {
    if (threadIdx.x < nhead && blockIdx.x == 0) head[threadIdx.x] = 0;
    if (threadIdx.x == 0 && blockIdx.x == 0) *clock0 = (int64_t)wall_clock64();
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct BatchData {
    int32_t B = 0;
    int64_t ntot = 0, mtot = 0;
    hipStream_t stream = nullptr;
    std::vector<int64_t> var_off, row_off;
    std::vector<double> normA, normQ, c_norm2, b_norm2, c_inf, b_inf;
    std::vector<int32_t> cls;                 // size class of each instance
    std::vector<std::vector<int32_t>> order;  // per class, by decreasing work
    // team size per class until qp_batch_autotune / qp_batch_set_threads: what the
    // autotuner chooses on uneven MPC batches (larger teams shorten the slowest solves)
    int32_t threads[NCLASS] = {256, 1024, 1024, 1024};
    DevMem var_off_d, row_off_d, a_rowptr, a_col, a_val, p_rowptr, p_col, p_val;
    DevMem c, b, l, u, rt, normA_d, normQ_d, b_inf_d, c_inf_d, omega0_d, has_x0, has_y0, x0, y0;
    DevMem x, xbar, xt, xmd0, xmd1, xrs, y, ybar, yrs, x_out, y_out, res, order_d, head, clock0;
    DevMem dscale;                   // preconditioning (D2 of all variables, then D1), or empty
    std::vector<double> h_d;         // host copy of dscale (empty: not preconditioned)
    std::vector<double> h_c, h_b;    // the given c and b
    DevMem lrA_off, lrA, lrP_off, lrP;  // long-row lists (rows > LONG_ROW nonzeros)
    DevMem sa_inst, sa_start, sa_width, sa_col, sa_val;  // sliced A (build_sliced)
    DevMem sp_inst, sp_start, sp_width, sp_col, sp_val;  // sliced P
    std::vector<int32_t> order_off;  // offsets of each class in order_d
    int32_t launch_order[NCLASS] = {NCLASS - 1, NCLASS - 2, NCLASS - 3, NCLASS - 4};
    std::vector<double> h_omega;     // staging of per-solve scalars (outlive async copies)
    std::vector<uint8_t> h_hx, h_hy;
    int wall_khz = 100000;
    int num_cu = 256;
    int use_lds = 1;
    int32_t lds_need[NCLASS] = {0, 0, 0, 0};  // doubles of dynamic LDS per class
    int32_t lds_cap = 0;  // bytes of dynamic LDS a team may have (the matrix cache's limit)
    // one stream per size class (default priority), forked from and joined to `stream`
    hipStream_t cls_stream[NCLASS] = {};
    hipEvent_t ev_fork = nullptr, ev_join[NCLASS] = {};
    ~BatchData() {
        for (int k = 0; k < NCLASS; ++k) {
            if (cls_stream[k]) (void)hipStreamDestroy(cls_stream[k]);
            if (ev_join[k]) (void)hipEventDestroy(ev_join[k]);
        }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
    }
};

static int class_of(int64_t rows) {
    for (int k = 0; k < NCLASS; ++k)
        if (rows <= CLASS_LIMIT[k]) return k;
    return NCLASS - 1;
}

static BatchDev make_dev(BatchData *bd) {
    BatchDev a;
    std::memset(&a, 0, sizeof(a));
    a.count = bd->B;
    a.var_off = bd->var_off_d.as<int32_t>();
    a.row_off = bd->row_off_d.as<int32_t>();
    a.a_rowptr = bd->a_rowptr.as<int32_t>();
    a.a_col = bd->a_col.as<int32_t>();
    a.a_val = bd->a_val.as<double>();
    a.p_rowptr = bd->p_rowptr.as<int32_t>();
    a.p_col = bd->p_col.as<int32_t>();
    a.p_val = bd->p_val.as<double>();
    a.c = bd->c.as<double>();
    a.b = bd->b.as<double>();
    a.l = bd->l.as<double>();
    a.u = bd->u.as<double>();
    a.rt = bd->rt.as<uint8_t>();
    a.normA = bd->normA_d.as<double>();
    a.normQ = bd->normQ_d.as<double>();
    a.b_inf = bd->b_inf_d.as<double>();
    a.c_inf = bd->c_inf_d.as<double>();
    a.omega0 = bd->omega0_d.as<double>();
    a.has_x0 = bd->has_x0.as<uint8_t>();
    a.has_y0 = bd->has_y0.as<uint8_t>();
    a.x0 = bd->x0.as<double>();
    a.y0 = bd->y0.as<double>();
    a.x = bd->x.as<double>();
    a.xbar = bd->xbar.as<double>();
    a.xt = bd->xt.as<double>();
    a.xmd0 = bd->xmd0.as<double>();
    a.xmd1 = bd->xmd1.as<double>();
    a.xrs = bd->xrs.as<double>();
    a.y = bd->y.as<double>();
    a.ybar = bd->ybar.as<double>();
    a.yrs = bd->yrs.as<double>();
    a.x_out = bd->x_out.as<double>();
    a.y_out = bd->y_out.as<double>();
    a.res = bd->res.as<State>();
    a.head = bd->head.as<int32_t>();
    a.clock0 = bd->clock0.as<int64_t>();
    a.lrA_off = bd->lrA_off.as<int32_t>();
    a.lrA = bd->lrA.as<int32_t>();
    a.lrP_off = bd->lrP_off.as<int32_t>();
    a.lrP = bd->lrP.as<int32_t>();
    a.dscale = bd->h_d.empty() ? nullptr : bd->dscale.as<double>();
    a.ntot = bd->ntot;
    a.sa_inst = bd->sa_inst.as<int32_t>();
    a.sa_start = bd->sa_start.as<int32_t>();
    a.sa_width = bd->sa_width.as<int32_t>();
    a.sa_col = bd->sa_col.as<int32_t>();
    a.sa_val = bd->sa_val.as<double>();
    a.sp_inst = bd->sp_inst.as<int32_t>();
    a.sp_start = bd->sp_start.as<int32_t>();
    a.sp_width = bd->sp_width.as<int32_t>();
    a.sp_col = bd->sp_col.as<int32_t>();
    a.sp_val = bd->sp_val.as<double>();
    return a;
}

// Sliced copy of a batch CSR matrix (rows of all instances concatenated, off[B+1]
// instance offsets) for the row loops of k_batch: each instance's rows are cut into
// slices of SLICE rows, one row per lane of a wavefront; entry k of the row in lane l
// of a slice sits at start[slice] + SLICE * k + l, so the lanes of a load read
// consecutive addresses.  A slice's width is its longest row, rows longer than
// LONG_ROW left out (the whole team sums those from the CSR arrays).  Padding holds
// column 0 and is never added.  src[e] is the CSR entry
// copied to sliced position e (-1 for padding), so values can be gathered on the
// device after preprocessing has scaled the CSR values.
struct HostSliced {
    std::vector<int32_t> inst, start, width, col;
    std::vector<int64_t> src;
};

static int build_sliced(const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                        const std::vector<int64_t> &off, int B, HostSliced &h) {
    h.inst.assign(B + 1, 0);
    int64_t pos = 0;
    for (int i = 0; i < B; ++i) {
        h.inst[i] = (int32_t)h.start.size();
        for (int64_t r0 = off[i]; r0 < off[i + 1]; r0 += SLICE) {
            const int64_t r1 = std::min<int64_t>(r0 + SLICE, off[i + 1]);
            int64_t w = 0;
            for (int64_t r = r0; r < r1; ++r) {
                const int64_t len = rp[r + 1] - rp[r];
                if (len <= LONG_ROW) w = std::max(w, len);
            }
            if (pos + w * SLICE > INT32_MAX)
                return fail(QP_ERR_INVALID_ARGUMENT, "batch too large for the sliced layout");
            h.start.push_back((int32_t)pos);
            h.width.push_back((int32_t)w);
            pos += w * SLICE;
        }
    }
    h.inst[B] = (int32_t)h.start.size();
    h.col.assign((size_t)pos, 0);
    h.src.assign((size_t)pos, -1);
    for (int i = 0; i < B; ++i) {
        int32_t sl = h.inst[i];
        for (int64_t r0 = off[i]; r0 < off[i + 1]; r0 += SLICE, ++sl) {
            const int64_t r1 = std::min<int64_t>(r0 + SLICE, off[i + 1]);
            for (int64_t r = r0; r < r1; ++r) {
                const int64_t len = rp[r + 1] - rp[r];
                if (len > LONG_ROW) continue;
                for (int64_t k = 0; k < len; ++k) {
                    const int64_t e = h.start[sl] + SLICE * k + (r - r0);
                    h.col[(size_t)e] = col[(size_t)(rp[r] + k)];
                    h.src[(size_t)e] = rp[r] + k;
                }
            }
        }
    }
    return QP_OK;
}

__global__ void k_sliced_gather(double *__restrict__ out, const double *__restrict__ val,
                                const int64_t *__restrict__ src, int64_t len) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) out[e] = src[e] >= 0 ? val[src[e]] : 0.0;
}

// uploads the layout and gathers its values from the (possibly scaled) CSR values
static int upload_sliced(const HostSliced &h, const double *csr_val, hipStream_t s,
                         DevMem &inst, DevMem &start, DevMem &width, DevMem &col, DevMem &val) {
    int rc;
    DevMem src;
    const int64_t len = (int64_t)h.col.size();
    if ((rc = inst.upload(h.inst.data(), h.inst.size() * 4)) ||
        (rc = start.upload(h.start.data(), h.start.size() * 4)) ||
        (rc = width.upload(h.width.data(), h.width.size() * 4)) ||
        (rc = col.upload(h.col.data(), h.col.size() * 4)) ||
        (rc = src.upload(h.src.data(), h.src.size() * 8)) || (rc = val.alloc((size_t)len * 8 + 16)))
        return rc;
    (void)hipGetLastError();  // launch errors are read below: drop any earlier one
    if (len > 0)
        hipLaunchKernelGGL(k_sliced_gather, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s,
                           val.as<double>(), csr_val, src.as<int64_t>(), len);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return QP_OK;
}

template <class K>
static int persistent_grid(K kernel, int nt, int count, int num_cu, size_t lds = 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int g = per_cu * num_cu;
    return g < count ? g : count;
}

// Dynamic LDS of a class whose vectors fit: the cap when the occupancy query gives as
// many resident teams per CU with it as with the vectors alone (the rest then caches
// matrix slices), else the vectors' share.
template <int NT>
static size_t cache_lds(size_t need, size_t cap, int32_t *lds_doubles) {
    int occ_need = 0, occ_cap = 0;
    if (hipFuncSetAttribute((const void *)k_batch<NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)cap) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_need, k_batch<NT>, NT, need) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_cap, k_batch<NT>, NT, cap) !=
            hipSuccess ||
        occ_cap < 1 || occ_cap < occ_need) {
        (void)hipGetLastError();
        return need;
    }
    *lds_doubles = (int32_t)(cap / 8);
    return cap;
}

// launches one persistent kernel over the instances order[lo, hi) of size class k on
// stream s, with queue head k (reset beforehand by run_classes)
static void launch_class(BatchData *bd, BatchDev a, const DevSettings &ds, int nt, int lo, int hi,
                         int k, hipStream_t s, bool norms, int32_t maxit, double rtol) {
    a.order = bd->order_d.as<int32_t>() + lo;
    a.order_count = hi - lo;
    if (a.order_count <= 0) return;
    a.head = bd->head.as<int32_t>() + k;
#define QPB_LAUNCH(NT)                                                                           \
    do {                                                                                         \
        if (norms) {                                                                             \
            int g = persistent_grid(k_batch_norms<NT>, NT, a.order_count, bd->num_cu);           \
            hipLaunchKernelGGL(k_batch_norms<NT>, dim3(g), dim3(NT), 0, s, a, maxit, rtol,       \
                               bd->normA_d.as<double>(), bd->normQ_d.as<double>());              \
        } else {                                                                                 \
            size_t lds = (size_t)a.lds_doubles * 8;                                              \
            if (lds > 0 && (size_t)bd->lds_cap > lds)                                            \
                lds = cache_lds<NT>(lds, (size_t)bd->lds_cap, &a.lds_doubles);                   \
            if (lds > 64 * 1024 &&                                                               \
                hipFuncSetAttribute((const void *)k_batch<NT>,                                   \
                                    hipFuncAttributeMaxDynamicSharedMemorySize,                  \
                                    (int)lds) != hipSuccess) {                                   \
                a.lds_doubles = 0; /* larger LDS refused: gathered vectors stay in HBM */        \
            }                                                                                    \
            const size_t lds_use = (size_t)a.lds_doubles * 8;                                    \
            int g = persistent_grid(k_batch<NT>, NT, a.order_count, bd->num_cu, lds_use);        \
            hipLaunchKernelGGL(k_batch<NT>, dim3(g), dim3(NT), lds_use, s, a, ds);               \
        }                                                                                        \
    } while (0)
    switch (nt) {
    case 64: QPB_LAUNCH(64); break;
    case 128: QPB_LAUNCH(128); break;
    case 256: QPB_LAUNCH(256); break;
    case 512: QPB_LAUNCH(512); break;
    default: QPB_LAUNCH(1024); break;
    }
#undef QPB_LAUNCH
}

// Gives each size class's hardware queue its private-memory (scratch) backing at create.
// The solve kernel's out-of-line calls and spilled registers use private memory, and the
// first dispatch of such a kernel on a queue has the runtime allocate it, which otherwise
// falls into the first solve and delays the start of that class.  Every class stream runs
// k_batch<1024> (the largest private segment per lane) at its full persistent grid over
// an empty queue: each workgroup takes no instance and exits.  The queue heads it counts
// up are reset before every solve.
static int warm_class_queues(BatchData *bd) {
    BatchDev a = make_dev(bd);
    a.order = bd->order_d.as<int32_t>();
    a.order_count = 0;
    a.lds_doubles = 0;
    DevSettings ds;
    std::memset(&ds, 0, sizeof(ds));
    const int g = persistent_grid(k_batch<1024>, 1024, 1 << 30, bd->num_cu);
    for (int k = 0; k < NCLASS; ++k) {
        if (bd->order_off[k + 1] == bd->order_off[k]) continue;
        a.head = bd->head.as<int32_t>() + k;
        hipLaunchKernelGGL(k_batch<1024>, dim3(g), dim3(1024), 0, bd->cls_stream[k], a, ds);
    }
    HIPCHK(hipGetLastError());
    for (int k = 0; k < NCLASS; ++k) HIPCHK(hipStreamSynchronize(bd->cls_stream[k]));
    return QP_OK;
}

// Runs launch(k, stream) for every size class, each on its own stream so that the
// classes overlap: when the workgroups of one persistent launch run out of
// instances they exit and the next class's workgroups take their place, instead of
// the GPU idling behind one class's slowest instance.  The class with the most
// estimated work starts first.  The caller's stream waits for all of them.
template <class F>
static int run_classes(BatchData *bd, F launch) {
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, bd->stream, bd->head.as<int32_t>(),
                       NCLASS, bd->clock0.as<int64_t>());
    HIPCHK(hipEventRecord(bd->ev_fork, bd->stream));
    // Wait for the reset (and the uploads before it) here: while it is pending, every class
    // kernel gets enqueued behind the fork, all become ready at once and their workgroups
    // interleave, so the first class no longer takes the free CUs first.
    HIPCHK(hipStreamSynchronize(bd->stream));
    for (int q = 0; q < NCLASS; ++q) {
        const int k = bd->launch_order[q];
        HIPCHK(hipStreamWaitEvent(bd->cls_stream[k], bd->ev_fork, 0));
        launch(k, bd->cls_stream[k]);
        HIPCHK(hipEventRecord(bd->ev_join[k], bd->cls_stream[k]));
    }
    // The handle's stream waits for the classes only after every class is launched: with
    // more streams than hardware queues a class stream may share a queue with it, and a
    // wait queued there earlier would hold that class back until the previous one ends.
    for (int k = NCLASS - 1; k >= 0; --k) HIPCHK(hipStreamWaitEvent(bd->stream, bd->ev_join[k], 0));
    return QP_OK;
}

static DevSettings batch_settings(const qp_settings *s) {
    DevSettings ds;
    std::memset(&ds, 0, sizeof(ds));
    ds.eps = s->eps;
    ds.beta_sufficient = s->beta_sufficient;
    ds.beta_necessary = s->beta_necessary;
    ds.beta_artificial = s->beta_artificial;
    ds.pw_smoothing = s->pw_smoothing;
    ds.eps_zero = s->eps_zero;
    ds.step_safety = s->step_safety;
    ds.max_iter = s->max_iter;
    ds.restart_mode = s->restart_mode;
    ds.fixed_K = s->fixed_K;
    ds.interval = s->restart_mode == QP_RESTART_FIXED_K ? s->fixed_K : s->check_every;
    ds.momentum = s->momentum;
    ds.detect_infeas = s->detect_infeasibility;
    ds.eps_infeas = s->eps_infeasible;
    return ds;
}

template <class T>
static int fetch_vec(std::vector<T> &dst, const T *src, int64_t count, int ms) {
    if (count == 0) {
        dst.clear();
        return QP_OK;
    }
    if (!src) return fail(QP_ERR_INVALID_ARGUMENT, "missing batch array");
    if (ms == QP_MEM_HOST) {
        dst.assign(src, src + count);  // one pass, no zero fill before the copy
    } else {
        dst.resize((size_t)count);
        HIPCHK(hipMemcpy(dst.data(), src, (size_t)count * sizeof(T), hipMemcpyDeviceToHost));
    }
    return QP_OK;
}

// Uploads the c and b the iteration runs on (with preconditioning D2 c and D1 b) and
// the per-instance statistics: infinity norms of the given vectors (relKKT), 2-norms of
// the iterated ones (initial primal weight).
static int upload_vectors(BatchData *bd, const std::vector<double> &c, const std::vector<double> &b) {
    const int64_t n = bd->ntot, m = bd->mtot;
    std::vector<double> cs(c), bs(b);
    if (!bd->h_d.empty()) {
        for (int64_t j = 0; j < n; ++j) cs[j] = c[j] * bd->h_d[j];
        for (int64_t r = 0; r < m; ++r) bs[r] = b[r] * bd->h_d[n + r];
    }
    auto put = [&](DevMem &dm, const std::vector<double> &v) -> int {
        if (!dm.p) return dm.upload(v.data(), v.size() * 8);
        if (!v.empty()) HIPCHK(hipMemcpy(dm.p, v.data(), v.size() * 8, hipMemcpyHostToDevice));
        return QP_OK;
    };
    int rc;
    if ((rc = put(bd->c, cs)) || (rc = put(bd->b, bs))) return rc;
    for (int i = 0; i < bd->B; ++i) {
        double cn = 0.0, ci = 0.0, bn = 0.0, bi = 0.0;
        for (int64_t j = bd->var_off[i]; j < bd->var_off[i + 1]; ++j) {
            cn += cs[j] * cs[j];
            if (std::fabs(c[j]) > ci) ci = std::fabs(c[j]);
        }
        for (int64_t r = bd->row_off[i]; r < bd->row_off[i + 1]; ++r) {
            bn += bs[r] * bs[r];
            if (std::fabs(b[r]) > bi) bi = std::fabs(b[r]);
        }
        bd->c_norm2[i] = std::sqrt(cn);
        bd->b_norm2[i] = std::sqrt(bn);
        bd->c_inf[i] = ci;
        bd->b_inf[i] = bi;
    }
    return QP_OK;
}

// Host checks of a batch descriptor's arrays (no device work): offsets, row pointers,
// row types, bounds, per-instance column ranges, int32 limits, and Q's symmetry when
// settings.check_symmetry is set.
int validate_batch_arrays(const qp_problem_desc *d, const qp_settings *s, const BatchArrays &a) {
    const int32_t B = d->num_instances;
    const int64_t n = d->n, m = d->m;
    const int64_t *vo = d->var_off, *ro = d->row_off;
    if (!vo || !ro) return fail(QP_ERR_INVALID_ARGUMENT, "batch problems need var_off and row_off");
    if (vo[0] != 0 || ro[0] != 0 || vo[B] != n || ro[B] != m)
        return fail(QP_ERR_BATCH_MISMATCH, "var_off/row_off do not span [0,n) and [0,m)");
    for (int i = 0; i < B; ++i)
        if (vo[i + 1] <= vo[i] || ro[i + 1] < ro[i])
            return fail(QP_ERR_BATCH_MISMATCH, "every instance needs n_i > 0 and m_i >= 0");
    if (n + m >= ((int64_t)1 << 31)) return fail(QP_ERR_INVALID_ARGUMENT, "batch exceeds int32");
    const int64_t pnnz = d->Q.nnz + (m > 0 ? d->A.nnz : 0);
    if (pnnz >= ((int64_t)1 << 31)) return fail(QP_ERR_INVALID_ARGUMENT, "batch exceeds int32");
    if (a.qr[0] != 0 || a.qr[n] != d->Q.nnz || (m > 0 && (a.ar[0] != 0 || a.ar[m] != d->A.nnz)))
        return fail(QP_ERR_INVALID_ARGUMENT, "row pointers do not match nnz");
    for (int64_t j = 0; j < n; ++j)
        if (a.qr[j + 1] < a.qr[j]) return fail(QP_ERR_INVALID_ARGUMENT, "Q.row_ptr decreases");
    for (int64_t i = 0; i < m; ++i) {
        if (a.ar[i + 1] < a.ar[i]) return fail(QP_ERR_INVALID_ARGUMENT, "A.row_ptr decreases");
        if (a.rt[i] > 1) return fail(QP_ERR_INVALID_ARGUMENT, "row_type must be 0 or 1");
    }
    for (int64_t j = 0; j < n; ++j)
        if (!(a.l[j] <= a.u[j]) || a.l[j] == INFINITY || a.u[j] == -INFINITY)
            return fail(QP_ERR_INVALID_ARGUMENT, "invalid bounds at variable %lld", (long long)j);
    for (int i = 0; i < B; ++i) {
        const int64_t nv = vo[i + 1] - vo[i];
        for (int64_t r = ro[i]; r < ro[i + 1]; ++r)
            for (int64_t e = a.ar[r]; e < a.ar[r + 1]; ++e)
                if (a.ac[e] < 0 || a.ac[e] >= nv)
                    return fail(QP_ERR_INVALID_ARGUMENT, "A column index outside its instance");
        for (int64_t j = vo[i]; j < vo[i + 1]; ++j)
            for (int64_t e = a.qr[j]; e < a.qr[j + 1]; ++e)
                if (a.qc[e] < 0 || a.qc[e] >= nv)
                    return fail(QP_ERR_INVALID_ARGUMENT, "Q column index outside its instance");
    }
    if (s->check_symmetry)
        for (int i = 0; i < B; ++i) {
            int rc = qph::check_symmetric(vo[i + 1] - vo[i], a.qr + vo[i], a.qc, a.qv, i);
            if (rc) return rc;
        }
    return QP_OK;
}

int validate_batch_host(const qp_problem_desc *d, const qp_settings *s) {
    const int64_t m = d->m;
    static const int32_t zero = 0;
    std::vector<uint8_t> rt;
    std::vector<double> l, u;
    if (!d->row_type) rt.assign((size_t)m, 0);
    if (!d->l) l.assign((size_t)d->n, -INFINITY);
    if (!d->u) u.assign((size_t)d->n, INFINITY);
    if (m > 0 && (!d->A.row_ptr || !d->b || (d->A.nnz > 0 && (!d->A.col_idx || !d->A.val))))
        return fail(QP_ERR_INVALID_ARGUMENT, "A arrays and b are required when m > 0");
    if (!d->c) return fail(QP_ERR_INVALID_ARGUMENT, "c is required");
    BatchArrays arr{d->Q.row_ptr, d->Q.col_idx, d->Q.val, m > 0 ? d->A.row_ptr : &zero,
                    d->A.col_idx, d->row_type ? d->row_type : rt.data(),
                    d->l ? d->l : l.data(), d->u ? d->u : u.data()};
    return validate_batch_arrays(d, s, arr);
}

int create_batch(const qp_problem_desc *d, const qp_settings *s, hipStream_t stream,
                 BatchData **out) {
    *out = nullptr;
    if (!d->var_off || !d->row_off)
        return fail(QP_ERR_INVALID_ARGUMENT, "batch problems need var_off and row_off");
    const int32_t B = d->num_instances;
    const int ms = d->mem_space;
    BatchData *bd = new BatchData();
    bd->B = B;
    bd->stream = stream;
    // The size classes run concurrently on streams of their own.  Ordinary streams share
    // the process's few hardware queues (4 by default), and two classes whose streams
    // land on one queue run one after the other (measured: 4096 MPC QPs in 0.73 s against
    // 0.50 s with a queue each).  A stream with a CU mask gets a hardware queue of its
    // own; the mask enables every CU, so nothing else changes.
    int ncu = 0, cdev = 0;
    (void)hipGetDevice(&cdev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, cdev) != hipSuccess ||
        ncu < 1)
        ncu = 256;
    std::vector<uint32_t> cu_mask((size_t)(ncu + 31) / 32, 0u);
    for (int c = 0; c < ncu; ++c) cu_mask[(size_t)c / 32] |= 1u << (c % 32);
    for (int k = 0; k < NCLASS; ++k) {
        if (hipExtStreamCreateWithCUMask(&bd->cls_stream[k], (uint32_t)cu_mask.size(),
                                         cu_mask.data()) != hipSuccess) {
            (void)hipGetLastError();
            bd->cls_stream[k] = nullptr;
            if (hipStreamCreateWithFlags(&bd->cls_stream[k], hipStreamNonBlocking) != hipSuccess) {
                delete bd;
                return fail(QP_ERR_DEVICE, "batch: stream creation failed");
            }
        }
        if (hipEventCreateWithFlags(&bd->ev_join[k], hipEventDisableTiming) != hipSuccess) {
            delete bd;
            return fail(QP_ERR_DEVICE, "batch: stream or event creation failed");
        }
    }
    if (hipEventCreateWithFlags(&bd->ev_fork, hipEventDisableTiming) != hipSuccess) {
        delete bd;
        return fail(QP_ERR_DEVICE, "batch: event creation failed");
    }
    bd->var_off.assign(d->var_off, d->var_off + B + 1);
    bd->row_off.assign(d->row_off, d->row_off + B + 1);
    const int64_t n = d->n, m = d->m;
    bd->ntot = n;
    bd->mtot = m;
    std::vector<int32_t> qr, qc, ar, ac;
    std::vector<double> qv, av, c, b, l, u;
    std::vector<uint8_t> rt;
    int rc;
    if ((rc = fetch_vec(qr, d->Q.row_ptr, n + 1, ms)) || (rc = fetch_vec(qc, d->Q.col_idx, d->Q.nnz, ms)) ||
        (rc = fetch_vec(qv, d->Q.val, d->Q.nnz, ms)) || (rc = fetch_vec(c, d->c, n, ms))) {
        delete bd;
        return rc;
    }
    if (m > 0) {
        if ((rc = fetch_vec(ar, d->A.row_ptr, m + 1, ms)) ||
            (rc = fetch_vec(ac, d->A.col_idx, d->A.nnz, ms)) ||
            (rc = fetch_vec(av, d->A.val, d->A.nnz, ms)) || (rc = fetch_vec(b, d->b, m, ms))) {
            delete bd;
            return rc;
        }
        if (d->row_type) {
            if ((rc = fetch_vec(rt, d->row_type, m, ms))) {
                delete bd;
                return rc;
            }
        } else {
            rt.assign(m, 0);
        }
    } else {
        ar.assign(1, 0);
    }
    if (d->l) {
        if ((rc = fetch_vec(l, d->l, n, ms))) { delete bd; return rc; }
    } else {
        l.assign(n, -INFINITY);
    }
    if (d->u) {
        if ((rc = fetch_vec(u, d->u, n, ms))) { delete bd; return rc; }
    } else {
        u.assign(n, INFINITY);
    }
    {
        BatchArrays arr{qr.data(), qc.data(), qv.data(), ar.data(), ac.data(), rt.data(),
                        l.data(), u.data()};
        if ((rc = validate_batch_arrays(d, s, arr))) {
            delete bd;
            return rc;
        }
    }
    const int64_t pnnz = d->Q.nnz + (m > 0 ? d->A.nnz : 0);
    std::vector<int32_t> pr(n + 1, 0), pc((size_t)pnnz);
    std::vector<double> pv((size_t)pnnz);
    {
        // (indices were validated above)
        std::vector<int64_t> acount(n, 0);
        for (int i = 0; i < B; ++i)
            for (int64_t r = bd->row_off[i]; r < bd->row_off[i + 1]; ++r)
                for (int64_t e = ar[r]; e < ar[r + 1]; ++e) acount[bd->var_off[i] + ac[e]]++;
        for (int64_t j = 0; j < n; ++j) pr[j + 1] = (int32_t)(pr[j] + (qr[j + 1] - qr[j]) + acount[j]);
        std::vector<int64_t> next(n);
        for (int64_t j = 0; j < n; ++j) {
            int64_t pos = pr[j];
            for (int64_t e = qr[j]; e < qr[j + 1]; ++e, ++pos) {
                pc[pos] = qc[e];
                pv[pos] = qv[e];
            }
            next[j] = pos;
        }
        for (int i = 0; i < B; ++i) {
            const int64_t v0 = bd->var_off[i], r0 = bd->row_off[i];
            const int64_t nv = bd->var_off[i + 1] - v0;
            for (int64_t r = r0; r < bd->row_off[i + 1]; ++r)
                for (int64_t e = ar[r]; e < ar[r + 1]; ++e) {
                    const int64_t pos = next[v0 + ac[e]]++;
                    pc[pos] = (int32_t)(nv + (r - r0));
                    pv[pos] = -av[e];
                }
        }
    }
    // rows longer than LONG_ROW nonzeros, per instance (local row ids)
    std::vector<int32_t> lao(B + 1, 0), la, lpo(B + 1, 0), lp;
    for (int i = 0; i < B; ++i) {
        for (int64_t r = bd->row_off[i]; r < bd->row_off[i + 1]; ++r)
            if (ar[r + 1] - ar[r] > LONG_ROW) la.push_back((int32_t)(r - bd->row_off[i]));
        for (int64_t j = bd->var_off[i]; j < bd->var_off[i + 1]; ++j)
            if (pr[j + 1] - pr[j] > LONG_ROW) lp.push_back((int32_t)(j - bd->var_off[i]));
        lao[i + 1] = (int32_t)la.size();
        lpo[i + 1] = (int32_t)lp.size();
    }
    if ((rc = bd->lrA_off.upload(lao.data(), lao.size() * 4)) ||
        (rc = bd->lrA.upload(la.data(), la.size() * 4)) ||
        (rc = bd->lrP_off.upload(lpo.data(), lpo.size() * 4)) ||
        (rc = bd->lrP.upload(lp.data(), lp.size() * 4))) {
        delete bd;
        return rc;
    }
    std::vector<int32_t> vo(B + 1), ro(B + 1);
    for (int i = 0; i <= B; ++i) {
        vo[i] = (int32_t)bd->var_off[i];
        ro[i] = (int32_t)bd->row_off[i];
    }
    const size_t nb = (size_t)n * 8, mb = (size_t)std::max<int64_t>(m, 1) * 8;
    if ((rc = bd->var_off_d.upload(vo.data(), vo.size() * 4)) ||
        (rc = bd->row_off_d.upload(ro.data(), ro.size() * 4)) ||
        (rc = bd->a_rowptr.upload(ar.data(), ar.size() * 4)) ||
        (rc = bd->a_col.upload(ac.data(), ac.size() * 4)) ||
        (rc = bd->a_val.upload(av.data(), av.size() * 8)) ||
        (rc = bd->p_rowptr.upload(pr.data(), pr.size() * 4)) ||
        (rc = bd->p_col.upload(pc.data(), pc.size() * 4)) ||
        (rc = bd->p_val.upload(pv.data(), pv.size() * 8)) ||
        (rc = bd->rt.upload(rt.data(), rt.size()))) {
        delete bd;
        return rc;
    }
    bd->c_norm2.assign(B, 0.0);
    bd->b_norm2.assign(B, 0.0);
    bd->c_inf.assign(B, 0.0);
    bd->b_inf.assign(B, 0.0);
    // Sec. 5 preprocessing, per instance (each instance's own K), on the device
    std::vector<double> ls(l), us(u);
    if (s->precondition) {
        DevMem work;
        if ((rc = work.alloc((size_t)(n + m) * 16)) ||
            (rc = bd->dscale.alloc((size_t)(n + m) * 8))) {
            delete bd;
            return rc;
        }
        ScaleInput in{};
        in.n = n;
        in.m = m;
        in.a_rowptr = bd->a_rowptr.as<int32_t>();
        in.a_col = bd->a_col.as<int32_t>();
        in.a_val = bd->a_val.as<double>();
        in.p_rowptr = bd->p_rowptr.as<int32_t>();
        in.p_col = bd->p_col.as<int32_t>();
        in.p_val = bd->p_val.as<double>();
        in.var_off = bd->var_off_d.as<int32_t>();
        in.row_off = bd->row_off_d.as<int32_t>();
        in.count = B;
        in.ruiz_iters = s->ruiz_iters;
        in.l2 = 1;
        in.pc = 1;
        if (precondition_device(stream, in, work.as<double>(), bd->dscale.as<double>())) {
            delete bd;
            return fail(QP_ERR_DEVICE, "preconditioning kernels failed to launch");
        }
        bd->h_d.resize((size_t)(n + m));
        if (hipStreamSynchronize(stream) != hipSuccess ||
            hipMemcpy(bd->h_d.data(), bd->dscale.p, (size_t)(n + m) * 8, hipMemcpyDeviceToHost) !=
                hipSuccess) {
            delete bd;
            return fail(QP_ERR_DEVICE, "preconditioning failed");
        }
        for (int64_t j = 0; j < n; ++j) {
            ls[j] = l[j] / bd->h_d[j];
            us[j] = u[j] / bd->h_d[j];
        }
    }
    {
        HostSliced sa, sp;
        std::vector<int64_t> voff(bd->var_off.begin(), bd->var_off.end());
        std::vector<int64_t> roff(bd->row_off.begin(), bd->row_off.end());
        if ((rc = build_sliced(ar, ac, roff, B, sa)) || (rc = build_sliced(pr, pc, voff, B, sp)) ||
            (rc = upload_sliced(sa, bd->a_val.as<double>(), stream, bd->sa_inst, bd->sa_start,
                                bd->sa_width, bd->sa_col, bd->sa_val)) ||
            (rc = upload_sliced(sp, bd->p_val.as<double>(), stream, bd->sp_inst, bd->sp_start,
                                bd->sp_width, bd->sp_col, bd->sp_val))) {
            delete bd;
            return rc;
        }
    }
    bd->h_c = c;
    bd->h_b = b;
    if ((rc = upload_vectors(bd, c, b)) || (rc = bd->l.upload(ls.data(), nb)) ||
        (rc = bd->u.upload(us.data(), nb)) || (rc = bd->x.alloc(nb)) || (rc = bd->xbar.alloc(nb)) || (rc = bd->xt.alloc(nb)) ||
        (rc = bd->xmd0.alloc(nb)) || (rc = bd->xmd1.alloc(nb)) || (rc = bd->xrs.alloc(nb)) ||
        (rc = bd->y.alloc(mb)) || (rc = bd->ybar.alloc(mb)) || (rc = bd->yrs.alloc(mb)) ||
        (rc = bd->x_out.alloc(nb)) || (rc = bd->y_out.alloc(mb)) || (rc = bd->x0.alloc(nb)) ||
        (rc = bd->y0.alloc(mb)) || (rc = bd->res.alloc((size_t)B * sizeof(State))) ||
        (rc = bd->head.alloc(NCLASS * 8)) || (rc = bd->clock0.alloc(8)) ||
        (rc = bd->normA_d.alloc((size_t)B * 8)) || (rc = bd->normQ_d.alloc((size_t)B * 8)) ||
        (rc = bd->b_inf_d.alloc((size_t)B * 8)) || (rc = bd->c_inf_d.alloc((size_t)B * 8)) ||
        (rc = bd->omega0_d.alloc((size_t)B * 8)) || (rc = bd->has_x0.alloc((size_t)B)) ||
        (rc = bd->has_y0.alloc((size_t)B))) {
        delete bd;
        return rc;
    }
    bd->normA.assign(B, 0.0);
    bd->normQ.assign(B, 0.0);
    // Size classes and queue order: decreasing estimated work, so that likely stragglers
    // start first.  The estimate is the instance's nonzeros times (1 + m_i / n_i)^8: the
    // rows per variable rank the iteration counts far better than the size does
    // (Spearman 0.82 against 0.50 for the nonzeros on the 4096-instance MPC batch, whose
    // slowest instances are underactuated horizons), and the order alone changes no result.
    bd->cls.resize(B);
    bd->order.assign(NCLASS, {});
    std::vector<double> work(B);
    for (int i = 0; i < B; ++i) {
        const int64_t nv = bd->var_off[i + 1] - bd->var_off[i];
        const int64_t mv = bd->row_off[i + 1] - bd->row_off[i];
        bd->cls[i] = class_of(nv + mv);
        const double f = 1.0 + (double)mv / (double)std::max<int64_t>(nv, 1);
        work[i] = (double)((pr[bd->var_off[i + 1]] - pr[bd->var_off[i]]) +
                           (ar[bd->row_off[i + 1]] - ar[bd->row_off[i]]) + nv + mv) *
                  (f * f) * (f * f) * (f * f) * (f * f);
        bd->order[bd->cls[i]].push_back(i);
    }
    // classes launch in decreasing order of their summed estimated work: the first
    // launched kernel takes the free CUs first, and the class with most of the work is
    // the one whose leading instances must not wait
    {
        double cw[NCLASS] = {0, 0, 0, 0};
        for (int i = 0; i < B; ++i) cw[bd->cls[i]] += work[i];
        std::stable_sort(bd->launch_order, bd->launch_order + NCLASS,
                         [&](int32_t p, int32_t q) { return cw[p] > cw[q]; });
    }
    std::vector<int32_t> flat;
    bd->order_off.assign(NCLASS + 1, 0);
    for (int k = 0; k < NCLASS; ++k) {
        auto &o = bd->order[k];
        std::stable_sort(o.begin(), o.end(), [&](int32_t p, int32_t q) { return work[p] > work[q]; });
        flat.insert(flat.end(), o.begin(), o.end());
        bd->order_off[k + 1] = (int32_t)flat.size();
    }
    if ((rc = bd->order_d.upload(flat.data(), flat.size() * 4))) {
        delete bd;
        return rc;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        // dynamic LDS per class: the most any instance can use (LdsMode) within the cap
        int max_lds = 65536;
        (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        const int cap = std::min(max_lds, 160 * 1024) - 8192;  // room for the static LDS
        bd->lds_cap = cap;
        for (int k = 0; k < NCLASS; ++k) {
            int64_t need = 0;
            for (int32_t id : bd->order[k]) {
                const int64_t nv = bd->var_off[id + 1] - bd->var_off[id];
                const int64_t mv = bd->row_off[id + 1] - bd->row_off[id];
                const int64_t cap_d = cap / 8;
                const int mode = lds_mode_of(nv, mv, cap_d);
                const int64_t w = mode == LDS_ALL ? 5 * nv + 2 * mv
                                  : mode == LDS_GATHERED ? 3 * nv + mv : 0;
                need = std::max(need, w);
            }
            bd->lds_need[k] = (int32_t)need;
        }
    }
    (void)hipDeviceGetAttribute(&bd->wall_khz, hipDeviceAttributeWallClockRate, dev);
    (void)hipDeviceGetAttribute(&bd->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (bd->wall_khz <= 0) bd->wall_khz = 100000;
    // operator norms: overrides, else a batched power iteration
    if (s->norm_A > 0.0 && s->norm_Q > 0.0) {
        bd->normA.assign(B, s->norm_A);
        bd->normQ.assign(B, s->norm_Q);
    } else {
        BatchDev a = make_dev(bd);
        DevSettings ds = batch_settings(s);
        rc = run_classes(bd, [&](int k, hipStream_t cs) {
            launch_class(bd, a, ds, bd->threads[k], bd->order_off[k], bd->order_off[k + 1], k, cs,
                         true, s->power_iter_max, s->power_iter_rtol);
        });
        if (rc) {
            delete bd;
            return rc;
        }
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            delete bd;
            return fail(QP_ERR_DEVICE, "batched power iteration: %s", hipGetErrorString(e));
        }
        if (hipMemcpy(bd->normA.data(), bd->normA_d.p, (size_t)B * 8, hipMemcpyDeviceToHost) !=
                hipSuccess ||
            hipMemcpy(bd->normQ.data(), bd->normQ_d.p, (size_t)B * 8, hipMemcpyDeviceToHost) !=
                hipSuccess) {
            delete bd;
            return fail(QP_ERR_DEVICE, "reading batched norms failed");
        }
        if (s->norm_A > 0.0) bd->normA.assign(B, s->norm_A);
        if (s->norm_Q > 0.0) bd->normQ.assign(B, s->norm_Q);
    }
    for (int i = 0; i < B; ++i)
        if (!(bd->normA[i] > 0.0) && !(bd->normQ[i] > 0.0)) {
            delete bd;
            return fail(QP_ERR_INVALID_ARGUMENT, "instance %d has ||A|| = ||Q|| = 0", i);
        }
    if ((rc = warm_class_queues(bd))) {
        delete bd;
        return rc;
    }
    *out = bd;
    return QP_OK;
}

void destroy_batch(BatchData *b) {
    if (b) {
        (void)hipStreamSynchronize(b->stream);
        delete b;
    }
}

int batch_norms(BatchData *b, double *norm_A, double *norm_Q) {
    if (norm_A) std::memcpy(norm_A, b->normA.data(), (size_t)b->B * 8);
    if (norm_Q) std::memcpy(norm_Q, b->normQ.data(), (size_t)b->B * 8);
    return QP_OK;
}

int batch_set_norms(BatchData *b, const double *norm_A, const double *norm_Q) {
    for (int i = 0; i < b->B; ++i) {
        const double a = norm_A ? norm_A[i] : b->normA[i];
        const double q = norm_Q ? norm_Q[i] : b->normQ[i];
        if (!(a >= 0.0) || !(q >= 0.0) || !(a > 0.0 || q > 0.0))
            return fail(QP_ERR_INVALID_ARGUMENT, "invalid norms for instance %d", i);
    }
    if (norm_A) std::memcpy(b->normA.data(), norm_A, (size_t)b->B * 8);
    if (norm_Q) std::memcpy(b->normQ.data(), norm_Q, (size_t)b->B * 8);
    return QP_OK;
}

int batch_scaling(BatchData *bd, double *d_var, double *d_row) {
    const int64_t n = bd->ntot, m = bd->mtot;
    for (int64_t j = 0; d_var && j < n; ++j) d_var[j] = bd->h_d.empty() ? 1.0 : bd->h_d[j];
    for (int64_t i = 0; d_row && i < m; ++i) d_row[i] = bd->h_d.empty() ? 1.0 : bd->h_d[n + i];
    return QP_OK;
}

int batch_update_vectors(BatchData *bd, const double *c, const double *bvec, int ms) {
    const hipMemcpyKind kind = ms == QP_MEM_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost;
    if (c) HIPCHK(hipMemcpy(bd->h_c.data(), c, (size_t)bd->ntot * 8, kind));
    if (bvec && bd->mtot) HIPCHK(hipMemcpy(bd->h_b.data(), bvec, (size_t)bd->mtot * 8, kind));
    return upload_vectors(bd, bd->h_c, bd->h_b);
}

int batch_set_threads(BatchData *b, const int32_t *threads) {
    for (int k = 0; k < NCLASS; ++k) {
        const int32_t v = threads[k];
        if (v != 64 && v != 128 && v != 256 && v != 512 && v != 1024)
            return fail(QP_ERR_INVALID_ARGUMENT,
                        "threads per instance must be 64, 128, 256, 512 or 1024");
    }
    std::memcpy(b->threads, threads, sizeof(b->threads));
    return QP_OK;
}

// uploads per-instance scalars and warm starts, runs every size class
// max_count[k]: instances of class k to run (-1: all, 0: none)
static int run_batch(BatchData *bd, const qp_settings *s, int ms, const qp_warm_start *ws,
                     const int32_t *threads, const int32_t *max_count) {
    const int B = bd->B;
    hipStream_t st = bd->stream;
    std::vector<double> &omega = bd->h_omega;
    std::vector<uint8_t> &hx = bd->h_hx, &hy = bd->h_hy;
    HIPCHK(hipStreamSynchronize(st));  // the staging vectors may still feed a previous solve
    omega.assign(B, 0.0);
    hx.assign(B, 0);
    hy.assign(B, 0);
    bool any_warm = false;
    const hipMemcpyKind kind = ms == QP_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    for (int i = 0; i < B; ++i) {
        const double w0 = ws ? ws[i].omega0 : 0.0;
        omega[i] = w0 > 0.0 ? w0
                   : (bd->c_norm2[i] > s->eps_zero && bd->b_norm2[i] > s->eps_zero)
                       ? bd->c_norm2[i] / bd->b_norm2[i]
                       : 1.0;
        if (ws && ws[i].x0) {
            const int64_t v0 = bd->var_off[i], nv = bd->var_off[i + 1] - v0;
            HIPCHK(hipMemcpyAsync(bd->x0.as<double>() + v0, ws[i].x0, nv * 8, kind, st));
            hx[i] = 1;
            any_warm = true;
        }
        if (ws && ws[i].y0) {
            const int64_t r0 = bd->row_off[i], nr = bd->row_off[i + 1] - r0;
            if (nr > 0) HIPCHK(hipMemcpyAsync(bd->y0.as<double>() + r0, ws[i].y0, nr * 8, kind, st));
            hy[i] = 1;
            any_warm = true;
        }
    }
    if (any_warm && !bd->h_d.empty()) {  // warm starts refer to the given problem
        launch_scale_pair(st, bd->x0.as<double>(), bd->x0.as<double>(), bd->dscale.as<double>(),
                          bd->ntot, 1);
        launch_scale_pair(st, bd->y0.as<double>(), bd->y0.as<double>(),
                          bd->dscale.as<double>() + bd->ntot, bd->mtot, 1);
    }
    HIPCHK(hipMemcpyAsync(bd->omega0_d.p, omega.data(), (size_t)B * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bd->has_x0.p, hx.data(), (size_t)B, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bd->has_y0.p, hy.data(), (size_t)B, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bd->normA_d.p, bd->normA.data(), (size_t)B * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bd->normQ_d.p, bd->normQ.data(), (size_t)B * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bd->b_inf_d.p, bd->b_inf.data(), (size_t)B * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bd->c_inf_d.p, bd->c_inf.data(), (size_t)B * 8, hipMemcpyHostToDevice, st));
    BatchDev a = make_dev(bd);
    a.warm_fallback = s->warm_fallback;
    a.any_warm = any_warm ? 1 : 0;
    a.deadline_ticks = s->time_limit_s > 0.0
                           ? (int64_t)(s->time_limit_s * 1000.0 * (double)bd->wall_khz)
                           : 0;
    DevSettings ds = batch_settings(s);
    (void)hipGetLastError();  // launch errors are read below: drop any earlier one
    int rc = run_classes(bd, [&](int k, hipStream_t cs) {
        int lo = bd->order_off[k], hi = bd->order_off[k + 1];
        if (max_count && max_count[k] >= 0 && hi - lo > max_count[k]) hi = lo + max_count[k];
        BatchDev ak = a;
        ak.lds_doubles = bd->use_lds ? bd->lds_need[k] : 0;
        launch_class(bd, ak, ds, threads[k], lo, hi, k, cs, false, 0, 0.0);
    });
    if (rc) return rc;
    HIPCHK(hipGetLastError());
    return QP_OK;
}

int batch_solve(BatchData *bd, const qp_settings *s, int ms, const qp_warm_start *ws,
                qp_result *res, double *x_out, double *y_out) {
    const double t0 = qph::now_s();
    int rc;
    if ((rc = run_batch(bd, s, ms, ws, bd->threads, nullptr))) return rc;
    HIPCHK(hipStreamSynchronize(bd->stream));
    const double dt = qph::now_s() - t0;
    std::vector<State> S(bd->B);
    HIPCHK(hipMemcpy(S.data(), bd->res.p, (size_t)bd->B * sizeof(State), hipMemcpyDeviceToHost));
    const hipMemcpyKind kind = ms == QP_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (!bd->h_d.empty()) {  // back to the given problem: x = D2 x~, y = D1 y~
        launch_scale_pair(bd->stream, bd->x_out.as<double>(), bd->x_out.as<double>(),
                          bd->dscale.as<double>(), bd->ntot, 0);
        launch_scale_pair(bd->stream, bd->y_out.as<double>(), bd->y_out.as<double>(),
                          bd->dscale.as<double>() + bd->ntot, bd->mtot, 0);
        HIPCHK(hipStreamSynchronize(bd->stream));
    }
    if (x_out) HIPCHK(hipMemcpy(x_out, bd->x_out.p, (size_t)bd->ntot * 8, kind));
    if (y_out && bd->mtot) HIPCHK(hipMemcpy(y_out, bd->y_out.p, (size_t)bd->mtot * 8, kind));
    for (int i = 0; i < bd->B; ++i) {
        qp_result &r = res[i];
        std::memset(&r, 0, sizeof(r));
        const State &Z = S[i];
        r.status = Z.status;
        r.used_warm_start = Z.used_warm;
        r.iterations = Z.total;
        r.restarts = Z.restarts;
        r.kkt_evals = Z.kkt_evals;
        const double *k = Z.kkt[Z.cand ? 1 : 0];
        r.r_primal = k[0];
        r.r_dual = k[1];
        r.r_gap = k[2];
        r.rel_kkt = k[3];
        r.primal_obj = k[4];
        r.dual_obj = k[5];
        r.omega = Z.omega;
        r.norm_A = bd->normA[i];
        r.norm_Q = bd->normQ[i];
        r.solve_time_s = dt;
        r.start_s = (double)Z.t_start / (1000.0 * (double)bd->wall_khz);
        r.end_s = (double)Z.t_end / (1000.0 * (double)bd->wall_khz);
    }
    return QP_OK;
}

int batch_autotune(BatchData *bd, const qp_settings *s, int32_t sample, int32_t iters,
                   int32_t *threads_out) {
    // fixed work per trial: `iters` iterations (eps = 0) on up to `sample` instances per class
    qp_settings ts = *s;
    ts.eps = 0.0;
    ts.max_iter = iters > 0 ? iters : 256;
    ts.time_limit_s = 0.0;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int32_t best[NCLASS];
    std::memcpy(best, bd->threads, sizeof(best));
    for (int k = 0; k < NCLASS; ++k) {
        if (bd->order_off[k + 1] == bd->order_off[k]) continue;
        float best_ms = 1e30f;
        for (int c = 0; c < NCHOICE; ++c) {
            int32_t thr[NCLASS], cnt[NCLASS];
            for (int q = 0; q < NCLASS; ++q) {
                thr[q] = THREAD_CHOICES[c];
                cnt[q] = q == k ? (sample > 0 ? sample : -1) : 0;  // only class k runs
            }
            for (int rep = 0; rep < 2; ++rep) {  // the first pass warms up
                HIPCHK(hipEventRecord(e0, bd->stream));
                int rc = run_batch(bd, &ts, QP_MEM_HOST, nullptr, thr, cnt);
                if (rc) return rc;
                HIPCHK(hipEventRecord(e1, bd->stream));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                if (rep == 1 && ms < best_ms) {
                    best_ms = ms;
                    best[k] = THREAD_CHOICES[c];
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::memcpy(bd->threads, best, sizeof(best));
    if (threads_out) std::memcpy(threads_out, best, sizeof(best));
    return QP_OK;
}

}  // namespace qpb
