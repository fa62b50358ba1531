// qp_decide.h -- device-side scalar logic shared by the single-instance and the
// batched solvers: relative KKT error from reduced quantities (Sec. 5), restart
// candidate, criteria and primal weight (Sec. 6), and the step-size table
// (Sec. 6 rule; Thm 1 / eq. (param-choice) for beta_k, theta_k and fixed K).
#pragma once

#include <math.h>

#include "qp_internal.h"

namespace qpk {

// Sec. 6 cap at inner index k: 0.99 (k+2) / (||Q||/w + sqrt(||A||^2 (k+2)^2 + ||Q||^2/w^2))
__device__ __forceinline__ double pdqp_cap(const DevSettings &s, double omega, int64_t k) {
    const double kk = (double)(k + 2);
    const double qw = s.norm_Q / omega;
    return s.step_safety * kk / (qw + sqrt(s.norm_A * s.norm_A * kk * kk + qw * qw));
}

// primal step p and dual step d at inner index k; *s_last carries the scale of
// index k-1 of the same cycle (Sec. 6: min{(1 + 1/k) eta_{k-1}, cap_k}).  Plain PDHG
// (momentum off) keeps the cap of beta = 1, i.e. (k+2) replaced by 2, for every k.
__device__ __forceinline__ void step_at(const DevSettings &s, double omega, int64_t k,
                                        double *s_last, double *p, double *d) {
    if (!s.momentum) {
        const double qw = s.norm_Q / omega;
        const double sk = s.step_safety * 2.0 / (qw + sqrt(4.0 * s.norm_A * s.norm_A + qw * qw));
        *s_last = sk;
        *p = sk / omega;
        *d = sk * omega;
        return;
    }
    if (s.restart_mode == MODE_FIXED_K) {  // Theorem 1 / eq. (param-choice)
        const double Kf = (double)s.fixed_K;
        *p = (double)(k + 1) / (2.0 * (s.norm_Q + Kf * s.norm_A));
        *d = s.norm_A > 0.0 ? (double)(k + 1) / (2.0 * Kf * s.norm_A) : 0.0;
        *s_last = 0.0;
        return;
    }
    const double cap = pdqp_cap(s, omega, k);
    double sk;
    if (k == 0) {
        sk = cap;
    } else {
        const double grown = (1.0 + 1.0 / (double)k) * (*s_last);
        sk = grown < cap ? grown : cap;
    }
    *s_last = sk;
    *p = sk / omega;
    *d = sk * omega;
}

// Scalars of inner iteration kj.  w is the weight of the new iterate in the running
// average z-bar; theta_next and w_next (the weight of x in x_md) belong to iteration
// kj+1.  Algorithm 1: w = 1/beta_k, theta_{k+1} = (k+1)/(k+2), w_next = 1/beta_{k+1}.
// Plain PDHG: beta = theta = 1 (x_md = x, x~ = 2x - x_prev) and z-bar is the uniform
// average of the cycle, w = 1/(k+1).
__device__ __forceinline__ Step step_record(const DevSettings &s, int64_t kj, double p, double d) {
    Step e;
    e.p = p;
    e.d = d;
    if (s.momentum) {
        e.w = 2.0 / (double)(kj + 2);
        e.theta_next = (double)(kj + 1) / (double)(kj + 2);
        e.w_next = 2.0 / (double)(kj + 3);
    } else {
        e.w = 1.0 / (double)(kj + 1);
        e.theta_next = 1.0;
        e.w_next = 1.0;
    }
    e.pad[0] = e.pad[1] = e.pad[2] = 0.0;
    return e;
}

__device__ __forceinline__ Step make_step(const DevSettings &s, double omega, int64_t kj,
                                          double *s_last) {
    double p, d;
    step_at(s, omega, kj, s_last, &p, &d);
    return step_record(s, kj, p, d);
}

// relKKT of point p (0 = z, 1 = z-bar) from the reduced quantities
// (out: r_primal, r_dual, r_gap, rel_kkt, primal_obj, dual_obj)
__device__ __forceinline__ void rel_kkt_point(const double *ra, const double *rp, int p,
                                              const DevSettings &s, double *out) {
    const double res_p = ra[RA_RES0 + p], ax = ra[RA_AX0 + p], by = ra[RA_BY0 + p];
    const double dres = rp[RP_DRES0 + p], qx = rp[RP_QX0 + p], aty = rp[RP_ATY0 + p];
    const double xqx = rp[RP_XQX0 + p], cx = rp[RP_CX0 + p], bnd = rp[RP_BND0 + p];
    const double P = 0.5 * xqx + cx;
    const double D = -0.5 * xqx + by + bnd;
    const double r_p = res_p / (1.0 + fmax(ax, s.b_inf));
    const double r_d = dres / (1.0 + fmax(fmax(qx, aty), s.c_inf));
    const double r_g = fabs(P - D) / (1.0 + fmax(fabs(P), fabs(D)));
    double r = r_p;
    if (r_d > r) r = r_d;
    if (r_g > r) r = r_g;
    if (isnan(r_p) || isnan(r_d) || isnan(r_g)) r = NAN;
    out[0] = r_p;
    out[1] = r_d;
    out[2] = r_g;
    out[3] = r;
    out[4] = P;
    out[5] = D;
}

// Infeasibility certificates from S.inf (the paper is silent; the quantities are those
// of the drift z - z_restart, projected): primal infeasible when the dual direction is a
// Farkas ray, max |A'dy+| over unbounded components <= tol (b'dy+ - support), with
// b'dy+ - support > 0; dual infeasible when the primal direction descends without
// bound, max(||Q dx+||, A dx+ violation) <= tol (-c'dx+), with c'dx+ < 0.
__device__ __forceinline__ int infeas_status(const State &S, const DevSettings &s) {
    const double farkas = S.inf[INF_BDY] - S.inf[INF_SUPP];
    if (farkas > 0.0 && S.inf[INF_GVIOL] / farkas <= s.eps_infeas) return ST_PRIMAL_INFEASIBLE;
    const double cdx = S.inf[INF_CDX];
    const double dviol = fmax(S.inf[INF_QDX], S.inf[INF_AVIOL]);
    if (cdx < 0.0 && dviol / -cdx <= s.eps_infeas) return ST_DUAL_INFEASIBLE;
    return -1;
}

// One evaluation (DECIDE_INIT / DECIDE_CHECK / DECIDE_FALLBACK) applied to S.
// Returns the restart flag (the caller copies the candidate if set).
__device__ __forceinline__ int decide_update(int mode, const double *ra, const double *rp,
                                             State &S, const DevSettings &s, int32_t len) {
    double k0[6], k1[6];
    rel_kkt_point(ra, rp, 0, s, k0);
    rel_kkt_point(ra, rp, 1, s, k1);
    int restart = 0;
    if (mode == DECIDE_FALLBACK) {
        // point 0 = warm start, point 1 = cold start
        S.used_warm = k0[3] < k1[3] ? 1 : 0;
        S.kkt_evals += 2;
        S.restart_flag = 0;
        return 0;
    }
    if (mode == DECIDE_INIT) {
        S.kkt_evals += 1;
        S.r0 = k0[3];
        S.prev_cand = INFINITY;
        S.total = 0;
        S.k = 0;
        S.cand = 0;
        S.r_cur = S.r_avg = k0[3];
        for (int i = 0; i < 6; ++i) S.kkt[0][i] = S.kkt[1][i] = k0[i];
        if (isnan(k0[3])) {
            S.status = ST_NUMERICAL;
            S.done = 1;
        } else if (k0[3] <= s.eps) {
            S.status = ST_OPTIMAL;
            S.done = 1;
        } else if (s.max_iter <= 0) {
            S.status = ST_ITER_LIMIT;
            S.done = 1;
        }
    } else {  // DECIDE_CHECK after `len` iterations
        S.total += len;
        S.k += len;
        S.kkt_evals += 2;
        S.checks += 1;
        const double r = k0[3], rb = k1[3];
        const bool fixed = s.restart_mode == MODE_FIXED_K;
        // Algorithm 1 and the Sec. 5 methods (fixed frequency, halving, no restart) are
        // measured at the average; the better of iterate and average is the Sec. 6 rule
        // GetRestartCandidate (ties: average)
        const int cand_avg = s.restart_mode != MODE_ADAPTIVE ? 1 : !(r < rb);
        const double rc = cand_avg ? rb : r;
        if (isnan(r) || isnan(rb)) {
            S.status = ST_NUMERICAL;
            S.done = 1;
        } else if (rc <= s.eps) {
            S.status = ST_OPTIMAL;
            S.done = 1;
        } else if (s.detect_infeas && infeas_status(S, s) >= 0) {
            S.status = infeas_status(S, s);
            S.done = 1;
        } else if (S.total >= s.max_iter) {
            S.status = ST_ITER_LIMIT;
            S.done = 1;
        } else if (s.restart_mode == MODE_ADAPTIVE) {  // Sec. 6 criteria (i), (ii), (iii)
            restart = (rc <= s.beta_sufficient * S.r0) ||
                      (rc <= s.beta_necessary * S.r0 && rc > S.prev_cand) ||
                      ((double)S.k >= s.beta_artificial * (double)S.total);
        } else if (s.restart_mode == MODE_HALVING) {   // Sec. 5 adaptive restart
            restart = rb <= 0.5 * S.r0;
        } else if (fixed) {                            // Algorithm 1
            restart = 1;
        }
        if (restart) {
            if (!fixed) {  // Sec. 6 PrimalWeightUpdate
                const double dx = sqrt(rp[RP_DX0 + cand_avg]);
                const double dy = sqrt(ra[RA_DY0 + cand_avg]);
                if (dx > s.eps_zero && dy > s.eps_zero)
                    S.omega = exp(s.pw_smoothing * log(dy / dx) +
                                  (1.0 - s.pw_smoothing) * log(S.omega));
            }
            S.k = 0;
            S.r0 = rc;
            S.prev_cand = INFINITY;
            S.restarts += 1;
        } else if (!S.done) {
            S.prev_cand = rc;
        }
        S.cand = cand_avg;
        S.r_cur = r;
        S.r_avg = rb;
        for (int i = 0; i < 6; ++i) {
            S.kkt[0][i] = k0[i];
            S.kkt[1][i] = k1[i];
        }
    }
    S.restart_flag = restart;
    return restart;
}

}  // namespace qpk
