// qp_kernels.hip -- gfx950 kernels of the single-instance rAPDHG hot path.
//
// Per iteration (Algorithm 1 of Lu & Yang, arXiv 2311.07710, in the
// EQ/GE + bounds form L(x,y) = 1/2 x'Qx + c'x - y'(Ax - b)):
//   dual phase   (k_dual):   y+ = proj_Y(y - d_k (A x~ - b)),  y-bar averaging
//   primal phase (k_primal): x+ = proj_X(x - p_k (Q x_md + c - A'y+)),  x-bar
//                            averaging, and the NEXT iteration's x~ and x_md
// Every KKT check (Sec. 5 relative KKT error for z and z-bar):
//   k_kkt_rows (A x, A x-bar), k_kkt_cols (Q x, A'y for both points), then the
//   single-workgroup k_decide (Sec. 6 restart candidate, criteria (i)-(iii),
//   primal weight update, step-size table for the next interval) and k_apply.
//
// Memory layout: A is CSR (m rows); Q and -A' are fused into ONE CSR matrix
// P = [Q | -A'] (n rows, columns >= n address y), so the primal phase is a
// single streaming pass gathering from (x_md, y).  Rows are grouped on the
// host into blocks of <= NNZ_BLK nonzeros and <= BS rows; a workgroup streams
// its nonzeros with coalesced loads, gathers the vector entries
// and stages the products in LDS, then each row is summed in CSR order
// (several lanes per row only when a block holds few rows).
//
// Large instances run both phases on column panels (the second half of this file):
// the columns are split into ranges pinned to groups of XCDs so each XCD gathers from
// a slice that stays in its L2; persistent, software-pipelined k_panel_spmv<0/1> write
// per-panel row sums that k_dual_combine / k_primal_combine add in panel order before
// the same epilogues.  The KKT evaluation then gathers (x, x-bar) and (y, y-bar) as
// 16-byte pairs (k_interleave, k_panel_kkt<0/1>).  The path is bound by HBM streams
// and, on the large instances, by the L2 request rate of the random gathers: no MFMA
// anywhere on it.
#include <math.h>

#include "qp_decide.h"
#include "qp_internal.h"

namespace qpk {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of row blocks so neighbouring rows share an L2.
__device__ __forceinline__ int xcd_block(int bid, int nb) {
    const int X = 8;
    const int q = nb / X, r = nb % X;
    const int x = bid % X, local = bid / X;
    return x * q + min(x, r) + local;
}

// max that keeps a NaN once seen (the reductions must report NaN)
__device__ __forceinline__ double nmax(double a, double b) {
    return (b > a || b != b) ? b : a;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = nmax(v, __shfl_xor(v, off, 64));
    return v;
}

// group reduction over G lanes (G a power of two dividing 64)
__device__ __forceinline__ double group_sum(double v, int G) {
    for (int off = G >> 1; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int lanes_per_row(int nrows) {
    int g = BS / (nrows > 0 ? nrows : 1);
    g = g > 64 ? 64 : g;
    return 1 << (31 - __clz(g));
}

// Deterministic block sum of the staged products prod[0..cnt).
__device__ double block_sum_lds(const double *prod, int cnt, double *scratch) {
    double s = 0.0;
    for (int e = threadIdx.x; e < cnt; e += BS) s = s + prod[e];
    s = wave_sum(s);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) scratch[wid] = s;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BS / 64; ++w) t = t + scratch[w];
    __syncthreads();
    return t;  // valid in thread 0
}

// Deterministic block sum of one value per thread (valid in thread 0).
__device__ double block_sum_value(double s, double *scratch) {
    s = wave_sum(s);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) scratch[wid] = s;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BS / 64; ++w) t = t + scratch[w];
    __syncthreads();
    return t;
}

// Chunk partial sums of a long row: thread 0 publishes the chunk's W partial sums;
// the last chunk to arrive (atomic counter) adds all partials of the row.  The whole
// last workgroup reads them in parallel (thread t adds partials t, t + BS, ... in
// order, then a fixed reduction tree over the threads), so a row of many chunks costs
// one memory round trip instead of one per chunk; the order is fixed, so the result
// is deterministic.  Returns true in thread 0 of the last workgroup, with the row
// totals in tot[].
//
// The chunks of a row run on different XCDs, whose L2s are not coherent with each
// other.  The partials are therefore written and read with agent-scope atomic
// accesses (write-through / cache-bypassing), and the writer waits for its stores to
// be acknowledged before it bumps the counter.  No agent-scope fence is used: on this
// GPU one writes back and invalidates the whole L2 of the XCD, which evicted the
// gathered vector of every other workgroup there.
template <int W>
__device__ bool finish_chunks(int32_t *count, const int32_t *first, const int32_t *nchunk,
                              double *partial, int bi, int lr, const double *part, double *tot) {
    __shared__ int is_last;
    __shared__ double scratch[BS / 64];
    if (threadIdx.x == 0) {
        for (int v = 0; v < W; ++v)
            __hip_atomic_store(&partial[(size_t)bi * 4 + v], part[v], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // keeps the order in code
        __builtin_amdgcn_s_waitcnt(0);  // the partial stores are acknowledged
        const int old = atomicAdd(&count[lr], 1);
        is_last = (old == nchunk[lr] - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    const int f = first[lr], nc = nchunk[lr];
    double acc[W];
    for (int v = 0; v < W; ++v) acc[v] = 0.0;
    for (int ch = threadIdx.x; ch < nc; ch += BS)
        for (int v = 0; v < W; ++v)
            acc[v] = acc[v] + __hip_atomic_load(&partial[(size_t)(f + ch) * 4 + v],
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int v = 0; v < W; ++v) tot[v] = block_sum_value(acc[v], scratch);
    if (threadIdx.x == 0)
        __hip_atomic_store(&count[lr], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return threadIdx.x == 0;
}

template <int W>
__device__ bool chunk_finish(const Blocks &bk, int bi, int lr, const double *part, double *tot) {
    return finish_chunks<W>(bk.lr_count, bk.lr_first, bk.lr_nchunk, bk.lr_partial, bi, lr, part,
                            tot);
}

// ---------------------------------------------------------------------------
// dual phase: one pass over A
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dual_epilogue(int i, double v, double *__restrict__ y,
                                              double *__restrict__ ybar,
                                              const double *__restrict__ b,
                                              const uint8_t *__restrict__ rt, double d, double w) {
    double yn = y[i] - d * (v - b[i]);
    if (rt[i] == 1 && yn < 0.0) yn = 0.0;  // projection onto y_i >= 0 for >= rows
    ybar[i] = (1.0 - w) * ybar[i] + w * yn;
    y[i] = yn;
}

// Streams the (column, value) pairs of entries e0 + i*BS + t, i < EPT, of a block with
// every load issued before any result is used, so that the gathers that follow are all
// in flight together.  Lanes past the block's end read entry e0 (device arrays carry a
// zero pad entry, so e0 is readable even for an empty block at the end of an array) and
// get value 0: their products are zero and never summed.
//
// Cache policy (measured on the large random QP): P = [Q | -A'] is streamed with
// non-temporal loads so it does not evict the gathered vectors; A (a third of P's size)
// is streamed with ordinary loads, which lets it stay resident in the 256 MB MALL
// from one iteration to the next (dual phase 46.6 -> 42.1 us).  Ordinary loads for P
// as well were 7 % slower: the per-iteration working set then exceeds the MALL.
enum Stream { STREAM_A = 0, STREAM_P = 1 };

template <int SRC>
__device__ __forceinline__ void load_block(const int32_t *__restrict__ col,
                                           const double *__restrict__ val, int e0, int e1,
                                           int t, int (&cols)[EPT], double (&vals)[EPT]) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = e0 + i * BS + t;
        const int ee = e < e1 ? e : e0;
        double v;
        if (SRC == STREAM_P) {
            cols[i] = __builtin_nontemporal_load(&col[ee]);
            v = __builtin_nontemporal_load(&val[ee]);
        } else {
            cols[i] = col[ee];
            v = val[ee];
        }
        vals[i] = e < e1 ? v : 0.0;
    }
}

__global__ __launch_bounds__(BS) void k_dual(Blocks bk, Csr A, const double *__restrict__ xt,
                                             double *__restrict__ y, double *__restrict__ ybar,
                                             const double *__restrict__ b,
                                             const uint8_t *__restrict__ rt,
                                             const Step *__restrict__ step,
                                             const State *__restrict__ st) {
    if (st->done) return;
    __shared__ double prod[NNZ_BLK];
    __shared__ double scratch[BS / 64];
    const int bi = xcd_block(blockIdx.x, gridDim.x);
    const Block B = bk.blk[bi];
    const int t = threadIdx.x;
    int cols[EPT];
    double vals[EPT];
    load_block<STREAM_A>(A.col, A.val, B.e0, B.e1, t, cols, vals);
    double g[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) g[i] = xt[cols[i]];
#pragma unroll
    for (int i = 0; i < EPT; ++i) prod[i * BS + t] = vals[i] * g[i];
    __syncthreads();
    const double d = step->d, w = step->w;
    const int lr = bk.lr[bi];
    if (lr < 0) {
        const int nrows = B.row1 - B.row0;
        const int G = lanes_per_row(nrows);
        const int rl = t / G, lane = t % G;
        double s = 0.0;
        if (rl < nrows) {
            const int row = B.row0 + rl;
            const int s1 = A.rowptr[row + 1] - B.e0;
            for (int e = A.rowptr[row] - B.e0 + lane; e < s1; e += G) s = s + prod[e];
        }
        s = group_sum(s, G);
        if (rl < nrows && lane == 0) dual_epilogue(B.row0 + rl, s, y, ybar, b, rt, d, w);
    } else {
        double part = block_sum_lds(prod, B.e1 - B.e0, scratch);
        double tot;
        if (chunk_finish<1>(bk, bi, lr, &part, &tot)) dual_epilogue(B.row0, tot, y, ybar, b, rt, d, w);
    }
}

// ---------------------------------------------------------------------------
// primal phase: one pass over P = [Q | -A'] gathering (x_md, y+)
// ---------------------------------------------------------------------------
struct PrimalArgs {
    const double *xmd_in;
    const double *y;
    double *x, *xbar, *xt, *xmd_out;
    const double *c, *l, *u;
    int32_t ub;      // 1: every l_j = lo and every u_j = hi (l and u are not read)
    double lo, hi;
};

static PrimalArgs primal_args(const Vecs &v, int md_in) {
    PrimalArgs a;
    a.xmd_in = v.xmd[md_in];
    a.y = v.y;
    a.x = v.x;
    a.xbar = v.xbar;
    a.xt = v.xt;
    a.xmd_out = v.xmd[md_in ^ 1];
    a.c = v.c;
    a.l = v.l;
    a.u = v.u;
    a.ub = v.uniform_bounds;
    a.lo = v.lo_all;
    a.hi = v.hi_all;
    return a;
}

__device__ __forceinline__ void primal_epilogue(int j, double s, const PrimalArgs &a, double p,
                                                double w, double th1, double w1) {
    const double g = s + a.c[j];
    const double xo = a.x[j];
    double xn = xo - p * g;
    const double lo = a.ub ? a.lo : a.l[j], hi = a.ub ? a.hi : a.u[j];
    if (xn < lo) xn = lo;
    if (xn > hi) xn = hi;
    const double xb = (1.0 - w) * a.xbar[j] + w * xn;
    a.x[j] = xn;
    a.xbar[j] = xb;
    a.xt[j] = xn + th1 * (xn - xo);          // x~ of the next iteration
    a.xmd_out[j] = (1.0 - w1) * xb + w1 * xn;  // x_md of the next iteration
}

__global__ __launch_bounds__(BS) void k_primal(Blocks bk, Csr P, PrimalArgs a,
                                               const Step *__restrict__ step,
                                               const State *__restrict__ st, int32_t n) {
    if (st->done) return;
    __shared__ double prod[NNZ_BLK];
    __shared__ double scratch[BS / 64];
    const int bi = xcd_block(blockIdx.x, gridDim.x);
    const Block B = bk.blk[bi];
    const int t = threadIdx.x;
    int cols[EPT];
    double vals[EPT];
    load_block<STREAM_P>(P.col, P.val, B.e0, B.e1, t, cols, vals);
    double g[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int cc = cols[i];
        g[i] = *(cc < n ? a.xmd_in + cc : a.y + (cc - n));
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) prod[i * BS + t] = vals[i] * g[i];
    __syncthreads();
    const double p = step->p, w = step->w, th1 = step->theta_next, w1 = step->w_next;
    const int lr = bk.lr[bi];
    if (lr < 0) {
        const int nrows = B.row1 - B.row0;
        const int G = lanes_per_row(nrows);
        const int rl = t / G, lane = t % G;
        double s = 0.0;
        if (rl < nrows) {
            const int row = B.row0 + rl;
            const int s1 = P.rowptr[row + 1] - B.e0;
            for (int e = P.rowptr[row] - B.e0 + lane; e < s1; e += G) s = s + prod[e];
        }
        s = group_sum(s, G);
        if (rl < nrows && lane == 0) primal_epilogue(B.row0 + rl, s, a, p, w, th1, w1);
    } else {
        double part = block_sum_lds(prod, B.e1 - B.e0, scratch);
        double tot;
        if (chunk_finish<1>(bk, bi, lr, &part, &tot)) primal_epilogue(B.row0, tot, a, p, w, th1, w1);
    }
}

// ---------------------------------------------------------------------------
// KKT evaluation, rows of A: A x and A x-bar in one pass
// ---------------------------------------------------------------------------
struct KktRowArgs {
    const double *x, *xbar, *y, *ybar, *yrs, *b;
    const uint8_t *rt;
    const double *dr;  // row scaling D1 of a preconditioned problem, or nullptr
    double *partials;  // [(nblk + nlr) * RA_NV]
};

__device__ __forceinline__ void kkt_row_contrib(int i, double s0, double s1, const KktRowArgs &a,
                                                double *cv) {
    const double bi = a.b[i];
    const bool ge = a.rt[i] == 1;
    double r0 = s0 - bi, r1 = s1 - bi;
    if (ge) {
        r0 = (r0 < 0.0) ? -r0 : 0.0;
        r1 = (r1 < 0.0) ? -r1 : 0.0;
    }
    // preconditioned: the original problem's row i is row i of the scaled one divided
    // by D1_i (relKKT is measured on the given problem; dot products are invariant)
    const double sr = a.dr ? a.dr[i] : 1.0;
    cv[RA_RES0] = fabs(r0) / sr;
    cv[RA_RES1] = fabs(r1) / sr;
    cv[RA_AX0] = fabs(s0) / sr;
    cv[RA_AX1] = fabs(s1) / sr;
    const double yi = a.y[i], ybi = a.ybar[i], yr = a.yrs[i];
    cv[RA_BY0] = bi * yi;
    cv[RA_BY1] = bi * ybi;
    const double d0 = yi - yr, d1 = ybi - yr;
    cv[RA_DY0] = d0 * d0;
    cv[RA_DY1] = d1 * d1;
}

// block reduction of NV contributions (first NMAX are maxima, the rest sums),
// written by thread 0 to out[0..NV)
template <int NV, int NMAX>
__device__ void block_reduce_write(double *cv, double *out) {
    __shared__ double red[NV][BS / 64];
#pragma unroll
    for (int v = 0; v < NV; ++v) cv[v] = v < NMAX ? wave_max(cv[v]) : wave_sum(cv[v]);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int v = 0; v < NV; ++v) red[v][wid] = cv[v];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 0; v < NV; ++v) {
            double acc = red[v][0];
            for (int w = 1; w < BS / 64; ++w) acc = v < NMAX ? nmax(acc, red[v][w]) : acc + red[v][w];
            out[v] = acc;
        }
    }
}

__global__ __launch_bounds__(BS) void k_kkt_rows(Blocks bk, Csr A, KktRowArgs a,
                                                 const State *__restrict__ st) {
    if (st->done) return;
    __shared__ double prod0[NNZ_BLK];
    __shared__ double prod1[NNZ_BLK];
    __shared__ double scratch[BS / 64];
    const int bi = xcd_block(blockIdx.x, gridDim.x);
    const Block B = bk.blk[bi];
    const int t = threadIdx.x;
    {
        int cols[EPT];
        double vals[EPT], g0[EPT], g1[EPT];
        load_block<STREAM_A>(A.col, A.val, B.e0, B.e1, t, cols, vals);
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            g0[i] = a.x[cols[i]];
            g1[i] = a.xbar[cols[i]];
        }
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            prod0[i * BS + t] = vals[i] * g0[i];
            prod1[i * BS + t] = vals[i] * g1[i];
        }
    }
    __syncthreads();
    double cv[RA_NV];
    for (int v = 0; v < RA_NV; ++v) cv[v] = 0.0;
    const int lr = bk.lr[bi];
    if (lr < 0) {
        const int nrows = B.row1 - B.row0;
        const int G = lanes_per_row(nrows);
        const int rl = t / G, lane = t % G;
        double s0 = 0.0, s1 = 0.0;
        if (rl < nrows) {
            const int row = B.row0 + rl;
            const int e1 = A.rowptr[row + 1] - B.e0;
            for (int e = A.rowptr[row] - B.e0 + lane; e < e1; e += G) {
                s0 = s0 + prod0[e];
                s1 = s1 + prod1[e];
            }
        }
        s0 = group_sum(s0, G);
        s1 = group_sum(s1, G);
        if (rl < nrows && lane == 0) kkt_row_contrib(B.row0 + rl, s0, s1, a, cv);
        block_reduce_write<RA_NV, 4>(cv, a.partials + (size_t)bi * RA_NV);
    } else {
        double part[2];
        part[0] = block_sum_lds(prod0, B.e1 - B.e0, scratch);
        part[1] = block_sum_lds(prod1, B.e1 - B.e0, scratch);
        if (t == 0)
            for (int v = 0; v < RA_NV; ++v) a.partials[(size_t)bi * RA_NV + v] = 0.0;
        double tot[2];
        if (chunk_finish<2>(bk, bi, lr, part, tot)) {
            kkt_row_contrib(B.row0, tot[0], tot[1], a, cv);
            for (int v = 0; v < RA_NV; ++v)
                a.partials[(size_t)(bk.nblk + lr) * RA_NV + v] = cv[v];
        }
    }
}

// ---------------------------------------------------------------------------
// KKT evaluation, rows of P = [Q | -A']: Q x and A'y for z and z-bar
// ---------------------------------------------------------------------------
struct KktColArgs {
    const double *x, *xbar, *y, *ybar, *xrs, *c, *l, *u;
    const double *dv;  // column scaling D2 of a preconditioned problem, or nullptr
    double *partials;  // [(nblk + nlr) * RP_NV]
};

__device__ __forceinline__ void kkt_col_contrib(int j, const double *qx, const double *naty,
                                                const KktColArgs &a, double *cv) {
    const double cj = a.c[j], lj = a.l[j], uj = a.u[j];
    const bool lo_fin = isfinite(lj), hi_fin = isfinite(uj);
    const double sv = a.dv ? a.dv[j] : 1.0;  // original column j = scaled one / D2_j
    for (int p = 0; p < 2; ++p) {
        const double xp = p == 0 ? a.x[j] : a.xbar[j];
        const double aty = -naty[p];
        const double lam = qx[p] + cj - aty;  // reduced cost Qx + c - A'y
        double lam_hat;
        if (lo_fin && hi_fin) lam_hat = lam;
        else if (lo_fin) lam_hat = lam > 0.0 ? lam : 0.0;
        else if (hi_fin) lam_hat = lam < 0.0 ? lam : 0.0;
        else lam_hat = 0.0;
        cv[RP_DRES0 + p] = fabs(lam - lam_hat) / sv;
        cv[RP_QX0 + p] = fabs(qx[p]) / sv;
        cv[RP_ATY0 + p] = fabs(aty) / sv;
        cv[RP_XQX0 + p] = xp * qx[p];
        cv[RP_CX0 + p] = cj * xp;
        double bnd = 0.0;
        if (lo_fin && lam_hat > 0.0) bnd = lj * lam_hat;
        if (hi_fin && lam_hat < 0.0) bnd = uj * lam_hat;
        cv[RP_BND0 + p] = bnd;
        const double dx = xp - a.xrs[j];
        cv[RP_DX0 + p] = dx * dx;
    }
}

__global__ __launch_bounds__(BS) void k_kkt_cols(Blocks bk, Csr P, KktColArgs a,
                                                 const State *__restrict__ st, int32_t n) {
    if (st->done) return;
    __shared__ double prod0[NNZ_BLK];
    __shared__ double prod1[NNZ_BLK];
    __shared__ uint8_t isA[NNZ_BLK];
    __shared__ double scratch[BS / 64];
    const int bi = xcd_block(blockIdx.x, gridDim.x);
    const Block B = bk.blk[bi];
    const int t = threadIdx.x;
    {
        int cols[EPT];
        double vals[EPT], g0[EPT], g1[EPT];
        load_block<STREAM_P>(P.col, P.val, B.e0, B.e1, t, cols, vals);
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int cc = cols[i];
            const bool ya = cc >= n;
            g0[i] = *(ya ? a.y + (cc - n) : a.x + cc);
            g1[i] = *(ya ? a.ybar + (cc - n) : a.xbar + cc);
        }
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            prod0[i * BS + t] = vals[i] * g0[i];
            prod1[i * BS + t] = vals[i] * g1[i];
            isA[i * BS + t] = cols[i] >= n;
        }
    }
    __syncthreads();
    double cv[RP_NV];
    for (int v = 0; v < RP_NV; ++v) cv[v] = 0.0;
    const int lr = bk.lr[bi];
    if (lr < 0) {
        const int nrows = B.row1 - B.row0;
        const int G = lanes_per_row(nrows);
        const int rl = t / G, lane = t % G;
        double q[2] = {0.0, 0.0}, na[2] = {0.0, 0.0};
        if (rl < nrows) {
            const int row = B.row0 + rl;
            const int e1 = P.rowptr[row + 1] - B.e0;
            for (int e = P.rowptr[row] - B.e0 + lane; e < e1; e += G) {
                if (isA[e]) {
                    na[0] = na[0] + prod0[e];
                    na[1] = na[1] + prod1[e];
                } else {
                    q[0] = q[0] + prod0[e];
                    q[1] = q[1] + prod1[e];
                }
            }
        }
        for (int p = 0; p < 2; ++p) {
            q[p] = group_sum(q[p], G);
            na[p] = group_sum(na[p], G);
        }
        if (rl < nrows && lane == 0) kkt_col_contrib(B.row0 + rl, q, na, a, cv);
        block_reduce_write<RP_NV, 6>(cv, a.partials + (size_t)bi * RP_NV);
    } else {
        // split the staged products of this chunk into the Q part and the A' part
        double part[4];
        for (int p = 0; p < 4; ++p) {
            double s = 0.0;
            const double *src = (p & 1) ? prod1 : prod0;
            const bool wantA = p >= 2;
            for (int e = t; e < B.e1 - B.e0; e += BS)
                if ((bool)isA[e] == wantA) s = s + src[e];
            s = wave_sum(s);
            if ((t & 63) == 0) scratch[t >> 6] = s;
            __syncthreads();
            if (t == 0) {
                double acc = 0.0;
                for (int w = 0; w < BS / 64; ++w) acc = acc + scratch[w];
                part[p] = acc;
            }
            __syncthreads();
        }
        if (t == 0)
            for (int v = 0; v < RP_NV; ++v) a.partials[(size_t)bi * RP_NV + v] = 0.0;
        double tot[4];
        if (chunk_finish<4>(bk, bi, lr, part, tot)) {
            double q[2] = {tot[0], tot[1]}, na[2] = {tot[2], tot[3]};
            kkt_col_contrib(B.row0, q, na, a, cv);
            for (int v = 0; v < RP_NV; ++v)
                a.partials[(size_t)(bk.nblk + lr) * RP_NV + v] = cv[v];
        }
    }
}

// ---------------------------------------------------------------------------
// decision kernel (one workgroup): relKKT, candidate, restart, primal weight,
// step table for the next interval
// ---------------------------------------------------------------------------
// First stage of the partial reduction: workgroup g folds the per-block KKT partials of
// slots [g*per, min((g+1)*per, nslot)) into one slot of out (the first NMAX entries of a
// slot are maxima, the rest sums), in a fixed order.
template <int NV, int NMAX>
__global__ __launch_bounds__(BS) void k_fold_slots(const double *__restrict__ part, int32_t nslot,
                                                   int32_t per, double *__restrict__ out,
                                                   const State *__restrict__ st) {
    if (st->done) return;
    __shared__ double red[NV][BS];
    const int t = threadIdx.x;
    const int i0 = blockIdx.x * per;
    const int i1 = min(nslot, i0 + per);
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int i = i0 + t; i < i1; i += BS) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double z = part[(size_t)i * NV + v];
            acc[v] = v < NMAX ? nmax(acc[v], z) : acc[v] + z;
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) red[v][t] = acc[v];
    __syncthreads();
    for (int h = BS / 2; h >= 1; h >>= 1) {
        if (t < h) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                red[v][t] = v < NMAX ? nmax(red[v][t], red[v][t + h]) : red[v][t] + red[v][t + h];
        }
        __syncthreads();
    }
    if (t < NV) out[(size_t)blockIdx.x * NV + t] = red[t][0];
}

__global__ __launch_bounds__(BS) void k_decide(int mode, const double *__restrict__ partA,
                                               int32_t nslotA, const double *__restrict__ partP,
                                               int32_t nslotP, State *st, Step *table,
                                               DevSettings s, int32_t len) {
    if (st->done) return;
    __shared__ double red[RA_NV + RP_NV][BS];
    const int t = threadIdx.x;
    // fixed-order reduction of the block partials
    for (int v = 0; v < RA_NV; ++v) {
        const bool mx = v < 4;
        double acc = 0.0;
        for (int i = t; i < nslotA; i += BS) {
            const double z = partA[(size_t)i * RA_NV + v];
            acc = mx ? nmax(acc, z) : acc + z;
        }
        red[v][t] = acc;
    }
    for (int v = 0; v < RP_NV; ++v) {
        const bool mx = v < 6;
        double acc = 0.0;
        for (int i = t; i < nslotP; i += BS) {
            const double z = partP[(size_t)i * RP_NV + v];
            acc = mx ? nmax(acc, z) : acc + z;
        }
        red[RA_NV + v][t] = acc;
    }
    __syncthreads();
    for (int h = BS / 2; h >= 1; h >>= 1) {
        if (t < h) {
            for (int v = 0; v < RA_NV + RP_NV; ++v) {
                const bool mx = v < RA_NV ? v < 4 : (v - RA_NV) < 6;
                red[v][t] = mx ? nmax(red[v][t], red[v][t + h]) : red[v][t] + red[v][t + h];
            }
        }
        __syncthreads();
    }
    __shared__ State S;
    if (t == 0) {
        double ra[RA_NV], rp[RP_NV];
        for (int v = 0; v < RA_NV; ++v) ra[v] = red[v][0];
        for (int v = 0; v < RP_NV; ++v) rp[v] = red[RA_NV + v][0];
        S = *st;
        decide_update(mode, ra, rp, S, s, len);
    }
    __syncthreads();
    if (mode != DECIDE_FALLBACK && !S.done) {
        // The next interval's step table, the same values as make_step called in order:
        // with the Sec. 6 rule only the scale's min-recurrence is sequential (thread 0,
        // a multiply and a compare per entry); the caps, the growth factors and each
        // entry's divisions are computed by the whole workgroup.
        const double om = S.omega;
        const int64_t k0 = S.k;
        if (s.momentum && s.restart_mode != MODE_FIXED_K) {
            __shared__ double cap[BS], grow[BS];
            double sl = S.s_last;  // thread 0's carry
            for (int c0 = 0; c0 < s.interval; c0 += BS) {
                const int j = c0 + t;
                const int64_t kj = k0 + j;
                if (j < s.interval) {
                    cap[t] = pdqp_cap(s, om, kj);
                    grow[t] = kj > 0 ? 1.0 + 1.0 / (double)kj : 0.0;
                }
                __syncthreads();
                if (t == 0) {
                    const int cnt = s.interval - c0 < BS ? s.interval - c0 : BS;
                    for (int i = 0; i < cnt; ++i) {
                        double sk = cap[i];
                        if (k0 + c0 + i > 0) {
                            const double grown = grow[i] * sl;
                            sk = grown < sk ? grown : sk;
                        }
                        sl = sk;
                        cap[i] = sk;
                    }
                }
                __syncthreads();
                if (j < s.interval) table[j] = step_record(s, kj, cap[t] / om, cap[t] * om);
                __syncthreads();
            }
            if (t == 0) S.s_last = sl;
        } else {
            // no recurrence: every entry is independent
            for (int j = t; j < s.interval; j += BS) {
                double sl = S.s_last;
                table[j] = make_step(s, om, k0 + j, &sl);
                if (j == s.interval - 1) S.s_last = sl;
            }
            __syncthreads();
        }
    }
    if (t == 0) *st = S;
}

// ---------------------------------------------------------------------------
// infeasibility certificates (the paper is silent; see the decision in
// qp_decide.h): the drift z - z_restart, projected onto the dual cone (dy+) and
// onto the recession cone of X (dx+), and the products A dx+, Q dx+, A'dy+
// ---------------------------------------------------------------------------
__global__ void k_infeas_dirs(const double *__restrict__ x, const double *__restrict__ xrs,
                              const double *__restrict__ l, const double *__restrict__ u,
                              const double *__restrict__ y, const double *__restrict__ yrs,
                              const uint8_t *__restrict__ rt, double *__restrict__ dxh,
                              double *__restrict__ dyh, int64_t n, int64_t m,
                              const State *__restrict__ st) {
    if (st->done) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const bool lo = isfinite(l[k]), hi = isfinite(u[k]);
        double v = x[k] - xrs[k];
        if (lo && hi) v = 0.0;
        else if (lo && v < 0.0) v = 0.0;
        else if (hi && v > 0.0) v = 0.0;
        dxh[k] = v;
    }
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += stride) {
        const double v = y[k] - yrs[k];
        dyh[k] = (rt[k] == 1 && v < 0.0) ? 0.0 : v;
    }
}

struct InfRowArgs {
    const double *dxh, *dyh, *b, *dr;
    const uint8_t *rt;
    double *partials;  // [(nblk + nlr) * IA_NV]
};

__device__ __forceinline__ void infeas_row_contrib(int i, double s, const InfRowArgs &a,
                                                   double *cv) {
    const double viol = a.rt[i] == 1 ? (s < 0.0 ? -s : 0.0) : fabs(s);
    cv[IA_AVIOL] = viol / (a.dr ? a.dr[i] : 1.0);
    cv[IA_BDY] = a.b[i] * a.dyh[i];
}

__global__ __launch_bounds__(BS) void k_infeas_rows(Blocks bk, Csr A, InfRowArgs a,
                                                    const State *__restrict__ st) {
    if (st->done) return;
    __shared__ double prod[NNZ_BLK];
    __shared__ double scratch[BS / 64];
    const int bi = xcd_block(blockIdx.x, gridDim.x);
    const Block B = bk.blk[bi];
    const int t = threadIdx.x;
    {
        int cols[EPT];
        double vals[EPT], g[EPT];
        load_block<STREAM_A>(A.col, A.val, B.e0, B.e1, t, cols, vals);
#pragma unroll
        for (int i = 0; i < EPT; ++i) g[i] = a.dxh[cols[i]];
#pragma unroll
        for (int i = 0; i < EPT; ++i) prod[i * BS + t] = vals[i] * g[i];
    }
    __syncthreads();
    double cv[IA_NV] = {0.0, 0.0};
    const int lr = bk.lr[bi];
    if (lr < 0) {
        const int nrows = B.row1 - B.row0;
        const int G = lanes_per_row(nrows);
        const int rl = t / G, lane = t % G;
        double sum = 0.0;
        if (rl < nrows) {
            const int row = B.row0 + rl;
            const int e1 = A.rowptr[row + 1] - B.e0;
            for (int e = A.rowptr[row] - B.e0 + lane; e < e1; e += G) sum = sum + prod[e];
        }
        sum = group_sum(sum, G);
        if (rl < nrows && lane == 0) infeas_row_contrib(B.row0 + rl, sum, a, cv);
        block_reduce_write<IA_NV, 1>(cv, a.partials + (size_t)bi * IA_NV);
    } else {
        const double part = block_sum_lds(prod, B.e1 - B.e0, scratch);
        if (t == 0)
            for (int v = 0; v < IA_NV; ++v) a.partials[(size_t)bi * IA_NV + v] = 0.0;
        double tot;
        if (chunk_finish<1>(bk, bi, lr, &part, &tot)) {
            infeas_row_contrib(B.row0, tot, a, cv);
            for (int v = 0; v < IA_NV; ++v)
                a.partials[(size_t)(bk.nblk + lr) * IA_NV + v] = cv[v];
        }
    }
}

struct InfColArgs {
    const double *dxh, *dyh, *c, *l, *u, *dv;
    double *partials;  // [(nblk + nlr) * IP_NV]
};

// qd = (Q dx+)_j, nat = (-A'dy+)_j (P stores -A')
__device__ __forceinline__ void infeas_col_contrib(int j, double qd, double nat,
                                                   const InfColArgs &a, double *cv) {
    const double sv = a.dv ? a.dv[j] : 1.0;
    const double g = -nat;
    const double lj = a.l[j], uj = a.u[j];
    double viol = 0.0, supp = 0.0;
    if (g > 0.0) {
        if (isfinite(uj)) supp = uj * g;
        else viol = g;
    } else if (g < 0.0) {
        if (isfinite(lj)) supp = lj * g;
        else viol = -g;
    }
    cv[IP_QDX] = fabs(qd) / sv;
    cv[IP_GVIOL] = viol / sv;
    cv[IP_SUPP] = supp;
    cv[IP_CDX] = a.c[j] * a.dxh[j];
}

__global__ __launch_bounds__(BS) void k_infeas_cols(Blocks bk, Csr P, InfColArgs a,
                                                    const State *__restrict__ st, int32_t n) {
    if (st->done) return;
    __shared__ double prod[NNZ_BLK];
    __shared__ uint8_t isA[NNZ_BLK];
    __shared__ double scratch[BS / 64];
    const int bi = xcd_block(blockIdx.x, gridDim.x);
    const Block B = bk.blk[bi];
    const int t = threadIdx.x;
    {
        int cols[EPT];
        double vals[EPT], g[EPT];
        load_block<STREAM_P>(P.col, P.val, B.e0, B.e1, t, cols, vals);
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int cc = cols[i];
            g[i] = *(cc >= n ? a.dyh + (cc - n) : a.dxh + cc);
        }
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            prod[i * BS + t] = vals[i] * g[i];
            isA[i * BS + t] = cols[i] >= n;
        }
    }
    __syncthreads();
    double cv[IP_NV] = {0.0, 0.0, 0.0, 0.0};
    const int lr = bk.lr[bi];
    if (lr < 0) {
        const int nrows = B.row1 - B.row0;
        const int G = lanes_per_row(nrows);
        const int rl = t / G, lane = t % G;
        double q = 0.0, na = 0.0;
        if (rl < nrows) {
            const int row = B.row0 + rl;
            const int e1 = P.rowptr[row + 1] - B.e0;
            for (int e = P.rowptr[row] - B.e0 + lane; e < e1; e += G) {
                if (isA[e]) na = na + prod[e];
                else q = q + prod[e];
            }
        }
        q = group_sum(q, G);
        na = group_sum(na, G);
        if (rl < nrows && lane == 0) infeas_col_contrib(B.row0 + rl, q, na, a, cv);
        block_reduce_write<IP_NV, 2>(cv, a.partials + (size_t)bi * IP_NV);
    } else {
        // long row: the chunk's Q and -A' products summed separately
        double part[2];
        double qs = 0.0, as = 0.0;
        for (int k = t; k < B.e1 - B.e0; k += BS) {
            if (isA[k]) as = as + prod[k];
            else qs = qs + prod[k];
        }
        part[0] = block_sum_value(qs, scratch);
        part[1] = block_sum_value(as, scratch);
        if (t == 0)
            for (int v = 0; v < IP_NV; ++v) a.partials[(size_t)bi * IP_NV + v] = 0.0;
        double tot[2];
        if (chunk_finish<2>(bk, bi, lr, part, tot)) {
            infeas_col_contrib(B.row0, tot[0], tot[1], a, cv);
            for (int v = 0; v < IP_NV; ++v)
                a.partials[(size_t)(bk.nblk + lr) * IP_NV + v] = cv[v];
        }
    }
}

// folds the (already folded) per-block partials of both kernels into st->inf
__global__ __launch_bounds__(BS) void k_infeas_final(const double *__restrict__ pa, int32_t na,
                                                     const double *__restrict__ pp, int32_t np,
                                                     State *st) {
    if (st->done) return;
    __shared__ double red[INF_NV][BS];
    const int t = threadIdx.x;
    double acc[INF_NV] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = t; i < na; i += BS) {
        acc[INF_AVIOL] = nmax(acc[INF_AVIOL], pa[(size_t)i * IA_NV + IA_AVIOL]);
        acc[INF_BDY] = acc[INF_BDY] + pa[(size_t)i * IA_NV + IA_BDY];
    }
    for (int i = t; i < np; i += BS) {
        acc[INF_QDX] = nmax(acc[INF_QDX], pp[(size_t)i * IP_NV + IP_QDX]);
        acc[INF_GVIOL] = nmax(acc[INF_GVIOL], pp[(size_t)i * IP_NV + IP_GVIOL]);
        acc[INF_SUPP] = acc[INF_SUPP] + pp[(size_t)i * IP_NV + IP_SUPP];
        acc[INF_CDX] = acc[INF_CDX] + pp[(size_t)i * IP_NV + IP_CDX];
    }
    for (int v = 0; v < INF_NV; ++v) red[v][t] = acc[v];
    __syncthreads();
    for (int h = BS / 2; h >= 1; h >>= 1) {
        if (t < h)
            for (int v = 0; v < INF_NV; ++v) {
                const bool mx = v == INF_AVIOL || v == INF_QDX || v == INF_GVIOL;
                red[v][t] = mx ? nmax(red[v][t], red[v][t + h]) : red[v][t] + red[v][t + h];
            }
        __syncthreads();
    }
    if (t < INF_NV) st->inf[t] = red[t][0];
}

// ---------------------------------------------------------------------------
// restart application, initialisation, state reset
// ---------------------------------------------------------------------------
__global__ void k_apply(Vecs v, double *xmd_out, const State *__restrict__ st, int64_t n,
                        int64_t m) {
    if (!st->restart_flag) return;
    const int avg = st->cand;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        const double xc = avg ? v.xbar[j] : v.x[j];
        v.x[j] = xc;
        v.xbar[j] = xc;
        v.xt[j] = xc;
        xmd_out[j] = xc;
        v.xrs[j] = xc;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const double yc = avg ? v.ybar[i] : v.y[i];
        v.y[i] = yc;
        v.ybar[i] = yc;
        v.yrs[i] = yc;
    }
}

__device__ __forceinline__ double proj_box(double v, double lo, double hi) {
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

__global__ void k_init(Vecs v, const double *x0, const double *y0, int64_t n, int64_t m,
                       int pair) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        const double lo = v.l[j], hi = v.u[j];
        const double xc = proj_box(0.0, lo, hi);
        const double xw = x0 ? proj_box(x0[j], lo, hi) : xc;
        v.x[j] = xw;
        v.xbar[j] = pair ? xc : xw;
        v.xt[j] = xw;
        v.xmd[0][j] = xw;
        v.xrs[j] = xw;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        double yw = y0 ? y0[i] : 0.0;
        if (v.rt[i] == 1 && yw < 0.0) yw = 0.0;
        v.y[i] = yw;
        v.ybar[i] = pair ? 0.0 : yw;
        v.yrs[i] = yw;
    }
}

__global__ void k_fallback_apply(Vecs v, const State *__restrict__ st, int64_t n, int64_t m) {
    const int take = st->used_warm;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        const double xv = take ? v.x[j] : v.xbar[j];
        v.x[j] = xv;
        v.xbar[j] = xv;
        v.xt[j] = xv;
        v.xmd[0][j] = xv;
        v.xrs[j] = xv;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const double yv = take ? v.y[i] : v.ybar[i];
        v.y[i] = yv;
        v.ybar[i] = yv;
        v.yrs[i] = yv;
    }
}

__global__ void k_state_reset(State *st, double omega, int64_t max_iter) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    State S;
    S.omega = omega;
    S.r0 = 0.0;
    S.prev_cand = INFINITY;
    S.s_last = 0.0;
    S.r_cur = S.r_avg = 0.0;
    for (int p = 0; p < 2; ++p)
        for (int i = 0; i < 6; ++i) S.kkt[p][i] = 0.0;
    S.total = 0;
    S.k = 0;
    S.restarts = 0;
    S.kkt_evals = 0;
    S.done = 0;
    S.status = -1;
    S.cand = 0;
    S.restart_flag = 0;
    S.used_warm = 0;
    S.checks = 0;
    S.pad0 = S.pad1 = 0;
    (void)max_iter;
    *st = S;
}

// ---------------------------------------------------------------------------
// power iteration helpers
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void k_spmv_plain(Blocks bk, Csr M, const double *x,
                                                   const double *x2, int32_t split, double *y,
                                                   double sign2) {
    __shared__ double prod[NNZ_BLK];
    __shared__ double scratch[BS / 64];
    const int bi = xcd_block(blockIdx.x, gridDim.x);
    const Block B = bk.blk[bi];
    const int t = threadIdx.x;
    {
        int cols[EPT];
        double vals[EPT], g[EPT];
        load_block<STREAM_P>(M.col, M.val, B.e0, B.e1, t, cols, vals);
        // a missing operand contributes zero; its entries read a valid dummy address
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int cc = cols[i];
            const bool first = cc < split;
            const double *src = first ? (x ? x + cc : M.val) : (x2 ? x2 + (cc - split) : M.val);
            g[i] = *src;
        }
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const bool first = cols[i] < split;
            const double pr = first ? (x ? vals[i] * g[i] : 0.0)
                                    : (x2 ? sign2 * (vals[i] * g[i]) : 0.0);
            prod[i * BS + t] = pr;
        }
    }
    __syncthreads();
    const int lr = bk.lr[bi];
    if (lr < 0) {
        const int nrows = B.row1 - B.row0;
        const int G = lanes_per_row(nrows);
        const int rl = t / G, lane = t % G;
        double s = 0.0;
        if (rl < nrows) {
            const int row = B.row0 + rl;
            const int e1 = M.rowptr[row + 1] - B.e0;
            for (int e = M.rowptr[row] - B.e0 + lane; e < e1; e += G) s = s + prod[e];
        }
        s = group_sum(s, G);
        if (rl < nrows && lane == 0) y[B.row0 + rl] = s;
    } else {
        double part = block_sum_lds(prod, B.e1 - B.e0, scratch);
        double tot;
        if (chunk_finish<1>(bk, bi, lr, &part, &tot)) y[B.row0] = tot;
    }
}

int dot_nparts(int64_t n) {
    int64_t p = (n + 8191) / 8192;
    if (p < 1) p = 1;
    if (p > 1024) p = 1024;
    return (int)p;
}

__global__ __launch_bounds__(BS) void k_dot_partials(const double *a, const double *b, int64_t n,
                                                     double *partials, int32_t nparts) {
    __shared__ double scratch[BS / 64];
    const int64_t chunk = (n + nparts - 1) / nparts;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += BS) s = s + a[i] * b[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int w = 0; w < BS / 64; ++w) acc = acc + scratch[w];
        partials[blockIdx.x] = acc;
    }
}

__global__ void k_div(double *dst, const double *src, int64_t n, double den) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i] / den;
}

__global__ void k_fill(double *dst, int64_t n, double value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = value;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

void launch_dual(hipStream_t s, const Blocks &bk, const Csr &A, const Vecs &v, const Step *step,
                 const State *st) {
    if (bk.nblk == 0) return;
    hipLaunchKernelGGL(k_dual, dim3(bk.nblk), dim3(BS), 0, s, bk, A, v.xt, v.y, v.ybar, v.b, v.rt,
                       step, st);
}

void launch_primal(hipStream_t s, const Blocks &bk, const Csr &P, const Vecs &v, int md_in,
                   const Step *step, const State *st, int64_t n) {
    if (bk.nblk == 0) return;
    const PrimalArgs a = primal_args(v, md_in);
    hipLaunchKernelGGL(k_primal, dim3(bk.nblk), dim3(BS), 0, s, bk, P, a, step, st, (int32_t)n);
}

void launch_kkt_rows(hipStream_t s, const Blocks &bk, const Csr &A, const Vecs &v,
                     double *partials, const State *st) {
    if (bk.nblk == 0) return;
    KktRowArgs a;
    a.x = v.x;
    a.xbar = v.xbar;
    a.y = v.y;
    a.ybar = v.ybar;
    a.yrs = v.yrs;
    a.b = v.b;
    a.rt = v.rt;
    a.dr = v.dr;
    a.partials = partials;
    hipLaunchKernelGGL(k_kkt_rows, dim3(bk.nblk), dim3(BS), 0, s, bk, A, a, st);
}

void launch_kkt_cols(hipStream_t s, const Blocks &bk, const Csr &P, const Vecs &v,
                     double *partials, const State *st, int64_t n) {
    if (bk.nblk == 0) return;
    KktColArgs a;
    a.x = v.x;
    a.xbar = v.xbar;
    a.y = v.y;
    a.ybar = v.ybar;
    a.xrs = v.xrs;
    a.c = v.c;
    a.l = v.l;
    a.u = v.u;
    a.dv = v.dv;
    a.partials = partials;
    hipLaunchKernelGGL(k_kkt_cols, dim3(bk.nblk), dim3(BS), 0, s, bk, P, a, st, (int32_t)n);
}

void launch_infeas(hipStream_t s, const Blocks &bkA, const Csr &A, const Blocks &bkP,
                   const Csr &P, const Vecs &v, double *dxh, double *dyh, double *part_a,
                   int32_t nslotA, double *part_p, int32_t nslotP, State *st, int64_t n,
                   int64_t m) {
    hipLaunchKernelGGL(k_infeas_dirs, dim3(grid_for(n > m ? n : m)), dim3(256), 0, s, v.x, v.xrs,
                       v.l, v.u, v.y, v.yrs, v.rt, dxh, dyh, n, m, st);
    if (bkA.nblk > 0) {
        InfRowArgs a;
        a.dxh = dxh;
        a.dyh = dyh;
        a.b = v.b;
        a.dr = v.dr;
        a.rt = v.rt;
        a.partials = part_a;
        hipLaunchKernelGGL(k_infeas_rows, dim3(bkA.nblk), dim3(BS), 0, s, bkA, A, a, st);
    }
    if (bkP.nblk > 0) {
        InfColArgs a;
        a.dxh = dxh;
        a.dyh = dyh;
        a.c = v.c;
        a.l = v.l;
        a.u = v.u;
        a.dv = v.dv;
        a.partials = part_p;
        hipLaunchKernelGGL(k_infeas_cols, dim3(bkP.nblk), dim3(BS), 0, s, bkP, P, a, st,
                           (int32_t)n);
    }
    // fold many block partials first (same scheme as the KKT reduction)
    auto fold = [&](double *part, int32_t nslot, int nv) -> int32_t {
        if (nslot <= 2 * BS) return nslot;
        const int32_t per = std::max<int32_t>(2 * BS, (nslot + FOLD_SLOTS - 1) / FOLD_SLOTS);
        const int32_t g = (nslot + per - 1) / per;
        double *out = part + (size_t)nslot * nv;
        if (nv == IA_NV)
            hipLaunchKernelGGL((k_fold_slots<IA_NV, 1>), dim3(g), dim3(BS), 0, s, part, nslot,
                               per, out, st);
        else
            hipLaunchKernelGGL((k_fold_slots<IP_NV, 2>), dim3(g), dim3(BS), 0, s, part, nslot,
                               per, out, st);
        return -g;
    };
    const int32_t fa = fold(part_a, nslotA, IA_NV), fp = fold(part_p, nslotP, IP_NV);
    const double *pa = fa < 0 ? part_a + (size_t)nslotA * IA_NV : part_a;
    const double *pp = fp < 0 ? part_p + (size_t)nslotP * IP_NV : part_p;
    hipLaunchKernelGGL(k_infeas_final, dim3(1), dim3(BS), 0, s, pa, fa < 0 ? -fa : fa, pp,
                       fp < 0 ? -fp : fp, st);
}

// The partial buffers hold FOLD_SLOTS spare slots after the nslot block partials: many
// partials are first folded there by up to FOLD_SLOTS workgroups, so the single-workgroup
// decision reads few.
void launch_decide(hipStream_t s, int mode, double *partA, int32_t nslotA, double *partP,
                   int32_t nslotP, State *st, Step *table, const DevSettings &ds, int32_t len) {
    auto fold = [&](double *part, int32_t nslot, int nv) -> int32_t {
        if (nslot <= 2 * BS) return 0;
        const int32_t per = std::max<int32_t>(2 * BS, (nslot + FOLD_SLOTS - 1) / FOLD_SLOTS);
        const int32_t g = (nslot + per - 1) / per;
        double *out = part + (size_t)nslot * nv;
        if (nv == RA_NV)
            hipLaunchKernelGGL((k_fold_slots<RA_NV, 4>), dim3(g), dim3(BS), 0, s, part, nslot, per,
                               out, st);
        else
            hipLaunchKernelGGL((k_fold_slots<RP_NV, 6>), dim3(g), dim3(BS), 0, s, part, nslot, per,
                               out, st);
        return g;
    };
    const int32_t gA = fold(partA, nslotA, RA_NV);
    const int32_t gP = fold(partP, nslotP, RP_NV);
    const double *pa = gA ? partA + (size_t)nslotA * RA_NV : partA;
    const double *pp = gP ? partP + (size_t)nslotP * RP_NV : partP;
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(BS), 0, s, mode, pa, gA ? gA : nslotA, pp,
                       gP ? gP : nslotP, st, table, ds, len);
}

void launch_apply(hipStream_t s, const Vecs &v, int md_out, const State *st, int64_t n,
                  int64_t m) {
    hipLaunchKernelGGL(k_apply, dim3(grid_for(n > m ? n : m)), dim3(256), 0, s, v, v.xmd[md_out],
                       st, n, m);
}

void launch_init(hipStream_t s, const Vecs &v, const double *x0, const double *y0, int64_t n,
                 int64_t m, int pair_with_cold) {
    hipLaunchKernelGGL(k_init, dim3(grid_for(n > m ? n : m)), dim3(256), 0, s, v, x0, y0, n, m,
                       pair_with_cold);
}

void launch_fallback_apply(hipStream_t s, const Vecs &v, const State *st, int64_t n, int64_t m) {
    hipLaunchKernelGGL(k_fallback_apply, dim3(grid_for(n > m ? n : m)), dim3(256), 0, s, v, st, n,
                       m);
}

void launch_state_reset(hipStream_t s, State *st, double omega, int64_t max_iter) {
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, st, omega, max_iter);
}

void launch_spmv_plain(hipStream_t s, const Blocks &bk, const Csr &M, const double *x,
                       const double *x2, int64_t split, double *y, double sign2) {
    if (bk.nblk == 0) return;
    hipLaunchKernelGGL(k_spmv_plain, dim3(bk.nblk), dim3(BS), 0, s, bk, M, x, x2, (int32_t)split,
                       y, sign2);
}

void launch_dot_partials(hipStream_t s, const double *a, const double *b, int64_t n,
                         double *partials, int32_t nparts) {
    hipLaunchKernelGGL(k_dot_partials, dim3(nparts), dim3(BS), 0, s, a, b, n, partials, nparts);
}

void launch_div(hipStream_t s, double *dst, const double *src, int64_t n, double den) {
    hipLaunchKernelGGL(k_div, dim3(grid_for(n)), dim3(256), 0, s, dst, src, n, den);
}

void launch_fill(hipStream_t s, double *dst, int64_t n, double value) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, dst, n, value);
}

}  // namespace qpk

// ---------------------------------------------------------------------------
// column-panel phases: per-panel partial row sums, then a combine + epilogue
// ---------------------------------------------------------------------------
namespace qpk {

// chunk partials (W <= 4 values) of a long row in a panel (same protocol as chunk_finish)
template <int W>
__device__ bool panel_chunk_finish_w(const Panels &pn, int bi, int lr, const double *part,
                                     double *tot) {
    return finish_chunks<W>(pn.lr_count, pn.lr_first, pn.lr_nchunk, pn.lr_partial, bi, lr, part,
                            tot);
}

__device__ bool panel_chunk_finish(const Panels &pn, int bi, int lr, double part, double *tot) {
    return panel_chunk_finish_w<1>(pn, bi, lr, &part, tot);
}

// PHASE 0: rows of A (dual phase, ordinary loads); PHASE 1: rows of P (primal phase,
// non-temporal loads).  Gathers v1[c] for c < split and v2[c - split] otherwise.
//
// Persistent and software-pipelined: workgroup w walks the slots w, w + nwg, w + 2 nwg,
// ... of the block map (nwg a multiple of 8, so every slot it takes belongs to its own
// XCD).  For the current block it issues the gathers, then the loads of the current
// block's values and of the NEXT block's column indices, so the matrix stream and the
// random gathers of one workgroup are in flight together.  (With one block per workgroup
// the blocks that start together stream together and then gather together: measured on
// the large random QP, the stream alone took 42 us and the gathers alone about 75 us, and
// the kernel took their sum.)  When there is no next block an empty range is loaded,
// which reads the block's first entry and yields nothing.
template <int SRC>
__device__ __forceinline__ void load_cols(const int32_t *__restrict__ col, int e0, int e1, int t,
                                          int (&cols)[EPT]) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = e0 + i * BS + t;
        const int ee = e < e1 ? e : e0;
        cols[i] = SRC == STREAM_P ? __builtin_nontemporal_load(&col[ee]) : col[ee];
    }
}

// values of entries e0 + i*BS + t; lanes past e1 read entry e0 (their products are
// masked where they are formed, so no loaded value is consumed before its use)
template <int SRC>
__device__ __forceinline__ void load_vals(const double *__restrict__ val, int e0, int e1, int t,
                                          double (&vals)[EPT]) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = e0 + i * BS + t;
        const int ee = e < e1 ? e : e0;
        vals[i] = SRC == STREAM_P ? __builtin_nontemporal_load(&val[ee]) : val[ee];
    }
}

// The block map and descriptors are read-only during the launch and passed as restrict
// kernel arguments, so the compiler reads them with scalar loads: waiting for them does
// not wait for the vector loads (gathers, stream) in flight.
__device__ __forceinline__ int next_slot(const int32_t *__restrict__ map, int grid, int idx,
                                         int nwg) {
    while (idx < grid && map[idx] < 0) idx += nwg;
    return idx;
}

template <int PHASE>
__global__ __launch_bounds__(BS) void k_panel_spmv(Panels pn, const int32_t *__restrict__ map,
                                                   const PBlock *__restrict__ blk,
                                                   const double *__restrict__ v1,
                                                   const double *__restrict__ v2, int32_t split,
                                                   int32_t nwg, const State *__restrict__ st) {
    if (st->done) return;
    constexpr int SRC = PHASE == 0 ? STREAM_A : STREAM_P;
    __shared__ double prod[NNZ_BLK];
    __shared__ double scratch[BS / 64];
    const int t = threadIdx.x;
    const int grid = pn.grid;
    int idx = next_slot(map, grid, blockIdx.x, nwg);
    if (idx >= grid) return;
    int bi = map[idx];
    PBlock B = blk[bi];
    int cols[EPT];
    load_cols<SRC>(pn.col, B.e0, B.e1, t, cols);
    while (true) {
        // next block's descriptor first: its loads complete together with this block's
        // column indices, which the gathers need anyway
        const int nidx = next_slot(map, grid, idx + nwg, nwg);
        const bool more = nidx < grid;
        const int nbi = more ? map[nidx] : bi;
        const PBlock NB = blk[nbi];
        __builtin_amdgcn_sched_barrier(0);
        double g[EPT];
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int cc = cols[i];
            if (PHASE == 0)
                g[i] = v1[cc];
            else
                g[i] = *(cc < split ? v1 + cc : v2 + (cc - split));
        }
        __builtin_amdgcn_sched_barrier(0);  // the gathers are issued before the stream loads
        double vals[EPT];
        load_vals<SRC>(pn.val, B.e0, B.e1, t, vals);
        int ncols[EPT];
        load_cols<SRC>(pn.col, NB.e0, more ? NB.e1 : NB.e0, t, ncols);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < EPT; ++i)
            prod[i * BS + t] = B.e0 + i * BS + t < B.e1 ? vals[i] * g[i] : 0.0;
        __syncthreads();
        const int32_t *rp = pn.rowptr + (size_t)B.panel * (size_t)(pn.R + 1);
        double *out = pn.part + (size_t)B.panel * (size_t)pn.R;
        if (B.lr < 0) {
            const int nrows = B.row1 - B.row0;
            if (nrows >= BS) {
                for (int rl = t; rl < nrows; rl += BS) {
                    const int row = B.row0 + rl;
                    const int e1 = rp[row + 1] - B.e0;
                    double s = 0.0;
                    for (int e = rp[row] - B.e0; e < e1; ++e) s = s + prod[e];
                    out[row] = s;
                }
            } else {
                const int G = lanes_per_row(nrows);
                const int rl = t / G, lane = t % G;
                double s = 0.0;
                if (rl < nrows) {
                    const int row = B.row0 + rl;
                    const int e1 = rp[row + 1] - B.e0;
                    for (int e = rp[row] - B.e0 + lane; e < e1; e += G) s = s + prod[e];
                }
                s = group_sum(s, G);
                if (rl < nrows && lane == 0) out[B.row0 + rl] = s;
            }
        } else {
            const double part = block_sum_lds(prod, B.e1 - B.e0, scratch);
            double tot;
            if (panel_chunk_finish(pn, bi, B.lr, part, &tot)) out[B.row0] = tot;
        }
        if (!more) break;
        __syncthreads();  // prod is rewritten by the next block
        idx = nidx;
        bi = nbi;
        B = NB;
#pragma unroll
        for (int i = 0; i < EPT; ++i) cols[i] = ncols[i];
    }
}

__global__ __launch_bounds__(256) void k_dual_combine(const double *__restrict__ part, int32_t np,
                                                      int64_t m, double *__restrict__ y,
                                                      double *__restrict__ ybar,
                                                      const double *__restrict__ b,
                                                      const uint8_t *__restrict__ rt,
                                                      const Step *__restrict__ step,
                                                      const State *__restrict__ st) {
    if (st->done) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double s = part[i];
    for (int k = 1; k < np; ++k) s = s + part[(size_t)k * m + i];
    dual_epilogue((int)i, s, y, ybar, b, rt, step->d, step->w);
}

__global__ __launch_bounds__(256) void k_primal_combine(const double *__restrict__ part,
                                                        int32_t np, int64_t n, PrimalArgs a,
                                                        const Step *__restrict__ step,
                                                        const State *__restrict__ st) {
    if (st->done) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = part[j];
    for (int k = 1; k < np; ++k) s = s + part[(size_t)k * n + j];
    primal_epilogue((int)j, s, a, step->p, step->w, step->theta_next, step->w_next);
}

// KKT products on the column panels.  KIND 0 (rows of A): sums of A x and A x-bar;
// KIND 1 (rows of P = [Q | -A']): sums of Q x, -A'y, Q x-bar, -A'y-bar, the column
// deciding the part.  Panel k's sums of row r go to kpart[(w*np + k)*R + r] for output w;
// the combine kernels add the panels in order and evaluate the rows' KKT terms.
//
// Both points are gathered at once from the pairs zz[c] = (x_c, x-bar_c) (c < n) and
// zz[n + i] = (y_i, y-bar_i), written just before by k_interleave: one 16-byte random
// load per nonzero instead of two 8-byte ones, half the L2 requests of the gathers that
// bound these kernels; the column indexes the pairs directly.
__global__ void k_interleave(const double *__restrict__ x, const double *__restrict__ xbar,
                             const double *__restrict__ y, const double *__restrict__ ybar,
                             int64_t n, int64_t m, double2 *__restrict__ zz,
                             const State *__restrict__ st) {
    if (st->done) return;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n + m;
         j += (int64_t)gridDim.x * blockDim.x)
        zz[j] = j < n ? make_double2(x[j], xbar[j]) : make_double2(y[j - n], ybar[j - n]);
}

template <int KIND>
__global__ __launch_bounds__(BS) void k_panel_kkt(Panels pn, const double2 *__restrict__ zz,
                                                  int32_t n, double *__restrict__ kpart,
                                                  const State *__restrict__ st) {
    if (st->done) return;
    const int bi = pn.map[blockIdx.x];
    if (bi < 0) return;
    constexpr int W = KIND == 0 ? 2 : 4;
    __shared__ double prod0[NNZ_BLK];
    __shared__ double prod1[NNZ_BLK];
    __shared__ uint8_t isA[KIND == 0 ? 1 : NNZ_BLK];
    __shared__ double scratch[BS / 64];
    const PBlock B = pn.blk[bi];
    const int t = threadIdx.x;
    {
        int cols[EPT];
        double vals[EPT], g0[EPT], g1[EPT];
        load_block<KIND == 0 ? STREAM_A : STREAM_P>(pn.col, pn.val, B.e0, B.e1, t, cols, vals);
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const double2 g = zz[cols[i]];
            g0[i] = g.x;
            g1[i] = g.y;
        }
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            prod0[i * BS + t] = vals[i] * g0[i];
            prod1[i * BS + t] = vals[i] * g1[i];
            if (KIND == 1) isA[i * BS + t] = cols[i] >= n;
        }
    }
    __syncthreads();
    const int32_t *rp = pn.rowptr + (size_t)B.panel * (size_t)(pn.R + 1);
    const size_t stride = (size_t)pn.np * (size_t)pn.R;
    double *out = kpart + (size_t)B.panel * (size_t)pn.R;
    if (B.lr < 0) {
        const int nrows = B.row1 - B.row0;
        const int G = nrows >= BS ? 1 : lanes_per_row(nrows);
        for (int rl0 = 0; rl0 < nrows; rl0 += BS / G) {
            const int rl = rl0 + t / G, lane = t % G;
            double sv[W];
#pragma unroll
            for (int w = 0; w < W; ++w) sv[w] = 0.0;
            if (rl < nrows) {
                const int row = B.row0 + rl;
                const int e1 = rp[row + 1] - B.e0;
                for (int e = rp[row] - B.e0 + lane; e < e1; e += G) {
                    if (KIND == 0) {
                        sv[0] = sv[0] + prod0[e];
                        sv[1] = sv[1] + prod1[e];
                    } else if (isA[e]) {
                        sv[1] = sv[1] + prod0[e];
                        sv[3] = sv[3] + prod1[e];
                    } else {
                        sv[0] = sv[0] + prod0[e];
                        sv[2] = sv[2] + prod1[e];
                    }
                }
            }
#pragma unroll
            for (int w = 0; w < W; ++w) sv[w] = group_sum(sv[w], G);
            if (rl < nrows && lane == 0)
                for (int w = 0; w < W; ++w) out[w * stride + B.row0 + rl] = sv[w];
        }
    } else {
        double ps[W];
        if (KIND == 0) {
            ps[0] = block_sum_lds(prod0, B.e1 - B.e0, scratch);
            ps[1] = block_sum_lds(prod1, B.e1 - B.e0, scratch);
        } else {
            double q0 = 0.0, a0 = 0.0, q1 = 0.0, a1 = 0.0;
            for (int e = t; e < B.e1 - B.e0; e += BS) {
                if (isA[e]) {
                    a0 = a0 + prod0[e];
                    a1 = a1 + prod1[e];
                } else {
                    q0 = q0 + prod0[e];
                    q1 = q1 + prod1[e];
                }
            }
            ps[0] = block_sum_value(q0, scratch);
            ps[1] = block_sum_value(a0, scratch);
            ps[W > 2 ? 2 : 0] = block_sum_value(q1, scratch);
            ps[W > 3 ? 3 : 0] = block_sum_value(a1, scratch);
        }
        double tot[W];
        if (panel_chunk_finish_w<W>(pn, bi, B.lr, ps, tot))
            for (int w = 0; w < W; ++w) out[w * stride + B.row0] = tot[w];
    }
}

__global__ __launch_bounds__(BS) void k_kkt_rows_combine(const double *__restrict__ kpart,
                                                         int32_t np, int64_t m, KktRowArgs a,
                                                         const State *__restrict__ st) {
    if (st->done) return;
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    double cv[RA_NV];
    for (int v = 0; v < RA_NV; ++v) cv[v] = 0.0;
    if (i < m) {
        double s0 = kpart[i], s1 = kpart[(size_t)np * m + i];
        for (int k = 1; k < np; ++k) {
            s0 = s0 + kpart[(size_t)k * m + i];
            s1 = s1 + kpart[(size_t)(np + k) * m + i];
        }
        kkt_row_contrib((int)i, s0, s1, a, cv);
    }
    block_reduce_write<RA_NV, 4>(cv, a.partials + (size_t)blockIdx.x * RA_NV);
}

__global__ __launch_bounds__(BS) void k_kkt_cols_combine(const double *__restrict__ kpart,
                                                         int32_t np, int64_t n, KktColArgs a,
                                                         const State *__restrict__ st) {
    if (st->done) return;
    const int64_t j = (int64_t)blockIdx.x * BS + threadIdx.x;
    double cv[RP_NV];
    for (int v = 0; v < RP_NV; ++v) cv[v] = 0.0;
    if (j < n) {
        const size_t sn = (size_t)np * n;
        double q[2] = {kpart[j], kpart[2 * sn + j]};
        double na[2] = {kpart[sn + j], kpart[3 * sn + j]};
        for (int k = 1; k < np; ++k) {
            const size_t o = (size_t)k * n + j;
            q[0] = q[0] + kpart[o];
            na[0] = na[0] + kpart[sn + o];
            q[1] = q[1] + kpart[2 * sn + o];
            na[1] = na[1] + kpart[3 * sn + o];
        }
        kkt_col_contrib((int)j, q, na, a, cv);
    }
    block_reduce_write<RP_NV, 6>(cv, a.partials + (size_t)blockIdx.x * RP_NV);
}

// Persistent workgroups of the panel phases: as many as can be resident at once (the
// occupancy both phase kernels reach, times the CU count), a multiple of 8 so each keeps
// to one XCD, at most the map size.
int32_t panel_resident_workgroups(int device) {
    int per_cu0 = 0, per_cu1 = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu0, k_panel_spmv<0>, BS, 0) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu1, k_panel_spmv<1>, BS, 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    const int per_cu = per_cu0 < per_cu1 ? per_cu0 : per_cu1;
    return (per_cu * cus) / 8 * 8;
}

static int32_t panel_workgroups(const Panels &pn) {
    return pn.grid < pn.nwg ? pn.grid : pn.nwg;
}

void launch_interleave(hipStream_t s, const Vecs &v, const State *st, int64_t n, int64_t m) {
    hipLaunchKernelGGL(k_interleave, dim3(grid_for(n + m)), dim3(256), 0, s, (const double *)v.x,
                       (const double *)v.xbar, (const double *)v.y, (const double *)v.ybar, n, m,
                       v.zz, st);
}

int32_t launch_kkt_rows_panels(hipStream_t s, const Panels &pn, const Vecs &v, double *kpart,
                               double *partials, const State *st, int64_t n, int64_t m) {
    if (m == 0) return 0;
    if (pn.grid > 0)
        hipLaunchKernelGGL(k_panel_kkt<0>, dim3(pn.grid), dim3(BS), 0, s, pn,
                           (const double2 *)v.zz, (int32_t)n, kpart, st);
    KktRowArgs a;
    a.x = v.x;
    a.xbar = v.xbar;
    a.y = v.y;
    a.ybar = v.ybar;
    a.yrs = v.yrs;
    a.b = v.b;
    a.rt = v.rt;
    a.dr = v.dr;
    a.partials = partials;
    const int32_t g = (int32_t)((m + BS - 1) / BS);
    hipLaunchKernelGGL(k_kkt_rows_combine, dim3(g), dim3(BS), 0, s, (const double *)kpart,
                       pn.np, m, a, st);
    return g;
}

int32_t launch_kkt_cols_panels(hipStream_t s, const Panels &pn, const Vecs &v, double *kpart,
                               double *partials, const State *st, int64_t n) {
    if (pn.grid > 0)
        hipLaunchKernelGGL(k_panel_kkt<1>, dim3(pn.grid), dim3(BS), 0, s, pn,
                           (const double2 *)v.zz, (int32_t)n, kpart, st);
    KktColArgs a;
    a.x = v.x;
    a.xbar = v.xbar;
    a.y = v.y;
    a.ybar = v.ybar;
    a.xrs = v.xrs;
    a.c = v.c;
    a.l = v.l;
    a.u = v.u;
    a.dv = v.dv;
    a.partials = partials;
    const int32_t g = (int32_t)((n + BS - 1) / BS);
    hipLaunchKernelGGL(k_kkt_cols_combine, dim3(g), dim3(BS), 0, s, (const double *)kpart,
                       pn.np, n, a, st);
    return g;
}

void launch_dual_panels(hipStream_t s, const Panels &pn, const Vecs &v, int64_t n,
                        const Step *step, const State *st) {
    if (pn.R == 0) return;
    if (pn.grid > 0)
        hipLaunchKernelGGL(k_panel_spmv<0>, dim3(panel_workgroups(pn)), dim3(BS), 0, s, pn,
                           pn.map, pn.blk, (const double *)v.xt, (const double *)nullptr,
                           (int32_t)n, panel_workgroups(pn), st);
    hipLaunchKernelGGL(k_dual_combine, dim3((unsigned)((pn.R + 255) / 256)), dim3(256), 0, s,
                       (const double *)pn.part, pn.np, pn.R, v.y, v.ybar, v.b, v.rt, step, st);
}

void launch_primal_panels(hipStream_t s, const Panels &pn, const Vecs &v, int md_in, int64_t n,
                          const Step *step, const State *st) {
    const PrimalArgs a = primal_args(v, md_in);
    if (pn.grid > 0)
        hipLaunchKernelGGL(k_panel_spmv<1>, dim3(panel_workgroups(pn)), dim3(BS), 0, s, pn,
                           pn.map, pn.blk, (const double *)v.xmd[md_in], (const double *)v.y,
                           (int32_t)n, panel_workgroups(pn), st);
    hipLaunchKernelGGL(k_primal_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (const double *)pn.part, pn.np, n, a, step, st);
}

}  // namespace qpk
