// qp_scale.hip -- diagonal preconditioning on the device (Lu & Yang, arXiv 2311.07710,
// Sec. 5 "Preprocessing", used unchanged by the Sec. 6 solver): one symmetric
// diagonal scaling d = (D2, D1) of K = [[Q, A'], [A, 0]] built from Ruiz steps
// (row maxima), an l2 step (row 2-norms) and a Pock-Chambolle step with alpha = 1
// (row 1-norms; K is symmetric, so its column sums equal its row sums).
//
// K is never formed: its variable row j is row j of P = [Q | -A'] (Q's row in stored
// order, then A's column j by increasing row index, exactly how P is assembled) and
// its constraint row i is row i of A.  Each step computes one statistic per row of K
// (one wavefront per row: lane-strided partial results combined by a fixed butterfly,
// so sums are deterministic), turns it into f = 1/sqrt(stat) (1 for an empty row),
// multiplies d by f and rescales every stored value as k * (f_row * f_col).  The
// product f_row * f_col is commutative, so the copy of A inside P stays the exact
// negative of A.
//
// Batches: rows of all instances are concatenated, columns are local to the
// instance; a row finds its instance by binary search over the offset arrays.
#include <math.h>

#include "qp_internal.h"

namespace qpk {

namespace {

struct ScaleView {
    int64_t n, m;                          // variables / constraint rows (all instances)
    const int32_t *a_rowptr, *a_col;       // A: m rows
    double *a_val;
    const int32_t *p_rowptr, *p_col;       // P = [Q | -A']: n rows
    double *p_val;
    const int32_t *var_off, *row_off;      // batch offsets [count+1] or nullptr
    int32_t count;
    double *st, *f, *d;                    // [n+m] statistic, step factor, cumulative scale
};

// instance of a global index (offsets off[0..count], increasing)
__device__ __forceinline__ int find_instance(const int32_t *off, int32_t count, int64_t g) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ double stat_add(int kind, double a, double v) {
    v = fabs(v);
    if (kind == SCALE_MAX) return v > a ? v : a;
    if (kind == SCALE_L2) return a + v * v;
    return a + v;
}

constexpr int WAVES = 4;  // rows per 256-thread workgroup, one wavefront each

__global__ __launch_bounds__(64 * WAVES) void k_row_stats(ScaleView s, int kind) {
    const int64_t r = (int64_t)blockIdx.x * WAVES + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= s.n + s.m) return;
    const int32_t *rp = r < s.n ? s.p_rowptr : s.a_rowptr;
    const double *val = r < s.n ? s.p_val : s.a_val;
    const int64_t row = r < s.n ? r : r - s.n;
    double a = 0.0;
    for (int32_t e = rp[row] + lane; e < rp[row + 1]; e += 64) a = stat_add(kind, a, val[e]);
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(a, off, 64);
        a = kind == SCALE_MAX ? (o > a ? o : a) : a + o;
    }
    if (lane != 0) return;
    if (kind == SCALE_L2) a = sqrt(a);
    s.st[r] = a;
    const double fr = a > 0.0 ? 1.0 / sqrt(a) : 1.0;
    s.f[r] = fr;
    s.d[r] = s.d[r] * fr;
}

__global__ __launch_bounds__(64 * WAVES) void k_apply_scale(ScaleView s) {
    const int64_t r = (int64_t)blockIdx.x * WAVES + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= s.n + s.m) return;
    if (r < s.n) {
        // row r of P: local columns < n_i address variables, the rest constraint rows
        int64_t vb = 0, rb = 0, nl = s.n;
        if (s.var_off) {
            const int q = find_instance(s.var_off, s.count, r);
            vb = s.var_off[q];
            rb = s.row_off[q];
            nl = s.var_off[q + 1] - vb;
        }
        const double fr = s.f[r];
        for (int32_t e = s.p_rowptr[r] + lane; e < s.p_rowptr[r + 1]; e += 64) {
            const int64_t c = s.p_col[e];
            const double fc = c < nl ? s.f[vb + c] : s.f[s.n + rb + (c - nl)];
            s.p_val[e] = s.p_val[e] * (fr * fc);
        }
    } else {
        const int64_t i = r - s.n;
        int64_t vb = 0;
        if (s.row_off) vb = s.var_off[find_instance(s.row_off, s.count, i)];
        const double fr = s.f[r];
        for (int32_t e = s.a_rowptr[i] + lane; e < s.a_rowptr[i + 1]; e += 64)
            s.a_val[e] = s.a_val[e] * (fr * s.f[vb + s.a_col[e]]);
    }
}

__global__ void k_fill_one(double *d, int64_t len) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < len) d[r] = 1.0;
}

__global__ void k_scale_pair(double *__restrict__ out, const double *__restrict__ in,
                             const double *__restrict__ d, int64_t len, int divide) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) out[e] = divide ? in[e] / d[e] : in[e] * d[e];
}

unsigned grid_of(int64_t len) { return (unsigned)((len + 255) / 256); }

}  // namespace

int precondition_device(hipStream_t s, const ScaleInput &in, double *work, double *d) {
    const int64_t R = in.n + in.m;
    if (R == 0) return 0;
    ScaleView v;
    v.n = in.n;
    v.m = in.m;
    v.a_rowptr = in.a_rowptr;
    v.a_col = in.a_col;
    v.a_val = in.a_val;
    v.p_rowptr = in.p_rowptr;
    v.p_col = in.p_col;
    v.p_val = in.p_val;
    v.var_off = in.var_off;
    v.row_off = in.row_off;
    v.count = in.count;
    v.st = work;
    v.f = work + R;
    v.d = d;
    (void)hipGetLastError();  // launch errors are read below: drop any earlier one
    hipLaunchKernelGGL(k_fill_one, dim3(grid_of(R)), dim3(256), 0, s, d, R);
    const unsigned rows_grid = (unsigned)((R + WAVES - 1) / WAVES);
    auto step = [&](int kind) {
        hipLaunchKernelGGL(k_row_stats, dim3(rows_grid), dim3(64 * WAVES), 0, s, v, kind);
        hipLaunchKernelGGL(k_apply_scale, dim3(rows_grid), dim3(64 * WAVES), 0, s, v);
    };
    for (int t = 0; t < in.ruiz_iters; ++t) step(SCALE_MAX);
    if (in.l2) step(SCALE_L2);
    if (in.pc) step(SCALE_SUM);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

void launch_scale_pair(hipStream_t s, double *out, const double *in, const double *d,
                       int64_t len, int divide) {
    if (len > 0)
        hipLaunchKernelGGL(k_scale_pair, dim3(grid_of(len)), dim3(256), 0, s, out, in, d, len,
                           divide);
}

}  // namespace qpk
