// qp_api.cpp -- host side of the C-ABI declared in include/qp.h.
//
// qp_create validates the CSR input, builds the device layouts (A as CSR and
// P = [Q | -A'] as one CSR matrix whose A' entries appear in increasing row
// order of A), partitions the rows of both into nnz-balanced blocks, uploads
// everything and estimates ||A||_2, ||Q||_2 by power iteration.
//
// qp_solve runs rAPDHG (Algorithm 1 inner loop, Sec. 6 restarts/step sizes/
// primal weight, Sec. 5 relKKT termination) entirely on the device: one check
// interval = `interval` x (dual kernel, primal kernel) + KKT kernels + the
// single-workgroup decision kernel + the restart kernel, replayed as one
// captured hipGraph.  The host only enqueues intervals (two in flight) and
// reads a small status record per interval.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <string>
#include <thread>
#include <vector>

#include "../../include/qp.h"
#include "qp_batch.h"
#include "qp_host.h"
#include "qp_internal.h"

using namespace qpk;

namespace qph {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace qph

using qph::DevMem;
using qph::fail;
using qph::now_s;

namespace {

struct HostPartition {
    std::vector<Block> blk;
    std::vector<int32_t> lr, lr_first, lr_nchunk;
};

// Group consecutive rows into blocks of <= NNZ_BLK nonzeros and <= BS rows; a
// longer row becomes its own sequence of NNZ_BLK-sized chunks.
HostPartition partition_rows(const int32_t *rowptr, int64_t nrows) {
    HostPartition hp;
    int64_t r = 0;
    while (r < nrows) {
        const int64_t len = (int64_t)rowptr[r + 1] - rowptr[r];
        if (len > NNZ_BLK) {
            const int32_t nch = (int32_t)((len + NNZ_BLK - 1) / NNZ_BLK);
            const int32_t id = (int32_t)hp.lr_first.size();
            hp.lr_first.push_back((int32_t)hp.blk.size());
            hp.lr_nchunk.push_back(nch);
            for (int32_t ch = 0; ch < nch; ++ch) {
                Block b;
                b.row0 = (int32_t)r;
                b.row1 = (int32_t)r + 1;
                b.e0 = rowptr[r] + ch * NNZ_BLK;
                b.e1 = std::min<int64_t>((int64_t)b.e0 + NNZ_BLK, rowptr[r + 1]);
                hp.blk.push_back(b);
                hp.lr.push_back(id);
            }
            ++r;
        } else {
            const int64_t r0 = r;
            const int64_t e0 = rowptr[r];
            while (r < nrows && r - r0 < BS && (int64_t)rowptr[r + 1] - e0 <= NNZ_BLK) ++r;
            Block b;
            b.row0 = (int32_t)r0;
            b.row1 = (int32_t)r;
            b.e0 = (int32_t)e0;
            b.e1 = rowptr[r];
            hp.blk.push_back(b);
            hp.lr.push_back(-1);
        }
    }
    return hp;
}

struct DevPartition {
    DevMem blk, lr, lr_first, lr_nchunk, lr_count, lr_partial;
    Blocks view{};
    int upload(const HostPartition &hp) {
        const size_t nb = hp.blk.size(), nl = hp.lr_first.size();
        int rc;
        if ((rc = blk.alloc(std::max<size_t>(nb, 1) * sizeof(Block)))) return rc;
        if ((rc = lr.alloc(std::max<size_t>(nb, 1) * sizeof(int32_t)))) return rc;
        if ((rc = lr_first.alloc(std::max<size_t>(nl, 1) * sizeof(int32_t)))) return rc;
        if ((rc = lr_nchunk.alloc(std::max<size_t>(nl, 1) * sizeof(int32_t)))) return rc;
        if ((rc = lr_count.alloc(std::max<size_t>(nl, 1) * sizeof(int32_t)))) return rc;
        if ((rc = lr_partial.alloc(std::max<size_t>(nb, 1) * 4 * sizeof(double)))) return rc;
        if (nb) {
            HIPCHK(hipMemcpy(blk.p, hp.blk.data(), nb * sizeof(Block), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(lr.p, hp.lr.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice));
        }
        if (nl) {
            HIPCHK(hipMemcpy(lr_first.p, hp.lr_first.data(), nl * sizeof(int32_t),
                             hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(lr_nchunk.p, hp.lr_nchunk.data(), nl * sizeof(int32_t),
                             hipMemcpyHostToDevice));
        }
        HIPCHK(hipMemset(lr_count.p, 0, lr_count.bytes));
        view.blk = blk.as<Block>();
        view.lr = lr.as<int32_t>();
        view.lr_first = lr_first.as<int32_t>();
        view.lr_nchunk = lr_nchunk.as<int32_t>();
        view.lr_count = lr_count.as<int32_t>();
        view.lr_partial = lr_partial.as<double>();
        view.nblk = (int32_t)nb;
        view.nlr = (int32_t)nl;
        return QP_OK;
    }
};

// Runs f(r0, r1) over [0, R) split into contiguous ranges on up to 16 host threads
// (the caller's thread takes the first range).  Every row belongs to exactly one
// range, so loops that write only their own rows' slots give the serial result.
template <class F>
void parallel_rows(int64_t R, F f) {
    const int64_t hc = (int64_t)std::max(1u, std::thread::hardware_concurrency());
    const int64_t T = std::min<int64_t>({hc, 16, std::max<int64_t>(1, R / 65536)});
    if (T <= 1) {
        f((int64_t)0, R);
        return;
    }
    std::vector<std::thread> th;
    for (int64_t t = 1; t < T; ++t) th.emplace_back(f, R * t / T, R * (t + 1) / T);
    f((int64_t)0, R / T);
    for (auto &x : th) x.join();
}

struct HostPanels {
    int np = 1;
    std::vector<PBlock> blk;
    std::vector<int32_t> map, rowptr, col, lr_first, lr_nchunk;
    std::vector<double> val;
    int grid = 0;
};

// Splits the columns of an R x C CSR matrix into np ranges of equal nonzero
// count and builds one CSR per range plus row blocks pinned to XCD groups.
HostPanels build_panels(const int32_t *rowptr, const int32_t *col, const double *val, int64_t R,
                        int64_t C, int np) {
    HostPanels hp;
    hp.np = np;
    const int64_t nnz = rowptr[R];
    std::vector<int64_t> cum(C + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) cum[col[e] + 1]++;
    for (int64_t c = 0; c < C; ++c) cum[c + 1] += cum[c];
    std::vector<int64_t> bound(np + 1, C);
    bound[0] = 0;
    for (int k = 1; k < np; ++k) {
        const int64_t target = (nnz * k + np - 1) / np;
        bound[k] = std::lower_bound(cum.begin(), cum.end(), target) - cum.begin();
        if (bound[k] < bound[k - 1]) bound[k] = bound[k - 1];
        if (bound[k] > C) bound[k] = C;
    }
    std::vector<int32_t> pcol(C);
    for (int k = 0; k < np; ++k)
        for (int64_t c = bound[k]; c < bound[k + 1]; ++c) pcol[c] = k;
    // per-panel row counts -> global row pointers
    hp.rowptr.assign((size_t)np * (R + 1), 0);
    std::vector<int64_t> base(np + 1, 0);
    {
        std::vector<int64_t> cnt((size_t)np * R, 0);
        parallel_rows(R, [&](int64_t r0, int64_t r1) {
            for (int64_t r = r0; r < r1; ++r)
                for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e)
                    cnt[(size_t)pcol[col[e]] * R + r]++;
        });
        int64_t pos = 0;
        for (int k = 0; k < np; ++k) {
            base[k] = pos;
            for (int64_t r = 0; r < R; ++r) {
                hp.rowptr[(size_t)k * (R + 1) + r] = (int32_t)pos;
                pos += cnt[(size_t)k * R + r];
            }
            hp.rowptr[(size_t)k * (R + 1) + R] = (int32_t)pos;
        }
        base[np] = pos;
    }
    hp.col.resize(nnz);
    hp.val.resize(nnz);
    {
        std::vector<int64_t> next((size_t)np * R);
        for (int k = 0; k < np; ++k)
            for (int64_t r = 0; r < R; ++r) next[(size_t)k * R + r] = hp.rowptr[(size_t)k * (R + 1) + r];
        parallel_rows(R, [&](int64_t r0, int64_t r1) {
            for (int64_t r = r0; r < r1; ++r)
                for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
                    const int k = pcol[col[e]];
                    const int64_t q = next[(size_t)k * R + r]++;
                    hp.col[q] = col[e];
                    hp.val[q] = val[e];
                }
        });
    }
    // row blocks of each panel
    std::vector<std::vector<int32_t>> per_panel(np);
    for (int k = 0; k < np; ++k) {
        const int32_t *rp = hp.rowptr.data() + (size_t)k * (R + 1);
        int64_t r = 0;
        while (r < R) {
            const int64_t len = (int64_t)rp[r + 1] - rp[r];
            if (len > NNZ_BLK) {
                const int32_t nch = (int32_t)((len + NNZ_BLK - 1) / NNZ_BLK);
                const int32_t id = (int32_t)hp.lr_first.size();
                hp.lr_first.push_back((int32_t)hp.blk.size());
                hp.lr_nchunk.push_back(nch);
                for (int32_t ch = 0; ch < nch; ++ch) {
                    PBlock b{};
                    b.row0 = (int32_t)r;
                    b.row1 = (int32_t)r + 1;
                    b.e0 = rp[r] + ch * NNZ_BLK;
                    b.e1 = (int32_t)std::min<int64_t>((int64_t)b.e0 + NNZ_BLK, rp[r + 1]);
                    b.panel = k;
                    b.lr = id;
                    per_panel[k].push_back((int32_t)hp.blk.size());
                    hp.blk.push_back(b);
                }
                ++r;
            } else {
                const int64_t r0 = r, e0 = rp[r];
                while (r < R && r - r0 < PANEL_ROWS && (int64_t)rp[r + 1] - e0 <= NNZ_BLK) ++r;
                PBlock b{};
                b.row0 = (int32_t)r0;
                b.row1 = (int32_t)r;
                b.e0 = (int32_t)e0;
                b.e1 = rp[r];
                b.panel = k;
                b.lr = -1;
                per_panel[k].push_back((int32_t)hp.blk.size());
                hp.blk.push_back(b);
            }
        }
    }
    // workgroup w runs on XCD w % 8: XCD x serves panel x / (8/np), every (8/np)-th block
    const int s = 8 / np;
    std::vector<std::vector<int32_t>> lists(8);
    for (int x = 0; x < 8; ++x) {
        const int k = x / s, xo = x % s;
        for (size_t b = 0; b < per_panel[k].size(); ++b)
            if ((int)(b % s) == xo) lists[x].push_back(per_panel[k][b]);
    }
    size_t maxlen = 0;
    for (auto &l : lists) maxlen = std::max(maxlen, l.size());
    hp.grid = (int)(8 * maxlen);
    hp.map.assign(hp.grid, -1);
    for (int x = 0; x < 8; ++x)
        for (size_t l = 0; l < lists[x].size(); ++l) hp.map[l * 8 + x] = lists[x][l];
    return hp;
}

struct DevPanels {
    DevMem blk, map, rowptr, col, val, lr_first, lr_nchunk, lr_count, lr_partial, part;
    Panels view{};
    int upload(const HostPanels &hp, int64_t R) {
        int rc;
        if ((rc = blk.upload(hp.blk.data(), hp.blk.size() * sizeof(PBlock))) ||
            (rc = map.upload(hp.map.data(), hp.map.size() * 4)) ||
            (rc = rowptr.upload(hp.rowptr.data(), hp.rowptr.size() * 4)) ||
            (rc = col.upload(hp.col.data(), hp.col.size() * 4)) ||
            (rc = val.upload(hp.val.data(), hp.val.size() * 8)) ||
            (rc = lr_first.upload(hp.lr_first.data(), hp.lr_first.size() * 4)) ||
            (rc = lr_nchunk.upload(hp.lr_nchunk.data(), hp.lr_nchunk.size() * 4)) ||
            (rc = lr_count.alloc(std::max<size_t>(hp.lr_first.size(), 1) * 4)) ||
            (rc = lr_partial.alloc(std::max<size_t>(hp.blk.size(), 1) * 4 * 8)) ||
            (rc = part.alloc(std::max<size_t>((size_t)hp.np * R, 1) * 8)))
            return rc;
        HIPCHK(hipMemset(lr_count.p, 0, lr_count.bytes));
        view.blk = blk.as<PBlock>();
        view.map = map.as<int32_t>();
        view.rowptr = rowptr.as<int32_t>();
        view.col = col.as<int32_t>();
        view.val = val.as<double>();
        view.lr_first = lr_first.as<int32_t>();
        view.lr_nchunk = lr_nchunk.as<int32_t>();
        view.lr_count = lr_count.as<int32_t>();
        view.lr_partial = lr_partial.as<double>();
        view.part = part.as<double>();
        view.np = hp.np;
        view.nblk = (int32_t)hp.blk.size();
        view.grid = hp.grid;
        view.nlr = (int32_t)hp.lr_first.size();
        view.R = R;
        return QP_OK;
    }
};

// panel count: explicit setting, else 4 (two XCDs per panel) when the gathered
// vector exceeds 6 MB, or exceeds 1.75 MB with rows of at least 256 entries on average.
// Measured: one panel ties or wins up to 4.8 MB on random and equality QPs (n + m up
// to 6e5, rows of 4-20 entries), where the gathers still mostly hit L2 and the
// combine kernel is pure cost; 4 wins among 1/2/4/8 at 8-12 MB (n = 1e6).  With long
// rows (factor-model portfolio QPs: a thousand factor rows of thousands of entries
// and the budget row) the partial sums are a few thousand values, so the XCD-local
// gather slices pay off from a smaller vector: 4 panels take the dual phase of a
// 1000-factor portfolio from 40.6 to 36.1 us per iteration at 2.5e5 assets (1.9 MB
// gathered) and from 68.6 to 59.4 us at 5e5 (3.8 MB), but not at 2e5 (1.5 MB: 31.1 vs
// 32.1 us).  (The row kernel made persistent and pipelined like the panel kernels,
// without panels, stays at 69.8 us there: the gain is the slices' L2 hits.)
int choose_panels(int32_t setting, int64_t gathered_len, int64_t nnz, int64_t rows) {
    if (setting == 1 || setting == 2 || setting == 4 || setting == 8) return setting;
    const int64_t bytes = gathered_len * 8;
    if (bytes > ((int64_t)6 << 20)) return 4;
    if (rows > 0 && nnz >= 256 * rows && bytes > ((int64_t)7 << 18)) return 4;
    return 1;
}

// copies `count` elements of an input array (host or device) to a host vector
template <class T>
int fetch(std::vector<T> &dst, const T *src, int64_t count, int mem_space) {
    if (count == 0) {
        dst.clear();
        return QP_OK;
    }
    if (!src)
        return fail(QP_ERR_INVALID_ARGUMENT, "null input array where %lld elements are expected",
                    (long long)count);
    if (mem_space == QP_MEM_HOST) {
        dst.assign(src, src + count);  // one pass, no zero fill before the copy
    } else {
        dst.resize((size_t)count);
        HIPCHK(hipMemcpy(dst.data(), src, (size_t)count * sizeof(T), hipMemcpyDeviceToHost));
    }
    return QP_OK;
}

int validate_csr(const char *name, const std::vector<int32_t> &rowptr, int64_t nrows,
                 int64_t nnz, const std::vector<int32_t> &col, int64_t ncols) {
    if (rowptr[0] != 0) return fail(QP_ERR_INVALID_ARGUMENT, "%s.row_ptr[0] must be 0", name);
    for (int64_t i = 0; i < nrows; ++i)
        if (rowptr[i + 1] < rowptr[i])
            return fail(QP_ERR_INVALID_ARGUMENT, "%s.row_ptr decreases at row %lld", name,
                        (long long)i);
    if (rowptr[nrows] != nnz)
        return fail(QP_ERR_INVALID_ARGUMENT, "%s.row_ptr[nrows] = %d but nnz = %lld", name,
                    rowptr[nrows], (long long)nnz);
    for (int64_t e = 0; e < nnz; ++e)
        if (col[e] < 0 || col[e] >= ncols)
            return fail(QP_ERR_INVALID_ARGUMENT, "%s.col_idx[%lld] = %d out of range [0,%lld)",
                        name, (long long)e, col[e], (long long)ncols);
    return QP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// the handle
// ---------------------------------------------------------------------------
struct qp_handle {
    int64_t n = 0, m = 0;
    int32_t mem_space = QP_MEM_HOST;
    int32_t device = 0;
    qp_settings set{};
    hipStream_t stream = nullptr;

    // problem data
    DevMem a_rowptr, a_col, a_val, p_rowptr, p_col, p_val;
    DevMem c, b, l, u, rt;
    DevMem dscale;              // preconditioning d = (D2 [n], D1 [m]) on the device
    std::vector<double> h_d;    // its host copy (empty: not preconditioned)
    std::vector<double> h_c, h_b;  // the given c and b (host copies)
    DevPartition partA, partP;
    DevPanels panA, panP;    // column-panel layouts of A and P (np > 1)
    int npA = 1, npP = 1;
    Csr A{}, P{};
    double norm_A = 0.0, norm_Q = 0.0, c_inf = 0.0, b_inf = 0.0, c_norm2 = 0.0, b_norm2 = 0.0;
    double dual_bytes = 0.0, primal_bytes = 0.0;  // algorithmic HBM bytes of one launch
    int32_t uniform_bounds = 0;
    double lo_all = 0.0, hi_all = 0.0;

    // solver vectors
    DevMem x, xbar, xt, xmd0, xmd1, xrs, y, ybar, yrs, x0buf, y0buf;
    DevMem partials_a, partials_p, state, table;
    DevMem ipart_a, ipart_p;    // infeasibility partials (when detection is on)
    DevMem kpart_a, kpart_p;    // KKT panel partial sums (2 np m and 4 np n doubles)
    DevMem zz;                  // (x, x-bar) and (y, y-bar) pairs gathered by the KKT panels
    Vecs vecs{};
    int32_t nslotA = 0, nslotP = 0;
    State *h_state = nullptr;  // pinned ring of status records
    static constexpr int RING = 8;
    hipEvent_t ring_ev[RING]{};
    hipGraphExec_t graph[2]{nullptr, nullptr};
    int32_t graph_interval = 0;
    DevSettings graph_ds{};

    // profiling
    std::vector<hipEvent_t> prof_ev;
    qp_profile prof{};
    std::vector<qp_check_info> log;

    // batch mode
    qpb::BatchData *batch = nullptr;

    ~qp_handle() {
        for (auto &g : graph)
            if (g) (void)hipGraphExecDestroy(g);
        for (auto &e : ring_ev)
            if (e) (void)hipEventDestroy(e);
        for (auto &e : prof_ev) (void)hipEventDestroy(e);
        if (h_state) (void)hipHostFree(h_state);
        qpb::destroy_batch(batch);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

extern "C" {

void qp_default_settings(qp_settings *s) {
    if (!s) return;
    std::memset(s, 0, sizeof(*s));
    s->eps = 1e-6;
    s->max_iter = 200000;
    s->time_limit_s = 3600.0;
    s->check_every = 64;
    s->restart_mode = QP_RESTART_ADAPTIVE;
    s->fixed_K = 100;
    s->beta_sufficient = 0.2;
    s->beta_necessary = 0.8;
    s->beta_artificial = 0.36;
    s->pw_smoothing = 0.2;
    s->eps_zero = 1e-10;
    s->step_safety = 0.99;
    s->norm_A = 0.0;
    s->norm_Q = 0.0;
    s->power_iter_max = 1000;
    s->power_iter_rtol = 1e-7;
    s->warm_fallback = 1;
    s->use_graph = 1;
    s->profile = 0;
    s->log_checks = 0;
    s->device = 0;
    s->panels_dual = 0;
    s->panels_primal = 0;
    s->momentum = 1;
    s->precondition = 0;
    s->ruiz_iters = 10;
    s->detect_infeasibility = 0;
    s->eps_infeasible = 1e-8;
    s->check_symmetry = 0;
    s->log_cb = nullptr;
    s->log_user = nullptr;
}

const char *qp_last_error(void) { return qph::g_err.c_str(); }

int qp_version(void) { return QP_ABI_VERSION; }

}  // extern "C"

namespace {

int check_settings(const qp_settings &s) {
    if (!(s.eps >= 0.0)) return fail(QP_ERR_INVALID_ARGUMENT, "eps must be >= 0");
    if (s.check_every <= 0) return fail(QP_ERR_INVALID_ARGUMENT, "check_every must be > 0");
    if (s.restart_mode < 0 || s.restart_mode > 3)
        return fail(QP_ERR_INVALID_ARGUMENT, "unknown restart_mode %d", s.restart_mode);
    if (s.restart_mode == QP_RESTART_FIXED_K && s.fixed_K <= 0)
        return fail(QP_ERR_INVALID_ARGUMENT, "fixed_K must be > 0");
    if (s.check_every > 4096 || (s.restart_mode == QP_RESTART_FIXED_K && s.fixed_K > 4096))
        return fail(QP_ERR_INVALID_ARGUMENT, "evaluation interval above 4096 is not supported");
    if (!(s.step_safety > 0.0)) return fail(QP_ERR_INVALID_ARGUMENT, "step_safety must be > 0");
    // Sec. 6 restart criteria compare relKKT against fractions of earlier values, and
    // the primal-weight update is a convex combination in log space
    if (!(s.beta_sufficient > 0.0 && s.beta_sufficient <= 1.0) ||
        !(s.beta_necessary > 0.0 && s.beta_necessary <= 1.0) ||
        !(s.beta_artificial > 0.0 && s.beta_artificial <= 1.0))
        return fail(QP_ERR_INVALID_ARGUMENT, "beta_sufficient, beta_necessary and "
                                             "beta_artificial must be in (0, 1]");
    if (!(s.pw_smoothing >= 0.0 && s.pw_smoothing <= 1.0))
        return fail(QP_ERR_INVALID_ARGUMENT, "pw_smoothing must be in [0, 1]");
    if (!(s.eps_zero >= 0.0)) return fail(QP_ERR_INVALID_ARGUMENT, "eps_zero must be >= 0");
    if (s.power_iter_max < 1)
        return fail(QP_ERR_INVALID_ARGUMENT, "power_iter_max must be >= 1");
    if (!(s.power_iter_rtol >= 0.0))
        return fail(QP_ERR_INVALID_ARGUMENT, "power_iter_rtol must be >= 0");
    if (s.momentum != 0 && s.momentum != 1)
        return fail(QP_ERR_INVALID_ARGUMENT, "momentum must be 0 or 1");
    if (s.profile < 0) return fail(QP_ERR_INVALID_ARGUMENT, "profile must be >= 0");
    if (s.precondition != 0 && s.precondition != 1)
        return fail(QP_ERR_INVALID_ARGUMENT, "precondition must be 0 or 1");
    if (s.ruiz_iters < 0 || s.ruiz_iters > 100)
        return fail(QP_ERR_INVALID_ARGUMENT, "ruiz_iters must be in [0, 100]");
    if (s.detect_infeasibility != 0 && s.detect_infeasibility != 1)
        return fail(QP_ERR_INVALID_ARGUMENT, "detect_infeasibility must be 0 or 1");
    if (!(s.eps_infeasible > 0.0))
        return fail(QP_ERR_INVALID_ARGUMENT, "eps_infeasible must be > 0");
    return QP_OK;
}

// power iteration for ||A||_2 (Rayleigh quotient of A'A) and ||Q||_2
int estimate_norms(qp_handle *h) {
    const int64_t n = h->n, m = h->m;
    hipStream_t s = h->stream;
    DevMem v, w, z, parts;
    const int np_n = dot_nparts(n), np_m = dot_nparts(std::max<int64_t>(m, 1));
    int rc;
    if ((rc = v.alloc(n * 8)) || (rc = z.alloc(n * 8)) || (rc = w.alloc(std::max<int64_t>(m, 1) * 8)) ||
        (rc = parts.alloc(2048 * 8)))
        return rc;
    std::vector<double> hp(2048);
    // the two dot products of a step: partials of a1.b1 in parts[0, np1) and of a2.b2 in
    // parts[1024, 1024 + np2) (at most 1024 partials each), one copy and one host wait per
    // step; each is then summed on the host in partial order
    auto dots = [&](const double *a1, const double *b1, int64_t len1, int np1, double *out1,
                    const double *a2, const double *b2, int64_t len2, int np2,
                    double *out2) -> int {
        launch_dot_partials(s, a1, b1, len1, parts.as<double>(), np1);
        launch_dot_partials(s, a2, b2, len2, parts.as<double>() + 1024, np2);
        HIPCHK(hipMemcpyAsync(hp.data(), parts.p, (size_t)(1024 + np2) * 8,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double acc1 = 0.0, acc2 = 0.0;
        for (int i = 0; i < np1; ++i) acc1 = acc1 + hp[i];
        for (int i = 0; i < np2; ++i) acc2 = acc2 + hp[1024 + i];
        *out1 = acc1;
        *out2 = acc2;
        return QP_OK;
    };
    const int maxit = h->set.power_iter_max;
    const double rtol = h->set.power_iter_rtol;
    if (!(h->set.norm_A > 0.0)) {
        double lam = 0.0;
        const int64_t annz = h->partA.view.nblk ? 1 : 0;
        if (m > 0 && annz) {
            launch_fill(s, v.as<double>(), n, 1.0 / std::sqrt((double)n));
            double lam_prev = 0.0;
            for (int it = 1; it <= maxit; ++it) {
                launch_spmv_plain(s, h->partA.view, h->A, v.as<double>(), nullptr, n,
                                  w.as<double>(), 1.0);
                launch_spmv_plain(s, h->partP.view, h->P, nullptr, w.as<double>(), n,
                                  z.as<double>(), -1.0);
                double nz2;
                if ((rc = dots(w.as<double>(), w.as<double>(), m, np_m, &lam, z.as<double>(),
                               z.as<double>(), n, np_n, &nz2)))
                    return rc;
                const double nz = std::sqrt(nz2);
                if (nz == 0.0) break;
                launch_div(s, v.as<double>(), z.as<double>(), n, nz);
                if (it > 1 && std::fabs(lam - lam_prev) <= rtol * lam) break;
                lam_prev = lam;
            }
        }
        h->norm_A = std::sqrt(lam);
    } else {
        h->norm_A = h->set.norm_A;
    }
    if (!(h->set.norm_Q > 0.0)) {
        double lam = 0.0;
        launch_fill(s, v.as<double>(), n, 1.0 / std::sqrt((double)n));
        double lam_prev = 0.0;
        for (int it = 1; it <= maxit; ++it) {
            launch_spmv_plain(s, h->partP.view, h->P, v.as<double>(), nullptr, n, z.as<double>(),
                              1.0);
            double nw2;
            if ((rc = dots(v.as<double>(), z.as<double>(), n, np_n, &lam, z.as<double>(),
                           z.as<double>(), n, np_n, &nw2)))
                return rc;
            const double nw = std::sqrt(nw2);
            if (nw == 0.0) break;
            launch_div(s, v.as<double>(), z.as<double>(), n, nw);
            if (it > 1 && std::fabs(lam - lam_prev) <= rtol * std::fabs(lam)) break;
            lam_prev = lam;
        }
        h->norm_Q = std::fabs(lam);
    } else {
        h->norm_Q = h->set.norm_Q;
    }
    return QP_OK;
}

// Uploads c and b (and the bounds when given) of the problem the iteration runs on:
// the given vectors, or with preconditioning c~ = D2 c, b~ = D1 b, l~ = l / D2,
// u~ = u / D2.  relKKT's ||c||_inf and ||b||_inf are the given problem's; the 2-norms
// for the initial primal weight are those of the iterated (scaled) problem.
int upload_vectors(qp_handle *h, const std::vector<double> &c, const std::vector<double> &b,
                   const std::vector<double> *l, const std::vector<double> *u) {
    const int64_t n = h->n, m = h->m;
    const bool sc = !h->h_d.empty();
    std::vector<double> cs(c), bs(b);
    if (sc) {
        for (int64_t j = 0; j < n; ++j) cs[j] = c[j] * h->h_d[j];
        for (int64_t i = 0; i < m; ++i) bs[i] = b[i] * h->h_d[n + i];
    }
    auto put = [&](DevMem &dm, const std::vector<double> &v) -> int {
        if (!dm.p) return dm.upload(v.data(), v.size() * 8);
        if (!v.empty()) HIPCHK(hipMemcpy(dm.p, v.data(), v.size() * 8, hipMemcpyHostToDevice));
        return QP_OK;
    };
    int rc;
    if ((rc = put(h->c, cs)) || (rc = put(h->b, bs))) return rc;
    if (l && u) {
        std::vector<double> ls(*l), us(*u);
        if (sc)
            for (int64_t j = 0; j < n; ++j) {
                ls[j] = (*l)[j] / h->h_d[j];
                us[j] = (*u)[j] / h->h_d[j];
            }
        if ((rc = put(h->l, ls)) || (rc = put(h->u, us))) return rc;
        // bounds equal for every variable (x >= 0, or all free) let the primal epilogue
        // skip reading l and u; compared bitwise, so -0.0 and 0.0 count as different
        bool uni = n > 0;
        for (int64_t j = 1; j < n && uni; ++j)
            uni = std::memcmp(&ls[j], &ls[0], 8) == 0 && std::memcmp(&us[j], &us[0], 8) == 0;
        h->uniform_bounds = uni ? 1 : 0;
        h->lo_all = uni ? ls[0] : 0.0;
        h->hi_all = uni ? us[0] : 0.0;
    }
    double cn = 0.0, bn = 0.0, ci = 0.0, bi = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        cn += cs[j] * cs[j];
        if (std::fabs(c[j]) > ci) ci = std::fabs(c[j]);
    }
    for (int64_t i = 0; i < m; ++i) {
        bn += bs[i] * bs[i];
        if (std::fabs(b[i]) > bi) bi = std::fabs(b[i]);
    }
    h->c_norm2 = std::sqrt(cn);
    h->b_norm2 = std::sqrt(bn);
    h->c_inf = ci;
    h->b_inf = bi;
    return QP_OK;
}

struct HostProblem {
    std::vector<int32_t> qr, qc, ar, ac;
    std::vector<double> qv, av, c, b, l, u;
    std::vector<uint8_t> rt;
};

// Copies the problem to host vectors and validates it (no device work for host input).
int gather_single(const qp_problem_desc *d, HostProblem &hp, const qp_settings &s) {
    const int64_t n = d->n, m = d->m;
    const int ms = d->mem_space;
    auto &qr = hp.qr, &qc = hp.qc, &ar = hp.ar, &ac = hp.ac;
    auto &qv = hp.qv, &av = hp.av, &c = hp.c, &b = hp.b, &l = hp.l, &u = hp.u;
    auto &rt = hp.rt;
    int rc;
    if ((rc = fetch(qr, d->Q.row_ptr, n + 1, ms))) return rc;
    if (qr[n] != d->Q.nnz || d->Q.nnz < 0)
        return fail(QP_ERR_INVALID_ARGUMENT, "Q.nnz (%lld) disagrees with Q.row_ptr[n] (%d)",
                    (long long)d->Q.nnz, qr[n]);
    if ((rc = fetch(qc, d->Q.col_idx, d->Q.nnz, ms)) || (rc = fetch(qv, d->Q.val, d->Q.nnz, ms)))
        return rc;
    if ((rc = validate_csr("Q", qr, n, d->Q.nnz, qc, n))) return rc;
    if (m > 0) {
        if (!d->A.row_ptr || !d->b)
            return fail(QP_ERR_INVALID_ARGUMENT, "A.row_ptr and b are required when m > 0");
        if (d->A.nnz > 0 && (!d->A.col_idx || !d->A.val))
            return fail(QP_ERR_INVALID_ARGUMENT, "A.col_idx and A.val are required when A.nnz > 0");
        if ((rc = fetch(ar, d->A.row_ptr, m + 1, ms))) return rc;
        if (ar[m] != d->A.nnz || d->A.nnz < 0)
            return fail(QP_ERR_INVALID_ARGUMENT, "A.nnz (%lld) disagrees with A.row_ptr[m] (%d)",
                        (long long)d->A.nnz, ar[m]);
        if ((rc = fetch(ac, d->A.col_idx, d->A.nnz, ms)) || (rc = fetch(av, d->A.val, d->A.nnz, ms)))
            return rc;
        if ((rc = validate_csr("A", ar, m, d->A.nnz, ac, n))) return rc;
        if ((rc = fetch(b, d->b, m, ms))) return rc;
        if (d->row_type) {
            if ((rc = fetch(rt, d->row_type, m, ms))) return rc;
            for (int64_t i = 0; i < m; ++i)
                if (rt[i] > 1)
                    return fail(QP_ERR_INVALID_ARGUMENT, "row_type[%lld] = %d is not 0 (EQ) or 1 (GE)",
                                (long long)i, rt[i]);
        } else {
            rt.assign(m, 0);
        }
    } else {
        ar.assign(1, 0);
    }
    if (!d->c) return fail(QP_ERR_INVALID_ARGUMENT, "c is required");
    if ((rc = fetch(c, d->c, n, ms))) return rc;
    if (d->l) {
        if ((rc = fetch(l, d->l, n, ms))) return rc;
    } else {
        l.assign(n, -INFINITY);
    }
    if (d->u) {
        if ((rc = fetch(u, d->u, n, ms))) return rc;
    } else {
        u.assign(n, INFINITY);
    }
    for (int64_t j = 0; j < n; ++j)
        if (!(l[j] <= u[j]) || l[j] == INFINITY || u[j] == -INFINITY)
            return fail(QP_ERR_INVALID_ARGUMENT, "invalid bounds at variable %lld: [%g, %g]",
                        (long long)j, l[j], u[j]);
    const int64_t pnnz = d->Q.nnz + (m > 0 ? d->A.nnz : 0);
    if (pnnz >= ((int64_t)1 << 31) || n + m >= ((int64_t)1 << 31))
        return fail(QP_ERR_INVALID_ARGUMENT, "problem exceeds int32 indexing");
    if (s.check_symmetry)
        if ((rc = qph::check_symmetric(n, qr.data(), qc.data(), qv.data(), 0))) return rc;
    return QP_OK;
}

// P = [Q | -A']: row j holds Q's row j followed by the entries of column j of A, negated,
// in increasing row index of A, with column index n + i.
void build_p(int64_t n, int64_t m, int64_t annz, const int32_t *qr, const int32_t *qc,
             const double *qv, const int32_t *ar, const int32_t *ac, const double *av,
             std::vector<int32_t> &pr, std::vector<int32_t> &pc, std::vector<double> &pv) {
    // Each host thread owns a range of P's rows (A's columns) and scans all of A in row
    // order, so every row gets its entries in the serial order.
    const int64_t pnnz = (int64_t)qr[n] + annz;
    pr.assign(n + 1, 0);
    pc.resize((size_t)pnnz);
    pv.resize((size_t)pnnz);
    std::vector<int64_t> acount(n, 0);
    parallel_rows(n, [&](int64_t j0, int64_t j1) {
        for (int64_t e = 0; e < annz; ++e) {
            const int64_t j = ac[e];
            if (j >= j0 && j < j1) acount[j]++;
        }
    });
    for (int64_t j = 0; j < n; ++j) pr[j + 1] = (int32_t)(pr[j] + (qr[j + 1] - qr[j]) + acount[j]);
    std::vector<int64_t> next(n);
    parallel_rows(n, [&](int64_t j0, int64_t j1) {
        for (int64_t j = j0; j < j1; ++j) {
            int64_t pos = pr[j];
            for (int64_t e = qr[j]; e < qr[j + 1]; ++e, ++pos) {
                pc[pos] = qc[e];
                pv[pos] = qv[e];
            }
            next[j] = pos;
        }
        for (int64_t i = 0; i < m; ++i)
            for (int64_t e = ar[i]; e < ar[i + 1]; ++e) {
                const int64_t j = ac[e];
                if (j < j0 || j >= j1) continue;
                const int64_t pos = next[j]++;
                pc[pos] = (int32_t)(n + i);
                pv[pos] = -av[e];
            }
    });
}

int64_t annz_of(const qp_problem_desc *d) { return d->m > 0 ? d->A.nnz : 0; }

int create_single(const qp_problem_desc *d, qp_handle *h, HostProblem &hp) {
    const int64_t n = d->n, m = d->m;
    const auto &qr = hp.qr, &qc = hp.qc, &ar = hp.ar, &ac = hp.ac;
    const auto &qv = hp.qv, &av = hp.av, &c = hp.c, &b = hp.b, &l = hp.l, &u = hp.u;
    const auto &rt = hp.rt;
    int rc;
    const int64_t pnnz = d->Q.nnz + (m > 0 ? d->A.nnz : 0);

    std::vector<int32_t> pr, pc;
    std::vector<double> pv;
    build_p(n, m, annz_of(d), qr.data(), qc.data(), qv.data(), ar.data(), ac.data(), av.data(),
            pr, pc, pv);

    auto up = [&](DevMem &dm, const void *src, size_t bytes) -> int { return dm.upload(src, bytes); };
    if ((rc = up(h->a_rowptr, ar.data(), ar.size() * 4)) || (rc = up(h->a_col, ac.data(), ac.size() * 4)) ||
        (rc = up(h->a_val, av.data(), av.size() * 8)) || (rc = up(h->p_rowptr, pr.data(), pr.size() * 4)) ||
        (rc = up(h->p_col, pc.data(), pc.size() * 4)) || (rc = up(h->p_val, pv.data(), pv.size() * 8)) ||
        (rc = up(h->rt, rt.data(), rt.size())))
        return rc;
    h->A = Csr{h->a_rowptr.as<int32_t>(), h->a_col.as<int32_t>(), h->a_val.as<double>(), m};
    h->P = Csr{h->p_rowptr.as<int32_t>(), h->p_col.as<int32_t>(), h->p_val.as<double>(), n};
    // Sec. 5 preprocessing: scale A and P in place on the device; the panel copies below
    // are built from the scaled values
    std::vector<double> av_s, pv_s;
    const double *avp = av.data(), *pvp = pv.data();
    if (h->set.precondition) {
        DevMem work;
        if ((rc = work.alloc((size_t)(n + m) * 16)) || (rc = h->dscale.alloc((size_t)(n + m) * 8)))
            return rc;
        ScaleInput in{};
        in.n = n;
        in.m = m;
        in.a_rowptr = h->A.rowptr;
        in.a_col = h->A.col;
        in.a_val = h->a_val.as<double>();
        in.p_rowptr = h->P.rowptr;
        in.p_col = h->P.col;
        in.p_val = h->p_val.as<double>();
        in.ruiz_iters = h->set.ruiz_iters;
        in.l2 = 1;
        in.pc = 1;
        if (precondition_device(h->stream, in, work.as<double>(), h->dscale.as<double>()))
            return fail(QP_ERR_DEVICE, "preconditioning kernels failed to launch");
        HIPCHK(hipStreamSynchronize(h->stream));
        h->h_d.resize((size_t)(n + m));
        HIPCHK(hipMemcpy(h->h_d.data(), h->dscale.p, (size_t)(n + m) * 8, hipMemcpyDeviceToHost));
        av_s.resize(av.size());
        pv_s.resize(pv.size());
        if (!av_s.empty())
            HIPCHK(hipMemcpy(av_s.data(), h->a_val.p, av_s.size() * 8, hipMemcpyDeviceToHost));
        if (!pv_s.empty())
            HIPCHK(hipMemcpy(pv_s.data(), h->p_val.p, pv_s.size() * 8, hipMemcpyDeviceToHost));
        avp = av_s.data();
        pvp = pv_s.data();
    }
    h->h_c = c;
    h->h_b = b;
    if ((rc = upload_vectors(h, c, b, &l, &u))) return rc;
    HostPartition hpA = partition_rows(ar.data(), m), hpP = partition_rows(pr.data(), n);
    {
        // Algorithmic bytes of one launch: matrix values (8 B) + column indices (4 B) per
        // nonzero, row pointers (4 B per row), every distinct gathered vector entry once
        // (8 B), and the per-row vector traffic of the fused epilogue:
        //   dual:   read y, y-bar, b (24 B) + row type (1 B), write y, y-bar (16 B)
        //   primal: read x, x-bar, c, l, u (40 B), write x, x-bar, x~, x_md (32 B)
        std::vector<uint8_t> seen((size_t)(n + m), 0);
        int64_t gA = 0, gP = 0;
        for (int64_t e = 0; e < (m > 0 ? d->A.nnz : 0); ++e)
            if (!seen[ac[e]]) { seen[ac[e]] = 1; ++gA; }
        std::fill(seen.begin(), seen.end(), 0);
        for (int64_t e = 0; e < pnnz; ++e)
            if (!seen[pc[e]]) { seen[pc[e]] = 1; ++gP; }
        const double annz = (double)(m > 0 ? d->A.nnz : 0);
        h->dual_bytes = m > 0 ? 12.0 * annz + 4.0 * (double)(m + 1) + 8.0 * (double)gA +
                                    41.0 * (double)m : 0.0;
        // (with bounds equal for every variable, l and u are two scalars: 56 B per row)
        h->primal_bytes = 12.0 * (double)pnnz + 4.0 * (double)(n + 1) + 8.0 * (double)gP +
                          (h->uniform_bounds ? 56.0 : 72.0) * (double)n;
    }
    if ((rc = h->partA.upload(hpA)) || (rc = h->partP.upload(hpP))) return rc;
    h->npA = m > 0 ? choose_panels(h->set.panels_dual, n, d->A.nnz, m) : 1;
    h->npP = choose_panels(h->set.panels_primal, n + m, pnnz, n);
    {
        // the two panel layouts are independent: A's is built on a second thread
        HostPanels pa, pp;
        std::thread ta;
        if (h->npA > 1)
            ta = std::thread([&] { pa = build_panels(ar.data(), ac.data(), avp, m, n, h->npA); });
        if (h->npP > 1) pp = build_panels(pr.data(), pc.data(), pvp, n, n + m, h->npP);
        if (ta.joinable()) ta.join();
        if (h->npA > 1 && (rc = h->panA.upload(pa, m))) return rc;
        if (h->npP > 1 && (rc = h->panP.upload(pp, n))) return rc;
        if (h->npA > 1 || h->npP > 1) {
            const int32_t nwg = panel_resident_workgroups(h->device);
            if (nwg < 8)
                return fail(QP_ERR_DEVICE, "occupancy query of the panel kernels failed");
            h->panA.view.nwg = nwg;
            h->panP.view.nwg = nwg;
        }
    }

    // solver vectors
    const size_t nb = (size_t)n * 8, mb = (size_t)std::max<int64_t>(m, 1) * 8;
    if ((rc = h->x.alloc(nb)) || (rc = h->xbar.alloc(nb)) || (rc = h->xt.alloc(nb)) ||
        (rc = h->xmd0.alloc(nb)) || (rc = h->xmd1.alloc(nb)) || (rc = h->xrs.alloc(nb)) ||
        (rc = h->y.alloc(mb)) || (rc = h->ybar.alloc(mb)) || (rc = h->yrs.alloc(mb)) ||
        (rc = h->x0buf.alloc(nb)) || (rc = h->y0buf.alloc(mb)))
        return rc;
    h->nslotA = h->partA.view.nblk + h->partA.view.nlr;
    h->nslotP = h->partP.view.nblk + h->partP.view.nlr;
    // slots: one per row block, or one per 256 rows when the KKT runs on the panels
    const int64_t slA = std::max<int64_t>(h->nslotA, (m + BS - 1) / BS);
    const int64_t slP = std::max<int64_t>(h->nslotP, (n + BS - 1) / BS);
    if (h->npA > 1 && (rc = h->kpart_a.alloc((size_t)2 * h->npA * m * 8))) return rc;
    if (h->npP > 1 && (rc = h->kpart_p.alloc((size_t)4 * h->npP * n * 8))) return rc;
    if ((h->npA > 1 || h->npP > 1) && (rc = h->zz.alloc((size_t)(n + m) * 16))) return rc;
    if ((rc = h->partials_a.alloc((size_t)(slA + FOLD_SLOTS) * RA_NV * 8)) ||
        (rc = h->partials_p.alloc((size_t)(slP + FOLD_SLOTS) * RP_NV * 8)) ||
        (rc = h->state.alloc(sizeof(State))) || (rc = h->table.alloc(4096 * sizeof(Step))))
        return rc;
    if (h->set.detect_infeasibility &&
        ((rc = h->ipart_a.alloc((size_t)(h->nslotA + FOLD_SLOTS) * IA_NV * 8)) ||
         (rc = h->ipart_p.alloc((size_t)(h->nslotP + FOLD_SLOTS) * IP_NV * 8))))
        return rc;
    Vecs &v = h->vecs;
    v.x = h->x.as<double>();
    v.xbar = h->xbar.as<double>();
    v.xt = h->xt.as<double>();
    v.xmd[0] = h->xmd0.as<double>();
    v.xmd[1] = h->xmd1.as<double>();
    v.xrs = h->xrs.as<double>();
    v.y = h->y.as<double>();
    v.ybar = h->ybar.as<double>();
    v.yrs = h->yrs.as<double>();
    v.c = h->c.as<double>();
    v.b = h->b.as<double>();
    v.l = h->l.as<double>();
    v.u = h->u.as<double>();
    v.rt = h->rt.as<uint8_t>();
    v.dv = h->h_d.empty() ? nullptr : h->dscale.as<double>();
    v.dr = h->h_d.empty() ? nullptr : h->dscale.as<double>() + n;
    v.uniform_bounds = h->uniform_bounds;
    v.lo_all = h->lo_all;
    v.hi_all = h->hi_all;
    v.zz = (h->npA > 1 || h->npP > 1) ? reinterpret_cast<double2 *>(h->zz.p) : nullptr;
    return QP_OK;
}

DevSettings dev_settings(const qp_handle *h) {
    DevSettings ds;
    std::memset(&ds, 0, sizeof(ds));  // padding bytes take part in the graph-cache comparison
    const qp_settings &s = h->set;
    ds.eps = s.eps;
    ds.beta_sufficient = s.beta_sufficient;
    ds.beta_necessary = s.beta_necessary;
    ds.beta_artificial = s.beta_artificial;
    ds.pw_smoothing = s.pw_smoothing;
    ds.eps_zero = s.eps_zero;
    ds.step_safety = s.step_safety;
    ds.norm_A = h->norm_A;
    ds.norm_Q = h->norm_Q;
    ds.b_inf = h->b_inf;
    ds.c_inf = h->c_inf;
    ds.max_iter = s.max_iter;
    ds.restart_mode = s.restart_mode;
    ds.fixed_K = s.fixed_K;
    ds.interval = s.restart_mode == QP_RESTART_FIXED_K ? s.fixed_K : s.check_every;
    ds.momentum = s.momentum;
    ds.detect_infeas = s.detect_infeasibility;
    ds.eps_infeas = s.eps_infeasible;
    return ds;
}

// one interval of `len` iterations starting with x_md in buffer md_in
// KKT products of (x, y) and (x-bar, y-bar) reduced into per-block slots (through the
// column panels when they exist, so the gathers stay in each XCD's L2); *sa and *sp
// receive the slot counts for launch_decide.
void enqueue_kkt(qp_handle *h, hipStream_t s, State *st, int32_t *sa, int32_t *sp) {
    if (h->npA > 1 || h->npP > 1) launch_interleave(s, h->vecs, st, h->n, h->m);
    if (h->npA > 1) {
        *sa = launch_kkt_rows_panels(s, h->panA.view, h->vecs, h->kpart_a.as<double>(),
                                     h->partials_a.as<double>(), st, h->n, h->m);
    } else {
        launch_kkt_rows(s, h->partA.view, h->A, h->vecs, h->partials_a.as<double>(), st);
        *sa = h->nslotA;
    }
    if (h->npP > 1) {
        *sp = launch_kkt_cols_panels(s, h->panP.view, h->vecs, h->kpart_p.as<double>(),
                                     h->partials_p.as<double>(), st, h->n);
    } else {
        launch_kkt_cols(s, h->partP.view, h->P, h->vecs, h->partials_p.as<double>(), st, h->n);
        *sp = h->nslotP;
    }
}

// ev: with profiling, 3 events per timed iteration (before the dual phase, between
// the phases, after the primal phase) for iterations j with j % stride == 0;
// nullptr otherwise
void enqueue_interval(qp_handle *h, const DevSettings &ds, int md_in, int len,
                      hipEvent_t *ev, int stride) {
    hipStream_t s = h->stream;
    const Step *tab = h->table.as<Step>();
    State *st = h->state.as<State>();
    int md = md_in;
    for (int j = 0; j < len; ++j) {
        const bool timed = ev && j % stride == 0;
        if (timed) (void)hipEventRecord(ev[3 * j + 0], s);
        if (h->npA > 1) launch_dual_panels(s, h->panA.view, h->vecs, h->n, tab + j, st);
        else launch_dual(s, h->partA.view, h->A, h->vecs, tab + j, st);
        if (timed) (void)hipEventRecord(ev[3 * j + 1], s);
        if (h->npP > 1) launch_primal_panels(s, h->panP.view, h->vecs, md, h->n, tab + j, st);
        else launch_primal(s, h->partP.view, h->P, h->vecs, md, tab + j, st, h->n);
        if (timed) (void)hipEventRecord(ev[3 * j + 2], s);
        md ^= 1;
    }
    int32_t sa, sp;
    enqueue_kkt(h, s, st, &sa, &sp);
    if (h->set.detect_infeasibility)  // directions in the warm-start buffers (free here)
        launch_infeas(s, h->partA.view, h->A, h->partP.view, h->P, h->vecs,
                      h->x0buf.as<double>(), h->y0buf.as<double>(), h->ipart_a.as<double>(),
                      h->nslotA, h->ipart_p.as<double>(), h->nslotP, st, h->n, h->m);
    launch_decide(s, DECIDE_CHECK, h->partials_a.as<double>(), sa, h->partials_p.as<double>(),
                  sp, st, h->table.as<Step>(), ds, len);
    launch_apply(s, h->vecs, md, st, h->n, h->m);
}

int get_graph(qp_handle *h, const DevSettings &ds, int md_in, hipGraphExec_t *out) {
    if (h->graph_interval != ds.interval || std::memcmp(&h->graph_ds, &ds, sizeof(ds)) != 0) {
        for (auto &g : h->graph)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
        h->graph_interval = ds.interval;
        h->graph_ds = ds;  // captured kernel arguments are frozen: re-capture on any change
    }
    if (!h->graph[md_in]) {
        hipGraph_t g;
        HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        enqueue_interval(h, ds, md_in, ds.interval, nullptr, 1);
        HIPCHK(hipStreamEndCapture(h->stream, &g));
        hipError_t e = hipGraphInstantiate(&h->graph[md_in], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess)
            return fail(QP_ERR_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    *out = h->graph[md_in];
    return QP_OK;
}

void fill_result(const qp_handle *h, const State &S, double t, qp_result *res) {
    std::memset(res, 0, sizeof(*res));
    res->status = S.status;
    res->used_warm_start = S.used_warm;
    res->iterations = S.total;
    res->restarts = S.restarts;
    res->kkt_evals = S.kkt_evals;
    const double *k = S.kkt[S.cand ? 1 : 0];
    res->r_primal = k[0];
    res->r_dual = k[1];
    res->r_gap = k[2];
    res->rel_kkt = k[3];
    res->primal_obj = k[4];
    res->dual_obj = k[5];
    res->omega = S.omega;
    res->norm_A = h->norm_A;
    res->norm_Q = h->norm_Q;
    res->solve_time_s = t;
    res->start_s = 0.0;
    res->end_s = t;
}

}  // namespace

extern "C" {

int qp_create(const qp_problem_desc *d, const qp_settings *settings, qp_handle **out) {
    if (!d || !out) return fail(QP_ERR_INVALID_ARGUMENT, "desc and out must be non-null");
    *out = nullptr;
    qp_settings s;
    if (settings) s = *settings;
    else qp_default_settings(&s);
    int rc;
    if ((rc = check_settings(s))) return rc;
    if (d->n <= 0) return fail(QP_ERR_INVALID_ARGUMENT, "n must be positive");
    if (d->m < 0) return fail(QP_ERR_INVALID_ARGUMENT, "m must be >= 0");
    // P = [Q | -A'] is indexed with int32: its columns run over (x, y) and its entries
    // over the nonzeros of Q and A; checked before any array is read
    if (d->n + d->m >= ((int64_t)1 << 31) ||
        d->Q.nnz + (d->m > 0 ? d->A.nnz : 0) >= ((int64_t)1 << 31))
        return fail(QP_ERR_INVALID_ARGUMENT, "problem exceeds int32 indexing");
    if (d->mem_space != QP_MEM_HOST && d->mem_space != QP_MEM_DEVICE)
        return fail(QP_ERR_INVALID_ARGUMENT, "unknown mem_space %d", d->mem_space);
    if (!d->Q.row_ptr || (d->Q.nnz > 0 && (!d->Q.col_idx || !d->Q.val)))
        return fail(QP_ERR_INVALID_ARGUMENT, "Q arrays are required");
    if (d->num_instances < 1) return fail(QP_ERR_INVALID_ARGUMENT, "num_instances must be >= 1");
    HostProblem hp;
    if (d->num_instances == 1 && d->mem_space == QP_MEM_HOST)
        if ((rc = gather_single(d, hp, s))) return rc;  // validation before any device work
    if (d->num_instances > 1 && d->mem_space == QP_MEM_HOST)
        if ((rc = qpb::validate_batch_host(d, &s))) return rc;
    HIPCHK(hipSetDevice(s.device));
    qp_handle *h = new qp_handle();
    h->n = d->n;
    h->m = d->m;
    h->mem_space = d->mem_space;
    h->device = s.device;
    h->set = s;
    hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete h;
        return fail(QP_ERR_DEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
    }
    if (d->stream) {
        // the caller's arrays are ordered on its stream: wait for them
        e = hipStreamSynchronize((hipStream_t)d->stream);
        if (e != hipSuccess) {
            delete h;
            return fail(QP_ERR_DEVICE, "caller stream: %s", hipGetErrorString(e));
        }
    }
    if (d->num_instances > 1) {
        rc = qpb::create_batch(d, &h->set, h->stream, &h->batch);
    } else {
        if (d->mem_space == QP_MEM_DEVICE) rc = gather_single(d, hp, s);
        if (!rc) rc = create_single(d, h, hp);
        if (!rc) rc = estimate_norms(h);
        if (!rc && !(h->norm_A > 0.0) && !(h->norm_Q > 0.0))
            rc = fail(QP_ERR_INVALID_ARGUMENT, "both ||A|| and ||Q|| are zero: nothing to solve");
        if (!rc) {
            e = hipHostMalloc((void **)&h->h_state, sizeof(State) * qp_handle::RING, 0);
            if (e != hipSuccess) rc = fail(QP_ERR_OUT_OF_MEMORY, "hipHostMalloc failed");
            for (int i = 0; !rc && i < qp_handle::RING; ++i)
                if (hipEventCreateWithFlags(&h->ring_ev[i], hipEventDisableTiming) != hipSuccess)
                    rc = fail(QP_ERR_DEVICE, "hipEventCreate failed");
        }
    }
    if (!rc) {
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) rc = fail(QP_ERR_DEVICE, "create: %s", hipGetErrorString(e));
    }
    if (rc) {
        delete h;
        return rc;
    }
    *out = h;
    qph::clear_error();
    return QP_OK;
}

void qp_free(qp_handle *h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

int qp_get_scaling(qp_handle *h, double *d_var, double *d_row) {
    if (!h) return fail(QP_ERR_INVALID_ARGUMENT, "null handle");
    if (h->batch) return qpb::batch_scaling(h->batch, d_var, d_row);
    for (int64_t j = 0; d_var && j < h->n; ++j) d_var[j] = h->h_d.empty() ? 1.0 : h->h_d[j];
    for (int64_t i = 0; d_row && i < h->m; ++i) d_row[i] = h->h_d.empty() ? 1.0 : h->h_d[h->n + i];
    return QP_OK;
}

int qp_get_norms(qp_handle *h, double *norm_A, double *norm_Q) {
    if (!h) return fail(QP_ERR_INVALID_ARGUMENT, "null handle");
    if (h->batch) return qpb::batch_norms(h->batch, norm_A, norm_Q);
    if (norm_A) *norm_A = h->norm_A;
    if (norm_Q) *norm_Q = h->norm_Q;
    return QP_OK;
}

int qp_update_vectors(qp_handle *h, const double *c, const double *b) {
    if (!h) return fail(QP_ERR_INVALID_ARGUMENT, "null handle");
    HIPCHK(hipSetDevice(h->device));
    if (h->batch) return qpb::batch_update_vectors(h->batch, c, b, h->mem_space);
    std::vector<double> hc(h->n), hb(h->m);
    int rc;
    if (c) {
        if ((rc = fetch(hc, c, h->n, h->mem_space))) return rc;
    } else {
        hc = h->h_c;
    }
    if (b && h->m) {
        if ((rc = fetch(hb, b, h->m, h->mem_space))) return rc;
    } else {
        hb = h->h_b;
    }
    h->h_c = hc;
    h->h_b = hb;
    return upload_vectors(h, hc, hb, nullptr, nullptr);
}

int qp_set_norms(qp_handle *h, const double *norm_A, const double *norm_Q) {
    if (!h) return fail(QP_ERR_INVALID_ARGUMENT, "null handle");
    if (h->batch) return qpb::batch_set_norms(h->batch, norm_A, norm_Q);
    const double a = norm_A ? norm_A[0] : h->norm_A, q = norm_Q ? norm_Q[0] : h->norm_Q;
    if (!(a >= 0.0) || !(q >= 0.0) || !(a > 0.0 || q > 0.0))
        return fail(QP_ERR_INVALID_ARGUMENT, "invalid norms");
    h->norm_A = a;
    h->norm_Q = q;
    return QP_OK;
}

int qp_batch_autotune(qp_handle *h, int32_t sample, int32_t iters, int32_t *threads_out) {
    if (!h) return fail(QP_ERR_INVALID_ARGUMENT, "null handle");
    if (!h->batch) return fail(QP_ERR_BATCH_MISMATCH, "qp_batch_autotune needs a batch handle");
    HIPCHK(hipSetDevice(h->device));
    return qpb::batch_autotune(h->batch, &h->set, sample, iters, threads_out);
}

int qp_batch_set_threads(qp_handle *h, const int32_t *threads) {
    if (!h || !threads) return fail(QP_ERR_INVALID_ARGUMENT, "null argument");
    if (!h->batch) return fail(QP_ERR_BATCH_MISMATCH, "qp_batch_set_threads needs a batch handle");
    return qpb::batch_set_threads(h->batch, threads);
}

int qp_get_check_log(qp_handle *h, qp_check_info *buf, int64_t cap, int64_t *len) {
    if (!h) return fail(QP_ERR_INVALID_ARGUMENT, "null handle");
    const int64_t k = std::min<int64_t>(cap, (int64_t)h->log.size());
    if (buf && k > 0) std::memcpy(buf, h->log.data(), (size_t)k * sizeof(qp_check_info));
    if (len) *len = (int64_t)h->log.size();
    return QP_OK;
}

int qp_get_profile(qp_handle *h, qp_profile *out) {
    if (!h || !out) return fail(QP_ERR_INVALID_ARGUMENT, "null argument");
    *out = h->prof;
    return QP_OK;
}

int qp_solve(qp_handle *h, const qp_warm_start *ws, qp_result *res, double *x_out,
             double *y_out) {
    if (!h || !res) return fail(QP_ERR_INVALID_ARGUMENT, "null handle or result");
    if (h->batch) return fail(QP_ERR_BATCH_MISMATCH, "qp_solve on a batch handle: use qp_batch_solve");
    HIPCHK(hipSetDevice(h->device));
    const double t0 = now_s();
    const int64_t n = h->n, m = h->m;
    hipStream_t s = h->stream;
    DevSettings ds = dev_settings(h);
    const int L = ds.interval;
    const bool profile = h->set.profile != 0;
    const int stride = profile ? h->set.profile : 1;  // time every stride-th iteration
    const bool use_graph = h->set.use_graph != 0 && !profile;
    State *st = h->state.as<State>();
    h->log.clear();
    h->prof = qp_profile{};
    h->prof.dual_bytes = 0.0;
    // profiling: two event sets of 3 per iteration, alternating between intervals, so
    // one interval stays in flight while the previous one is read (as without profiling)
    if (profile && (int)h->prof_ev.size() < 6 * L) {
        for (auto &e : h->prof_ev) (void)hipEventDestroy(e);
        h->prof_ev.assign(6 * L, nullptr);
        for (auto &e : h->prof_ev) HIPCHK(hipEventCreate(&e));
    }

    // initial primal weight (Sec. 6 InitializePrimalWeight) unless given
    double omega = (ws && ws->omega0 > 0.0) ? ws->omega0
                   : (h->c_norm2 > h->set.eps_zero && h->b_norm2 > h->set.eps_zero)
                       ? h->c_norm2 / h->b_norm2
                       : 1.0;
    const double *x0 = nullptr, *y0 = nullptr;
    if (ws && (ws->x0 || ws->y0)) {
        const hipMemcpyKind kind = h->mem_space == QP_MEM_HOST ? hipMemcpyHostToDevice
                                                               : hipMemcpyDeviceToDevice;
        const bool sc = !h->h_d.empty();  // warm starts refer to the given problem
        if (ws->x0) {
            HIPCHK(hipMemcpyAsync(h->x0buf.p, ws->x0, n * 8, kind, s));
            x0 = h->x0buf.as<double>();
            if (sc) launch_scale_pair(s, h->x0buf.as<double>(), x0, h->dscale.as<double>(), n, 1);
        }
        if (ws->y0 && m) {
            HIPCHK(hipMemcpyAsync(h->y0buf.p, ws->y0, m * 8, kind, s));
            y0 = h->y0buf.as<double>();
            if (sc)
                launch_scale_pair(s, h->y0buf.as<double>(), y0, h->dscale.as<double>() + n, m, 1);
        }
    }
    const bool warm = ws && (ws->x0 || ws->y0);
    launch_state_reset(s, st, omega, ds.max_iter);
    if (warm && h->set.warm_fallback) {
        launch_init(s, h->vecs, x0, y0, n, m, 1);
        int32_t sa, sp;
        enqueue_kkt(h, s, st, &sa, &sp);
        launch_decide(s, DECIDE_FALLBACK, h->partials_a.as<double>(), sa,
                      h->partials_p.as<double>(), sp, st, h->table.as<Step>(), ds, 0);
        launch_fallback_apply(s, h->vecs, st, n, m);
    } else {
        launch_init(s, h->vecs, x0, y0, n, m, 0);
        if (warm) {
            // warm start taken unconditionally
            State one{};
            HIPCHK(hipStreamSynchronize(s));
            HIPCHK(hipMemcpy(&one, st, sizeof(State), hipMemcpyDeviceToHost));
            one.used_warm = 1;
            HIPCHK(hipMemcpy(st, &one, sizeof(State), hipMemcpyHostToDevice));
        }
    }
    {
        int32_t sa, sp;
        enqueue_kkt(h, s, st, &sa, &sp);
        launch_decide(s, DECIDE_INIT, h->partials_a.as<double>(), sa,
                      h->partials_p.as<double>(), sp, st, h->table.as<Step>(), ds, 0);
    }
    HIPCHK(hipMemcpyAsync(&h->h_state[0], st, sizeof(State), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    State last = h->h_state[0];

    int64_t enqueued = 0;
    int md = 0;
    int slot = 0;
    struct Inflight {
        int slot, len, evset;  // ring slot, interval length, profiling event set
    };
    std::deque<Inflight> inflight;
    int evset = 0;
    bool stop = last.done != 0;
    bool time_up = false;
    int32_t seen_checks = 0;
    auto process = [&](const Inflight &f) -> int {
        const int sl = f.slot, len = f.len;
        HIPCHK(hipEventSynchronize(h->ring_ev[sl]));
        const State &S = h->h_state[sl];
        // an interval enqueued after the solve ended ran as no-ops: not timed
        if (profile && !last.done) {
            const hipEvent_t *ev = h->prof_ev.data() + (size_t)f.evset * 3 * L;
            int timed = 0;
            for (int j = 0; j < len; j += stride, ++timed) {
                float a = 0.f, b = 0.f;
                HIPCHK(hipEventElapsedTime(&a, ev[3 * j + 0], ev[3 * j + 1]));
                HIPCHK(hipEventElapsedTime(&b, ev[3 * j + 1], ev[3 * j + 2]));
                h->prof.dual_ms += a;
                h->prof.primal_ms += b;
            }
            if (m > 0) h->prof.dual_launches += timed;
            h->prof.primal_launches += timed;
        }
        if (S.checks > seen_checks) {
            seen_checks = S.checks;
            if (h->set.log_checks || h->set.log_cb) {
                qp_check_info ci;
                ci.total = S.total;
                ci.k = S.k;
                ci.r_cur = S.r_cur;
                ci.r_avg = S.r_avg;
                ci.candidate = S.cand;
                ci.restarted = S.restart_flag;
                ci.omega = S.omega;
                if (h->set.log_checks) h->log.push_back(ci);
                if (h->set.log_cb) h->set.log_cb(&ci, h->set.log_user);
            }
        }
        last = S;
        if (S.done) stop = true;
        if (h->set.time_limit_s > 0.0 && now_s() - t0 >= h->set.time_limit_s) time_up = true;
        return QP_OK;
    };
    int rc;
    while (!stop && !time_up && enqueued < ds.max_iter) {
        const int len = (int)std::min<int64_t>(L, ds.max_iter - enqueued);
        if (use_graph && len == L) {
            hipGraphExec_t g;
            if ((rc = get_graph(h, ds, md, &g))) return rc;
            HIPCHK(hipGraphLaunch(g, s));
        } else {
            enqueue_interval(h, ds, md, len,
                             profile ? h->prof_ev.data() + (size_t)evset * 3 * L : nullptr,
                             stride);
        }
        md = (md + len) & 1;
        enqueued += len;
        HIPCHK(hipMemcpyAsync(&h->h_state[slot], st, sizeof(State), hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(h->ring_ev[slot], s));
        inflight.push_back(Inflight{slot, len, evset});
        slot = (slot + 1) % qp_handle::RING;
        evset ^= 1;
        // one interval in flight while the previous one is read (with profiling, its
        // event set is the other one of the two)
        while (inflight.size() > 1) {
            const Inflight f = inflight.front();
            inflight.pop_front();
            if ((rc = process(f))) return rc;
        }
    }
    while (!inflight.empty()) {
        const Inflight f = inflight.front();
        inflight.pop_front();
        if ((rc = process(f))) return rc;
    }
    HIPCHK(hipStreamSynchronize(s));
    if (!last.done) last.status = time_up ? QP_TIME_LIMIT : QP_ITERATION_LIMIT;
    if (profile) {
        h->prof.dual_bytes = h->dual_bytes;
        h->prof.primal_bytes = h->primal_bytes;
    }
    // outputs: the candidate of the last evaluation
    const hipMemcpyKind kind = h->mem_space == QP_MEM_HOST ? hipMemcpyDeviceToHost
                                                           : hipMemcpyDeviceToDevice;
    const double *xs = last.cand ? h->vecs.xbar : h->vecs.x;
    const double *ys = last.cand ? h->vecs.ybar : h->vecs.y;
    if (!h->h_d.empty()) {  // back to the given problem: x = D2 x~, y = D1 y~
        launch_scale_pair(s, h->x0buf.as<double>(), xs, h->dscale.as<double>(), n, 0);
        if (m) launch_scale_pair(s, h->y0buf.as<double>(), ys, h->dscale.as<double>() + n, m, 0);
        HIPCHK(hipStreamSynchronize(s));
        xs = h->x0buf.as<double>();
        ys = h->y0buf.as<double>();
    }
    if (x_out) HIPCHK(hipMemcpy(x_out, xs, n * 8, kind));
    if (y_out && m) HIPCHK(hipMemcpy(y_out, ys, m * 8, kind));
    fill_result(h, last, now_s() - t0, res);
    qph::clear_error();
    return QP_OK;
}

int qp_batch_solve(qp_handle *h, const qp_warm_start *ws_array, qp_result *res_array,
                   double *x_out, double *y_out) {
    if (!h || !res_array) return fail(QP_ERR_INVALID_ARGUMENT, "null handle or result array");
    if (!h->batch) return fail(QP_ERR_BATCH_MISMATCH, "qp_batch_solve needs a batch handle");
    HIPCHK(hipSetDevice(h->device));
    return qpb::batch_solve(h->batch, &h->set, h->mem_space, ws_array, res_array, x_out, y_out);
}

}  // extern "C"
