// Host-side code of qp_create checked without a GPU: input validation (invalid host
// problems are rejected before any device call), and the layout builders against their
// definitions: the row-threaded P = [Q | -A'] build and the column-panel split.  Built by
// tests/test_host_layouts.py with hipcc against the library, plainly and with host-side
// AddressSanitizer and UndefinedBehaviorSanitizer; no GPU call is made.
#include "../paper_2311_07710_amd/csrc/qp_api.cpp"

#include <random>
#include <utility>

static int check_build_p(std::mt19937_64 &g) {
    for (int trial = 0; trial < 3; ++trial) {
        const int64_t n = 150000 + trial * 70001, m = trial == 2 ? 0 : n / 2 + 17;
        std::vector<int32_t> qr(n + 1, 0), qc, ar(m + 1, 0), ac;
        std::vector<double> qv, av;
        for (int64_t j = 0; j < n; ++j) {
            const int len = (int)(g() % 12);
            for (int k = 0; k < len; ++k) {
                qc.push_back((int32_t)(g() % n));
                qv.push_back((double)(g() % 999983));
            }
            qr[j + 1] = (int32_t)qc.size();
        }
        for (int64_t i = 0; i < m; ++i) {
            const int len = (int)(g() % 15);
            for (int k = 0; k < len; ++k) {
                ac.push_back((int32_t)(g() % n));
                av.push_back((double)(g() % 999979));
            }
            ar[i + 1] = (int32_t)ac.size();
        }
        std::vector<int32_t> pr, pc;
        std::vector<double> pv;
        build_p(n, m, (int64_t)ac.size(), qr.data(), qc.data(), qv.data(), ar.data(), ac.data(),
                av.data(), pr, pc, pv);
        // definition: row j = Q's row j, then A's entries of column j in increasing row order
        std::vector<std::vector<std::pair<int32_t, double>>> rows(n);
        for (int64_t j = 0; j < n; ++j)
            for (int64_t e = qr[j]; e < qr[j + 1]; ++e) rows[j].push_back({qc[e], qv[e]});
        for (int64_t i = 0; i < m; ++i)
            for (int64_t e = ar[i]; e < ar[i + 1]; ++e)
                rows[ac[e]].push_back({(int32_t)(n + i), -av[e]});
        int64_t pos = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (pr[j] != pos) return printf("build_p: row pointer %ld\n", (long)j), 1;
            for (auto &x : rows[j]) {
                if (pc[pos] != x.first || pv[pos] != x.second)
                    return printf("build_p: entry of row %ld\n", (long)j), 1;
                ++pos;
            }
        }
        if (pr[n] != pos || (int64_t)pc.size() != pos) return printf("build_p: total\n"), 1;
        printf("build_p n=%ld m=%ld ok\n", (long)n, (long)m);
    }
    return 0;
}

static int check_panels(std::mt19937_64 &g) {
    for (int trial = 0; trial < 2; ++trial) {
        const int64_t R = 200000 + trial * 77777, C = 300000 + trial * 1234;
        std::vector<int32_t> rp(R + 1, 0), col;
        std::vector<double> val;
        for (int64_t r = 0; r < R; ++r) {
            int len = (int)(g() % 20);
            if (r == 5 || r == R - 3) len = 5000 + trial;  // rows longer than one block
            std::vector<int32_t> cs;
            for (int k = 0; k < len; ++k) cs.push_back((int32_t)(g() % C));
            std::sort(cs.begin(), cs.end());
            for (int32_t c : cs) {
                col.push_back(c);
                val.push_back((double)(g() % 1000003));
            }
            rp[r + 1] = (int32_t)col.size();
        }
        for (int np : {2, 4, 8}) {
            HostPanels hp = build_panels(rp.data(), col.data(), val.data(), R, C, np);
            std::vector<int> pk(C, -1);  // the panel of each column, read back from hp
            for (int k = 0; k < np; ++k)
                for (int64_t e = hp.rowptr[(size_t)k * (R + 1)]; e < hp.rowptr[(size_t)k * (R + 1) + R];
                     ++e) {
                    if (pk[hp.col[e]] != -1 && pk[hp.col[e]] != k)
                        return printf("panels: column in two panels\n"), 1;
                    pk[hp.col[e]] = k;
                }
            for (int64_t c = 1; c < C; ++c)
                if (pk[c] != -1 && pk[c - 1] != -1 && pk[c] < pk[c - 1])
                    return printf("panels: ranges not ordered\n"), 1;
            // definition: panel k's row r = row r's entries whose column lies in panel k, in order
            for (int64_t r = 0; r < R; ++r)
                for (int k = 0; k < np; ++k) {
                    int64_t q = hp.rowptr[(size_t)k * (R + 1) + r];
                    for (int64_t e = rp[r]; e < rp[r + 1]; ++e)
                        if (pk[col[e]] == k) {
                            if (hp.col[q] != col[e] || hp.val[q] != val[e])
                                return printf("panels: entry r=%ld k=%d\n", (long)r, k), 1;
                            ++q;
                        }
                    if (q != hp.rowptr[(size_t)k * (R + 1) + r + 1])
                        return printf("panels: count r=%ld k=%d\n", (long)r, k), 1;
                }
            printf("panels R=%ld np=%d ok\n", (long)R, np);
        }
    }
    return 0;
}

// qp_create on host input that fails validation: every case is rejected with
// QP_ERR_INVALID_ARGUMENT before any device call (so this runs without a GPU), and the
// validation reads no array beyond what the descriptor promises
static int check_validation() {
    const int32_t qr[4] = {0, 1, 2, 3}, qc[3] = {0, 1, 2};
    const double qv[3] = {1.0, 2.0, 3.0};
    const int32_t ar[3] = {0, 2, 3}, ac[3] = {0, 2, 1};
    const double av[3] = {1.0, -1.0, 0.5}, c[3] = {1, 2, 3}, b[2] = {0, 1};
    const uint8_t rt[2] = {0, 1};
    auto base = [&]() {
        qp_problem_desc d;
        std::memset(&d, 0, sizeof(d));
        d.n = 3;
        d.m = 2;
        d.num_instances = 1;
        d.mem_space = QP_MEM_HOST;
        d.Q.row_ptr = qr; d.Q.col_idx = qc; d.Q.val = qv; d.Q.nnz = 3;
        d.A.row_ptr = ar; d.A.col_idx = ac; d.A.val = av; d.A.nnz = 3;
        d.c = c; d.b = b; d.row_type = rt;
        return d;
    };
    const int32_t qr_desc[4] = {0, 2, 1, 3}, ac_bad[3] = {0, 3, 1}, ar_bad[3] = {1, 2, 3};
    const uint8_t rt_bad[2] = {0, 7};
    struct Case { const char *name; void (*edit)(qp_problem_desc &, const void *); const void *arg; };
    int bad = 0, ncase = 0;
    auto expect = [&](const char *name, qp_problem_desc d) {
        qp_handle *h = nullptr;
        const int rc = qp_create(&d, nullptr, &h);
        ++ncase;
        if (rc != QP_ERR_INVALID_ARGUMENT || h) {
            printf("validation: %s returned %d\n", name, rc);
            ++bad;
        }
    };
    { auto d = base(); d.n = 0; expect("n = 0", d); }
    { auto d = base(); d.m = -1; expect("m < 0", d); }
    { auto d = base(); d.Q.row_ptr = qr_desc; expect("Q row_ptr decreasing", d); }
    { auto d = base(); d.Q.nnz = 2; expect("Q nnz mismatch", d); }
    { auto d = base(); d.A.col_idx = ac_bad; expect("A column out of range", d); }
    { auto d = base(); d.A.row_ptr = ar_bad; expect("A row_ptr[0] != 0", d); }
    { auto d = base(); d.A.col_idx = nullptr; expect("A col_idx null", d); }
    { auto d = base(); d.A.val = nullptr; expect("A val null", d); }
    { auto d = base(); d.Q.val = nullptr; expect("Q val null", d); }
    { auto d = base(); d.c = nullptr; expect("c null", d); }
    { auto d = base(); d.b = nullptr; expect("b null", d); }
    { auto d = base(); d.row_type = rt_bad; expect("row type 7", d); }
    { auto d = base(); d.mem_space = 9; expect("mem_space", d); }
    { auto d = base(); d.n = (int64_t)1 << 31; expect("n beyond int32", d); }
    (void)sizeof(Case);
    printf("validation: %d cases rejected%s\n", ncase, bad ? " (FAILURES)" : "");
    return bad ? 1 : 0;
}

// The automatic panel count: explicit settings kept; 4 panels above 6 MB of gathered
// vector; between 1.75 and 6 MB only for rows of at least 256 entries on average.
static int check_choose_panels() {
    struct Case { int32_t setting; int64_t len, nnz, rows; int want; };
    const int64_t MB = 1 << 20;
    const Case cases[] = {
        {1, 10 * MB, 1000, 10, 1}, {2, 100, 100, 10, 2}, {4, 100, 100, 10, 4},
        {8, 100, 100, 10, 8},                                  // explicit
        {0, 6 * MB / 8 + 1, 10, 10, 4}, {0, 6 * MB / 8, 10, 10, 1},   // size rule at 6 MB
        {0, 4 * MB / 8, 256 * 1001, 1001, 4},                 // long rows, 4 MB
        {0, 4 * MB / 8, 255 * 1001, 1001, 1},                 // rows just too short
        {0, 7 * MB / 32 + 1, 5000 * 1001, 1001, 4},           // long rows above 1.75 MB
        {0, 7 * MB / 32, 5000 * 1001, 1001, 1},               // long rows at 1.75 MB
        {0, 4 * MB / 8, 1000, 0, 1},                          // no rows
    };
    for (const Case &c : cases) {
        const int got = choose_panels(c.setting, c.len, c.nnz, c.rows);
        if (got != c.want) {
            fprintf(stderr, "choose_panels(%d, %lld, %lld, %lld) = %d, want %d\n", c.setting,
                    (long long)c.len, (long long)c.nnz, (long long)c.rows, got, c.want);
            return 1;
        }
    }
    return 0;
}

int main() {
    std::mt19937_64 g(11);
    if (check_validation()) return 1;
    if (check_choose_panels()) return 1;
    if (check_build_p(g) || check_panels(g)) return 1;
    printf("all ok\n");
    return 0;
}
