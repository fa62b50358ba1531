// Host-side layout builders of qp_create checked against their definitions: the
// row-threaded P = [Q | -A'] build and the column-panel split.  Built by
// tests/test_host_layouts.py with hipcc against the library; no GPU call is made.
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

int main() {
    std::mt19937_64 g(11);
    if (check_build_p(g) || check_panels(g)) return 1;
    printf("all ok\n");
    return 0;
}
