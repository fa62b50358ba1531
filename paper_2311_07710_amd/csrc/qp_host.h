// qp_host.h -- host-side helpers shared by the single-instance and batched
// solvers: thread-local error reporting, HIP error mapping, device buffers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <tuple>
#include <vector>

#include "../../include/qp.h"

namespace qph {

// records a formatted message for qp_last_error() and returns `code`
int fail(int code, const char *fmt, ...);
void clear_error();
double now_s();

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess)                                                                 \
            return ::qph::fail(_e == hipErrorOutOfMemory ? QP_ERR_OUT_OF_MEMORY : QP_ERR_DEVICE, \
                               "%s failed: %s", #expr, hipGetErrorString(_e));                \
    } while (0)

struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    DevMem(DevMem &&o) noexcept : p(o.p), bytes(o.bytes) {
        o.p = nullptr;
        o.bytes = 0;
    }
    DevMem &operator=(DevMem &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            o.p = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DevMem() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    int alloc(size_t b) {
        release();
        bytes = b;
        if (b == 0) return QP_OK;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(QP_ERR_OUT_OF_MEMORY, "hipMalloc(%zu) failed: %s", b, hipGetErrorString(e));
        }
        return QP_OK;
    }
    // Copies b bytes from the host and appends UPLOAD_PAD zero bytes: kernels that
    // read one entry past a range (an empty block at the end of an array) stay in bounds.
    static constexpr size_t UPLOAD_PAD = 16;
    int upload(const void *src, size_t b) {
        int rc = alloc(b + UPLOAD_PAD);
        if (rc) return rc;
        if (b) HIPCHK(hipMemcpy(p, src, b, hipMemcpyHostToDevice));
        HIPCHK(hipMemset((char *)p + b, 0, UPLOAD_PAD));
        return QP_OK;
    }
    template <class T> T *as() const { return (T *)p; }
};

// Q (n x n, rows rowptr[0..n], which may be offsets into a larger array) must equal its
// transpose exactly, entry by entry (duplicates are summed on both sides).
inline int check_symmetric(int64_t n, const int32_t *rowptr, const int32_t *col,
                           const double *val, int instance) {
    std::vector<std::tuple<int32_t, int32_t, double>> e, t;
    const int64_t base = rowptr[0];
    e.reserve((size_t)(rowptr[n] - base));
    for (int64_t r = 0; r < n; ++r)
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
            e.emplace_back((int32_t)r, col[k], val[k]);
            t.emplace_back(col[k], (int32_t)r, val[k]);
        }
    auto canon = [](std::vector<std::tuple<int32_t, int32_t, double>> &v) {
        std::sort(v.begin(), v.end());
        std::vector<std::tuple<int32_t, int32_t, double>> out;
        for (auto &x : v) {
            if (!out.empty() && std::get<0>(out.back()) == std::get<0>(x) &&
                std::get<1>(out.back()) == std::get<1>(x))
                std::get<2>(out.back()) += std::get<2>(x);
            else
                out.push_back(x);
        }
        v.swap(out);
    };
    canon(e);
    canon(t);
    if (e.size() != t.size())
        return fail(QP_ERR_INVALID_ARGUMENT, "Q of instance %d is not symmetric (pattern)", instance);
    for (size_t k = 0; k < e.size(); ++k)
        if (std::get<0>(e[k]) != std::get<0>(t[k]) || std::get<1>(e[k]) != std::get<1>(t[k]) ||
            std::get<2>(e[k]) != std::get<2>(t[k]))
            return fail(QP_ERR_INVALID_ARGUMENT, "Q of instance %d is not symmetric at (%d, %d)",
                        instance, (int)std::get<0>(e[k]), (int)std::get<1>(e[k]));
    return QP_OK;
}

}  // namespace qph
