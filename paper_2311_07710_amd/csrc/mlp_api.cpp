// mlp_api.cpp -- host side of include/qp_mlp.h: buffers, forward, backward
// (mean squared error), Adam, all on the handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/qp_mlp.h"
#include "mlp_internal.h"
#include "qp_host.h"

using qph::DevMem;
using qph::fail;
using namespace mlpk;

static int pad32(int v) { return (v + 31) / 32 * 32; }
static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Workspace of qp_mlp_forward_noalloc: static device memory, one copy per GPU for the
// life of the process.  In host code `scratch` names a host-side stand-in, not a device
// address; its address on each device comes from hipGetSymbolAddress, taken once per
// device by qp_mlp_create with that device current, and only that address is used.
static __device__ __align__(256) unsigned char scratch[QP_MLP_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[MAX_DEVICES];

// the calling thread's current device must be `device`
static int scratch_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES)
        return fail(QP_ERR_INVALID_ARGUMENT, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return QP_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(QP_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", device,
                    hipGetErrorString(e));
    g_scratch_dev[device] = ptr;
    return QP_OK;
}

static void *scratch_of(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_dev[device];
}

struct qp_mlp {
    int L = 0;
    std::vector<int> sz, pad;
    int maxB = 0, Bpad = 0, maxdim = 0, maxpad = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t nparams = 0;
    std::vector<int64_t> w_off, b_off;
    DevMem theta, grad, m1, m2;
    std::vector<DevMem> Wb, WbT, H;
    DevMem outf, dzf, dzb, dzT, HT, dH, part, lpart;
    DevMem bad;  // set by the row-gathering kernels when a row index is out of range
    size_t part_elems = 0;
    int lastB = 0;
    ~qp_mlp() {
        if (stream) (void)hipStreamDestroy(stream);
    }
};

static int zero(DevMem &d, hipStream_t s) {
    HIPCHK(hipMemsetAsync(d.p, 0, d.bytes, s));
    return QP_OK;
}

// refresh the BF16 weight copies (and their transposes) from the FP32 master
static void refresh_bf16(qp_mlp *h) {
    for (int l = 0; l < h->L; ++l) {
        weights_bf16(h->stream, h->theta.as<float>() + h->w_off[l], h->sz[l + 1], h->sz[l],
                     h->Wb[l].as<bf16>(), h->pad[l]);
        transpose_bf16(h->stream, h->Wb[l].as<bf16>(), h->sz[l + 1], h->sz[l], h->pad[l],
                       h->WbT[l].as<bf16>(), h->pad[l + 1]);
    }
}

extern "C" {

int qp_mlp_create(int32_t n_layers, const int32_t *sizes, int32_t max_batch, int32_t device,
                  qp_mlp **out) {
    if (!out || !sizes || n_layers < 1 || max_batch < 1)
        return fail(QP_ERR_INVALID_ARGUMENT, "qp_mlp_create: bad arguments");
    *out = nullptr;
    for (int i = 0; i <= n_layers; ++i)
        if (sizes[i] < 1) return fail(QP_ERR_INVALID_ARGUMENT, "layer size must be >= 1");
    HIPCHK(hipSetDevice(device));
    if (int rc0 = scratch_setup(device)) return rc0;
    qp_mlp *h = new qp_mlp();
    h->L = n_layers;
    h->device = device;
    h->maxB = max_batch;
    h->Bpad = pad32(max_batch);
    for (int i = 0; i <= n_layers; ++i) {
        h->sz.push_back(sizes[i]);
        h->pad.push_back(pad32(sizes[i]));
        h->maxdim = std::max(h->maxdim, (int)sizes[i]);
        h->maxpad = std::max(h->maxpad, pad32(sizes[i]));
    }
    int64_t off = 0;
    for (int l = 0; l < n_layers; ++l) {
        h->w_off.push_back(off);
        off += (int64_t)sizes[l + 1] * sizes[l];
        h->b_off.push_back(off);
        off += sizes[l + 1];
    }
    h->nparams = off;
    int rc = QP_OK;
    auto done = [&](int code) {
        delete h;
        return code;
    };
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
        return done(fail(QP_ERR_DEVICE, "hipStreamCreate failed"));
    const size_t P = (size_t)off * 4;
    if ((rc = h->theta.alloc(P)) || (rc = h->grad.alloc(P)) || (rc = h->m1.alloc(P)) ||
        (rc = h->m2.alloc(P)))
        return done(rc);
    h->Wb.resize(n_layers);
    h->WbT.resize(n_layers);
    h->H.resize(n_layers + 1);
    for (int l = 0; l < n_layers; ++l) {
        if ((rc = h->Wb[l].alloc((size_t)sizes[l + 1] * h->pad[l] * 2)) ||
            (rc = h->WbT[l].alloc((size_t)sizes[l] * h->pad[l + 1] * 2)))
            return done(rc);
    }
    for (int l = 0; l <= n_layers; ++l)
        if ((rc = h->H[l].alloc((size_t)h->maxB * h->pad[l] * 2))) return done(rc);
    // split-K partial buffer: the largest S*M*N over the planned products
    size_t pe = 0;
    for (int l = 0; l < n_layers; ++l) {
        const int M = h->maxB, N = sizes[l + 1], K = h->pad[l];
        pe = std::max(pe, (size_t)splitk_for(M, N, K) * M * N);          // forward
        pe = std::max(pe, (size_t)splitk_for(N, sizes[l], h->Bpad) * N * sizes[l]);  // dW
        pe = std::max(pe, (size_t)splitk_for(M, sizes[l], h->pad[l + 1]) * M * sizes[l]);  // dH
    }
    h->part_elems = pe;
    if ((rc = h->outf.alloc((size_t)h->maxB * sizes[n_layers] * 4)) ||
        (rc = h->dzf.alloc((size_t)h->maxB * h->maxdim * 4)) ||
        (rc = h->dzb.alloc((size_t)h->maxB * h->maxpad * 2)) ||
        (rc = h->dzT.alloc((size_t)h->maxdim * h->Bpad * 2)) ||
        (rc = h->HT.alloc((size_t)h->maxdim * h->Bpad * 2)) ||
        (rc = h->dH.alloc((size_t)h->maxB * h->maxdim * 4)) || (rc = h->part.alloc(pe * 4)) ||
        (rc = h->lpart.alloc(1024 * 8)) || (rc = h->bad.alloc(4)))
        return done(rc);
    DevMem *all[] = {&h->theta, &h->grad, &h->m1, &h->m2, &h->dzb, &h->dzT, &h->HT, &h->bad};
    for (DevMem *d : all)
        if ((rc = zero(*d, h->stream))) return done(rc);
    for (auto &d : h->Wb)
        if ((rc = zero(d, h->stream))) return done(rc);
    for (auto &d : h->WbT)
        if ((rc = zero(d, h->stream))) return done(rc);
    for (auto &d : h->H)
        if ((rc = zero(d, h->stream))) return done(rc);
    if (hipStreamSynchronize(h->stream) != hipSuccess)
        return done(fail(QP_ERR_DEVICE, "qp_mlp_create: device error"));
    *out = h;
    return QP_OK;
}

void qp_mlp_free(qp_mlp *h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

int64_t qp_mlp_num_params(const qp_mlp *h) { return h ? h->nparams : 0; }

int qp_mlp_set_params(qp_mlp *h, const float *params) {
    if (!h || !params) return fail(QP_ERR_INVALID_ARGUMENT, "null argument");
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipMemcpyAsync(h->theta.p, params, (size_t)h->nparams * 4, hipMemcpyHostToDevice,
                          h->stream));
    int rc;
    if ((rc = zero(h->m1, h->stream)) || (rc = zero(h->m2, h->stream))) return rc;
    refresh_bf16(h);
    HIPCHK(hipStreamSynchronize(h->stream));
    return QP_OK;
}

int qp_mlp_get_params(qp_mlp *h, float *params) {
    if (!h || !params) return fail(QP_ERR_INVALID_ARGUMENT, "null argument");
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipMemcpy(params, h->theta.p, (size_t)h->nparams * 4, hipMemcpyDeviceToHost));
    return QP_OK;
}

int qp_mlp_get_grads(qp_mlp *h, float *grads) {
    if (!h || !grads) return fail(QP_ERR_INVALID_ARGUMENT, "null argument");
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipMemcpy(grads, h->grad.p, (size_t)h->nparams * 4, hipMemcpyDeviceToHost));
    return QP_OK;
}

int qp_mlp_set_grads(qp_mlp *h, const float *grads) {
    if (!h || !grads) return fail(QP_ERR_INVALID_ARGUMENT, "null argument");
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipMemcpyAsync(h->grad.p, grads, (size_t)h->nparams * 4, hipMemcpyHostToDevice,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return QP_OK;
}

}  // extern "C"

// reads the out-of-range flag of the row-gathering kernels (the stream is synchronised)
static int check_rows(qp_mlp *h, const char *who) {
    int32_t bad = 0;
    HIPCHK(hipMemcpy(&bad, h->bad.p, 4, hipMemcpyDeviceToHost));
    if (bad) {
        HIPCHK(hipMemset(h->bad.p, 0, 4));
        return fail(QP_ERR_INVALID_ARGUMENT, "%s: a row index is outside [0, n_rows)", who);
    }
    return QP_OK;
}

static int forward_impl(qp_mlp *h, const float *x, const int32_t *rows, int64_t n_rows,
                        int32_t batch, float *out) {
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = h->stream;
    to_bf16(s, x, batch, h->sz[0], h->H[0].as<bf16>(), h->pad[0], rows, n_rows,
            h->bad.as<int32_t>());
    for (int l = 0; l < h->L; ++l) {
        const int N = h->sz[l + 1], K = h->pad[l];
        const int S = splitk_for(batch, N, K);
        gemm_nt(s, h->H[l].as<bf16>(), h->pad[l], h->Wb[l].as<bf16>(), h->pad[l],
                h->part.as<float>(), batch, N, K, S);
        const bool last = l == h->L - 1;
        reduce_epi(s, h->part.as<float>(), S, batch, N, h->theta.as<float>() + h->b_off[l],
                   last ? 0 : 1, last ? h->outf.as<float>() : nullptr, N,
                   last ? nullptr : h->H[l + 1].as<bf16>(), h->pad[l + 1]);
    }
    if (out)
        HIPCHK(hipMemcpyAsync(out, h->outf.p, (size_t)batch * h->sz[h->L] * 4,
                              hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    int rc;
    if (rows && (rc = check_rows(h, "qp_mlp_forward_rows"))) {
        h->lastB = 0;
        return rc;
    }
    h->lastB = batch;
    return QP_OK;
}

extern "C" {

int qp_mlp_forward(qp_mlp *h, const float *x, int32_t batch, float *out) {
    if (!h || !x) return fail(QP_ERR_INVALID_ARGUMENT, "null argument");
    if (batch < 1 || batch > h->maxB) return fail(QP_ERR_INVALID_ARGUMENT, "batch out of range");
    return forward_impl(h, x, nullptr, 0, batch, out);
}

int qp_mlp_forward_rows(qp_mlp *h, const float *x_all, int64_t n_rows, const int32_t *rows,
                        int32_t batch, float *out) {
    if (!h || !x_all || !rows) return fail(QP_ERR_INVALID_ARGUMENT, "null argument");
    if (batch < 1 || batch > h->maxB) return fail(QP_ERR_INVALID_ARGUMENT, "batch out of range");
    if (n_rows < 1) return fail(QP_ERR_INVALID_ARGUMENT, "n_rows must be >= 1");
    return forward_impl(h, x_all, rows, n_rows, batch, out);
}

int qp_mlp_forward_noalloc(qp_mlp *h, const float *x, int32_t batch, float *out) {
    if (!h || !x || !out) return fail(QP_ERR_INVALID_ARGUMENT, "null argument");
    if (batch < 1 || batch > h->maxB) return fail(QP_ERR_INVALID_ARGUMENT, "batch out of range");
    // workspace: BF16 activations of even layers' inputs, of odd layers' inputs, and the
    // split-K partial tiles of the largest product
    size_t act[2] = {0, 0}, part = 0;
    for (int l = 0; l < h->L; ++l) {
        act[l & 1] = std::max(act[l & 1], (size_t)batch * h->pad[l] * 2);
        const int N = h->sz[l + 1];
        part = std::max(part, (size_t)splitk_for(batch, N, h->pad[l]) * batch * N * 4);
    }
    const size_t off1 = align256(act[0]), offp = off1 + align256(act[1]);
    const size_t need = offp + part;
    if (need > (size_t)QP_MLP_NOALLOC_SCRATCH_BYTES)
        return fail(QP_ERR_INVALID_ARGUMENT,
                    "qp_mlp_forward_noalloc: batch %d needs %zu bytes of workspace, above the "
                    "%zu-byte limit",
                    (int)batch, need, (size_t)QP_MLP_NOALLOC_SCRATCH_BYTES);
    HIPCHK(hipSetDevice(h->device));
    unsigned char *ws = (unsigned char *)scratch_of(h->device);
    if (!ws) return fail(QP_ERR_DEVICE, "no workspace address for device %d", h->device);
    bf16 *bufs[2] = {(bf16 *)ws, (bf16 *)(ws + off1)};
    float *pt = (float *)(ws + offp);
    hipStream_t s = h->stream;
    to_bf16(s, x, batch, h->sz[0], bufs[0], h->pad[0]);
    for (int l = 0; l < h->L; ++l) {
        const int N = h->sz[l + 1], K = h->pad[l];
        const int S = splitk_for(batch, N, K);
        gemm_nt(s, bufs[l & 1], K, h->Wb[l].as<bf16>(), K, pt, batch, N, K, S);
        if (l == h->L - 1) {
            reduce_epi(s, pt, S, batch, N, h->theta.as<float>() + h->b_off[l], 0, out, N,
                       nullptr, 0);
        } else {
            bf16 *nx = bufs[(l + 1) & 1];
            // the workspace keeps the previous call's contents: the K padding of the next
            // layer's input must read as zeros
            zero_pad_bf16(s, nx, batch, N, h->pad[l + 1]);
            reduce_epi(s, pt, S, batch, N, h->theta.as<float>() + h->b_off[l], 1, nullptr, 0,
                       nx, h->pad[l + 1]);
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    return QP_OK;
}

}  // extern "C"

static int backward_impl(qp_mlp *h, const float *target, const int32_t *rows, int64_t n_rows,
                         int32_t batch, float *loss) {
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = h->stream;
    const int L = h->L, NO = h->sz[L];
    const float coef = 2.0f / ((float)batch * (float)NO);
    const int nb = mse_grad(s, h->outf.as<float>(), target, batch, NO, coef, h->dzf.as<float>(),
                            h->dzb.as<bf16>(), h->pad[L], h->lpart.as<double>(), rows, n_rows,
                            h->bad.as<int32_t>());
    for (int l = L - 1; l >= 0; --l) {
        const int No = h->sz[l + 1], Ni = h->sz[l];
        // dW_l = dZ_l' H_l  (K = batch)
        transpose_bf16(s, h->dzb.as<bf16>(), batch, No, h->pad[l + 1], h->dzT.as<bf16>(),
                       pad32(batch));
        transpose_bf16(s, h->H[l].as<bf16>(), batch, Ni, h->pad[l], h->HT.as<bf16>(),
                       pad32(batch));
        int S = splitk_for(No, Ni, pad32(batch));
        gemm_nt(s, h->dzT.as<bf16>(), pad32(batch), h->HT.as<bf16>(), pad32(batch),
                h->part.as<float>(), No, Ni, pad32(batch), S);
        reduce_epi(s, h->part.as<float>(), S, No, Ni, nullptr, 0,
                   h->grad.as<float>() + h->w_off[l], Ni, nullptr, 0);
        // the split-K partial buffer is free between the dW and dH products
        colsum(s, h->dzf.as<float>(), batch, No, h->part.as<float>(),
               h->grad.as<float>() + h->b_off[l]);
        if (l > 0) {
            // dH_l = dZ_l W_l, then the ReLU mask of H_l
            S = splitk_for(batch, Ni, h->pad[l + 1]);
            gemm_nt(s, h->dzb.as<bf16>(), h->pad[l + 1], h->WbT[l].as<bf16>(), h->pad[l + 1],
                    h->part.as<float>(), batch, Ni, h->pad[l + 1], S);
            reduce_epi(s, h->part.as<float>(), S, batch, Ni, nullptr, 0, h->dH.as<float>(), Ni,
                       nullptr, 0);
            relu_back(s, h->dH.as<float>(), h->H[l].as<bf16>(), h->pad[l], batch, Ni,
                      h->dzf.as<float>(), h->dzb.as<bf16>(), h->pad[l]);
        }
    }
    std::vector<double> lp(nb);
    HIPCHK(hipMemcpyAsync(lp.data(), h->lpart.p, nb * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double acc = 0.0;
    for (double v : lp) acc += v;
    if (loss) *loss = (float)(acc / ((double)batch * NO));
    if (rows) return check_rows(h, "qp_mlp_backward_rows");
    return QP_OK;
}

extern "C" {

int qp_mlp_backward(qp_mlp *h, const float *target, int32_t batch, float *loss) {
    if (!h || !target) return fail(QP_ERR_INVALID_ARGUMENT, "null argument");
    if (batch < 1 || batch != h->lastB)
        return fail(QP_ERR_INVALID_ARGUMENT, "backward needs the last forward batch");
    return backward_impl(h, target, nullptr, 0, batch, loss);
}

int qp_mlp_backward_rows(qp_mlp *h, const float *target_all, int64_t n_rows,
                         const int32_t *rows, int32_t batch, float *loss) {
    if (!h || !target_all || !rows) return fail(QP_ERR_INVALID_ARGUMENT, "null argument");
    if (batch < 1 || batch != h->lastB)
        return fail(QP_ERR_INVALID_ARGUMENT, "backward needs the last forward batch");
    if (n_rows < 1) return fail(QP_ERR_INVALID_ARGUMENT, "n_rows must be >= 1");
    return backward_impl(h, target_all, rows, n_rows, batch, loss);
}

int qp_mlp_adam_step(qp_mlp *h, float lr, float beta1, float beta2, float eps, int32_t step) {
    if (!h || step < 1) return fail(QP_ERR_INVALID_ARGUMENT, "bad Adam arguments");
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = h->stream;
    const float c1 = 1.0f - std::pow(beta1, (float)step), c2 = 1.0f - std::pow(beta2, (float)step);
    for (int l = 0; l < h->L; ++l) {
        const int64_t nw = (int64_t)h->sz[l + 1] * h->sz[l];
        float *th = h->theta.as<float>(), *g = h->grad.as<float>();
        float *m = h->m1.as<float>(), *v = h->m2.as<float>();
        adam(s, th + h->w_off[l], g + h->w_off[l], m + h->w_off[l], v + h->w_off[l], nw, lr,
             beta1, beta2, eps, c1, c2, h->Wb[l].as<bf16>(), h->sz[l], h->pad[l]);
        adam(s, th + h->b_off[l], g + h->b_off[l], m + h->b_off[l], v + h->b_off[l], h->sz[l + 1],
             lr, beta1, beta2, eps, c1, c2, nullptr, 1, 1);
        transpose_bf16(s, h->Wb[l].as<bf16>(), h->sz[l + 1], h->sz[l], h->pad[l],
                       h->WbT[l].as<bf16>(), h->pad[l + 1]);
    }
    HIPCHK(hipStreamSynchronize(s));
    return QP_OK;
}

}  // extern "C"
