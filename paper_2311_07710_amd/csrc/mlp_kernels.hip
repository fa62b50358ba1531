// mlp_kernels.hip -- BF16 MFMA kernels of the warm-start MLP (gfx950).
//
// GEMM: C = A * B^T with A (M x K) and B (N x K) both K-contiguous BF16, FP32
// accumulation on __builtin_amdgcn_mfma_f32_32x32x16_bf16.  A workgroup of 4
// wavefronts owns a 64 x 64 tile (each wave a 32 x 32 MFMA tile); K is
// streamed through LDS in steps of 32.  Large K is split over blockIdx.z into
// FP32 partial tiles that a second kernel adds in slice order (deterministic)
// while applying bias / ReLU and writing FP32 and/or BF16 outputs.  Every BF16
// matrix is stored with its row length padded to a multiple of 32 and zeros in
// the padding, so the K loop needs no bounds checks.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "mlp_internal.h"

namespace mlpk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float float16v __attribute__((ext_vector_type(16)));

constexpr int GBM = 64, GBN = 64, GBK = 32, GPAD = 8;

__global__ __launch_bounds__(256) void k_gemm_nt(const bf16 *__restrict__ A, int lda,
                                                 const bf16 *__restrict__ B, int ldb,
                                                 float *__restrict__ C, int M, int N, int Kpad,
                                                 int kchunk) {
    __shared__ __attribute__((aligned(16))) bf16 As[GBM][GBK + GPAD];
    __shared__ __attribute__((aligned(16))) bf16 Bs[GBN][GBK + GPAD];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int kb = blockIdx.z * kchunk;
    const int ke = min(Kpad, kb + kchunk);
    float16v acc = {};
    const int lr = t >> 2, lk = (t & 3) * 8;
    for (int k0 = kb; k0 < ke; k0 += GBK) {
        bf16x8 va = {}, vb = {};
        if (m0 + lr < M) va = *(const bf16x8 *)(A + (size_t)(m0 + lr) * lda + k0 + lk);
        if (n0 + lr < N) vb = *(const bf16x8 *)(B + (size_t)(n0 + lr) * ldb + k0 + lk);
        *(bf16x8 *)&As[lr][lk] = va;
        *(bf16x8 *)&Bs[lr][lk] = vb;
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 16) {
            const bf16x8 a = *(const bf16x8 *)&As[wm * 32 + (lane & 31)][kk + (lane >> 5) * 8];
            const bf16x8 b = *(const bf16x8 *)&Bs[wn * 32 + (lane & 31)][kk + (lane >> 5) * 8];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    float *Cz = C + (size_t)blockIdx.z * M * N;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int col = n0 + wn * 32 + (lane & 31);
        if (row < M && col < N) Cz[(size_t)row * N + col] = acc[v];
    }
}

// out = sum_z part[z] (+ bias) (ReLU), FP32 (ld ldf) and/or BF16 (ld ldb)
__global__ void k_reduce_epi(const float *__restrict__ part, int S, int M, int N,
                             const float *__restrict__ bias, int relu, float *__restrict__ outf,
                             int ldf, bf16 *__restrict__ outb, int ldb) {
    const int64_t total = (int64_t)M * N;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const int row = (int)(idx / N), col = (int)(idx % N);
        float s = part[idx];
        for (int z = 1; z < S; ++z) s += part[(size_t)z * total + idx];
        if (bias) s += bias[col];
        if (relu) s = s > 0.f ? s : 0.f;
        if (outf) outf[(size_t)row * ldf + col] = s;
        if (outb) outb[(size_t)row * ldb + col] = (bf16)s;
    }
}

// FP32 [rows x cols] -> BF16 [rows x ld] with zeros in columns [cols, ld).  With `sel`,
// row r of the output is row sel[r] of `in` (which has nsrc rows); an index outside
// [0, nsrc) gives a zero row and sets *bad.
__global__ void k_to_bf16(const float *__restrict__ in, int rows, int cols, bf16 *__restrict__ out,
                          int ld, const int32_t *__restrict__ sel, int64_t nsrc,
                          int32_t *__restrict__ bad) {
    const int64_t total = (int64_t)rows * ld;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const int r = (int)(idx / ld), c = (int)(idx % ld);
        int64_t src = r;
        if (sel) {
            src = sel[r];
            if (src < 0 || src >= nsrc) {
                *bad = 1;
                out[idx] = (bf16)0.f;
                continue;
            }
        }
        out[idx] = c < cols ? (bf16)in[src * cols + c] : (bf16)0.f;
    }
}

// out[c][r] = in[r][c] for r < rows, c < cols; zeros for r in [rows, ldo)
__global__ void k_transpose_bf16(const bf16 *__restrict__ in, int rows, int cols, int ldi,
                                 bf16 *__restrict__ out, int ldo) {
    __shared__ bf16 tile[32][33];
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
    for (int k = ty; k < 32; k += 8) {
        const int r = r0 + k, c = c0 + tx;
        tile[k][tx] = (r < rows && c < cols) ? in[(size_t)r * ldi + c] : (bf16)0.f;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int c = c0 + k, r = r0 + tx;
        if (c < cols && r < ldo) out[(size_t)c * ldo + r] = tile[tx][k];
    }
}

// dO = coef (O - T) (FP32 and padded BF16); per-block partial sums of (O - T)^2.  With
// `sel`, the target of sample r is row sel[r] of T (nsrc rows); an index outside
// [0, nsrc) gives a zero gradient row and sets *bad.
__global__ __launch_bounds__(256) void k_mse_grad(const float *__restrict__ O,
                                                  const float *__restrict__ T, int B, int N,
                                                  float coef, float *__restrict__ dzf,
                                                  bf16 *__restrict__ dzb, int ldb,
                                                  double *__restrict__ lpart,
                                                  const int32_t *__restrict__ sel, int64_t nsrc,
                                                  int32_t *__restrict__ bad) {
    __shared__ double red[256];
    const int64_t total = (int64_t)B * ldb;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double acc = 0.0;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const int r = (int)(idx / ldb), c = (int)(idx % ldb);
        int64_t tr = r;
        bool ok = true;
        if (sel) {
            tr = sel[r];
            ok = tr >= 0 && tr < nsrc;
            if (!ok) *bad = 1;
        }
        if (c < N && ok) {
            const float d = O[(size_t)r * N + c] - T[tr * N + c];
            acc += (double)d * (double)d;
            const float g = coef * d;
            dzf[(size_t)r * N + c] = g;
            dzb[idx] = (bf16)g;
        } else {
            if (c < N) dzf[(size_t)r * N + c] = 0.f;
            dzb[idx] = (bf16)0.f;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// dZ = dH * (H > 0): FP32 [B x N] and padded BF16 [B x ldb]; H is BF16 [B x ldh]
__global__ void k_relu_back(const float *__restrict__ dH, const bf16 *__restrict__ H, int ldh,
                            int B, int N, float *__restrict__ dzf, bf16 *__restrict__ dzb,
                            int ldb) {
    const int64_t total = (int64_t)B * ldb;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const int r = (int)(idx / ldb), c = (int)(idx % ldb);
        if (c < N) {
            const float g = (float)H[(size_t)r * ldh + c] > 0.f ? dH[(size_t)r * N + c] : 0.f;
            dzf[(size_t)r * N + c] = g;
            dzb[idx] = (bf16)g;
        } else {
            dzb[idx] = (bf16)0.f;
        }
    }
}

// db[j] = sum_b dZ[b][j] in two stages with a fixed order.  Stage 1: workgroup (x, y)
// sums rows [64y, 64y + 64) of columns [64x, 64x + 64): lane q of column j adds rows
// 64y + q, 64y + q + 4, ... in order, then the four lane sums are added in lane order
// into part[y][j].  Stage 2 adds the row chunks in order.
__global__ __launch_bounds__(256) void k_colsum_part(const float *__restrict__ dz, int B, int N,
                                                     float *__restrict__ part) {
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    const int r0 = blockIdx.y * 64, r1 = min(B, r0 + 64);
    float s = 0.f;
    if (j < N)
        for (int r = r0 + q; r < r1; r += 4) s += dz[(size_t)r * N + j];
    red[q][c] = s;
    __syncthreads();
    if (q == 0 && j < N)
        part[(size_t)blockIdx.y * N + j] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ void k_colsum_fin(const float *__restrict__ part, int chunks, int N,
                             float *__restrict__ db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = part[j];
    for (int y = 1; y < chunks; ++y) s += part[(size_t)y * N + j];
    db[j] = s;
}

// Adam (bias-corrected) on n parameters; optional BF16 copy of a [rows x cols]
// weight block into a padded [rows x ld] matrix
__global__ void k_adam(float *__restrict__ theta, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, bf16 *__restrict__ wb, int cols, int ld) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float th = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        theta[i] = th;
        if (wb) wb[(i / cols) * ld + (i % cols)] = (bf16)th;
    }
}

// zeros in columns [c0, ld) of every row of a BF16 [rows x ld] matrix
__global__ void k_zero_pad_bf16(bf16 *__restrict__ p, int rows, int c0, int ld) {
    const int w = ld - c0;
    const int64_t total = (int64_t)rows * w;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride)
        p[(idx / w) * ld + c0 + idx % w] = (bf16)0.f;
}

// BF16 copy of a [rows x cols] FP32 block into [rows x ld] (zeros in the padding)
__global__ void k_weights_bf16(const float *__restrict__ w, int rows, int cols,
                               bf16 *__restrict__ wb, int ld) {
    const int64_t total = (int64_t)rows * ld;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const int r = (int)(idx / ld), c = (int)(idx % ld);
        wb[idx] = c < cols ? (bf16)w[(size_t)r * cols + c] : (bf16)0.f;
    }
}

static unsigned grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}

int splitk_for(int M, int N, int Kpad) {
    const int tiles = ((M + GBM - 1) / GBM) * ((N + GBN - 1) / GBN);
    int s = (512 + tiles - 1) / tiles;
    if (s > 16) s = 16;
    const int ksteps = Kpad / GBK;
    if (s > ksteps) s = ksteps;
    return s < 1 ? 1 : s;
}

void gemm_nt(hipStream_t st, const bf16 *A, int lda, const bf16 *B, int ldb, float *part, int M,
             int N, int Kpad, int S) {
    const int steps = Kpad / GBK;
    const int kchunk = ((steps + S - 1) / S) * GBK;
    dim3 grid((N + GBN - 1) / GBN, (M + GBM - 1) / GBM, S);
    hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, A, lda, B, ldb, part, M, N, Kpad, kchunk);
}

void reduce_epi(hipStream_t st, const float *part, int S, int M, int N, const float *bias,
                int relu, float *outf, int ldf, bf16 *outb, int ldb) {
    hipLaunchKernelGGL(k_reduce_epi, dim3(grid_for((int64_t)M * N)), dim3(256), 0, st, part, S, M,
                       N, bias, relu, outf, ldf, outb, ldb);
}

void to_bf16(hipStream_t st, const float *in, int rows, int cols, bf16 *out, int ld,
             const int32_t *sel, int64_t nsrc, int32_t *bad) {
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for((int64_t)rows * ld)), dim3(256), 0, st, in, rows,
                       cols, out, ld, sel, nsrc, bad);
}

void transpose_bf16(hipStream_t st, const bf16 *in, int rows, int cols, int ldi, bf16 *out,
                    int ldo) {
    dim3 grid((cols + 31) / 32, (ldo + 31) / 32);
    hipLaunchKernelGGL(k_transpose_bf16, grid, dim3(256), 0, st, in, rows, cols, ldi, out, ldo);
}

int mse_grad(hipStream_t st, const float *O, const float *T, int B, int N, float coef, float *dzf,
             bf16 *dzb, int ldb, double *lpart, const int32_t *sel, int64_t nsrc, int32_t *bad) {
    const unsigned g = grid_for((int64_t)B * ldb) > 1024 ? 1024 : grid_for((int64_t)B * ldb);
    hipLaunchKernelGGL(k_mse_grad, dim3(g), dim3(256), 0, st, O, T, B, N, coef, dzf, dzb, ldb,
                       lpart, sel, nsrc, bad);
    return (int)g;
}

void relu_back(hipStream_t st, const float *dH, const bf16 *H, int ldh, int B, int N, float *dzf,
               bf16 *dzb, int ldb) {
    hipLaunchKernelGGL(k_relu_back, dim3(grid_for((int64_t)B * ldb)), dim3(256), 0, st, dH, H,
                       ldh, B, N, dzf, dzb, ldb);
}

void colsum(hipStream_t st, const float *dz, int B, int N, float *part, float *db) {
    const int chunks = (B + 63) / 64;
    hipLaunchKernelGGL(k_colsum_part, dim3((N + 63) / 64, chunks), dim3(256), 0, st, dz, B, N,
                       part);
    hipLaunchKernelGGL(k_colsum_fin, dim3((N + 255) / 256), dim3(256), 0, st, part, chunks, N, db);
}

void adam(hipStream_t st, float *theta, const float *g, float *m, float *v, int64_t n, float lr,
          float b1, float b2, float eps, float c1, float c2, bf16 *wb, int cols, int ld) {
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, st, theta, g, m, v, n, lr, b1, b2,
                       eps, c1, c2, wb, cols, ld);
}

void zero_pad_bf16(hipStream_t st, bf16 *p, int rows, int c0, int ld) {
    if (c0 >= ld || rows < 1) return;
    hipLaunchKernelGGL(k_zero_pad_bf16, dim3(grid_for((int64_t)rows * (ld - c0))), dim3(256), 0,
                       st, p, rows, c0, ld);
}

void weights_bf16(hipStream_t st, const float *w, int rows, int cols, bf16 *wb, int ld) {
    hipLaunchKernelGGL(k_weights_bf16, dim3(grid_for((int64_t)rows * ld)), dim3(256), 0, st, w,
                       rows, cols, wb, ld);
}

}  // namespace mlpk
