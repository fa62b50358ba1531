// mlp_internal.h -- launchers of the warm-start MLP kernels (mlp_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

namespace mlpk {

typedef __bf16 bf16;

int splitk_for(int M, int N, int Kpad);
// part[z][M][N] = A[M x Kpad] * B[N x Kpad]^T over K slice z (S slices)
void gemm_nt(hipStream_t st, const bf16 *A, int lda, const bf16 *B, int ldb, float *part, int M,
             int N, int Kpad, int S);
void reduce_epi(hipStream_t st, const float *part, int S, int M, int N, const float *bias,
                int relu, float *outf, int ldf, bf16 *outb, int ldb);
// sel (device, optional): output row r is input row sel[r] of nsrc rows; a bad index
// gives a zero row and sets *bad
void to_bf16(hipStream_t st, const float *in, int rows, int cols, bf16 *out, int ld,
             const int32_t *sel = nullptr, int64_t nsrc = 0, int32_t *bad = nullptr);
void transpose_bf16(hipStream_t st, const bf16 *in, int rows, int cols, int ldi, bf16 *out,
                    int ldo);
int mse_grad(hipStream_t st, const float *O, const float *T, int B, int N, float coef, float *dzf,
             bf16 *dzb, int ldb, double *lpart, const int32_t *sel = nullptr, int64_t nsrc = 0,
             int32_t *bad = nullptr);
void relu_back(hipStream_t st, const float *dH, const bf16 *H, int ldh, int B, int N, float *dzf,
               bf16 *dzb, int ldb);
// part: ceil(B / 64) * N floats of scratch
void colsum(hipStream_t st, const float *dz, int B, int N, float *part, float *db);
void adam(hipStream_t st, float *theta, const float *g, float *m, float *v, int64_t n, float lr,
          float b1, float b2, float eps, float c1, float c2, bf16 *wb, int cols, int ld);
void zero_pad_bf16(hipStream_t st, bf16 *p, int rows, int c0, int ld);
void weights_bf16(hipStream_t st, const float *w, int rows, int cols, bf16 *wb, int ld);

}  // namespace mlpk
