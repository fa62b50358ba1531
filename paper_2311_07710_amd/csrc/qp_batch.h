// qp_batch.h -- batched (segment-CSR, persistent-kernel) solver behind
// qp_create / qp_batch_solve when num_instances > 1.  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/qp.h"

namespace qpb {

struct BatchData;

// host pointers to a batch's arrays (Q and A row pointers over all instances, local
// column indices)
struct BatchArrays {
    const int32_t *qr, *qc;
    const double *qv;
    const int32_t *ar, *ac;
    const uint8_t *rt;
    const double *l, *u;
};
int validate_batch_arrays(const qp_problem_desc *d, const qp_settings *s, const BatchArrays &a);
// the same checks straight from a host-memory descriptor, before any device work
int validate_batch_host(const qp_problem_desc *d, const qp_settings *s);

int create_batch(const qp_problem_desc *d, const qp_settings *s, hipStream_t stream,
                 BatchData **out);
void destroy_batch(BatchData *b);
int batch_solve(BatchData *b, const qp_settings *s, int mem_space, const qp_warm_start *ws,
                qp_result *res, double *x_out, double *y_out);
int batch_norms(BatchData *b, double *norm_A, double *norm_Q);
int batch_scaling(BatchData *b, double *d_var, double *d_row);
int batch_update_vectors(BatchData *b, const double *c, const double *bvec, int mem_space);
int batch_set_norms(BatchData *b, const double *norm_A, const double *norm_Q);
int batch_autotune(BatchData *b, const qp_settings *s, int32_t sample, int32_t iters,
                   int32_t *threads_out);
int batch_set_threads(BatchData *b, const int32_t *threads);

}  // namespace qpb
