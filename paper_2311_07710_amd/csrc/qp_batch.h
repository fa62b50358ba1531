// qp_batch.h -- batched (segment-CSR, persistent-kernel) solver behind
// qp_create / qp_batch_solve when num_instances > 1.  Not part of the C-ABI.
#pragma once

#include "../../include/qp.h"

namespace qpb {

struct BatchData;

int create_batch(const qp_problem_desc *d, const qp_settings *s, BatchData **out);
void destroy_batch(BatchData *b);
int batch_solve(BatchData *b, const qp_settings *s, int mem_space, const qp_warm_start *ws,
                qp_result *res, double *x_out, double *y_out);
int batch_norms(BatchData *b, double *norm_A, double *norm_Q);
int batch_update_vectors(BatchData *b, const double *c, const double *bvec, int mem_space);

}  // namespace qpb
