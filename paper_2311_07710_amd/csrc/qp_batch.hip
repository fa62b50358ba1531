// qp_batch.hip -- batched rAPDHG (placeholder until the persistent kernel lands).
#include "qp_batch.h"

namespace qpb {

struct BatchData {
    int dummy = 0;
};

extern "C" const char *qp_last_error(void);

int create_batch(const qp_problem_desc *, const qp_settings *, BatchData **out) {
    *out = nullptr;
    return QP_ERR_UNSUPPORTED;
}
void destroy_batch(BatchData *b) { delete b; }
int batch_solve(BatchData *, const qp_settings *, int, const qp_warm_start *, qp_result *,
                double *, double *) {
    return QP_ERR_UNSUPPORTED;
}
int batch_norms(BatchData *, double *, double *) { return QP_ERR_UNSUPPORTED; }
int batch_update_vectors(BatchData *, const double *, const double *, int) {
    return QP_ERR_UNSUPPORTED;
}

}  // namespace qpb
