// Adjoint of the multipole estimator (placeholder until the kernels land).
#include "t3_internal.h"

namespace t3 {

int backward(t3_plan *plan, const t3_catalog &cat, const double *grad_ups, float *gg1, float *gg2,
             float *gw, hipStream_t s)
{
    (void)plan;
    (void)cat;
    (void)grad_ups;
    (void)gg1;
    (void)gg2;
    (void)gw;
    (void)s;
    return fail(T3_ERANGE, "t3_backward: not available in this build");
}

}  // namespace t3
