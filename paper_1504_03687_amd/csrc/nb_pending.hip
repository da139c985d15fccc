// Entry points whose kernels are not in this build yet.
#include "../../include/nbreg.h"
#include "nb_runtime.h"

namespace nbrt { void batched_release(nb_ctx *) {} }

extern "C" {
int nb_regular_force_batched(nb_ctx *, int32_t, const int64_t *, const int64_t *, const double *,
                             const double *, const double *, const int32_t *, const double *,
                             int32_t, nb_precision, double *, double *, int32_t *, int32_t *,
                             int32_t *, uint32_t *)
{
    return NB_ERR_UNSUPPORTED;
}
int nb_autotune(nb_ctx *, int64_t, const char *, int) { return NB_ERR_UNSUPPORTED; }
}
