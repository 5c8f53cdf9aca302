// Entry points whose kernels are not in this build yet.
#include "mgrt_internal.hpp"

extern "C" {

int mgrt_jacobian_coarse(mgrt_ctx *, int64_t, const double *, int32_t, const double *,
                         const double *, double, int64_t, int32_t, const int64_t *, int,
                         int64_t, const int64_t *, const mgrt_run_opts *, double *) {
    return MGRT_E_STATE;
}

int mgrt_misfit_gradient(mgrt_ctx *, int64_t, const double *, int32_t, const double *,
                         const double *, double, int64_t, const double *, int,
                         const mgrt_run_opts *, double *) {
    return MGRT_E_STATE;
}

int mgrt_tv_invert_level(mgrt_ctx *, int64_t, int64_t, const void *, int, int, const double *,
                         const int64_t *, const int32_t *, const double *, double, int, double,
                         int, double *, int32_t *) {
    return MGRT_E_STATE;
}

}
