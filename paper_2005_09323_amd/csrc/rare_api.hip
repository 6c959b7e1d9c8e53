// GKTL cloning, branching perturbation and AMS selection.
#include <hip/hip_runtime.h>

#include "../../include/lbm.h"
#include "api_internal.hpp"

extern "C" int gktl_select_clone(lbm_ctx*, double, uint64_t, int32_t, double, const float*, int32_t, int32_t*,
                                 double*) {
    return lbm_fail(LBM_EUNSUPPORTED, "gktl_select_clone: not built yet");
}
extern "C" int lbm_perturb(lbm_ctx*, const int32_t*, uint64_t, int32_t, double, const float*, int32_t) {
    return lbm_fail(LBM_EUNSUPPORTED, "lbm_perturb: not built yet");
}
extern "C" int ams_score_kill_branch(const float*, int32_t, int32_t, int32_t, uint64_t, int32_t, int32_t*, int32_t*,
                                     int32_t*, int32_t*, float*, float*, void*) {
    return lbm_fail(LBM_EUNSUPPORTED, "ams_score_kill_branch: not built yet");
}
