// C-ABI entry points of the GKTL / direct-sampling estimators.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/lbm.h"
#include "api_internal.hpp"
#include "estimators.hpp"

using namespace lbm;

extern "C" int gktl_rebuild(const int32_t* ancestors_dev, const double* integrals_dev, const double* ln_r_dev,
                            const float* series_dev, int32_t ld, int32_t col0, int32_t n, int32_t n_periods,
                            int32_t tau, double k, float* traj_dev, double* log_weight_dev,
                            double* traj_integral_dev, void* hip_stream) {
    if (!ancestors_dev || !integrals_dev || !ln_r_dev || !series_dev || !traj_dev || !log_weight_dev ||
        !traj_integral_dev)
        return lbm_fail(LBM_EINVAL, "NULL argument");
    if (n < 1 || n_periods < 1 || n_periods > MAX_PERIODS || tau < 1 || col0 < 0 ||
        (long long)col0 + (long long)n_periods * tau > ld)
        return lbm_fail(LBM_EINVAL, "bad sizes");
    RebuildArgs a;
    a.ancestors = ancestors_dev;
    a.integrals = integrals_dev;
    a.ln_r = ln_r_dev;
    a.series = series_dev;
    a.ld = ld;
    a.col0 = col0;
    a.n = n;
    a.n_periods = n_periods;
    a.tau = tau;
    a.k = k;
    a.traj = traj_dev;
    a.log_weight = log_weight_dev;
    a.traj_integral = traj_integral_dev;
    hipError_t e = launch_rebuild(a, (hipStream_t)hip_stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "lineage rebuild");
}

extern "C" int window_mean_max(const float* series_dev, int32_t rows, int32_t len, int32_t window,
                               double* prefix_scratch_dev, double* fmax_dev, void* hip_stream) {
    if (!series_dev || !prefix_scratch_dev || !fmax_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (rows < 1 || window < 1 || len < window) return lbm_fail(LBM_EINVAL, "bad sizes");
    WindowMaxArgs a;
    a.series = series_dev;
    a.len = len;
    a.window = window;
    a.prefix = prefix_scratch_dev;
    a.fmax = fmax_dev;
    hipError_t e = launch_window_max(a, rows, (hipStream_t)hip_stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "window maximum");
}

extern "C" int tail_probability(const double* fmax_dev, const double* log_weight_dev, int32_t n,
                                const double* levels_dev, int32_t n_levels, double* prob_dev, void* hip_stream) {
    if (!fmax_dev || !log_weight_dev || !levels_dev || !prob_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (n < 1 || n_levels < 1) return lbm_fail(LBM_EINVAL, "bad sizes");
    TailArgs a;
    a.fmax = fmax_dev;
    a.log_weight = log_weight_dev;
    a.levels = levels_dev;
    a.n = n;
    a.n_levels = n_levels;
    a.prob = prob_dev;
    hipError_t e = launch_tail(a, (hipStream_t)hip_stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "tail probability");
}

extern "C" int gktl_scgf(const double* ln_r_dev, int32_t n_periods, double t_a, double* out_dev, void* hip_stream) {
    if (!ln_r_dev || !out_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (n_periods < 1) return lbm_fail(LBM_EINVAL, "n_periods must be >= 1");
    if (!(t_a > 0.0) || !std::isfinite(t_a)) return lbm_fail(LBM_EINVAL, "T_a must be finite and > 0");
    hipError_t e = launch_scgf(ln_r_dev, n_periods, t_a, out_dev, (hipStream_t)hip_stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "SCGF");
}

extern "C" int return_times(const double* prob_dev, int32_t n, double t_a, double window, double* r_dev,
                            void* hip_stream) {
    if (n < 0) return lbm_fail(LBM_EINVAL, "negative count");
    if (!std::isfinite(t_a) || !std::isfinite(window) || !(window >= 0.0) || !(t_a > window))
        return lbm_fail(LBM_EINVAL, "need 0 <= window < T_a, both finite");
    if (n == 0) return LBM_OK;
    if (!prob_dev || !r_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    hipError_t e = launch_return_times(prob_dev, n, t_a, window, r_dev, (hipStream_t)hip_stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "return times");
}

extern "C" int ams_probability(const int32_t* k_history_dev, int32_t n_iter, int32_t n, const double* final_max_dev,
                               const double* levels_dev, int32_t n_levels, double* prob_dev, void* hip_stream) {
    if (n < 1 || n_iter < 0 || n_levels < 0) return lbm_fail(LBM_EINVAL, "bad sizes");
    if (n_levels == 0) return LBM_OK;
    if (!final_max_dev || !levels_dev || !prob_dev || (n_iter > 0 && !k_history_dev))
        return lbm_fail(LBM_EINVAL, "NULL argument");
    AmsProbArgs a;
    a.k_history = k_history_dev;
    a.n_iter = n_iter;
    a.n = n;
    a.final_max = final_max_dev;
    a.levels = levels_dev;
    a.n_levels = n_levels;
    a.prob = prob_dev;
    hipError_t e = launch_ams_probability(a, (hipStream_t)hip_stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "AMS probability");
}

extern "C" int ams_learned_score(const float* ghat_dev, const float* ft_dev, int64_t count, float level,
                                 float width, float* out_dev, void* hip_stream) {
    if (!ghat_dev || !ft_dev || !out_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (count < 0) return lbm_fail(LBM_EINVAL, "negative count");
    if (!std::isfinite(level)) return lbm_fail(LBM_EINVAL, "level must be finite");
    if (!(width > 0.0f) || !std::isfinite(width)) return lbm_fail(LBM_EINVAL, "width must be finite and > 0");
    if (count == 0) return LBM_OK;
    hipError_t e = launch_learned_score(ghat_dev, ft_dev, count, level, width, out_dev, (hipStream_t)hip_stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "learned score");
}
