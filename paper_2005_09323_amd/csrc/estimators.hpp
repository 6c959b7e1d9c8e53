// Argument blocks of the estimator kernels.
#pragma once

#include "common.hpp"

namespace lbm {

constexpr int MAX_PERIODS = 4096;

struct RebuildArgs {
    const int* ancestors;     // [n_periods][n]
    const double* integrals;  // [n_periods][n]  int A dt of each slot over each period
    const double* ln_r;       // [n_periods]
    const float* series;      // [n][ld] drag, period i at columns col0 + i*tau ...
    int ld, col0, n, n_periods, tau;
    double k;
    float* traj;              // [n][n_periods*tau]
    double* log_weight;       // [n]
    double* traj_integral;    // [n]
};

struct WindowMaxArgs {
    const float* series;  // [rows][len]
    int len, window;
    double* prefix;       // [rows][len+1] scratch
    double* fmax;         // [rows]
};

struct TailArgs {
    const double* fmax;
    const double* log_weight;
    const double* levels;
    int n, n_levels;
    double* prob;
};

struct AmsProbArgs {
    const int* k_history;   // [n_iter] trajectories discarded per iteration
    int n_iter, n;          // iterations, ensemble size
    const double* final_max;  // [n] maxima of the final ensemble
    const double* levels;   // [n_levels]
    int n_levels;
    double* prob;           // [n_levels]
};

hipError_t launch_scgf(const double* ln_r, int n_periods, double t_a, double* out, hipStream_t st);
hipError_t launch_return_times(const double* prob, int n, double t_a, double window, double* r, hipStream_t st);
hipError_t launch_ams_probability(const AmsProbArgs& a, hipStream_t st);
hipError_t launch_learned_score(const float* ghat, const float* ft, long long count, float a, float w, float* out,
                                hipStream_t st);
hipError_t launch_rebuild(const RebuildArgs& a, hipStream_t st);
hipError_t launch_window_max(const WindowMaxArgs& a, int rows, hipStream_t st);
hipError_t launch_tail(const TailArgs& a, hipStream_t st);

}  // namespace lbm
