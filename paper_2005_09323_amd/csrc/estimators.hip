// GKTL estimators on the device (paper Appendix C.1-C.2), in FP64.
//
// After a GKTL run the drag series of every slot is a patchwork of the
// trajectories that occupied the slot in each period.  The final ensemble's
// trajectories are rebuilt by walking the ancestors back; each carries the
// time integral of the observable along its lineage and the maximum of its
// window-averaged drag; the unbiased tail probability is the sum of
// exp(sum_i ln R_i - k int A) over trajectories above each level.
#include "estimators.hpp"

namespace lbm {

// Block = final trajectory j.  Lineage slot of each period, the rebuilt drag
// series and the integral of A along the lineage (added in period order).
__global__ __launch_bounds__(256) void gktl_rebuild_kernel(RebuildArgs a) {
    __shared__ int slot[MAX_PERIODS];
    const int j = (int)blockIdx.x;
    if (threadIdx.x == 0) {
        int s = j;
        for (int i = a.n_periods - 1; i >= 0; --i) {
            s = a.ancestors[(long long)i * a.n + s];
            slot[i] = s;
        }
        double integ = 0.0;
        for (int i = 0; i < a.n_periods; ++i) integ += a.integrals[(long long)i * a.n + slot[i]];
        double lz = 0.0;
        for (int i = 0; i < a.n_periods; ++i) lz += a.ln_r[i];
        a.log_weight[j] = lz - a.k * integ;
        a.traj_integral[j] = integ;
    }
    __syncthreads();
    const int len = a.n_periods * a.tau;
    for (int t = (int)threadIdx.x; t < len; t += (int)blockDim.x) {
        const int i = t / a.tau;
        a.traj[(long long)j * len + t] = a.series[(long long)slot[i] * a.ld + a.col0 + t];
    }
}

// Block = trajectory: FP64 running sums in time order, then the largest
// window mean (1/T) (S_t - S_{t-T}) over the windows inside [0, len).
__global__ __launch_bounds__(256) void window_max_kernel(WindowMaxArgs a) {
    const int j = (int)blockIdx.x;
    const float* row = a.series + (long long)j * a.len;
    double* pre = a.prefix + (long long)j * (a.len + 1);
    if (threadIdx.x == 0) {
        double s = 0.0;
        pre[0] = 0.0;
        for (int t = 0; t < a.len; ++t) {
            s += (double)row[t];
            pre[t + 1] = s;
        }
    }
    __syncthreads();
    __shared__ double sh[256];
    double best = -INFINITY;
    for (int t = a.window + (int)threadIdx.x; t <= a.len; t += (int)blockDim.x) {
        const double v = (pre[t] - pre[t - a.window]) / (double)a.window;
        best = fmax(best, v);
    }
    sh[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) a.fmax[j] = sh[0];
}

// Thread = level: (1/N) sum_j exp(log_weight_j) [fmax_j >= a], j in order.
__global__ void tail_probability_kernel(TailArgs a) {
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= a.n_levels) return;
    const double lev = a.levels[q];
    double s = 0.0;
    for (int j = 0; j < a.n; ++j)
        if (a.fmax[j] >= lev) s += exp(a.log_weight[j]);
    a.prob[q] = s / (double)a.n;
}

// SCGF estimate (paper Appendix C.1): lambda(k) = (1/T_a) sum_i ln R_i, the
// sum in period order (one thread).
__global__ void scgf_kernel(const double* ln_r, int n_periods, double t_a, double* out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n_periods; ++i) s += ln_r[i];
    out[0] = s / t_a;
}

// Return time of a level from the probability p that a block of length T_a
// holds a window of length T above it (paper Appendix C.2):
// r = -(T_a - T) / ln(1 - p); +inf where p = 0 (0 where p = 1).
__global__ void return_times_kernel(const double* prob, int n, double t_a, double window, double* r) {
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= n) return;
    const double p = prob[q];
    r[q] = p == 0.0 ? INFINITY : -(t_a - window) / log1p(-p);
}

// Unbiased AMS estimate of P(max >= a) (paper Appendix B): the product over
// the iterations of (1 - K_j / N), in order, times the fraction of the final
// ensemble whose maximum reaches a.  Thread = level.
__global__ void ams_probability_kernel(AmsProbArgs a) {
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= a.n_levels) return;
    double f = 1.0;
    for (int j = 0; j < a.n_iter; ++j) f *= 1.0 - (double)a.k_history[j] / (double)a.n;
    const double lev = a.levels[q];
    int c = 0;
    for (int m = 0; m < a.n; ++m) c += a.final_max[m] >= lev ? 1 : 0;
    a.prob[q] = f * (double)c / (double)a.n;
}

// AMS score from a learned predictor, kept consistent with the target event
// {max_t F_T(t) >= a}: the score is a once the time-averaged drag has reached a;
// before that the prediction g is mapped strictly increasingly into (-inf, a),
// a - w ln(1 + exp((a - g)/w)), so that max_t score >= a exactly when the event
// happened while over-predictions keep their order.  Evaluated in FP64 in the
// form whose exponential cannot overflow, rounded to FP32 (a monotone rounding)
// and held at or below the float just under a.
__global__ void learned_score_kernel(const float* ghat, const float* ft, long long count, float a, float w,
                                     float* out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float g = ghat[i];
    float s;
    if (ft[i] >= a) {
        s = a;
    } else if (!isfinite(g)) {
        s = -INFINITY;
    } else {
        const double x = ((double)a - (double)g) / (double)w;
        const double v = x > 0.0 ? (double)g - (double)w * log1p(exp(-x)) : (double)a - (double)w * log1p(exp(x));
        s = fminf((float)v, nextafterf(a, -INFINITY));
    }
    out[i] = s;
}

hipError_t launch_learned_score(const float* ghat, const float* ft, long long count, float a, float w, float* out,
                                hipStream_t st) {
    hipLaunchKernelGGL(learned_score_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, ghat, ft,
                       count, a, w, out);
    return hipGetLastError();
}

hipError_t launch_rebuild(const RebuildArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(gktl_rebuild_kernel, dim3(a.n), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_window_max(const WindowMaxArgs& a, int rows, hipStream_t st) {
    hipLaunchKernelGGL(window_max_kernel, dim3(rows), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_scgf(const double* ln_r, int n_periods, double t_a, double* out, hipStream_t st) {
    hipLaunchKernelGGL(scgf_kernel, dim3(1), dim3(64), 0, st, ln_r, n_periods, t_a, out);
    return hipGetLastError();
}
hipError_t launch_return_times(const double* prob, int n, double t_a, double window, double* r, hipStream_t st) {
    hipLaunchKernelGGL(return_times_kernel, dim3((n + 255) / 256), dim3(256), 0, st, prob, n, t_a, window, r);
    return hipGetLastError();
}
hipError_t launch_ams_probability(const AmsProbArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(ams_probability_kernel, dim3((a.n_levels + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_tail(const TailArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(tail_probability_kernel, dim3((a.n_levels + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace lbm
