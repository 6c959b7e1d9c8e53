// State copies (checkpoints) and the window-mean score of the drag series.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "../../include/lbm.h"
#include "api_internal.hpp"

using namespace lbm;

extern "C" int lbm_copy_state_out(const lbm_ctx* c, int32_t m, float* dst_dev) {
    if (!c || !dst_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (m < 0 || m >= c->n) return lbm_fail(LBM_EINVAL, "member %d out of range", m);
    const MemberDev& md = c->h_members[m];
    const size_t bytes = sizeof(float) * 9 * (size_t)md.nx * md.ny;
    hipError_t e = hipMemcpyAsync(dst_dev, c->pop[c->h_parity[m]] + md.off, bytes, hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "state copy out");
}

extern "C" int lbm_copy_state_in(lbm_ctx* c, int32_t m, const float* src_dev, int32_t t) {
    if (!c || !src_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (m < 0 || m >= c->n) return lbm_fail(LBM_EINVAL, "member %d out of range", m);
    if (t < 0 || t > c->cap) return lbm_fail(LBM_EINVAL, "time %d outside [0, %d]", t, c->cap);
    const MemberDev& md = c->h_members[m];
    const size_t bytes = sizeof(float) * 9 * (size_t)md.nx * md.ny;
    hipError_t e = hipMemcpyAsync(c->pop[c->h_parity[m]] + md.off, src_dev, bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return lbm_hip_fail(e, "state copy in");
    if ((e = set_int(c->d_cursor + m, t, c->stream)) != hipSuccess) return lbm_hip_fail(e, "cursor set");
    c->h_cursor[m] = t;
    return LBM_OK;
}

namespace lbm {

// One block per member; thread t owns output columns t, t + blockDim, ...
// Each window sum is formed afresh in FP64 (T adds), so every column is
// independent of the others' rounding.
// Each thread owns WM_RUN consecutive outputs: the first window is summed in
// order (FP64), the others slide (+ the new sample, - the oldest), so a row
// costs about t_len (window / WM_RUN + 1) loads instead of t_len window; the
// FP64 sliding error (a few ulps of the running sum) is far below the FP32
// output rounding.
constexpr int WM_RUN = 16;

__global__ __launch_bounds__(256) void window_mean_kernel(const float* series, int n, int ld, int t_len, int window,
                                                          float* out) {
    const long long t0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * WM_RUN;
    if (t0 >= t_len) return;
    const int t1 = (int)min((long long)t_len, t0 + WM_RUN);
    const double inv = 1.0 / (double)window;
    for (int m = (int)blockIdx.y; m < n; m += (int)gridDim.y) {  // rows beyond the grid's height
        const float* row = series + (long long)m * ld;
        float* orow = out + (long long)m * t_len;
        double acc = 0.0;
        bool have = false;
        for (int t = (int)t0; t < t1; ++t) {
            if (t < window - 1) {
                orow[t] = -INFINITY;
                continue;
            }
            if (!have) {
                for (int k = t - window + 1; k <= t; ++k) acc += (double)row[k];
                have = true;
            } else {
                acc += (double)row[t] - (double)row[t - window];
            }
            orow[t] = (float)(acc * inv);
        }
    }
}

}  // namespace lbm

extern "C" int lbm_window_mean(const float* series_dev, int32_t n, int32_t ld, int32_t t_len, int32_t window,
                               float* out_dev, void* hip_stream) {
    if (!series_dev || !out_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (n < 0 || t_len < 0 || ld < t_len || window < 1) return lbm_fail(LBM_EINVAL, "bad sizes");
    if (n == 0 || t_len == 0) return LBM_OK;
    const unsigned runs = (unsigned)((t_len + WM_RUN - 1) / WM_RUN);
    hipLaunchKernelGGL(window_mean_kernel, dim3((runs + 255) / 256, (unsigned)std::min(n, 65535)), dim3(256), 0,
                       (hipStream_t)hip_stream, series_dev, n, ld, t_len, window, out_dev);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "window mean kernel");
}
