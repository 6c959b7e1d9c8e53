// State copies (checkpoints) and the window-mean score of the drag series.
#include <hip/hip_runtime.h>

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
__global__ void window_mean_kernel(const float* series, int ld, int t_len, int window, float* out) {
    const int m = (int)blockIdx.x;
    const float* row = series + (long long)m * ld;
    float* orow = out + (long long)m * t_len;
    const double inv = 1.0 / (double)window;
    for (int t = (int)threadIdx.x; t < t_len; t += (int)blockDim.x) {
        if (t < window - 1) {
            orow[t] = -INFINITY;
            continue;
        }
        double acc = 0.0;
        for (int k = t - window + 1; k <= t; ++k) acc += (double)row[k];
        orow[t] = (float)(acc * inv);
    }
}

}  // namespace lbm

extern "C" int lbm_window_mean(const float* series_dev, int32_t n, int32_t ld, int32_t t_len, int32_t window,
                               float* out_dev, void* hip_stream) {
    if (!series_dev || !out_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (n < 0 || t_len < 0 || ld < t_len || window < 1) return lbm_fail(LBM_EINVAL, "bad sizes");
    if (n == 0 || t_len == 0) return LBM_OK;
    hipLaunchKernelGGL(window_mean_kernel, dim3(n), dim3(256), 0, (hipStream_t)hip_stream, series_dev, ld, t_len,
                       window, out_dev);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "window mean kernel");
}
