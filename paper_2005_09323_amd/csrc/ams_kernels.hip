// Trajectory-AMS selection (paper Section 4.1, Appendix B.1) on the device.
//
// The maxima are exact (max is order-free); the level is found by counting
// ranks; the kill and survivor lists keep slot order (block-wide exclusive
// scans); parents come from the counter-based Philox stream.  Every decision
// is therefore a fixed function of the score values and the key.
#include "ams_kernels.hpp"

namespace lbm {

// One block per member: max of the row; -inf if the row holds NaN or +inf (a
// blown-up trajectory).  -inf entries are ordinary lowest scores.
__global__ __launch_bounds__(256) void ams_maxima_kernel(const float* series, int t_len, float* maxima) {
    const int m = (int)blockIdx.x;
    const float* row = series + (long long)m * t_len;
    __shared__ float smax[256];
    __shared__ int sbad[256];
    float mx = -INFINITY;
    int bad = 0;
    for (int t = (int)threadIdx.x; t < t_len; t += 256) {
        const float v = row[t];
        if (isnan(v) || v == INFINITY) bad = 1; else mx = fmaxf(mx, v);
    }
    smax[threadIdx.x] = mx;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + s]);
            sbad[threadIdx.x] |= sbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) maxima[m] = sbad[0] ? -INFINITY : smax[0];
}

// Exclusive scan of flags[0..n) into out[0..n) (slot order), returns the total.
__device__ int block_exclusive_scan(const int* flags, int* out, int n, int* sh) {
    const int t = (int)threadIdx.x, nt = (int)blockDim.x;
    // each thread owns a contiguous run of slots
    const int per = (n + nt - 1) / nt;
    const int lo = min(n, t * per), hi = min(n, lo + per);
    int local = 0;
    for (int m = lo; m < hi; ++m) local += flags[m];
    sh[t] = local;
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int k = 0; k < nt; ++k) {
            const int v = sh[k];
            sh[k] = acc;
            acc += v;
        }
        sh[nt] = acc;
    }
    __syncthreads();
    int run = sh[t];
    for (int m = lo; m < hi; ++m) {
        out[m] = run;
        run += flags[m];
    }
    const int total = sh[nt];
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(1024) void ams_select_kernel(AmsArgs a) {
    __shared__ float q[MAX_AMS];
    __shared__ int flag[MAX_AMS];
    __shared__ int pos[MAX_AMS];
    __shared__ int surv[MAX_AMS];
    __shared__ int sh[1025];
    __shared__ float level_sh;
    const int t = (int)threadIdx.x, nt = (int)blockDim.x, n = a.n;
    for (int m = t; m < n; m += nt) q[m] = a.maxima[m];
    if (t == 0) level_sh = INFINITY;
    __syncthreads();
    // the n_kill-th lowest maximum: the value v with #{q < v} < n_kill <= #{q <= v}
    for (int m = t; m < n; m += nt) {
        int lt = 0, le = 0;
        for (int j = 0; j < n; ++j) {
            lt += q[j] < q[m];
            le += q[j] <= q[m];
        }
        if (lt < a.n_kill && a.n_kill <= le) level_sh = q[m];  // every writer stores the same value
    }
    __syncthreads();
    const float level = level_sh;
    // killed: at or below the level (ties together), in slot order
    for (int m = t; m < n; m += nt) flag[m] = q[m] <= level ? 1 : 0;
    __syncthreads();
    const int n_killed = block_exclusive_scan(flag, pos, n, sh);
    for (int m = t; m < n; m += nt)
        if (flag[m]) a.killed[pos[m]] = m;
    __syncthreads();
    // survivors, in slot order
    for (int m = t; m < n; m += nt) flag[m] = flag[m] ? 0 : 1;
    __syncthreads();
    const int n_surv = block_exclusive_scan(flag, pos, n, sh);
    for (int m = t; m < n; m += nt)
        if (flag[m]) surv[pos[m]] = m;
    __syncthreads();
    if (t == 0) {
        *a.n_killed = n_killed;
        *a.level = level;
    }
    // one wave per kill: its parent, and the parent's first crossing found 64
    // samples at a time (a wave-wide vote per block of samples)
    const int wave = t >> 6, lane = t & 63, nwaves = nt >> 6;
    for (int j = wave; j < n_killed; j += nwaves) {
        if (n_surv == 0) {  // extinction: nothing to branch from
            if (lane == 0) {
                a.parent[j] = -1;
                a.branch_t[j] = -1;
            }
            continue;
        }
        const U64x4 w = philox4x64_10((uint64_t)j, (uint64_t)a.iteration, 0, 0, a.key, PURPOSE_AMSP);
        const int p = surv[(int)index_below(w.v[0], (uint64_t)n_surv)];
        const float* row = a.series + (long long)p * a.t_len;
        int tb = -1;
        for (int t0 = 0; t0 < a.t_len && tb < 0; t0 += 64) {
            const int tt = t0 + lane;
            const unsigned long long hits = __ballot(tt < a.t_len && row[tt] > level);
            if (hits) tb = t0 + __ffsll(hits) - 1;
        }
        if (lane == 0) {
            a.parent[j] = p;
            a.branch_t[j] = tb;
        }
    }
}

hipError_t launch_ams(const AmsArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(ams_maxima_kernel, dim3(a.n), dim3(256), 0, st, a.series, a.t_len, a.maxima);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ams_select_kernel, dim3(1), dim3(1024), 0, st, a);
    return hipGetLastError();
}

}  // namespace lbm
