// C-ABI entry points of the learned score: features, forward, gradient, Adam.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/lbm.h"
#include "api_internal.hpp"
#include "cnn_kernels.hpp"

using namespace lbm;

namespace {
constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
struct WsLayout {
    size_t wt, act, gap, y, partial, total;
};
constexpr WsLayout layout(int batch) {
    WsLayout w{};
    size_t off = 0;
    w.wt = off;
    off += align256((size_t)CNN_WT_ELEMS * sizeof(unsigned short));
    w.act = off;
    off += align256((size_t)batch * 3 * 256 * 32 * sizeof(unsigned short));
    w.gap = off;
    off += align256((size_t)batch * 32 * sizeof(float));
    w.y = off;
    off += align256((size_t)batch * sizeof(float));
    w.partial = off;
    off += align256((size_t)cnn_partial_rows_cap(batch) * CNN_PART_STRIDE * sizeof(float));
    w.total = off;
    return w;
}

// Workspace of score_net_grad_noalloc: a file-scope device array with the
// layout of a caller's workspace for the largest batch that entry point
// accepts (each region of a smaller batch starts at the same or a lower
// offset and is shorter, so it fits too).  Every device the library runs on
// holds its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in, never the device memory: its device address is taken
// once per device with hipGetSymbolAddress and only that address is used.
constexpr int NOALLOC_MAX_BATCH = 256;
constexpr size_t NOALLOC_BYTES = layout(NOALLOC_MAX_BATCH).total;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, resolved on the first
// call per device (no allocation: the array is part of the loaded code object).
int scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return lbm_hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return lbm_fail(LBM_EUNSUPPORTED, "device %d beyond %d devices", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return lbm_hip_fail(e, "hipGetSymbolAddress of the static workspace");
        if (!p) return lbm_fail(LBM_EHIP, "hipGetSymbolAddress gave a NULL address for the static workspace");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return LBM_OK;
}

int check_ws(int batch, void* ws, size_t bytes) {
    if (batch < 1 || batch > (1 << 20)) return lbm_fail(LBM_EINVAL, "batch must be in [1, 2^20]");
    if (!ws) return lbm_fail(LBM_EINVAL, "NULL workspace");
    if (bytes < layout(batch).total) return lbm_fail(LBM_EINVAL, "workspace too small: %zu < %zu", bytes, layout(batch).total);
    if ((uintptr_t)ws & 255) return lbm_fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    return LBM_OK;
}
}  // namespace

extern "C" int32_t score_net_params(void) { return CNN_N_PARAMS; }

extern "C" size_t score_net_workspace_bytes(int32_t batch) { return batch < 1 ? 0 : layout(batch).total; }

extern "C" int score_features(const lbm_ctx* c, int32_t m0, int32_t n, int32_t px0, int32_t py0, int32_t patch,
                              int32_t pool, double u_scale, double rho_scale, float* out_dev) {
    if (!c || !out_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (m0 < 0 || n < 0 || m0 + n > c->n) return lbm_fail(LBM_EINVAL, "member range [%d, %d) outside the ensemble", m0, m0 + n);
    if (pool < 1 || patch < pool || patch % pool || patch / pool > 16)
        return lbm_fail(LBM_EINVAL, "patch must be a multiple of pool with patch/pool <= 16");
    for (int m = m0; m < m0 + n; ++m) {
        const lbm_member_desc& d = c->desc[m];
        if (px0 < 0 || py0 < 0 || px0 + patch > d.nx || py0 + patch > d.ny)
            return lbm_fail(LBM_EINVAL, "patch outside member %d", m);
    }
    if (n == 0) return LBM_OK;
    FeatureArgs a;
    a.members = c->d_members;
    a.parity = c->d_parity;
    a.pop0 = c->pop[0];
    a.pop1 = c->pop[1];
    a.m0 = m0;
    a.list = nullptr;
    a.px0 = px0;
    a.py0 = py0;
    a.patch = patch;
    a.pool = pool;
    a.u_scale = u_scale;
    a.rho_scale = rho_scale;
    a.out = out_dev;
    hipError_t e = launch_features(a, n, c->stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "feature kernel");
}

extern "C" int score_features_active(const lbm_ctx* c, int32_t px0, int32_t py0, int32_t patch, int32_t pool,
                                     double u_scale, double rho_scale, float* out_dev, int32_t max_rows,
                                     int32_t* n_rows) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    if (pool < 1 || patch < pool || patch % pool || patch / pool > 16)
        return lbm_fail(LBM_EINVAL, "patch must be a multiple of pool with patch/pool <= 16");
    if (n_rows) *n_rows = c->n_active;
    if (c->n_active > max_rows)
        return lbm_fail(LBM_EINVAL, "%d active members, the output holds %d rows", c->n_active, max_rows);
    if (c->n_active > 0 && !out_dev) return lbm_fail(LBM_EINVAL, "NULL output");
    for (int m = 0; m < c->n; ++m) {
        if (!c->h_active[m]) continue;
        const lbm_member_desc& d = c->desc[m];
        if (px0 < 0 || py0 < 0 || px0 + patch > d.nx || py0 + patch > d.ny)
            return lbm_fail(LBM_EINVAL, "patch outside member %d", m);
    }
    if (c->n_active == 0) return LBM_OK;
    FeatureArgs a;
    a.members = c->d_members;
    a.parity = c->d_parity;
    a.pop0 = c->pop[0];
    a.pop1 = c->pop[1];
    a.m0 = 0;
    a.list = c->d_active_list;
    a.px0 = px0;
    a.py0 = py0;
    a.patch = patch;
    a.pool = pool;
    a.u_scale = u_scale;
    a.rho_scale = rho_scale;
    a.out = out_dev;
    hipError_t e = launch_features(a, c->n_active, c->stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "feature kernel");
}

extern "C" int score_net_forward(const float* params_dev, const float* x_dev, int32_t batch, float* y_dev,
                                 void* workspace, size_t workspace_bytes, void* hip_stream) {
    if (!params_dev || !x_dev || !y_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    int rc = check_ws(batch, workspace, workspace_bytes);
    if (rc) return rc;
    const WsLayout w = layout(batch);
    CnnArgs a{};
    a.params = params_dev;
    a.x = x_dev;
    a.batch = batch;
    a.y = y_dev;
    a.gap = nullptr;
    a.act = nullptr;
    a.wt = (unsigned short*)((char*)workspace + w.wt);
    hipError_t e = launch_cnn_forward(a, (hipStream_t)hip_stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "score forward");
}

namespace {
// Forward (activations and averages saved) and backward of one batch into the
// workspace at `base` laid out by layout(batch); enqueued on the stream.
int grad_into(const float* params_dev, const float* x_dev, const float* labels_dev, int32_t batch, float* grads_dev,
              float* loss_dev, char* base, hipStream_t st) {
    const WsLayout w = layout(batch);
    CnnArgs a{};
    a.params = params_dev;
    a.x = x_dev;
    a.labels = labels_dev;
    a.batch = batch;
    a.y = (float*)(base + w.y);
    a.gap = (float*)(base + w.gap);
    a.act = (unsigned short*)(base + w.act);
    a.partial = (float*)(base + w.partial);
    a.grads = grads_dev;
    a.loss = loss_dev;
    a.wt = (unsigned short*)(base + w.wt);
    hipError_t e = launch_cnn_forward(a, st);
    if (e != hipSuccess) return lbm_hip_fail(e, "score forward");
    if ((e = launch_cnn_backward(a, st)) != hipSuccess) return lbm_hip_fail(e, "score backward");
    return LBM_OK;
}
}  // namespace

extern "C" int score_net_grad(const float* params_dev, const float* x_dev, const float* labels_dev, int32_t batch,
                              float* grads_dev, float* loss_dev, void* workspace, size_t workspace_bytes,
                              void* hip_stream) {
    if (!params_dev || !x_dev || !labels_dev || !grads_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    int rc = check_ws(batch, workspace, workspace_bytes);
    if (rc) return rc;
    return grad_into(params_dev, x_dev, labels_dev, batch, grads_dev, loss_dev, (char*)workspace,
                     (hipStream_t)hip_stream);
}

extern "C" int score_net_grad_noalloc(const float* params_dev, const float* x_dev, const float* labels_dev,
                                      int32_t batch, float* grads_dev, float* loss_dev, void* hip_stream) {
    if (!params_dev || !x_dev || !labels_dev || !grads_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (batch < 1 || batch > NOALLOC_MAX_BATCH)
        return lbm_fail(LBM_EINVAL, "batch %d outside [1, %d]: the static workspace holds %d images (%zu bytes)",
                        batch, NOALLOC_MAX_BATCH, NOALLOC_MAX_BATCH, NOALLOC_BYTES);
    void* ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    return grad_into(params_dev, x_dev, labels_dev, batch, grads_dev, loss_dev, (char*)ws, (hipStream_t)hip_stream);
}

extern "C" int score_net_adam(float* params_dev, float* m_dev, float* v_dev, const float* grads_dev, int32_t step,
                              double lr, double beta1, double beta2, double eps, void* hip_stream) {
    if (!params_dev || !m_dev || !v_dev || !grads_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (step < 1) return lbm_fail(LBM_EINVAL, "step must be >= 1");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return lbm_fail(LBM_EINVAL, "bad Adam hyper-parameters");
    AdamArgs a;
    a.params = params_dev;
    a.m = m_dev;
    a.v = v_dev;
    a.grads = grads_dev;
    a.step = step;
    a.lr = lr;
    a.beta1 = beta1;
    a.beta2 = beta2;
    a.eps = eps;
    hipError_t e = launch_cnn_adam(a, (hipStream_t)hip_stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "Adam kernel");
}
