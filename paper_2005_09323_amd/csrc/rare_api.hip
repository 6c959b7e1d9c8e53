// C-ABI entry points of GKTL cloning, in-place perturbation and AMS selection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "../../include/lbm.h"
#include "api_internal.hpp"
#include "ams_kernels.hpp"
#include "rare_kernels.hpp"

using namespace lbm;

// Library scratch of the cloning path, sized for the context on first use.
static int ensure_rare_scratch(lbm_ctx* c) {
    if (c->rare.ready) return LBM_OK;
    const int n = c->n;
    const long long floats = 9LL * c->h_members[0].nx * c->h_members[0].ny;
    c->rare.blocks_per_state = (int)((floats + MASS_CHUNK - 1) / MASS_CHUNK);
    hipError_t e;
    RareScratch& r = c->rare;
    if ((e = hipMalloc(&r.prefix, sizeof(double) * n)) != hipSuccess ||
        (e = hipMalloc(&r.alpha, sizeof(double) * (size_t)n * MAX_SNAP)) != hipSuccess ||
        (e = hipMalloc(&r.alpha_sum, sizeof(double) * n)) != hipSuccess ||
        (e = hipMalloc(&r.scale, sizeof(double) * n)) != hipSuccess ||
        (e = hipMalloc(&r.coef_w, sizeof(double) * n)) != hipSuccess ||
        (e = hipMalloc(&r.mass_partial, sizeof(double) * (size_t)(n + MAX_SNAP) * r.blocks_per_state)) != hipSuccess ||
        (e = hipMalloc(&r.mode, sizeof(int) * n)) != hipSuccess ||
        (e = hipMalloc(&r.src, sizeof(int) * n)) != hipSuccess ||
        (e = hipMalloc(&r.need_mass, sizeof(int) * n)) != hipSuccess ||
        (e = hipMalloc(&r.flags_new, sizeof(int) * n)) != hipSuccess ||
        (e = hipHostMalloc(&r.status_host, sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&r.status, sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&r.new_off, sizeof(long long) * n)) != hipSuccess ||
        (e = hipMalloc(&r.new_parity, sizeof(int) * n)) != hipSuccess ||
        (e = hipMalloc(&r.extra, sizeof(int) * n)) != hipSuccess ||
        (e = hipMalloc(&r.n_extra, sizeof(int))) != hipSuccess ||
        (e = hipHostMalloc(&r.new_off_host, sizeof(long long) * n)) != hipSuccess ||
        (e = hipHostMalloc(&r.new_parity_host, sizeof(int) * n)) != hipSuccess ||
        (e = hipHostMalloc(&r.n_extra_host, sizeof(int))) != hipSuccess)
        return lbm_hip_fail(e, "allocation of cloning scratch");
    r.ready = true;
    return LBM_OK;
}

void free_rare_scratch(lbm_ctx* c) {
    RareScratch& r = c->rare;
    hipFree(r.prefix);
    hipFree(r.alpha);
    hipFree(r.alpha_sum);
    hipFree(r.scale);
    hipFree(r.coef_w);
    hipFree(r.mass_partial);
    hipFree(r.mode);
    hipFree(r.src);
    hipFree(r.need_mass);
    hipFree(r.flags_new);
    hipFree(r.status);
    hipFree(r.new_off);
    hipFree(r.new_parity);
    hipFree(r.extra);
    hipFree(r.n_extra);
    if (r.status_host) hipHostFree(r.status_host);
    if (r.new_off_host) hipHostFree(r.new_off_host);
    if (r.new_parity_host) hipHostFree(r.new_parity_host);
    if (r.n_extra_host) hipHostFree(r.n_extra_host);
    r = RareScratch();
}

// Mass partials of the perturbed copies' parents and of the snapshots, and
// each perturbed copy's scale, for the modes already in r.mode/r.src.
static int run_mass_scale(lbm_ctx* c, double eps, const float* snapshots, int n_snap) {
    RareScratch& r = c->rare;
    hipError_t e;
    if (n_snap > 0 && eps != 0.0) {
        MassArgs ma;
        ma.members = c->d_members;
        ma.parity = c->d_parity;
        ma.need_mass = r.need_mass;
        ma.pop0 = c->pop[0];
        ma.pop1 = c->pop[1];
        ma.snapshots = snapshots;
        ma.partial = r.mass_partial;
        ma.n = c->n;
        ma.blocks_per_state = r.blocks_per_state;
        if ((e = launch_mass(ma, c->n + n_snap, c->stream)) != hipSuccess) return lbm_hip_fail(e, "mass kernel");
        ScaleArgs sa;
        sa.mode = r.mode;
        sa.src = r.src;
        sa.partial = r.mass_partial;
        sa.alpha = r.alpha;
        sa.alpha_sum = r.alpha_sum;
        sa.scale = r.scale;
        sa.coef_w = r.coef_w;
        const lbm_member_desc& d0 = c->desc[0];
        const MemberDev& m0 = c->h_members[0];
        long long grid_cells = 0;  // an open channel's grid bars (same rule as in_grid)
        for (int y = m0.bar / 2; m0.bar > 0 && y < d0.ny; ++y)
            if ((y - m0.bar / 2) % (2 * m0.bar) < m0.bar) grid_cells += m0.bar;
        sa.n_fluid = (double)d0.nx * d0.ny - (double)d0.sq_side * d0.sq_side - (double)grid_cells;
        sa.eps = eps;
        sa.n = c->n;
        sa.n_snap = n_snap;
        sa.blocks_per_state = r.blocks_per_state;
        if ((e = launch_scale(sa, c->stream)) != hipSuccess) return lbm_hip_fail(e, "scale kernel");
    }
    return LBM_OK;
}

// Mass partials, scales and the gather for the modes already in r.mode/r.src.
static int run_gather(lbm_ctx* c, double eps, const float* snapshots, int n_snap, int reset_accum) {
    RareScratch& r = c->rare;
    hipError_t e;
    int rc = run_mass_scale(c, eps, snapshots, n_snap);
    if (rc) return rc;
    GatherArgs ga;
    ga.members = c->d_members;
    ga.parity = c->d_parity;
    ga.mode = r.mode;
    ga.src = r.src;
    ga.pop0 = c->pop[0];
    ga.pop1 = c->pop[1];
    ga.snapshots = snapshots;
    ga.alpha = r.alpha;
    ga.scale = r.scale;
    ga.coef_w = r.coef_w;
    ga.eps = eps;
    ga.n = c->n;
    ga.n_snap = (eps != 0.0) ? n_snap : 0;
    if ((e = launch_gather(ga, 9LL * c->h_members[0].nx * c->h_members[0].ny, c->stream)) != hipSuccess)
        return lbm_hip_fail(e, "gather kernel");
    FinishArgs fa;
    fa.mode = r.mode;
    fa.src = r.src;
    fa.parity = c->d_parity;
    fa.accum = c->accum;
    fa.flags = c->d_flags;
    fa.flags_new = r.flags_new;
    fa.n = c->n;
    fa.reset_accum = reset_accum;
    if ((e = launch_finish(fa, c->stream)) != hipSuccess) return lbm_hip_fail(e, "finish kernel");
    return LBM_OK;
}

static int check_snapshots(const lbm_ctx* c, double eps, const float* snapshots, int32_t n_snap) {
    if (!std::isfinite(eps)) return lbm_fail(LBM_EINVAL, "eps must be finite");
    if (n_snap < 0 || n_snap > MAX_SNAP) return lbm_fail(LBM_EINVAL, "n_snap must be in [0, %d]", MAX_SNAP);
    if (eps != 0.0 && n_snap > 0 && !snapshots) return lbm_fail(LBM_EINVAL, "snapshots are NULL");
    if ((uintptr_t)snapshots & 15) return lbm_fail(LBM_EINVAL, "snapshots must be 16-byte aligned");
    if (!c->uniform_shape) return lbm_fail(LBM_EUNSUPPORTED, "cloning needs every member on one lattice shape");
    return LBM_OK;
}

extern "C" int gktl_select_clone(lbm_ctx* c, double k, uint64_t key, int32_t period, double eps,
                                 const float* snapshots, int32_t n_snap, int32_t* ancestors_dev, double* ln_r_dev) {
    if (!c || !ancestors_dev || !ln_r_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (!std::isfinite(k)) return lbm_fail(LBM_EINVAL, "k must be finite");
    if (c->n > MAX_SELECT) return lbm_fail(LBM_EUNSUPPORTED, "selection handles at most %d members", MAX_SELECT);
    int rc = check_snapshots(c, eps, snapshots, n_snap);
    if (rc) return rc;
    if ((rc = ensure_rare_scratch(c))) return rc;
    RareScratch& r = c->rare;
    SelectArgs sa;
    sa.accum = c->accum;
    sa.k = k;
    sa.key = key;
    sa.period = period;
    sa.n = c->n;
    sa.n_snap = n_snap;
    sa.eps = eps;
    sa.prefix = r.prefix;
    sa.ln_r = ln_r_dev;
    sa.ancestors = ancestors_dev;
    sa.status = r.status;
    sa.mode = r.mode;
    sa.src = r.src;
    sa.need_mass = r.need_mass;
    sa.alpha = r.alpha;
    sa.alpha_sum = r.alpha_sum;
    sa.members = c->d_members;
    sa.parity = c->d_parity;
    sa.relabel = c->relabel;
    sa.new_off = r.new_off;
    sa.new_parity = r.new_parity;
    sa.extra = r.extra;
    sa.n_extra = r.n_extra;
    hipError_t e;
    if ((e = launch_select(sa, c->stream)) != hipSuccess) return lbm_hip_fail(e, "selection kernel");
    // the all-non-finite case must leave the ensemble untouched: read the status (synchronises);
    // relabelling also reads back where every slot's state goes (the host mirrors follow it)
    const int n = c->n;
    if ((e = hipMemcpyAsync(r.status_host, r.status, sizeof(int), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
        return lbm_hip_fail(e, "selection status");
    if (c->relabel &&
        ((e = hipMemcpyAsync(r.n_extra_host, r.n_extra, sizeof(int), hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
         (e = hipMemcpyAsync(r.new_off_host, r.new_off, sizeof(long long) * n, hipMemcpyDeviceToHost, c->stream)) !=
             hipSuccess ||
         (e = hipMemcpyAsync(r.new_parity_host, r.new_parity, sizeof(int) * n, hipMemcpyDeviceToHost, c->stream)) !=
             hipSuccess))
        return lbm_hip_fail(e, "selection tables");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return lbm_hip_fail(e, "selection status");
    if (*r.status_host != 0) return lbm_fail(LBM_ENONFINITE, "every trajectory has a non-finite weight");
    if (!c->relabel) {
        if ((rc = run_gather(c, eps, snapshots, n_snap, 1))) return rc;
        for (int m = 0; m < n; ++m) c->h_parity[m] ^= 1;
        return LBM_OK;
    }
    // relabelling: the first copy of every ancestor keeps its block; the other
    // copies are written into blocks whose states left no descendant
    if ((rc = run_mass_scale(c, eps, snapshots, n_snap))) return rc;
    PlaceArgs pa;
    pa.members = c->d_members;
    pa.parity = c->d_parity;
    pa.extra = r.extra;
    pa.src = r.src;
    pa.mode = r.mode;
    pa.new_off = r.new_off;
    pa.pop0 = c->pop[0];
    pa.pop1 = c->pop[1];
    pa.snapshots = snapshots;
    pa.alpha = r.alpha;
    pa.scale = r.scale;
    pa.coef_w = r.coef_w;
    pa.eps = eps;
    pa.n_snap = (eps != 0.0) ? n_snap : 0;
    pa.n_extra = *r.n_extra_host;
    if (pa.n_extra < 0 || pa.n_extra > n)
        return lbm_fail(LBM_EHIP, "selection reported %d further copies of %d", pa.n_extra, n);
    if ((e = launch_place(pa, 9LL * c->h_members[0].nx * c->h_members[0].ny, c->stream)) != hipSuccess)
        return lbm_hip_fail(e, "placement kernel");
    FinishArgs fa;
    fa.mode = r.mode;
    fa.src = r.src;
    fa.parity = c->d_parity;
    fa.accum = c->accum;
    fa.flags = c->d_flags;
    fa.flags_new = r.flags_new;
    fa.n = n;
    fa.reset_accum = 1;
    CommitArgs ca;
    ca.members = c->d_members;
    ca.parity = c->d_parity;
    ca.new_off = r.new_off;
    ca.new_parity = r.new_parity;
    ca.accum = c->accum;
    ca.flags = c->d_flags;
    ca.flags_new = r.flags_new;
    ca.n = n;
    if ((e = launch_relabel_commit(fa, ca, c->stream)) != hipSuccess) return lbm_hip_fail(e, "relabelling commit");
    for (int m = 0; m < n; ++m) {
        c->h_members[m].off = r.new_off_host[m];
        c->h_parity[m] = r.new_parity_host[m];
    }
    return LBM_OK;
}

extern "C" int lbm_set_cloning(lbm_ctx* c, int32_t relabel) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    if (relabel != 0 && relabel != 1) return lbm_fail(LBM_EINVAL, "relabel must be 0 or 1");
    c->relabel = relabel;
    return LBM_OK;
}

extern "C" int lbm_perturb(lbm_ctx* c, const int32_t* mask_host, uint64_t key, int32_t period, double eps,
                           const float* snapshots, int32_t n_snap) {
    if (!c || !mask_host) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (c->n > MAX_SELECT) return lbm_fail(LBM_EUNSUPPORTED, "at most %d members", MAX_SELECT);
    int rc = check_snapshots(c, eps, snapshots, n_snap);
    if (rc) return rc;
    if (eps == 0.0 || n_snap == 0) return LBM_OK;  // the identity
    if ((rc = ensure_rare_scratch(c))) return rc;
    RareScratch& r = c->rare;
    PlanArgs pa{};
    for (int m = 0; m < c->n; ++m)
        if (mask_host[m]) pa.mask.w[m >> 5] |= 1u << (m & 31);
    pa.key = key;
    pa.period = period;
    pa.n = c->n;
    pa.n_snap = n_snap;
    pa.mode = r.mode;
    pa.src = r.src;
    pa.need_mass = r.need_mass;
    pa.alpha = r.alpha;
    pa.alpha_sum = r.alpha_sum;
    hipError_t e;
    if ((e = launch_plan(pa, c->stream)) != hipSuccess) return lbm_hip_fail(e, "perturbation plan");
    if ((rc = run_gather(c, eps, snapshots, n_snap, 0))) return rc;
    for (int m = 0; m < c->n; ++m)
        if (mask_host[m]) c->h_parity[m] ^= 1;
    return LBM_OK;
}

extern "C" int ams_score_kill_branch(const float* series_dev, int32_t n, int32_t t_len, int32_t n_kill, uint64_t key,
                                     int32_t iteration, int32_t* killed_dev, int32_t* parent_dev,
                                     int32_t* branch_t_dev, int32_t* n_killed_dev, float* level_dev,
                                     float* maxima_dev, void* hip_stream) {
    if (!series_dev || !killed_dev || !parent_dev || !branch_t_dev || !n_killed_dev || !level_dev || !maxima_dev)
        return lbm_fail(LBM_EINVAL, "NULL argument");
    if (n < 1 || n > MAX_AMS) return lbm_fail(LBM_EINVAL, "n must be in [1, %d]", MAX_AMS);
    if (t_len < 1) return lbm_fail(LBM_EINVAL, "t_len must be >= 1");
    if (n_kill < 1 || n_kill > n) return lbm_fail(LBM_EINVAL, "n_kill must be in [1, n]");
    AmsArgs a;
    a.series = series_dev;
    a.n = n;
    a.t_len = t_len;
    a.n_kill = n_kill;
    a.iteration = iteration;
    a.key = key;
    a.maxima = maxima_dev;
    a.killed = killed_dev;
    a.parent = parent_dev;
    a.branch_t = branch_t_dev;
    a.n_killed = n_killed_dev;
    a.level = level_dev;
    hipError_t e = launch_ams(a, (hipStream_t)hip_stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "AMS selection kernels");
}
