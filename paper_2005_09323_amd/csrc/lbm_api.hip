// C-ABI layer: context lifetime, argument validation, chunked stepping and
// the bookkeeping mirrors the host keeps of per-member device state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "api_internal.hpp"

using namespace lbm;

static thread_local std::string g_last_error;

int lbm_fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int lbm_hip_fail(hipError_t e, const char* what) {
    return lbm_fail(LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char* lbm_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// small device utilities

namespace lbm {

__global__ void fill_int_kernel(int* p, int n, int v) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = v;
}
__global__ void fill_double_kernel(double* p, int n, double v) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = v;
}
__global__ void set_int_kernel(int* p, int v) { *p = v; }
__global__ void iota_kernel(int* p, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = i;
}
__global__ void set_bits_kernel(int* p, int* list, int n, MaskBits bits) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const unsigned on = (bits.w[i >> 5] >> (i & 31)) & 1u;
    p[i] = (int)on;
    if (list && on) {  // position = set bits below i
        int pos = __popc(bits.w[i >> 5] & ((1u << (i & 31)) - 1u));
        for (int w = 0; w < (i >> 5); ++w) pos += __popc(bits.w[w]);
        list[pos] = i;
    }
}

hipError_t fill_int(int* p, int n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t fill_double(double* p, int n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_double_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t fill_iota(int* p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}
hipError_t set_int(int* p, int v, hipStream_t st) {
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, p, v);
    return hipGetLastError();
}
hipError_t set_bits(int* p, int* list, int n, const MaskBits& bits, hipStream_t st) {
    hipLaunchKernelGGL(set_bits_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, list, n, bits);
    return hipGetLastError();
}

}  // namespace lbm

// ---------------------------------------------------------------------------

static long long member_floats(const lbm_member_desc& d) { return 9LL * d.nx * d.ny; }

extern "C" size_t lbm_state_floats(const lbm_member_desc* members, int32_t n) {
    if (!members || n <= 0) return 0;
    size_t tot = 0;
    for (int i = 0; i < n; ++i) tot += (size_t)member_floats(members[i]);
    return tot;
}

static int validate_member(const lbm_member_desc& d, int i) {
    if (d.nx < 4 || d.ny < 4) return lbm_fail(LBM_EINVAL, "member %d: nx, ny must be >= 4", i);
    // the kernels index a member's 9 planes with 32-bit element offsets
    if (9LL * d.nx * d.ny > 0xFFFFFFFFLL)
        return lbm_fail(LBM_EINVAL, "member %d: lattice too large (at most %lld cells)", i, 0xFFFFFFFFLL / 9);
    if (d.reserved != 0) return lbm_fail(LBM_EINVAL, "member %d: reserved field must be 0", i);
    if (!(d.tau > 0.5) || !std::isfinite(d.tau)) return lbm_fail(LBM_EINVAL, "member %d: tau must be > 1/2", i);
    if (!std::isfinite(d.force_x)) return lbm_fail(LBM_EINVAL, "member %d: force must be finite", i);
    if (d.sq_side < 0) return lbm_fail(LBM_EINVAL, "member %d: negative square side", i);
    if (d.sq_side > 0) {
        if (d.sq_x0 < 1 || d.sq_x0 + d.sq_side > d.nx - 1 || d.sq_y0 < 1 || d.sq_y0 + d.sq_side > d.ny - 1)
            return lbm_fail(LBM_EINVAL, "member %d: square must keep one fluid cell on every side", i);
    }
    return LBM_OK;
}

// Rows per workgroup of a two-step shape's strips (0: whole strips).  The
// adaptive shape keeps whole strips when there are at least as many as
// workgroup slots (two per compute unit); otherwise it cuts them into the
// tallest row ranges (128, 64 or 32 rows) that give two workgroups per slot,
// or 32 rows when none does.  A few tall strips leave most slots idle, and a
// cut costs only the rows that both neighbours collide at phase A.  Measured
// on 16 to 96 members of 1024 x 256 and 64 to 128 of 512 x 128, this comes
// within 5 % of the best row range, at 1.2 to 1.9 x the speed of whole strips.
static int strip_rows(const lbm_ctx* c, const TileShape& ts) {
    if (ts.seg_rows >= 0) return ts.seg_rows;
    const long long slots = 2LL * c->cu_count;
    auto groups = [&](int h) {
        long long g = 0;
        for (int m = 0; m < c->n; ++m) {
            const auto& d = c->desc[m];
            const int rows = h > 0 ? std::min(h, d.ny) : d.ny;
            g += (long long)(d.nx / 256) * ((d.ny + rows - 1) / rows);
        }
        return g;
    };
    if (groups(0) >= slots) return 0;
    for (int h : {128, 64})
        if (groups(h) >= 2 * slots) return h;
    return 32;
}

// Segment table of one tiling: runs of consecutive members with the same
// lattice shape share it.  strips: the two-step kernel's tiling (one
// workgroup per 256-column strip, or per row range of one: Segment::rows).
static int build_table(lbm_ctx* c, const TileShape& ts, bool strips, Segment* seg, int& nseg, int& total) {
    const int rows = ts.tyt * ts.r;
    const int shape_split = strips ? strip_rows(c, ts) : 0;
    nseg = 0;
    int blocks = 0;
    for (int m = 0; m < c->n; ++m) {
        const auto& d = c->desc[m];
        const bool same = nseg > 0 && c->desc[seg[nseg - 1].member_begin].nx == d.nx &&
                          c->desc[seg[nseg - 1].member_begin].ny == d.ny;
        // strips: rows per workgroup, the run's own choice if it has one
        const int run = same ? nseg - 1 : nseg;
        const int split = strips && run < (int)c->run_rows.size() && c->run_rows[run] >= 0 ? c->run_rows[run]
                                                                                           : shape_split;
        const int hseg = split > 0 ? std::min(split, d.ny) : d.ny;
        const int tx = (d.nx + 255) / 256, ty = strips ? (d.ny + hseg - 1) / hseg : (d.ny + rows - 1) / rows;
        if (!same) {
            if (nseg == MAX_SEGMENTS)
                return lbm_fail(LBM_EUNSUPPORTED, "more than %d runs of distinct lattice shapes; group members by shape",
                                MAX_SEGMENTS);
            Segment s;
            s.block_begin = blocks;
            s.member_begin = m;
            s.tiles_per_member = tx * ty;
            s.tiles_x = tx;
            // four cells per lane needs 16-byte rows, and 32-bit byte offsets over the member's block
            s.vec = (d.nx % 4 == 0 && 36LL * d.nx * d.ny < (1LL << 31)) ? 1 : 0;
            s.rows = strips ? hseg : 0;
            seg[nseg++] = s;
        }
        if ((long long)blocks + (long long)tx * ty > (1LL << 31) - 1)
            return lbm_fail(LBM_EUNSUPPORTED, "ensemble needs more than 2^31 workgroups");
        blocks += tx * ty;
    }
    total = blocks;
    return LBM_OK;
}

// Whether the next batch makes two steps per launch.  The two-step kernel
// gives one workgroup per strip (or row range of a strip): with few active
// members (an AMS branch re-simulates a handful) that leaves most compute
// units idle, and one-step launches (many small tiles, the same results bit
// for bit) are faster.  The adaptive shape uses it once the active members
// give 1.5 workgroups per compute unit (measured with split strips: 0.8 x the
// one-step speed at 1 workgroup per CU, 1.1 x at 1.5, 1.2 to 1.5 x at 2).
static bool two_step_now(const lbm_ctx* c) {
    if (!c->two_step) return false;
    if (!TILE_SHAPES[c->tile_id].adaptive) return true;
    long long groups = 0;  // workgroups of the active members
    for (int s = 0; s < c->nseg2; ++s) {
        const int end = s + 1 < c->nseg2 ? c->seg2[s + 1].member_begin : c->n;
        for (int m = c->seg2[s].member_begin; m < end; ++m)
            if (c->h_active[m]) groups += c->seg2[s].tiles_per_member;
    }
    return 2 * groups >= 3LL * c->cu_count;
}

// Tables of the current tile shape.  A two-step shape applies when every
// member's width is a multiple of 256 and its block fits 32-bit byte
// offsets; otherwise (and for the last step of an odd chunk) the library
// steps with the one-step shape 0, which gives the same results.
static int build_segments(lbm_ctx* c) {
    const TileShape ts = TILE_SHAPES[c->tile_id];
    ++c->table_gen;
    c->two_step = false;
    c->one_tile = c->tile_id;
    if (ts.steps == 2) {
        c->one_tile = 0;
        bool ok = true;
        for (int m = 0; m < c->n; ++m)
            ok = ok && c->desc[m].nx % 256 == 0 && 36LL * c->desc[m].nx * c->desc[m].ny < (1LL << 31);
        if (ok) {
            int rc = build_table(c, ts, true, c->seg2, c->nseg2, c->total_blocks2);
            if (rc) return rc;
            c->two_step = true;
            c->split2 = false;
            for (int s = 0; s < c->nseg2; ++s)
                c->split2 = c->split2 || c->seg2[s].rows < c->desc[c->seg2[s].member_begin].ny;
        }
    }
    return build_table(c, TILE_SHAPES[c->one_tile], false, c->seg, c->nseg, c->total_blocks);
}

extern "C" int lbm_create(lbm_ctx** out, const lbm_member_desc* members, int32_t n_members, float* pop_a,
                          float* pop_b, size_t pop_floats, float* drag_series, int32_t series_capacity,
                          double* accum, void* hip_stream) {
    if (!out) return lbm_fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!members || n_members <= 0) return lbm_fail(LBM_EINVAL, "need at least one member");
    if (n_members > MAX_MEMBERS) return lbm_fail(LBM_EINVAL, "at most %d members", MAX_MEMBERS);
    if (!pop_a || !pop_b || !drag_series || !accum) return lbm_fail(LBM_EINVAL, "NULL device buffer");
    if (pop_a == pop_b) return lbm_fail(LBM_EINVAL, "pop_a and pop_b must be distinct buffers");
    if (((uintptr_t)pop_a | (uintptr_t)pop_b) & 15) return lbm_fail(LBM_EINVAL, "population buffers must be 16-byte aligned");
    if (series_capacity < 1) return lbm_fail(LBM_EINVAL, "series_capacity must be >= 1");
    for (int i = 0; i < n_members; ++i) {
        int rc = validate_member(members[i], i);
        if (rc) return rc;
    }
    const size_t need = lbm_state_floats(members, n_members);
    if (pop_floats < need) return lbm_fail(LBM_EINVAL, "population buffers hold %zu floats, need %zu", pop_floats, need);

    lbm_ctx* c = new lbm_ctx();
    c->n = n_members;
    c->desc.assign(members, members + n_members);
    c->pop[0] = pop_a;
    c->pop[1] = pop_b;
    c->pop_floats = pop_floats;
    c->series = drag_series;
    c->cap = series_capacity;
    c->accum = accum;
    c->stream = (hipStream_t)hip_stream;
    c->h_parity.assign(n_members, 0);
    c->h_cursor.assign(n_members, 0);
    c->h_active.assign(n_members, 1);

    long long off = 0, part = 0;
    c->h_members.resize(n_members);
    c->uniform_shape = true;
    for (int i = 0; i < n_members; ++i) {
        const auto& d = members[i];
        MemberDev& m = c->h_members[i];
        m.nx = d.nx;
        m.ny = d.ny;
        m.sx0 = d.sq_x0;
        m.sy0 = d.sq_y0;
        m.ss = d.sq_side;
        m.ring = d.sq_side > 0 ? 4 * d.sq_side + 4 : 0;
        const double omega = 1.0 / d.tau;
        m.omega = omega;
        m.half_fx = 0.5 * d.force_x;
        m.gf3 = (1.0 - 0.5 * omega) * 3.0 * d.force_x;
        m.gf9 = (1.0 - 0.5 * omega) * 9.0 * d.force_x;
        m.force = d.force_x;
        m.sb = m.s3 = m.s4 = 1.0;
        m.model = 0;
        m.open = 0;
        m.gx0 = m.bar = 0;
        m.sp_x0 = d.nx;
        m.out_rho = 0;
        m.tau = m.tau_sp = d.tau;
        m.sp_inv = 0.0;
        m.u_c = 0.0;
        m.ghost_off = 0;
        m.off = off;
        m.part_off = part;
        off += member_floats(d);
        part += (long long)m.ring * MAX_CHUNK;
        c->max_cells = std::max<long long>(c->max_cells, (long long)d.nx * d.ny);
        c->max_ny = std::max(c->max_ny, d.ny);
        if (d.nx != members[0].nx || d.ny != members[0].ny) c->uniform_shape = false;
    }
    c->partial_floats = std::max<long long>(part, 1);
    c->tile_id = DEFAULT_TILE;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            c->cu_count = cus;
    }
    int rc = build_segments(c);
    if (rc) {
        delete c;
        return rc;
    }

    hipError_t e;
    if ((e = hipMalloc(&c->d_members, sizeof(MemberDev) * n_members)) != hipSuccess ||
        (e = hipMalloc(&c->d_parity, sizeof(int) * n_members)) != hipSuccess ||
        (e = hipMalloc(&c->d_cursor, sizeof(int) * n_members)) != hipSuccess ||
        (e = hipMalloc(&c->d_active, sizeof(int) * n_members)) != hipSuccess ||
        (e = hipMalloc(&c->d_active_list, sizeof(int) * n_members)) != hipSuccess ||
        (e = hipMalloc(&c->d_flags, sizeof(int) * n_members)) != hipSuccess ||
        (e = hipMalloc(&c->d_partial, sizeof(double) * c->partial_floats)) != hipSuccess ||
        (e = hipMalloc(&c->d_scratch, sizeof(double) * (4 * (size_t)n_members + 64))) != hipSuccess ||
        (e = hipMalloc(&c->d_iscratch, sizeof(int) * (4 * (size_t)n_members + 64))) != hipSuccess) {
        lbm_destroy(c);
        return lbm_hip_fail(e, "hipMalloc of library scratch");
    }
    if ((e = hipMemcpy(c->d_members, c->h_members.data(), sizeof(MemberDev) * n_members, hipMemcpyHostToDevice)) !=
        hipSuccess) {
        lbm_destroy(c);
        return lbm_hip_fail(e, "upload of member table");
    }
    if ((e = fill_int(c->d_parity, n_members, 0, c->stream)) != hipSuccess ||
        (e = fill_int(c->d_cursor, n_members, 0, c->stream)) != hipSuccess ||
        (e = fill_int(c->d_active, n_members, 1, c->stream)) != hipSuccess ||
        (e = fill_iota(c->d_active_list, n_members, c->stream)) != hipSuccess ||
        (e = fill_int(c->d_flags, n_members, 0, c->stream)) != hipSuccess) {
        lbm_destroy(c);
        return lbm_hip_fail(e, "initialising bookkeeping");
    }
    c->n_active = n_members;
    *out = c;
    return LBM_OK;
}

extern "C" int lbm_destroy(lbm_ctx* c) {
    if (!c) return LBM_OK;
    if (c->stream) hipStreamSynchronize(c->stream); else hipDeviceSynchronize();
    hipFree(c->d_members);
    hipFree(c->d_parity);
    hipFree(c->d_cursor);
    hipFree(c->d_active);
    hipFree(c->d_active_list);
    hipFree(c->d_flags);
    hipFree(c->d_partial);
    hipFree(c->d_scratch);
    hipFree(c->d_iscratch);
    hipFree(c->d_ghost);
    free_chunk_graph(c);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    free_rare_scratch(c);
    delete c;
    return LBM_OK;
}

static FinalizeArgs finalize_args(lbm_ctx* c, int n, int accumulate, int swap_parity) {
    FinalizeArgs f;
    f.members = c->d_members;
    f.active = c->d_active;
    f.parity = c->d_parity;
    f.cursor = c->d_cursor;
    f.flags = c->d_flags;
    f.partial = c->d_partial;
    f.series = c->series;
    f.accum = c->accum;
    f.ld = c->cap;
    f.n = n;
    f.accumulate = accumulate;
    f.swap_parity = swap_parity;
    f.mu = c->mu;
    f.inv_sigma_dt = c->dt / c->sigma;
    return f;
}

extern "C" int lbm_init(lbm_ctx* c, uint64_t seed, double noise_amp) { return lbm_init_flow(c, seed, noise_amp, 0.0); }

extern "C" int lbm_init_flow(lbm_ctx* c, uint64_t seed, double noise_amp, double ux0) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    if (!std::isfinite(noise_amp) || noise_amp < 0 || noise_amp >= 0.5)
        return lbm_fail(LBM_EINVAL, "noise_amp must be in [0, 0.5)");
    if (!std::isfinite(ux0) || std::fabs(ux0) > 0.3) return lbm_fail(LBM_EINVAL, "|ux0| must be <= 0.3");
    if (c->open && ux0 != 0.0) return lbm_fail(LBM_EINVAL, "an open channel starts from its inlet profile: ux0 must be 0");
    hipError_t e;
    if ((e = fill_int(c->d_parity, c->n, 0, c->stream)) != hipSuccess ||
        (e = fill_int(c->d_cursor, c->n, 0, c->stream)) != hipSuccess ||
        (e = fill_int(c->d_active, c->n, 1, c->stream)) != hipSuccess ||
        (e = fill_iota(c->d_active_list, c->n, c->stream)) != hipSuccess ||
        (e = fill_int(c->d_flags, c->n, 0, c->stream)) != hipSuccess ||
        (e = fill_double(c->accum, c->n, 0.0, c->stream)) != hipSuccess)
        return lbm_hip_fail(e, "lbm_init bookkeeping");
    std::fill(c->h_parity.begin(), c->h_parity.end(), 0);
    std::fill(c->h_active.begin(), c->h_active.end(), 1);
    c->n_active = c->n;
    InitArgs a;
    a.members = c->d_members;
    a.pop0 = c->pop[0];
    a.partial = c->d_partial;
    a.seed = seed;
    a.noise_amp = noise_amp;
    a.ux0 = ux0;
    if ((e = launch_init(a, c->n, c->max_cells, c->stream)) != hipSuccess) return lbm_hip_fail(e, "init kernel");
    if ((e = launch_finalize(finalize_args(c, 1, 0, 0), c->n, c->stream)) != hipSuccess)
        return lbm_hip_fail(e, "drag reduction");
    std::fill(c->h_cursor.begin(), c->h_cursor.end(), 1);
    return LBM_OK;
}

extern "C" int lbm_set_observable(lbm_ctx* c, double mu, double sigma, double dt) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    if (!std::isfinite(mu) || !(sigma > 0) || !std::isfinite(sigma) || !(dt > 0) || !std::isfinite(dt))
        return lbm_fail(LBM_EINVAL, "need finite mu, sigma > 0, dt > 0");
    c->mu = mu;
    c->sigma = sigma;
    c->dt = dt;
    return LBM_OK;
}

extern "C" int lbm_set_active(lbm_ctx* c, const int32_t* active_host) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    MaskBits bits{};
    c->n_active = 0;
    for (int m = 0; m < c->n; ++m) {
        const int on = active_host ? (active_host[m] != 0) : 1;
        c->h_active[m] = on;
        c->n_active += on;
        if (on) bits.w[m >> 5] |= 1u << (m & 31);
    }
    hipError_t e = set_bits(c->d_active, c->d_active_list, c->n, bits, c->stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "active mask upload");
}

extern "C" int lbm_step_batch(lbm_ctx* c, int32_t n_steps) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    if (n_steps < 0) return lbm_fail(LBM_EINVAL, "n_steps must be >= 0");
    if (n_steps == 0) return LBM_OK;
    for (int m = 0; m < c->n; ++m)
        if (c->h_active[m] && (long long)c->h_cursor[m] + n_steps > c->cap)
            return lbm_fail(LBM_ERANGE, "member %d: drag column %d + %d steps exceeds capacity %d", m,
                            c->h_cursor[m], n_steps, c->cap);
    StepArgs a;
    a.members = c->d_members;
    a.parity = c->d_parity;
    a.active = c->d_active;
    a.pop0 = c->pop[0];
    a.pop1 = c->pop[1];
    a.partial = c->d_partial;
    a.xcd = TILE_SHAPES[c->one_tile].xcd;
    a.split = 0;
    a.total_blocks = c->total_blocks;
    a.nseg = c->nseg;
    for (int s = 0; s < c->nseg; ++s) a.seg[s] = c->seg[s];
    StepArgs a2 = a;
    if (c->two_step) {
        a2.xcd = TILE_SHAPES[c->tile_id].xcd;
        a2.split = c->split2 ? 1 : 0;
        a2.total_blocks = c->total_blocks2;
        a2.nseg = c->nseg2;
        for (int s = 0; s < c->nseg2; ++s) a2.seg[s] = c->seg2[s];
    }
    const int waves2 = TILE_SHAPES[c->tile_id].tyt;
    const bool two = two_step_now(c);
    a.active_list = nullptr;
    a2.active_list = nullptr;
    a.ghost = c->open ? c->d_ghost : nullptr;
    a2.ghost = a.ghost;
    GhostArgs g;
    g.members = c->d_members;
    g.parity = c->d_parity;
    g.active = c->d_active;
    g.pop0 = c->pop[0];
    g.pop1 = c->pop[1];
    g.ghost = c->d_ghost;
    if (c->n_active == 0) return LBM_OK;  // nothing steps (no drag column either)
    if (c->n_active < c->n && c->uniform_shape) {
        // launch the active members' tiles only: the inactive ones would cost a
        // workgroup dispatch each (the grid of a full ensemble) for no work
        a.active_list = c->d_active_list;
        a.total_blocks = c->n_active * c->seg[0].tiles_per_member;
        if (c->two_step) {
            a2.active_list = c->d_active_list;
            a2.total_blocks = c->n_active * c->seg2[0].tiles_per_member;
        }
    }
    // the launches of one chunk of steps on stream st; `launches` counts them
    // (every launch swaps the buffers once, whether it makes one step or two)
    auto enqueue = [&](int chunk, hipStream_t st, int& launches) -> hipError_t {
        hipError_t e;
        int s = 0;
        launches = 0;
        if (two)
            for (; s + 1 < chunk; s += 2, ++launches) {
                a2.slot = s;
                a2.flip = launches & 1;
                if (c->open) {  // the inlet's values and the outlet ghost column of the first of the two steps
                    g.flip = a2.flip;
                    if ((e = launch_outlet_ghost(g, c->n, c->max_ny, st)) != hipSuccess) return e;
                }
                if ((e = launch_step2(waves2, a2, c->model, st)) != hipSuccess) return e;
            }
        for (; s < chunk; ++s, ++launches) {
            a.slot = s;
            a.flip = launches & 1;
            if (c->open) {
                g.flip = a.flip;
                if ((e = launch_outlet_ghost(g, c->n, c->max_ny, st)) != hipSuccess) return e;
            }
            if ((e = launch_step(c->one_tile, a, c->model, st)) != hipSuccess) return e;
        }
        return launch_finalize(finalize_args(c, chunk, 1, launches & 1), c->n, st);
    };
    hipError_t e;
    int done = 0;
    while (done < n_steps) {
        const int chunk = std::min(n_steps - done, c->chunk);
        int launches = 0;
        if (c->graphs && chunk == c->chunk) {
            ChunkGraphKey key{c->tile_id, c->one_tile, two ? 1 : 0, waves2, c->model, c->open ? 1 : 0, chunk,
                              c->table_gen, a.total_blocks, a2.total_blocks, a.active_list ? 1 : 0, c->mu, c->dt / c->sigma,
                              (const void*)c->d_ghost};
            if (!c->graph_exec || !(key == c->graph_key)) {
                free_chunk_graph(c);
                if (!c->cap_stream && (e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != hipSuccess)
                    return lbm_hip_fail(e, "capture stream");
                if ((e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                    return lbm_hip_fail(e, "begin capture");
                int l = 0;
                const hipError_t ce = enqueue(chunk, c->cap_stream, l);
                hipGraph_t gr = nullptr;
                const hipError_t ee = hipStreamEndCapture(c->cap_stream, &gr);
                if (ce != hipSuccess || ee != hipSuccess) {
                    if (gr) hipGraphDestroy(gr);
                    return lbm_hip_fail(ce != hipSuccess ? ce : ee, "capture of a chunk of steps");
                }
                if ((e = hipGraphInstantiateWithFlags(&c->graph_exec, gr, 0)) != hipSuccess) {
                    hipGraphDestroy(gr);
                    c->graph_exec = nullptr;
                    return lbm_hip_fail(e, "graph instantiation");
                }
                c->graph = gr;
                c->graph_key = key;
                c->graph_launches = l;
            }
            if ((e = hipGraphLaunch(c->graph_exec, c->stream)) != hipSuccess) return lbm_hip_fail(e, "graph launch");
            launches = c->graph_launches;
        } else if ((e = enqueue(chunk, c->stream, launches)) != hipSuccess) {
            return lbm_hip_fail(e, "lattice step launches");
        }
        for (int m = 0; m < c->n; ++m)
            if (c->h_active[m]) {
                c->h_parity[m] ^= (launches & 1);
                c->h_cursor[m] += chunk;
            }
        done += chunk;
    }
    return LBM_OK;
}

void free_chunk_graph(lbm_ctx* c) {
    if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
    if (c->graph) hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}

extern "C" int lbm_set_graphs(lbm_ctx* c, int32_t on) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    c->graphs = on != 0;
    return LBM_OK;
}

extern "C" int lbm_drag(const lbm_ctx* c, int32_t t0, int32_t t1, float* out_dev) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    if (t0 < 0 || t1 < t0 || t1 > c->cap) return lbm_fail(LBM_EINVAL, "bad column range [%d, %d)", t0, t1);
    if (t1 == t0) return LBM_OK;
    if (!out_dev) return lbm_fail(LBM_EINVAL, "NULL output");
    hipError_t e = hipMemcpy2DAsync(out_dev, sizeof(float) * (t1 - t0), c->series + t0, sizeof(float) * c->cap,
                                    sizeof(float) * (t1 - t0), c->n, hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "drag copy");
}

extern "C" int lbm_member_state(const lbm_ctx* c, int32_t m, float** state_dev) {
    if (!c || !state_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (m < 0 || m >= c->n) return lbm_fail(LBM_EINVAL, "member %d out of range", m);
    *state_dev = c->pop[c->h_parity[m]] + c->h_members[m].off;
    return LBM_OK;
}

extern "C" int lbm_member_time(const lbm_ctx* c, int32_t m, int32_t* t) {
    if (!c || !t) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (m < 0 || m >= c->n) return lbm_fail(LBM_EINVAL, "member %d out of range", m);
    *t = c->h_cursor[m];
    return LBM_OK;
}

extern "C" int lbm_set_time(lbm_ctx* c, int32_t t) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    if (t < 0 || t > c->cap) return lbm_fail(LBM_EINVAL, "time %d outside [0, %d]", t, c->cap);
    hipError_t e = fill_int(c->d_cursor, c->n, t, c->stream);
    if (e != hipSuccess) return lbm_hip_fail(e, "cursor reset");
    std::fill(c->h_cursor.begin(), c->h_cursor.end(), t);
    return LBM_OK;
}

extern "C" int lbm_flags(const lbm_ctx* c, int32_t* out_dev) {
    if (!c || !out_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    hipError_t e = hipMemcpyAsync(out_dev, c->d_flags, sizeof(int) * c->n, hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "flags copy");
}

extern "C" int lbm_set_flags(lbm_ctx* c, const int32_t* flags_dev) {
    if (!c || !flags_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    hipError_t e = hipMemcpyAsync(c->d_flags, flags_dev, sizeof(int) * c->n, hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "flags copy");
}

extern "C" int lbm_set_collision(lbm_ctx* c, int32_t model, double s_bulk, double s_third, double s_fourth) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    if (model != 0 && model != 1) return lbm_fail(LBM_EINVAL, "collision model %d: 0 (BGK) or 1 (central moments)", model);
    if (model == 1)
        for (double s : {s_bulk, s_third, s_fourth})
            if (!(s > 0.0 && s < 2.0)) return lbm_fail(LBM_EINVAL, "relaxation rate %g outside (0, 2)", s);
    // unit bulk, third- and fourth-order rates: the shorter evaluation of the same collision
    const int internal = model == 1 && s_bulk == 1.0 && s_third == 1.0 && s_fourth == 1.0 ? 2 : model;
    c->model = internal;
    for (auto& m : c->h_members) {
        m.model = internal;
        if (model == 1) {
            m.sb = s_bulk;
            m.s3 = s_third;
            m.s4 = s_fourth;
        }
    }
    hipError_t e = hipMemcpyAsync(c->d_members, c->h_members.data(), sizeof(MemberDev) * c->n, hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "member table upload");
}

static int validate_open(const lbm_member_desc& d, int i, const lbm_open_channel& o) {
    if (d.ny > 2048) return lbm_fail(LBM_EUNSUPPORTED, "member %d: open channels support ny <= 2048", i);
    if (o.grid_bar > 0) {
        if (o.grid_x0 < 1 || o.grid_x0 + o.grid_bar > d.nx - 2)
            return lbm_fail(LBM_EINVAL, "member %d: the grid must lie within columns 1 .. nx - 3", i);
        if (d.sq_side > 0 && o.grid_x0 + o.grid_bar > d.sq_x0 - 2)
            return lbm_fail(LBM_EINVAL, "member %d: the grid must end at least two columns before the square", i);
    }
    if (d.sq_side > 0 && (d.sq_x0 < 2 || d.sq_x0 + d.sq_side > d.nx - 3))
        return lbm_fail(LBM_EINVAL, "member %d: an open channel needs two fluid columns before and three after the square", i);
    return LBM_OK;
}

extern "C" int lbm_set_open_channel(lbm_ctx* c, const lbm_open_channel* oc) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    if (oc) {
        if (oc->outlet_density != 0 && oc->outlet_density != 1)
            return lbm_fail(LBM_EINVAL, "outlet_density must be 0 (held at 1) or 1 (extrapolated)");
        if (!std::isfinite(oc->u_c) || oc->u_c < 0.0 || oc->u_c > 0.3)
            return lbm_fail(LBM_EINVAL, "inlet centre-line velocity must be in [0, 0.3]");
        if (oc->grid_bar < 0) return lbm_fail(LBM_EINVAL, "negative grid bar size");
        if (oc->sponge_x0 < 0) return lbm_fail(LBM_EINVAL, "negative sponge start");
        if (!(oc->sponge_tau > 0.5) || !std::isfinite(oc->sponge_tau))
            return lbm_fail(LBM_EINVAL, "sponge relaxation time must be > 1/2");
        for (int m = 0; m < c->n; ++m) {
            int rc = validate_open(c->desc[m], m, *oc);
            if (rc) return rc;
        }
    }
    hipError_t e = hipStreamSynchronize(c->stream);  // no launch may still read the table or the ghost columns
    if (e != hipSuccess) return lbm_hip_fail(e, "stream synchronisation");
    free_chunk_graph(c);  // it holds the old ghost pointer
    hipFree(c->d_ghost);
    c->d_ghost = nullptr;
    long long goff = 0;
    for (int m = 0; m < c->n; ++m) {
        MemberDev& md = c->h_members[m];
        const auto& d = c->desc[m];
        md.open = oc ? 1 : 0;
        md.gx0 = oc && oc->grid_bar > 0 ? oc->grid_x0 : 0;
        md.bar = oc ? oc->grid_bar : 0;
        md.sp_x0 = oc ? std::min(oc->sponge_x0, d.nx) : d.nx;
        md.tau_sp = oc ? oc->sponge_tau : d.tau;
        md.sp_inv = md.sp_x0 < d.nx - 1 ? 1.0 / (double)(d.nx - 1 - md.sp_x0) : 0.0;
        md.u_c = oc ? oc->u_c : 0.0;
        md.out_rho = oc ? oc->outlet_density : 0;
        md.ghost_off = goff;
        goff += 9LL * d.ny;
    }
    c->open = oc != nullptr;
    if (c->open && (e = hipMalloc(&c->d_ghost, sizeof(float) * (size_t)goff)) != hipSuccess) {
        c->open = false;
        for (auto& md : c->h_members) md.open = md.bar = 0;
        hipMemcpy(c->d_members, c->h_members.data(), sizeof(MemberDev) * c->n, hipMemcpyHostToDevice);
        build_segments(c);
        return lbm_hip_fail(e, "hipMalloc of outlet ghost columns");
    }
    e = hipMemcpy(c->d_members, c->h_members.data(), sizeof(MemberDev) * c->n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return lbm_hip_fail(e, "member table upload");
    return build_segments(c);
}

extern "C" int32_t lbm_tile_count(void) { return N_TILE_SHAPES; }

extern "C" int lbm_launch_steps(const lbm_ctx* c, int32_t* steps) {
    if (!c || !steps) return lbm_fail(LBM_EINVAL, "NULL argument");
    *steps = two_step_now(c) ? 2 : 1;
    return LBM_OK;
}

extern "C" int lbm_set_tile(lbm_ctx* c, int32_t tile_id) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    if (tile_id < 0 || tile_id >= N_TILE_SHAPES) return lbm_fail(LBM_EINVAL, "tile id %d out of range", tile_id);
    const int old = c->tile_id;
    c->tile_id = tile_id;
    int rc = build_segments(c);
    if (rc) {
        c->tile_id = old;
        build_segments(c);
    }
    return rc;
}

// Runs of consecutive members with one lattice shape (the segments of the tables).
static int count_runs(const lbm_ctx* c) {
    int runs = 0;
    for (int m = 0; m < c->n; ++m)
        if (m == 0 || c->desc[m].nx != c->desc[m - 1].nx || c->desc[m].ny != c->desc[m - 1].ny) ++runs;
    return runs;
}

extern "C" int lbm_run_count(const lbm_ctx* c, int32_t* n_runs) {
    if (!c || !n_runs) return lbm_fail(LBM_EINVAL, "NULL argument");
    *n_runs = count_runs(c);
    return LBM_OK;
}

extern "C" int lbm_set_run_rows(lbm_ctx* c, const int32_t* rows, int32_t n_runs) {
    if (!c) return lbm_fail(LBM_EINVAL, "NULL context");
    if (n_runs == 0) {
        c->run_rows.clear();
        return build_segments(c);
    }
    if (!rows) return lbm_fail(LBM_EINVAL, "NULL rows");
    if (n_runs != count_runs(c))
        return lbm_fail(LBM_EINVAL, "%d row ranges for %d runs of lattice shapes", n_runs, count_runs(c));
    for (int r = 0; r < n_runs; ++r)
        if (rows[r] < -1) return lbm_fail(LBM_EINVAL, "run %d: rows %d (-1 by the shape, 0 whole strips, >= 1)", r, rows[r]);
    const std::vector<int> old = c->run_rows;
    c->run_rows.assign(rows, rows + n_runs);
    int rc = build_segments(c);
    if (rc) {
        c->run_rows = old;
        build_segments(c);
    }
    return rc;
}

extern "C" int lbm_get_run_rows(const lbm_ctx* c, int32_t* rows, int32_t max_runs, int32_t* n_runs) {
    if (!c || !n_runs) return lbm_fail(LBM_EINVAL, "NULL argument");
    *n_runs = c->two_step ? c->nseg2 : count_runs(c);
    if (rows && max_runs < *n_runs) return lbm_fail(LBM_EINVAL, "room for %d runs, need %d", max_runs, *n_runs);
    if (rows)
        for (int s = 0; s < *n_runs; ++s) {
            if (!c->two_step) {
                rows[s] = -1;
                continue;
            }
            const int ny = c->desc[c->seg2[s].member_begin].ny;
            rows[s] = c->seg2[s].rows >= ny ? 0 : c->seg2[s].rows;
        }
    return LBM_OK;
}

extern "C" int lbm_autotune(lbm_ctx* c, int32_t n_steps, int32_t* best_tile) {
    if (!c || !best_tile) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (n_steps < 1) return lbm_fail(LBM_EINVAL, "n_steps must be >= 1");
    StepArgs a;
    a.members = c->d_members;
    a.parity = c->d_parity;
    a.active = c->d_active;
    a.pop0 = c->pop[0];
    a.pop1 = c->pop[1];
    a.partial = c->d_partial;
    a.active_list = nullptr;  // every member, whatever the mask
    a.ghost = c->open ? c->d_ghost : nullptr;
    GhostArgs g;
    g.members = c->d_members;
    g.parity = c->d_parity;
    g.active = c->d_active;
    g.pop0 = c->pop[0];
    g.pop1 = c->pop[1];
    g.ghost = c->d_ghost;
    // Launches are timed in pairs so every state ends in the buffer it
    // started in; the states do advance (untracked: no drag, no cursor), so
    // callers tune before lbm_init, which rebuilds step 0.
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return lbm_fail(LBM_EHIP, "event creation failed");
    float best_ms = 1e30f;  // per step
    int best = c->tile_id;
    const int pairs = std::max(1, n_steps / 2);
    c->run_rows.clear();  // the shapes first, each with its own row policy
    // time the current tables with shape t; ms per step, or a negative value
    // if the shape does not apply
    auto time_shape = [&](int t, float& ms) -> int {
        ms = -1.0f;
        if (build_segments(c) != LBM_OK) return LBM_OK;
        const TileShape ts = TILE_SHAPES[t];
        if (ts.steps == 2 && !c->two_step) return LBM_OK;  // it would run shape 0
        if (ts.adaptive) return LBM_OK;                    // a policy over shapes 16 and 0, not a shape
        const bool two = ts.steps == 2;
        a.total_blocks = two ? c->total_blocks2 : c->total_blocks;
        a.split = two && c->split2 ? 1 : 0;
        a.xcd = ts.xcd;
        a.nseg = two ? c->nseg2 : c->nseg;
        for (int s = 0; s < a.nseg; ++s) a.seg[s] = two ? c->seg2[s] : c->seg[s];
        a.slot = 0;
        auto launch = [&](int flip) {
            a.flip = flip;
            if (c->open) {  // the outlet ghost column the launch's first step pulls
                g.flip = flip;
                hipError_t ge = launch_outlet_ghost(g, c->n, c->max_ny, c->stream);
                if (ge != hipSuccess) return ge;
            }
            return two ? launch_step2(ts.tyt, a, c->model, c->stream) : launch_step(t, a, c->model, c->stream);
        };
        // warm-up pair
        launch(0);
        launch(1);
        hipEventRecord(e0, c->stream);
        for (int p = 0; p < pairs; ++p) {
            launch(0);
            launch(1);
        }
        hipEventRecord(e1, c->stream);
        hipError_t err = hipEventSynchronize(e1);
        if (err != hipSuccess) return lbm_hip_fail(err, "autotune timing");
        float t_ms = 0;
        hipEventElapsedTime(&t_ms, e0, e1);
        ms = t_ms / (float)(2 * pairs * ts.steps);
        return LBM_OK;
    };
    int rc = LBM_OK;
    for (int t = 0; t < N_TILE_SHAPES && rc == LBM_OK; ++t) {
        c->tile_id = t;
        float ms;
        rc = time_shape(t, ms);
        if (rc == LBM_OK && ms >= 0.0f && ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    // Runs of different lattice sizes (an uneven batch): each run's row range
    // on its own, one run at a time (whole strips, 128, 64 or 32 rows per
    // workgroup), keeping whatever times best for the whole ensemble.
    c->tile_id = best;
    const int runs = count_runs(c);
    if (rc == LBM_OK && TILE_SHAPES[best].steps == 2 && runs > 1 && build_segments(c) == LBM_OK && c->two_step) {
        c->run_rows.assign(runs, -1);
        for (int r = 0; r < runs; ++r) c->run_rows[r] = c->seg2[r].rows >= c->desc[c->seg2[r].member_begin].ny ? 0 : c->seg2[r].rows;
        rc = time_shape(best, best_ms);  // the reference, timed next to the variants
        for (int r = 0; r < runs && rc == LBM_OK; ++r) {
            const int ny = c->desc[c->seg2[r].member_begin].ny;
            int keep = c->run_rows[r];
            for (int h : {0, 128, 64, 32}) {
                if (h == keep || (h > 0 && h >= ny)) continue;
                c->run_rows[r] = h;
                float ms;
                rc = time_shape(best, ms);
                if (rc != LBM_OK) break;
                if (ms >= 0.0f && ms < 0.99f * best_ms) {  // a clear gain only
                    best_ms = ms;
                    keep = h;
                }
            }
            c->run_rows[r] = keep;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->tile_id = best;
    build_segments(c);
    *best_tile = best;
    return rc;
}

// What a tuned launch shape depends on: the runs of lattice shapes, the
// collision and whether the channels are open.
static std::string tune_key(const lbm_ctx* c) {
    std::ostringstream k;
    k << "model=" << c->model << " open=" << (c->open ? 1 : 0) << " shapes=";
    int run = 0;
    for (int m = 0; m < c->n; ++m) {
        ++run;
        if (m + 1 == c->n || c->desc[m + 1].nx != c->desc[m].nx || c->desc[m + 1].ny != c->desc[m].ny) {
            k << c->desc[m].nx << "x" << c->desc[m].ny << "*" << run << ";";
            run = 0;
        }
    }
    return k.str();
}

extern "C" int lbm_autotune_cached(lbm_ctx* c, int32_t n_steps, const char* path, int32_t* best_tile) {
    if (!c || !path || !best_tile) return lbm_fail(LBM_EINVAL, "NULL argument");
    const std::string key = tune_key(c);
    {
        std::ifstream in(path);
        std::string line;
        while (in && std::getline(in, line)) {
            const size_t tab = line.rfind('\t');
            if (tab == std::string::npos || line.compare(0, tab, key) != 0 || tab != key.size()) continue;
            // "<tile>" or "<tile> <rows of run 0>,<rows of run 1>,..."
            std::istringstream val(line.substr(tab + 1));
            int tile = -1;
            val >> tile;
            if (!val && !val.eof()) continue;
            if (tile < 0 || tile >= N_TILE_SHAPES) continue;  // a table from another build: tune again
            std::vector<int32_t> rows;
            std::string list;
            if (val >> list) {
                std::istringstream ls(list);
                std::string item;
                while (std::getline(ls, item, ',')) rows.push_back((int32_t)std::atoi(item.c_str()));
            }
            c->run_rows.clear();
            int rc = lbm_set_tile(c, tile);
            if (rc) return rc;
            if (!rows.empty() && (rc = lbm_set_run_rows(c, rows.data(), (int32_t)rows.size())) != LBM_OK) return rc;
            *best_tile = tile;
            return LBM_OK;
        }
    }
    const int rc = lbm_autotune(c, n_steps, best_tile);
    if (rc) return rc;
    std::ofstream out(path, std::ios::app);
    out << key << '\t' << *best_tile;
    for (size_t r = 0; r < c->run_rows.size(); ++r) out << (r ? ',' : ' ') << c->run_rows[r];
    out << '\n';
    if (!out) return lbm_fail(LBM_EINVAL, "cannot append the tuned shape to %s", path);
    return LBM_OK;
}
