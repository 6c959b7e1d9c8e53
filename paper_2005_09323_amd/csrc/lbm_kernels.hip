// Lattice-Boltzmann kernels: initial state, fused pull-stream + BGK collide
// step with momentum-exchange drag partials, and the per-chunk drag
// reduction with the FP64 observable integral.
//
// Paper Appendix A gives the scheme (exact streaming, BGK relaxation to the
// second-order equilibrium); Section 2 the halfway bounce-back on walls and
// obstacle; Section 2.1 the drag.  Populations are FP32 deviations
// d_i = f_i - w_i so that the O(1) rest weights never enter FP32 sums.
#include "kernels.hpp"

namespace lbm {

// BGK relaxation with Guo forcing of one cell, in deviation form:
//   rho = 1 + sum d_i,  j = sum c_i d_i,  u = (j + F/2) / rho,
//   d_i^eq = w_i [(rho - 1) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u^2)],
//   d_i <- d_i + omega (d_i^eq - d_i) + w_i (1 - omega/2) [3 (c_ix - u_x) + 9 (c.u) c_ix] F.
// (The w_i of f_i = w_i + d_i cancel exactly between f_i and f_i^eq.)
// The populations are stored in FP32 but the update is computed in FP64:
// the flow changes little from one step to the next, so FP32 rounding in
// the update repeats with the same sign step after step and its error grows
// linearly in time, while one rounding on store does not.
__device__ __forceinline__ void bgk_guo(const MemberDev& m, const float din[9], double d[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) d[i] = (double)din[i];
    const double drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    const double jx = ((d[1] - d[3]) + (d[5] - d[6])) + (d[8] - d[7]);
    const double jy = ((d[2] - d[4]) + (d[5] - d[7])) + (d[6] - d[8]);
    const double rho = 1.0 + drho;
    const double inv = 1.0 / rho;
    const double ux = (jx + m.half_fx) * inv;
    const double uy = jy * inv;
    const double usq = 1.5 * (ux * ux + uy * uy);
    const double om = m.omega;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double cu = (double)CX[i] * ux + (double)CY[i] * uy;
        const double deq = WD[i] * (drho + rho * (3.0 * cu + 4.5 * cu * cu - usq));
        const double src = WD[i] * (m.gf3 * ((double)CX[i] - ux) + m.gf9 * cu * (double)CX[i]);
        d[i] = d[i] + om * (deq - d[i]) + src;
    }
}

// Momentum handed to the square by one ring cell: sum over its links into
// the square of 2 c_ix f_i^out (the w_i parts cancel over the closed square,
// so deviations give the same total).
__device__ __forceinline__ double ring_drag(const MemberDev& m, const double d[9], int x, int y) {
    double acc = 0.0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        if (CX[i] == 0) continue;
        if (in_square(m, x + CX[i], y + CY[i])) acc += 2.0 * (double)CX[i] * d[i];
    }
    return acc;
}

// Workgroup -> (member, tile): members are grouped in segments of equal
// lattice shape; within a segment tiles run x-fastest, then y, then member.
__device__ __forceinline__ int block_to_member(const StepArgs& a, int b, int& tx, int& ty) {
    int s = 0;
#pragma unroll 1
    while (s + 1 < a.nseg && b >= a.seg[s + 1].block_begin) ++s;
    const int local = b - a.seg[s].block_begin;
    const int mloc = local / a.seg[s].tiles_per_member;
    const int tile = local - mloc * a.seg[s].tiles_per_member;
    ty = tile / a.seg[s].tiles_x;
    tx = tile - ty * a.seg[s].tiles_x;
    return a.seg[s].member_begin + mloc;
}

// Spread consecutive logical tiles over one XCD: the hardware deals
// workgroups round-robin to the 8 XCDs, so logical tile L runs on XCD
// (physical id % 8); give each XCD a contiguous range of logical tiles so
// that vertically adjacent tiles share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int total) {
    const int per = total / 8, rem = total % 8;
    const int xcd = b & 7, k = b >> 3;
    return (xcd < rem) ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

template <int TYT, int R>
__global__ __launch_bounds__(64 * TYT) void step_kernel(StepArgs a) {
    const int b = a.xcd ? xcd_remap((int)blockIdx.x, a.total_blocks) : (int)blockIdx.x;
    int tx, ty;
    const int mi = block_to_member(a, b, tx, ty);
    if (!a.active[mi]) return;
    const MemberDev m = a.members[mi];
    const int par = a.parity[mi] ^ a.flip;
    const float* __restrict__ src = (par ? a.pop1 : a.pop0) + m.off;
    float* __restrict__ dst = (par ? a.pop0 : a.pop1) + m.off;
    const int nx = m.nx, ny = m.ny;
    const long long plane = (long long)nx * ny;
    const int x = tx * 64 + (int)(threadIdx.x & 63);
    const int ly = (int)(threadIdx.x >> 6);
    if (x >= nx) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = ty * (TYT * R) + r * TYT + ly;
        if (y >= ny) break;
        if (in_square(m, x, y)) continue;
        float dl[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int xs = x - CX[i];
            xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
            const int ys = y - CY[i];
            const bool bounce = (ys < 0) | (ys >= ny) | in_square(m, xs, ys);
            const long long idx = bounce ? (long long)OPP[i] * plane + (long long)y * nx + x
                                         : (long long)i * plane + (long long)ys * nx + xs;
            dl[i] = src[idx];
        }
        double d[9];
        bgk_guo(m, dl, d);
        const long long cell = (long long)y * nx + x;
#pragma unroll
        for (int i = 0; i < 9; ++i) dst[(long long)i * plane + cell] = (float)d[i];
        const int ri = ring_index(m, x, y);
        if (ri >= 0) a.partial[m.part_off + (long long)a.slot * m.ring + ri] = ring_drag(m, d, x, y);
    }
}

// Step 0: equilibrium at rest with the seeded density, relaxed once.
__global__ __launch_bounds__(256) void init_kernel(InitArgs a) {
    const int mi = (int)blockIdx.y;
    const MemberDev m = a.members[mi];
    const long long plane = (long long)m.nx * m.ny;
    const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
    if (cell >= plane) return;
    const int y = (int)(cell / m.nx), x = (int)(cell - (long long)y * m.nx);
    if (in_square(m, x, y)) return;
    double drho = 0.0;
    if (a.noise_amp != 0.0) {
        const U64x4 w = philox4x64_10((uint64_t)cell, (uint64_t)mi, 0, 0, a.seed, PURPOSE_INIT);
        drho = a.noise_amp * (2.0 * uniform53(w.v[0]) - 1.0);
    }
    float d0[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) d0[i] = (float)(WD[i] * drho);
    double d[9];
    bgk_guo(m, d0, d);
    float* dst = a.pop0 + m.off;  // step 0 lives in buffer 0 (parity 0)
#pragma unroll
    for (int i = 0; i < 9; ++i) dst[(long long)i * plane + cell] = (float)d[i];
    const int ri = ring_index(m, x, y);
    if (ri >= 0) a.partial[m.part_off + ri] = ring_drag(m, d, x, y);
}

// Reduce the drag partials of a chunk of n steps for one member per block:
// f_d(s) = sum of ring partials in ring order (FP64), written to the series at
// the member's cursor; then, in step order, accum += (f_d - mu)/sigma * dt.
// The member's parity flips n times (not for step 0, which init wrote in
// place) and its cursor advances by n.
__global__ __launch_bounds__(256) void finalize_kernel(FinalizeArgs a) {
    const int mi = (int)blockIdx.x;
    if (!a.active[mi]) return;
    const MemberDev m = a.members[mi];
    __shared__ double fd[256];
    const int s = (int)threadIdx.x;
    const int cur = a.cursor[mi];
    if (s < a.n) {
        double acc = 0.0;
        const double* p = a.partial + m.part_off + (long long)s * m.ring;
        for (int r = 0; r < m.ring; ++r) acc += p[r];
        fd[s] = acc;
        a.series[(long long)mi * a.ld + cur + s] = (float)acc;
    }
    __syncthreads();
    if (s == 0) {
        bool bad = false;
        if (a.accumulate) {
            double tot = a.accum[mi];
            for (int t = 0; t < a.n; ++t) {
                tot += (fd[t] - a.mu) * a.inv_sigma_dt;
                bad |= !isfinite(fd[t]);
            }
            a.accum[mi] = tot;
        } else {
            for (int t = 0; t < a.n; ++t) bad |= !isfinite(fd[t]);
        }
        if (bad) a.flags[mi] = 1;
        a.parity[mi] ^= (a.n & a.advance_parity);
        a.cursor[mi] = cur + a.n;
    }
}

// ---------------------------------------------------------------------------
// launchers

template <int TYT, int R>
static hipError_t launch_step_t(const StepArgs& a, hipStream_t st) {
    hipLaunchKernelGGL((step_kernel<TYT, R>), dim3(a.total_blocks), dim3(64 * TYT), 0, st, a);
    return hipGetLastError();
}

// Table of step-kernel tile shapes: threads 64 x TYT, each thread R rows.
const TileShape TILE_SHAPES[] = {
    {4, 1}, {4, 2}, {4, 4}, {2, 4}, {8, 1}, {8, 2}, {16, 1}, {1, 8},
};
const int N_TILE_SHAPES = (int)(sizeof(TILE_SHAPES) / sizeof(TILE_SHAPES[0]));

hipError_t launch_step(int tile_id, const StepArgs& a, hipStream_t st) {
    switch (tile_id) {
        case 0: return launch_step_t<4, 1>(a, st);
        case 1: return launch_step_t<4, 2>(a, st);
        case 2: return launch_step_t<4, 4>(a, st);
        case 3: return launch_step_t<2, 4>(a, st);
        case 4: return launch_step_t<8, 1>(a, st);
        case 5: return launch_step_t<8, 2>(a, st);
        case 6: return launch_step_t<16, 1>(a, st);
        case 7: return launch_step_t<1, 8>(a, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(const InitArgs& a, int n_members, long long max_cells, hipStream_t st) {
    const unsigned gx = (unsigned)((max_cells + 255) / 256);
    hipLaunchKernelGGL(init_kernel, dim3(gx, n_members), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs& a, int n_members, hipStream_t st) {
    hipLaunchKernelGGL(finalize_kernel, dim3(n_members), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace lbm
