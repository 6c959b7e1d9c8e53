// Lattice-Boltzmann kernels: initial state, fused pull-stream + BGK collide
// step with momentum-exchange drag partials, and the per-chunk drag
// reduction with the FP64 observable integral.
//
// Paper Appendix A gives the scheme (exact streaming, BGK relaxation to the
// second-order equilibrium); Section 2 the halfway bounce-back on walls and
// obstacle; Section 2.1 the drag.  Populations are FP32 deviations
// d_i = f_i - w_i so that the O(1) rest weights never enter FP32 sums.
#include "lbm_device.hpp"

namespace lbm {

// One fluid-or-solid cell, one population per lane access: used for lattices
// whose width is not a multiple of 4.  OPEN: x is not periodic; populations
// entering at x = 0 come from the inlet ghost column, those entering at
// x = nx - 1 from the outlet ghost column (ghost: the member's [9][ny] block,
// +x movers from the inlet, -x movers from the outlet).
template <int MODEL, bool OPEN>
__device__ __forceinline__ void scalar_cell(const MemberDev& m, const float* __restrict__ src, float* __restrict__ dst,
                                            double* __restrict__ part, const float* __restrict__ ghost, int x, int y) {
    const int nx = m.nx, ny = m.ny;
    const long long plane = (long long)nx * ny;
    if (solid_at<OPEN>(m, x, y)) return;
    float dl[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int xs = x - CX[i];
        if (!OPEN) xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
        const int ys = y - CY[i];
        const bool wall = (ys < 0) | (ys >= ny);
        const bool inside = (unsigned)xs < (unsigned)nx;
        const bool bounce = wall || (inside && solid_at<OPEN>(m, xs, ys));
        if (bounce)
            dl[i] = src[(long long)OPP[i] * plane + (long long)y * nx + x];
        else if (OPEN && (xs < 0 || xs >= nx))
            dl[i] = ghost[(long long)i * ny + ys];
        else
            dl[i] = src[(long long)i * plane + (long long)ys * nx + xs];
    }
    const int ri = ring_index(m, x, y);
    const unsigned links = ri >= 0 ? square_links(m, x, y) : 0u;
    double drag;
    if (OPEN) {
        MemberDev mc = m;
        sponge_at(mc, x);
        drag = collide_cell<MODEL>(mc, dl, links);
    } else {
        drag = collide_cell<MODEL>(m, dl, links);
    }
    const long long cell = (long long)y * nx + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) dst[(long long)i * plane + cell] = dl[i];
    if (ri >= 0) part[ri] = drag;
}

// One row segment of up to 256 cells per wave, four consecutive cells per
// lane, 16-byte loads and stores.  A population moving along +x (c_x = 1) is
// pulled from x - 1: the lane's aligned float4 supplies three of its four
// cells and the fourth comes from the neighbouring lane through a wave
// shift; the first lane of the wave takes it from one wave-uniform load,
// which also carries the periodic wrap at x = 0 (OPEN: the inlet ghost
// column).  Likewise for c_x = -1 at the right end (OPEN: the outlet ghost
// column).
// Rows next to a wall are wave-uniform (the whole row bounces back); only
// waves touching a solid cell decide per cell.  OPEN also sets the
// relaxation rates per cell (sponge zone).
template <int MODEL, bool OPEN>
__device__ __forceinline__ void vec_row(const MemberDev& m, const float* __restrict__ src, float* __restrict__ dst,
                                        double* __restrict__ part, const float* __restrict__ ghost, int base, int y,
                                        int lane) {
    const int nx = m.nx, ny = m.ny;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const int nvalid = min(256, nx - base);  // a multiple of 4
    const int last = nvalid / 4 - 1;         // last lane holding cells
    const bool live = lane <= last;
    const int x0 = base + 4 * min(lane, last);
    const unsigned voff = 4u * (unsigned)x0;  // per-lane byte offset within a row
    const unsigned rowoff = (unsigned)y * (unsigned)nx;
    const bool left_end = base == 0, right_end = base + nvalid == nx;
    const int xl = (left_end ? nx : base) - 1;
    const int xr = right_end ? 0 : base + nvalid;
    const bool near_sq = m.ss > 0 && y >= m.sy0 - 1 && y <= m.sy0 + m.ss && base <= m.sx0 + m.ss &&
                         base + nvalid - 1 >= m.sx0 - 1;
    // which of the rows y - 1, y, y + 1 cross the grid's bars (wave-uniform)
    bool grow[3] = {false, false, false};
    if (OPEN) {
#pragma unroll
        for (int j = 0; j < 3; ++j) grow[j] = y - 1 + j >= 0 && y - 1 + j < ny && grid_row(m, y - 1 + j);
    }
    const bool near_grid = OPEN && (grow[0] || grow[1] || grow[2]) && base <= m.gx0 + m.bar &&
                           base + nvalid - 1 >= m.gx0 - 1;
    const bool near = near_sq || near_grid;
    // bit j: column x0 - 1 + j (j = 0..5, the lane's cells and their neighbours) holds grid bars
    unsigned gcols = 0;
    if (near_grid)
#pragma unroll
        for (int j = 0; j < 6; ++j) gcols |= ((unsigned)(x0 - 1 + j - m.gx0) < (unsigned)m.bar ? 1u : 0u) << j;
    // solid test of column x0 + dx (dx = -1 .. 4) in row y - 1 + j
    auto solid = [&](int dx, int j) {
        return (near_sq && in_square(m, x0 + dx, y - 1 + j)) || (OPEN && grow[j] && ((gcols >> (dx + 1)) & 1u));
    };
    // open channel: the columns of this segment reach the sponge zone (wave-uniform)
    const bool sponge_wave = OPEN && base + nvalid - 1 > m.sp_x0;
    // buffer resources over the member's whole block (range-checked by the hardware);
    // row offsets are wave-uniform (scalar), the lane offset is the only vector operand
    const unsigned bytes = 36u * plane;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)src, (short)0, (int)bytes, BUFFER_RSRC_WORD3);
    const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc((void*)dst, (short)0, (int)bytes, BUFFER_RSRC_WORD3);
    // load phase: nine 16-byte non-temporal loads and the edge elements, no
    // branches in between (row choice by wave-uniform selects), so all are in
    // flight at once
    f4 v[9];
    float e[9];
    bool wall[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ys = y - CY[i];
        wall[i] = ys < 0 || ys >= ny;  // the whole row takes its own opposite population
        const unsigned row = wall[i] ? (unsigned)OPP[i] * plane + rowoff : (unsigned)i * plane + (unsigned)ys * (unsigned)nx;
        v[i] = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, 4u * row, BUFFER_NT);
        // the edge element goes through the vector memory pipe like the rest
        // (every lane asks for the same word)
        if (CX[i] == 1) {
            if (OPEN && left_end) e[i] = ghost[(unsigned)i * (unsigned)ny + (unsigned)(wall[i] ? y : ys)];
            else e[i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, 4u * (unsigned)xl, 4u * row, 0));
        } else if (CX[i] == -1) {
            if (OPEN && right_end) e[i] = ghost[(unsigned)i * (unsigned)ny + (unsigned)(wall[i] ? y : ys)];
            else e[i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, 4u * (unsigned)xr, 4u * row, 0));
        } else {
            e[i] = 0.0f;
        }
    }
    // shift phase: +x movers take x - 1 from the left neighbour lane, -x movers x + 1 from the right
    f4 p[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (CX[i] == 1) {
            const float sh = wave_shr1(v[i].w);
            const f4 s4 = f4{lane == 0 ? e[i] : sh, v[i].x, v[i].y, v[i].z};
            p[i] = wall[i] ? v[i] : s4;
        } else if (CX[i] == -1) {
            const float sh = wave_shl1(v[i].x);
            const f4 s4 = f4{v[i].y, v[i].z, v[i].w, lane == last ? e[i] : sh};
            p[i] = wall[i] ? v[i] : s4;
        } else {
            p[i] = v[i];
        }
    }
    if (near) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (solid(k, 1)) continue;  // a solid cell's results are never stored
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const int ys = y - CY[i];
                if (ys < 0 || ys >= ny) continue;
                if (solid(k - CX[i], 1 - CY[i])) p[i][k] = src[(unsigned)OPP[i] * plane + rowoff + (unsigned)(x0 + k)];
            }
        }
    }
    // collide the four cells one after the other, in place
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
        float dl[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) dl[i] = p[i][k];
        const int ri = (near_sq && live && !in_square(m, x0 + k, y)) ? ring_index(m, x0 + k, y) : -1;
        const unsigned links = ri >= 0 ? square_links(m, x0 + k, y) : 0u;
        double drag;
        if (OPEN) {
            MemberDev mc = m;
            if (sponge_wave) sponge_at(mc, x0 + k);
            drag = collide_cell<MODEL>(mc, dl, links);
        } else {
            drag = collide_cell<MODEL>(m, dl, links);
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) p[i][k] = dl[i];
        if (ri >= 0) part[ri] = drag;
    }
    if (!live) return;
    // lanes whose four cells are all fluid store 16 bytes at a time, lanes
    // with only solid cells store nothing, and the rare mixed ones store cell
    // by cell, leaving the solid cells untouched
    unsigned smask = 0;  // bit k: cell x0 + k is solid
    if (near)
#pragma unroll
        for (int k = 0; k < 4; ++k) smask |= (solid(k, 1) ? 1u : 0u) << k;
    if (smask == 0) {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            __builtin_amdgcn_raw_buffer_store_b128(p[i], rd, voff, 4u * ((unsigned)i * plane + rowoff), BUFFER_NT);
    } else if (smask != 0xFu) {
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
            if (solid(k, 1)) continue;
#pragma unroll
            for (int i = 0; i < 9; ++i) dst[(unsigned)i * plane + rowoff + (unsigned)(x0 + k)] = p[i][k];
        }
    }
}

// Fused pull-stream + collide step over the whole ensemble.  Workgroup =
// TYT waves; a tile is 256 columns by TYT*R rows; wave w handles rows
// w, w + TYT, ... of the tile.
// One-row shapes are held to 96 VGPRs (5 waves per SIMD): the memory-bound
// step needs the waves in flight more than the registers.  OPEN: the
// open-channel instantiation (inlet, grid, sponge, outlet ghost column).
template <int TYT, int R, int MODEL, bool OPEN>
__global__ __launch_bounds__(64 * TYT) __attribute__((amdgpu_waves_per_eu(R == 1 && MODEL == 0 && !OPEN ? 5 : 4))) void step_kernel(StepArgs a) {
    const int b = a.xcd ? xcd_remap((int)blockIdx.x, a.total_blocks) : (int)blockIdx.x;
    int tx, ty, vec, seg_rows;
    const int mi = block_to_member(a, b, tx, ty, vec, seg_rows);
    // the three bookkeeping reads are independent: issue them together
    const int on = a.active[mi];
    const MemberDev m = a.members[mi];
    const int par = a.parity[mi] ^ a.flip;
    if (!on) return;
    const float* __restrict__ src = (par ? a.pop1 : a.pop0) + m.off;
    float* __restrict__ dst = (par ? a.pop0 : a.pop1) + m.off;
    double* __restrict__ part = a.partial + m.part_off + (long long)a.slot * m.ring;
    const float* __restrict__ ghost = OPEN ? a.ghost + m.ghost_off : nullptr;
    const int lane = (int)(threadIdx.x & 63);
    // the wave index is uniform across the wave: say so, so that all row logic stays scalar
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int base = tx * 256;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = ty * (TYT * R) + r * TYT + wv;
        if (y >= m.ny) break;
        if (vec) {
            vec_row<MODEL, OPEN>(m, src, dst, part, ghost, base, y, lane);
        } else {
#pragma unroll 1
            for (int k = 0; k < 4; ++k) {
                const int x = base + 64 * k + lane;
                if (x < m.nx) scalar_cell<MODEL, OPEN>(m, src, dst, part, ghost, x, y);
            }
        }
    }
}

// Open channel boundaries (paper Section 2), rebuilt before every step into
// the member's [9][ny] ghost block: the +x movers (i = 1, 5, 8) of the inlet
// column x = -1, which the cells of column 0 pull, and the -x movers
// (i = 3, 6, 7) of the outlet column x = nx, which the cells of column nx - 1
// pull.  The inlet is the equilibrium of the parabolic profile (inlet_dev);
// the outlet is outlet_ghost_value of the post-collision state about to be
// streamed.
// One workgroup per member: each thread takes rows t, t + 256, ... and puts
// the velocities of the last two columns into LDS ([4][ny] doubles); after a
// barrier every thread rebuilds the ghost populations of its rows from its
// own and its neighbours' entries.
__global__ __launch_bounds__(256) void outlet_ghost_kernel(GhostArgs a) {
    const int mi = (int)blockIdx.x;
    const MemberDev m = a.members[mi];
    if (!m.open || !a.active[mi]) return;  // the whole workgroup
    extern __shared__ OutletVel vel[];      // [ny]
    const int par = a.parity[mi] ^ a.flip;
    const float* __restrict__ src = (par ? a.pop1 : a.pop0) + m.off;
    const int nx = m.nx, ny = m.ny;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    for (int y = (int)threadIdx.x; y < ny; y += 256) {
        float d1[9], d2[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const unsigned row = (unsigned)i * plane + (unsigned)y * (unsigned)nx;
            d1[i] = src[row + (unsigned)(nx - 1)];
            d2[i] = src[row + (unsigned)(nx - 2)];
        }
        OutletVel v;
        stored_velocity(d1, v.ux1, v.uy1);
        stored_velocity(d2, v.ux2, v.uy2);
        vel[y] = v;
    }
    __syncthreads();
    float* __restrict__ g = a.ghost + m.ghost_off;
    for (int y = (int)threadIdx.x; y < ny; y += 256) {
        const OutletVel va = vel[y > 0 ? y - 1 : 0], v0 = vel[y], vb = vel[y + 1 < ny ? y + 1 : ny - 1];
        double rho_g = 1.0;
        if (m.out_rho) {  // the row's two cells again (the LDS table keeps velocities only)
            float d1[9], d2[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const unsigned row = (unsigned)i * plane + (unsigned)y * (unsigned)nx;
                d1[i] = src[row + (unsigned)(nx - 1)];
                d2[i] = src[row + (unsigned)(nx - 2)];
            }
            rho_g = outlet_density(m, d1, d2);
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            if (CX[i] == 1) g[i * ny + y] = inlet_dev(m, i, y);
            else if (CX[i] == -1) g[i * ny + y] = outlet_ghost_value(m, CX[i], CY[i], WD[i], y, va, v0, vb, rho_g);
        }
    }
}

// Step 0: equilibrium with the seeded density and a uniform velocity
// (u_x0, 0) (at rest for u_x0 = 0; an open channel's inlet profile
// (u_in(y), 0) instead), relaxed once.
__global__ __launch_bounds__(256) void init_kernel(InitArgs a) {
    const int mi = (int)blockIdx.y;
    const MemberDev m = a.members[mi];
    const long long plane = (long long)m.nx * m.ny;
    const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
    if (cell >= plane) return;
    const int y = (int)(cell / m.nx), x = (int)(cell - (long long)y * m.nx);
    if (in_solid(m, x, y)) return;
    double drho = 0.0;
    if (a.noise_amp != 0.0) {
        const U64x4 w = philox4x64_10((uint64_t)cell, (uint64_t)mi, 0, 0, a.seed, PURPOSE_INIT);
        drho = a.noise_amp * (2.0 * uniform53(w.v[0]) - 1.0);
    }
    // f_i = f_i^eq(rho, u0) - w_i = w_i [drho + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u^2)]
    double u0 = a.ux0;
    if (m.open) {
        const double yc = (double)y + 0.5;
        u0 = 4.0 * m.u_c * yc * ((double)m.ny - yc) / ((double)m.ny * (double)m.ny);
    }
    const double rho = 1.0 + drho;
    float d[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double cu = (double)CX[i] * u0;
        d[i] = (float)(WD[i] * (drho + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * u0 * u0)));
    }
    const int ri = ring_index(m, x, y);
    MemberDev mc = m;
    if (m.open) sponge_at(mc, x);
    const double drag = collide_member(mc, d, ri >= 0 ? square_links(m, x, y) : 0u);
    float* dst = a.pop0 + m.off;  // step 0 lives in buffer 0 (parity 0)
#pragma unroll
    for (int i = 0; i < 9; ++i) dst[(long long)i * plane + cell] = d[i];
    if (ri >= 0) a.partial[m.part_off + ri] = drag;
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
        a.parity[mi] ^= a.swap_parity;
        a.cursor[mi] = cur + a.n;
    }
}

// ---------------------------------------------------------------------------
// launchers

template <int TYT, int R>
static hipError_t launch_step_t(const StepArgs& a, int model, hipStream_t st) {
    const dim3 grid(a.total_blocks), block(64 * TYT);
    if (a.ghost) {
        if (model == 2) hipLaunchKernelGGL((step_kernel<TYT, R, 2, true>), grid, block, 0, st, a);
        else if (model == 1) hipLaunchKernelGGL((step_kernel<TYT, R, 1, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((step_kernel<TYT, R, 0, true>), grid, block, 0, st, a);
    } else {
        if (model == 2) hipLaunchKernelGGL((step_kernel<TYT, R, 2, false>), grid, block, 0, st, a);
        else if (model == 1) hipLaunchKernelGGL((step_kernel<TYT, R, 1, false>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((step_kernel<TYT, R, 0, false>), grid, block, 0, st, a);
    }
    return hipGetLastError();
}

// Table of step-kernel launch shapes: TYT waves per workgroup, R rows per
// wave, whether workgroups are remapped so each XCD gets contiguous tiles,
// and steps per launch.  Ids 0-15 are one-step shapes (launch_step switches
// on id % 8); ids 16-19 are the two-step kernel with TYT rows per iteration;
// id 20 is shape 16 while the active members fill the device, shape 0 otherwise.
const TileShape TILE_SHAPES[] = {
    {4, 1, 1, 1, 0}, {4, 2, 1, 1, 0}, {8, 1, 1, 1, 0}, {2, 2, 1, 1, 0},
    {16, 1, 1, 1, 0}, {1, 4, 1, 1, 0}, {4, 4, 1, 1, 0}, {8, 2, 1, 1, 0},
    {4, 1, 0, 1, 0}, {4, 2, 0, 1, 0}, {8, 1, 0, 1, 0}, {2, 2, 0, 1, 0},
    {16, 1, 0, 1, 0}, {1, 4, 0, 1, 0}, {4, 4, 0, 1, 0}, {8, 2, 0, 1, 0},
    {4, 1, 1, 2, 0}, {2, 1, 1, 2, 0}, {8, 1, 1, 2, 0}, {4, 1, 0, 2, 0},
    {4, 1, 1, 2, 1, -1}, {4, 1, 1, 2, 0, 128}, {4, 1, 1, 2, 0, 64}, {4, 1, 1, 2, 0, 32},
};
const int N_TILE_SHAPES = (int)(sizeof(TILE_SHAPES) / sizeof(TILE_SHAPES[0]));

hipError_t launch_step(int tile_id, const StepArgs& a, int model, hipStream_t st) {
    switch (tile_id % 8) {
        case 0: return launch_step_t<4, 1>(a, model, st);
        case 1: return launch_step_t<4, 2>(a, model, st);
        case 2: return launch_step_t<8, 1>(a, model, st);
        case 3: return launch_step_t<2, 2>(a, model, st);
        case 4: return launch_step_t<16, 1>(a, model, st);
        case 5: return launch_step_t<1, 4>(a, model, st);
        case 6: return launch_step_t<4, 4>(a, model, st);
        case 7: return launch_step_t<8, 2>(a, model, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_outlet_ghost(const GhostArgs& a, int n_members, int max_ny, hipStream_t st) {
    hipLaunchKernelGGL(outlet_ghost_kernel, dim3(n_members), dim3(256), sizeof(double) * 4 * max_ny, st, a);
    return hipGetLastError();
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
