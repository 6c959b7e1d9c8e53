// Two lattice steps per pass over the populations (temporal blocking of the
// fused pull-stream + BGK collide step of paper Appendix A).
//
// A workgroup of NW waves owns a strip of 256 columns of one member and
// sweeps it from the bottom row to the top, NW rows per iteration:
//
//   phase A  each wave pulls one row of the state at t from HBM and collides
//            it (step t+1) exactly as the one-step kernel does, and keeps the
//            result in an LDS ring of NW + 2 rows.  The two cells just outside
//            the strip (x0 - 1 and x0 + 256, periodic) are collided too, so
//            that phase B never needs a neighbouring strip;
//   phase B  each wave pulls the row below its phase-A row from the ring,
//            collides it (step t+2) and writes it to the other buffer.
//
// Every population is read from HBM once and written once per two steps
// (plus 2 x 9 words per row for the outside cells).  The arithmetic of every
// cell is the one-step kernel's, on the same FP32 inputs, so both paths give
// bit-identical states and drag.  The next iteration's row loads are issued
// before the current row is collided and stay in flight across the
// workgroup barriers, which wait for LDS traffic only.
#include "lbm_device.hpp"

namespace lbm {

// One direction row of the ring: [3] = cell x0 - 1, [4 .. 259] = cells
// x0 .. x0 + 255 (16-byte aligned), [260] = cell x0 + 256.
constexpr int RING_ROW = 264;
constexpr int RING_CELL0 = 4;
constexpr int RING_LEFT = 3;
constexpr int RING_RIGHT = 260;

struct RowLoads {
    f4 v[9];     // the lane's four cells of the pulled row of each direction
    float e[9];  // the word beyond the strip's edge for the +x / -x movers
};

__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Row loads of row y from the state at t: direction i comes from row y - c_iy
// (or, next to a wall, from the row's own opposite population).  The loads go
// through L2 (not non-temporal): the neighbouring strip, on the same XCD and
// near the same row, reads the words just outside this strip, and finds them
// there (measured: 7 % instead of 12 % extra HBM fetch, 1.6 % faster).
__device__ __forceinline__ void load_row(const MemberDev& m, __amdgpu_buffer_rsrc_t rs, unsigned voff, int xl, int xr,
                                         int y, RowLoads& L) {
    const unsigned plane = (unsigned)m.nx * (unsigned)m.ny;
    const unsigned rowoff = (unsigned)y * (unsigned)m.nx;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ys = y - CY[i];
        const bool wall = ys < 0 || ys >= m.ny;
        const unsigned row = wall ? (unsigned)OPP[i] * plane + rowoff : (unsigned)i * plane + (unsigned)ys * (unsigned)m.nx;
        L.v[i] = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, 4u * row, 0);
        L.e[i] = CX[i] == 1 ? __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, 4u * (unsigned)xl, 4u * row, 0))
                            : (CX[i] == -1 ? __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, 4u * (unsigned)xr, 4u * row, 0))
                                           : 0.0f);
    }
}

// Collide the lane's four cells of row y in place; ring cells leave their
// drag partial in part.
template <int MODEL>
__device__ __forceinline__ void collide_row(const MemberDev& m, f4 p[9], double* __restrict__ part, bool near_sq, int x0,
                                            int y) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float dl[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) dl[i] = p[i][k];
        const int ri = (near_sq && !in_square(m, x0 + k, y)) ? ring_index(m, x0 + k, y) : -1;
        const double drag = collide_cell<MODEL>(m, dl, ri >= 0 ? square_links(m, x0 + k, y) : 0u);
#pragma unroll
        for (int i = 0; i < 9; ++i) p[i][k] = dl[i];
        if (ri >= 0) part[ri] = drag;
    }
}

template <int NW, int MODEL>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2))) void step2_kernel(StepArgs a) {
    __shared__ f4 ring4[(NW + 2) * 9 * RING_ROW / 4];
    float* const ring = (float*)ring4;
    const int b = a.xcd ? xcd_remap((int)blockIdx.x, a.total_blocks) : (int)blockIdx.x;
    int tx, ty, vec;
    const int mi = block_to_member(a, b, tx, ty, vec);
    const int on = a.active[mi];
    const MemberDev m = a.members[mi];
    const int par = a.parity[mi] ^ a.flip;
    if (!on) return;  // the whole workgroup: no barrier is left waiting
    const float* __restrict__ src = (par ? a.pop1 : a.pop0) + m.off;
    float* __restrict__ dst = (par ? a.pop0 : a.pop1) + m.off;
    double* __restrict__ part0 = a.partial + m.part_off + (long long)a.slot * m.ring;  // step t+1
    double* __restrict__ part1 = part0 + m.ring;                                         // step t+2
    const int lane = (int)(threadIdx.x & 63);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nx = m.nx, ny = m.ny;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const unsigned bytes = 36u * plane;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)src, (short)0, (int)bytes, BUFFER_RSRC_WORD3);
    const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc((void*)dst, (short)0, (int)bytes, BUFFER_RSRC_WORD3);
    const int base = tx * 256;
    const int x0 = base + 4 * lane;
    const unsigned voff = 4u * (unsigned)x0;
    const int xl = (base == 0 ? nx : base) - 1;      // the cell left of the strip (periodic)
    const int xr = (base + 256 == nx) ? 0 : base + 256;  // the cell right of it
    const int xh = (lane & 1) ? xr : xl;             // lanes 0 / 1 collide the left / right outside cell
    const bool sq_cols = m.ss > 0 && base <= m.sx0 + m.ss && base + 255 >= m.sx0 - 1;
    const int iters = ny / NW + 1;                   // phase B of the last iteration reaches row ny - 1
    RowLoads cur;
    if (wv < ny) load_row(m, rs, voff, xl, xr, wv, cur);
#pragma unroll 1
    for (int j = 0; j < iters; ++j) {
        const int y = j * NW + wv;
        // phase A: row y at step t+1 into the ring.  Every gather this row
        // needs (the outside cell, the obstacle's bounce-back words) is
        // issued before the prefetch of the wave's next row: waits on memory
        // complete in issue order, so waiting for them leaves the prefetch in
        // flight.
        const bool row_a = y < ny;
        const bool near_sq = row_a && sq_cols && y >= m.sy0 - 1 && y <= m.sy0 + m.ss;
        float hv[9];
        f4 p[9];
        if (row_a) {
            load_cell<false>(m, src, xh, y, hv);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int ys = y - CY[i];
                const bool wall = ys < 0 || ys >= ny;
                const f4 v = cur.v[i];
                if (CX[i] == 1) {
                    const float sh = wave_shr1(v.w);
                    const f4 s4 = f4{lane == 0 ? cur.e[i] : sh, v.x, v.y, v.z};
                    p[i] = wall ? v : s4;
                } else if (CX[i] == -1) {
                    const float sh = wave_shl1(v.x);
                    const f4 s4 = f4{v.y, v.z, v.w, lane == 63 ? cur.e[i] : sh};
                    p[i] = wall ? v : s4;
                } else {
                    p[i] = v;
                }
            }
            if (near_sq) {
                const unsigned rowoff = (unsigned)y * (unsigned)nx;
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    const int ys = y - CY[i];
                    if (ys < 0 || ys >= ny) continue;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (in_square(m, x0 + k - CX[i], ys)) p[i][k] = src[(unsigned)OPP[i] * plane + rowoff + (unsigned)(x0 + k)];
                }
            }
        }
        RowLoads nxt;
        if (y + NW < ny) load_row(m, rs, voff, xl, xr, y + NW, nxt);
        if (row_a) {
            float* row = ring + (y % (NW + 2)) * 9 * RING_ROW;
            collide_row<MODEL>(m, p, part0, near_sq, x0, y);
#pragma unroll
            for (int i = 0; i < 9; ++i) *(f4*)(row + i * RING_ROW + RING_CELL0 + 4 * lane) = p[i];
            // the outside cells (their drag belongs to the neighbouring strip)
            collide_cell<MODEL>(m, hv, 0u);
            if (lane < 2 && !in_square(m, xh, y)) {
                const int at = lane ? RING_RIGHT : RING_LEFT;
#pragma unroll
                for (int i = 0; i < 9; ++i) row[i * RING_ROW + at] = hv[i];
            }
        }
        lds_barrier();
        // phase B: row y - 1 at step t+2 from the ring to the other buffer
        const int r = y - 1;
        if (r >= 0 && r < ny) {
            const float* own = ring + (r % (NW + 2)) * 9 * RING_ROW;
            const bool near_sq = sq_cols && r >= m.sy0 - 1 && r <= m.sy0 + m.ss;
            f4 p[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int rsrc = r - CY[i];
                if (rsrc < 0 || rsrc >= ny) {  // wall row: the cell's own opposite population
                    p[i] = *(const f4*)(own + OPP[i] * RING_ROW + RING_CELL0 + 4 * lane);
                    continue;
                }
                const float* srow = ring + (rsrc % (NW + 2)) * 9 * RING_ROW + i * RING_ROW;
                const f4 v = *(const f4*)(srow + RING_CELL0 + 4 * lane);
                if (CX[i] == 1) {
                    const float h = srow[RING_LEFT];
                    const float sh = wave_shr1(v.w);
                    p[i] = f4{lane == 0 ? h : sh, v.x, v.y, v.z};
                } else if (CX[i] == -1) {
                    const float h = srow[RING_RIGHT];
                    const float sh = wave_shl1(v.x);
                    p[i] = f4{v.y, v.z, v.w, lane == 63 ? h : sh};
                } else {
                    p[i] = v;
                }
            }
            if (near_sq) {
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    const int rsrc = r - CY[i];
                    if (rsrc < 0 || rsrc >= ny) continue;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (in_square(m, x0 + k - CX[i], rsrc)) p[i][k] = own[OPP[i] * RING_ROW + RING_CELL0 + 4 * lane + k];
                }
            }
            collide_row<MODEL>(m, p, part1, near_sq, x0, r);
            const unsigned rowoff = (unsigned)r * (unsigned)nx;
            if (!near_sq) {
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    __builtin_amdgcn_raw_buffer_store_b128(p[i], rd, voff, 4u * ((unsigned)i * plane + rowoff), BUFFER_NT);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (in_square(m, x0 + k, r)) continue;
#pragma unroll
                    for (int i = 0; i < 9; ++i) dst[(unsigned)i * plane + rowoff + (unsigned)(x0 + k)] = p[i][k];
                }
            }
        }
        lds_barrier();
        cur = nxt;
    }
}

template <int NW>
static hipError_t launch_step2_t(const StepArgs& a, int model, hipStream_t st) {
    if (model == 1)
        hipLaunchKernelGGL((step2_kernel<NW, 1>), dim3(a.total_blocks), dim3(64 * NW), 0, st, a);
    else
        hipLaunchKernelGGL((step2_kernel<NW, 0>), dim3(a.total_blocks), dim3(64 * NW), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_step2(int waves, const StepArgs& a, int model, hipStream_t st) {
    switch (waves) {
        case 2: return launch_step2_t<2>(a, model, st);
        case 4: return launch_step2_t<4>(a, model, st);
        case 8: return launch_step2_t<8>(a, model, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm
