// Two lattice steps per pass over the populations (temporal blocking of the
// fused pull-stream + BGK collide step of paper Appendix A).
//
// A workgroup of NW waves owns a strip of 256 columns of one member and
// sweeps it from the bottom row to the top, NW rows per iteration:
//
//   phase A  each wave pulls one row of the state at t from HBM and collides
//            it (step t+1) exactly as the one-step kernel does, and keeps the
//            result in an LDS ring of NW + 2 rows (NW + 3 for open channels).
//            The two cells just outside the strip (x0 - 1 and x0 + 256,
//            periodic) are collided too, so that phase B never needs a
//            neighbouring strip;
//   phase B  each wave pulls the row below its phase-A row (two rows below
//            for open channels) from the ring, collides it (step t+2) and
//            writes it to the other buffer.
//
// Every population is read from HBM once and written once per two steps
// (plus 2 x 9 words per row for the outside cells).  The arithmetic of every
// cell is the one-step kernel's, on the same FP32 inputs, so both paths give
// bit-identical states and drag.  The next iteration's row loads are issued
// before the current row is collided and stay in flight across the
// workgroup barriers, which wait for LDS traffic only.
//
// Open channels (OPEN): the strip at x = 0 takes the inlet's values from the
// ghost block for both steps (they are constant); the strip at the outlet
// takes the ghost column of step t+1 from the ghost block (built from the
// state at t by the ghost kernel) and builds that of step t+2 itself: phase A
// keeps the velocities of the last two columns of every row in a small LDS
// ring, and phase B trails phase A by two rows, so that the rows a ghost
// value needs (its own and the two neighbours of each of the three rows a
// cell pulls from) are collided before it is used.  Grid bars are solid like
// the square; sponge rates are set per cell.
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
// OPEN: at the channel's ends the edge words come from the ghost block (rg,
// [9][ny] floats: the strip at x = 0 (left_end) and the one ending at x = nx
// (right_end)).  Every edge word is one vector load, from the state or from
// the ghost block by a uniform choice of resource and offset: a scalar load
// there, or a load whose register another kind of load also writes, makes
// the compiler wait for every load in flight (the next row's prefetch
// included).
template <bool OPEN>
__device__ __forceinline__ void load_row(const MemberDev& m, __amdgpu_buffer_rsrc_t rs, __amdgpu_buffer_rsrc_t rg,
                                         unsigned voff, int xl, int xr, int y, RowLoads& L, bool left_end,
                                         bool right_end) {
    const unsigned plane = (unsigned)m.nx * (unsigned)m.ny;
    const unsigned rowoff = (unsigned)y * (unsigned)m.nx;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ys = y - CY[i];
        const bool wall = ys < 0 || ys >= m.ny;
        const unsigned row = wall ? (unsigned)OPP[i] * plane + rowoff : (unsigned)i * plane + (unsigned)ys * (unsigned)m.nx;
        L.v[i] = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, 4u * row, 0);
        if constexpr (OPEN) {
            const unsigned gi = (unsigned)i * (unsigned)m.ny + (unsigned)(wall ? y : ys);
            if (CX[i] != 0) {
                const bool from_ghost = CX[i] == 1 ? left_end : right_end;
                const unsigned xe = CX[i] == 1 ? (unsigned)xl : (unsigned)xr;
                L.e[i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                    from_ghost ? rg : rs, from_ghost ? 0u : 4u * xe, from_ghost ? 4u * gi : 4u * row, 0));
            } else {
                L.e[i] = 0.0f;
            }
        } else {
            if (CX[i] == 1)
                L.e[i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, 4u * (unsigned)xl, 4u * row, 0));
            else if (CX[i] == -1)
                L.e[i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, 4u * (unsigned)xr, 4u * row, 0));
            else
                L.e[i] = 0.0f;
        }
    }
}

// Collide the lane's four cells of row y in place; ring cells leave their
// drag partial in part.  sponge: the strip reaches an open channel's sponge
// zone (rates per cell).
template <int MODEL, bool OPEN>
__device__ __forceinline__ void collide_row(const MemberDev& m, f4 p[9], double* __restrict__ part, bool near_sq, int x0,
                                            int y, bool sponge) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float dl[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) dl[i] = p[i][k];
        const int ri = (near_sq && !in_square(m, x0 + k, y)) ? ring_index(m, x0 + k, y) : -1;
        const unsigned links = ri >= 0 ? square_links(m, x0 + k, y) : 0u;
        double drag;
        if (OPEN) {
            MemberDev mc = m;
            if (sponge) sponge_at(mc, x0 + k);
            drag = collide_cell<MODEL>(mc, dl, links);
        } else {
            drag = collide_cell<MODEL>(m, dl, links);
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) p[i][k] = dl[i];
        if (ri >= 0) part[ri] = drag;
    }
}

// Halfway bounce-back of the lane's four cells of row y from the solid mask
// mk of its rows (bit 6 j + dx + 1: column x0 + dx of row y - 1 + j): p[i][k]
// becomes own[i][k] (the cell's own opposite population) where the cell x0 + k
// is fluid and the cell it pulls from, x0 + k - c_ix in row y - c_iy, is
// solid.  For each direction the four cells' tests are one 4-bit field of mk;
// each choice is a sign-extended bit and a bitwise select, with no branch.
__device__ __forceinline__ void bounce_select(unsigned mk, int ny, int y, const f4 own[9], f4 p[9]) {
    const unsigned fluid = ~(mk >> 7) & 0xFu;  // row y, columns x0 .. x0 + 3
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int ys = y - CY[i];
        if (ys < 0 || ys >= ny) continue;  // a wall row: the whole row bounces back already
        const unsigned m = (mk >> (6 * (1 - CY[i]) + 1 - CX[i])) & fluid;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned sel = (unsigned)((int)(m << (31 - k)) >> 31);  // all ones where bit k is set
            p[i][k] = __uint_as_float((__float_as_uint(own[i][k]) & sel) | (__float_as_uint(p[i][k]) & ~sel));
        }
    }
}

// Velocity ring of the outlet strip: rows y & (VROWS - 1).  Phase B reads
// rows r - 2 .. r + 2 while phase A writes up to r + 2 + NW - 1, so 16 rows
// hold every row still needed for NW <= 8.
constexpr int VROWS = 16;

template <int NW, int MODEL, bool OPEN, bool SPLIT>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2))) void step2_kernel(StepArgs a) {
    constexpr int LAG = OPEN ? 2 : 1;          // phase B works on row y - LAG
    constexpr int RROWS = NW + 1 + LAG;        // ring rows: y - LAG - 1 .. y for the whole workgroup
    __shared__ f4 ring4[RROWS * 9 * RING_ROW / 4];
    __shared__ OutletVel vring[OPEN ? VROWS : 1];
    __shared__ double rring[OPEN ? VROWS : 1];  // the rows' outlet densities (1 when held)
    float* const ring = (float*)ring4;
    const int b = a.xcd ? xcd_remap((int)blockIdx.x, a.total_blocks) : (int)blockIdx.x;
    int tx, ty, vec, seg_rows;
    const int mi = block_to_member(a, b, tx, ty, vec, seg_rows);
    const int on = a.active[mi];
    const MemberDev m = a.members[mi];
    const int par = a.parity[mi] ^ a.flip;
    if (!on) return;  // the whole workgroup: no barrier is left waiting
    const float* __restrict__ src = (par ? a.pop1 : a.pop0) + m.off;
    float* __restrict__ dst = (par ? a.pop0 : a.pop1) + m.off;
    double* __restrict__ part0 = a.partial + m.part_off + (long long)a.slot * m.ring;  // step t+1
    double* __restrict__ part1 = part0 + m.ring;                                         // step t+2
    const float* __restrict__ ghost = OPEN ? a.ghost + m.ghost_off : nullptr;
    const int lane = (int)(threadIdx.x & 63);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nx = m.nx, ny = m.ny;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const unsigned bytes = 36u * plane;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)src, (short)0, (int)bytes, BUFFER_RSRC_WORD3);
    const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc((void*)dst, (short)0, (int)bytes, BUFFER_RSRC_WORD3);
    // OPEN: the member's ghost block, [9][ny] floats (the inlet's +x movers, the outlet's -x movers)
    const __amdgpu_buffer_rsrc_t rg =
        OPEN ? __builtin_amdgcn_make_buffer_rsrc((void*)ghost, (short)0, (int)(36u * (unsigned)ny), BUFFER_RSRC_WORD3) : rs;
    const int base = tx * 256;
    const int x0 = base + 4 * lane;
    const unsigned voff = 4u * (unsigned)x0;
    const bool left_end = base == 0, right_end = base + 256 == nx;
    const int xl = (left_end ? nx : base) - 1;      // the cell left of the strip (periodic)
    const int xr = right_end ? 0 : base + 256;      // the cell right of it
    const int xh = (lane & 1) ? xr : xl;             // lanes 0 / 1 collide the left / right outside cell
    // OPEN: an end of the channel has no outside cell to collide (the inlet's
    // values come from the ghost block, the outlet's are built in phase B)
    const bool own_h = !OPEN || !((lane & 1) ? right_end : left_end);
    const bool sq_cols = m.ss > 0 && base <= m.sx0 + m.ss && base + 255 >= m.sx0 - 1;
    // grid bars within the columns any cell of this workgroup pulls from: the
    // outside cells x0 - 1 and x0 + 256 reach one column further than the
    // strip's own cells (base - 2 .. base + 257)
    const bool grid_cols = OPEN && m.bar > 0 && base <= m.gx0 + m.bar + 1 && base + 255 >= m.gx0 - 2;
    const bool sponge = OPEN && base + 255 > m.sp_x0;
    // bit j: column x0 - 1 + j (j = 0..5) holds grid bars
    unsigned gcols = 0;
    if (grid_cols)
#pragma unroll
        for (int j = 0; j < 6; ++j) gcols |= ((unsigned)(x0 - 1 + j - m.gx0) < (unsigned)m.bar ? 1u : 0u) << j;
    // OPEN: which rows cross the grid's bars.  Row yy does when yy >= bar/2 and
    // its phase (yy - bar/2) mod 2 bar is below bar; the wave carries the phase of
    // its row (a scalar, advanced by NW rows per iteration), so that no row test
    // needs a division or a memory read
    const int gper = 2 * m.bar, ghalf = m.bar >> 1;
    auto grow_ph = [&](int yy, int ph) {  // false outside the lattice
        return OPEN && grid_cols && yy >= ghalf && yy < ny && ph < m.bar;
    };
    // bits 0, 1, 2: rows yy - 1, yy, yy + 1 cross the grid's bars; ph: the phase of yy
    auto rows3 = [&](int yy, int ph) -> unsigned {
        if (!OPEN || !grid_cols) return 0u;
        const int pm = ph == 0 ? gper - 1 : ph - 1, pp = ph + 1 == gper ? 0 : ph + 1;
        return (grow_ph(yy - 1, pm) ? 1u : 0u) | (grow_ph(yy, ph) ? 2u : 0u) | (grow_ph(yy + 1, pp) ? 4u : 0u);
    };
    // OPEN: bit j: column x0 - 1 + j (j = 0..5) crosses the square
    unsigned sqcols = 0;
    if (OPEN && sq_cols)
#pragma unroll
        for (int j = 0; j < 6; ++j) sqcols |= ((unsigned)(x0 - 1 + j - m.sx0) < (unsigned)m.ss ? 1u : 0u) << j;
    // OPEN: solid cells around the lane's four cells of row yy: bit 6 j + dx + 1 for column
    // x0 + dx (dx = -1 .. 4) of row yy - 1 + j (j = 0..2), from the grid rows g3 of
    // rows3(yy) and, if near (the row is near the square), the square's rows; built once
    // per row so that each bounce-back test is one bit
    auto solids = [&](int yy, bool near, unsigned g3) -> unsigned {
        unsigned mk = 0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            unsigned row = ((g3 >> j) & 1u) ? gcols : 0u;
            if (near && (unsigned)(yy - 1 + j - m.sy0) < (unsigned)m.ss) row |= sqcols;
            mk |= row << (6 * j);
        }
        return mk;
    };
    // solid test of column x0 + dx in row yy = row - 1 + j: from the mask mk of the row
    // (OPEN), or from the square's bounds if near (periodic x has only the square; the
    // mask measured slower there)
    auto solid = [&](unsigned mk, int dx, int yy, int j, bool near) {
        return OPEN ? ((mk >> (6 * j + dx + 1)) & 1u) != 0u : near && in_square(m, x0 + dx, yy);
    };
    // rows [ya, yb) of the strip are this workgroup's to write; phase A also
    // collides the LAG rows on either side that phase B (and the outlet's
    // velocity ring) pull from, which the neighbouring workgroups of a split
    // strip collide too, bit for bit the same
    // (SPLIT = false: whole strips, compiled without the row-range arithmetic)
    const int ya = SPLIT ? ty * seg_rows : 0, yb = SPLIT ? min(ya + seg_rows, ny) : ny;
    const int ya0 = SPLIT ? max(ya - LAG, 0) : 0, ya1 = SPLIT ? min(yb + LAG, ny) : ny;  // phase A rows
    // phase B of the last iteration reaches row yb - 1
    const int iters = SPLIT ? (yb + LAG - ya0 + NW - 1) / NW : (ny + LAG - 1) / NW + 1;
    // phase of the wave's phase-A row (once, by a division)
    int gph = 0;
    if (OPEN && grid_cols) {
        const int r0 = (ya0 + wv - ghalf) % gper;
        gph = r0 < 0 ? r0 + gper : r0;
    }
    RowLoads cur;
    if ((SPLIT ? ya0 + wv : wv) < ya1) load_row<OPEN>(m, rs, rg, voff, xl, xr, ya0 + wv, cur, left_end, right_end);
#pragma unroll 1
    for (int j = 0; j < iters; ++j) {
        const int y = ya0 + j * NW + wv;
        // phase A: row y at step t+1 into the ring.  Every gather this row
        // needs (the outside cell, the obstacle's bounce-back words) is
        // issued before the prefetch of the wave's next row: waits on memory
        // complete in issue order, so waiting for them leaves the prefetch in
        // flight.
        const bool row_a = y < ya1;
        const bool near_sq = row_a && sq_cols && y >= m.sy0 - 1 && y <= m.sy0 + m.ss;
        const unsigned gA = row_a ? rows3(y, gph) : 0u;
        const bool near_a = near_sq || gA != 0u;
        float hv[9];
        f4 p[9];
        if (row_a) {
            if (own_h) {
                if (OPEN) {  // an interior outside cell: no wrap; the grid's rows from the bit table
#pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        const int xs = xh - CX[i], ys = y - CY[i];
                        const bool bounce = ys < 0 || ys >= ny || in_square(m, xs, ys) ||
                                            ((unsigned)(xs - m.gx0) < (unsigned)m.bar && ((gA >> (1 - CY[i])) & 1u));
                        hv[i] = src[bounce ? (unsigned)OPP[i] * plane + (unsigned)y * (unsigned)nx + (unsigned)xh
                                           : (unsigned)i * plane + (unsigned)ys * (unsigned)nx + (unsigned)xs];
                    }
                } else {
                    load_cell<false>(m, src, xh, y, hv);
                }
            }
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
            if (near_a) {
                // the row's own populations at t for the bounce-back: the rows of the
                // +-x movers are row y already; the other six, one coalesced load each
                const unsigned rowoff = (unsigned)y * (unsigned)nx;
                f4 ownv[9];
#pragma unroll
                for (int i = 1; i < 9; ++i)
                    ownv[i] = CY[OPP[i]] == 0 ? cur.v[OPP[i]]
                                              : __builtin_amdgcn_raw_buffer_load_b128(rs, voff, 4u * ((unsigned)OPP[i] * plane + rowoff), 0);
                const unsigned mk = OPEN ? solids(y, near_sq, gA) : 0u;
                if (OPEN) {
                    bounce_select(mk, ny, y, ownv, p);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (solid(mk, k, y, 1, near_sq)) continue;  // a solid cell's results are never stored
#pragma unroll
                        for (int i = 1; i < 9; ++i) {
                            const int ys = y - CY[i];
                            if (ys < 0 || ys >= ny) continue;
                            if (solid(mk, k - CX[i], ys, 1 - CY[i], near_sq)) p[i][k] = ownv[i][k];
                        }
                    }
                }
            }
        }
        // OPEN: the inlet's +x movers of row y, which lane 0 of the inlet strip
        // puts in the ring's left slot for both steps.  Loaded by every strip and
        // row (row clamped into the block), before the prefetch: loads issued on
        // some paths only leave the compiler unable to count them, and it then
        // waits for every load in flight, the prefetch included.
        float gin[3] = {0.0f, 0.0f, 0.0f};
        if (OPEN) {
            const unsigned yg = (unsigned)min(y, ny - 1);
#pragma unroll
            for (int i = 0, n = 0; i < 9; ++i)
                if (CX[i] == 1)
                    gin[n++] = __uint_as_float(
                        __builtin_amdgcn_raw_buffer_load_b32(rg, 0u, 4u * ((unsigned)i * (unsigned)ny + yg), 0));
        }
        RowLoads nxt;
        if (OPEN)  // on every path (the row clamped; past the last row its words go unused): see gin
            load_row<OPEN>(m, rs, rg, voff, xl, xr, min(y + NW, ya1 - 1), nxt, left_end, right_end);
        else if (y + NW < ya1)
            load_row<OPEN>(m, rs, rg, voff, xl, xr, y + NW, nxt, left_end, right_end);
        if (row_a) {
            float* row = ring + (y % RROWS) * 9 * RING_ROW;
            collide_row<MODEL, OPEN>(m, p, part0, near_sq, x0, y, sponge);
#pragma unroll
            for (int i = 0; i < 9; ++i) *(f4*)(row + i * RING_ROW + RING_CELL0 + 4 * lane) = p[i];
            if (OPEN && right_end && lane == 63) {  // the velocities the outlet ghost of step t+2 needs
                float d1[9], d2[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    d1[i] = p[i][3];  // column nx - 1
                    d2[i] = p[i][2];  // column nx - 2
                }
                OutletVel v;
                stored_velocity(d1, v.ux1, v.uy1);
                stored_velocity(d2, v.ux2, v.uy2);
                vring[y & (VROWS - 1)] = v;
                rring[y & (VROWS - 1)] = outlet_density(m, d1, d2);
            }
            // the outside cells (their drag belongs to the neighbouring strip)
            if (own_h) {
                if (OPEN) {
                    MemberDev mc = m;
                    if (sponge || base + 256 > m.sp_x0) sponge_at(mc, xh);
                    collide_cell<MODEL>(mc, hv, 0u);
                } else {
                    collide_cell<MODEL>(m, hv, 0u);
                }
            }
            if (lane < 2) {
                const int at = lane ? RING_RIGHT : RING_LEFT;
                if (own_h) {
                    if (!(in_square(m, xh, y) || (OPEN && (unsigned)(xh - m.gx0) < (unsigned)m.bar && ((gA >> 1) & 1u))))
#pragma unroll
                        for (int i = 0; i < 9; ++i) row[i * RING_ROW + at] = hv[i];
                } else if (lane == 0) {  // the inlet's +x movers for both steps
#pragma unroll
                    for (int i = 0, n = 0; i < 9; ++i)
                        if (CX[i] == 1) row[i * RING_ROW + at] = gin[n++];
                }
            }
        }
        lds_barrier();
        // phase B: row y - LAG at step t+2 from the ring to the other buffer
        const int r = y - LAG;
        if (r >= ya && r < yb) {
            const float* own = ring + (r % RROWS) * 9 * RING_ROW;
            const bool near_sq = sq_cols && r >= m.sy0 - 1 && r <= m.sy0 + m.ss;
            int phb = gph - LAG;  // the phase of row r = y - LAG
            if (phb < 0) phb += gper;
            if (phb < 0) phb += gper;
            const unsigned gB = rows3(r, phb);
            const bool near_b = near_sq || gB != 0u;
            const unsigned mkb = OPEN && near_b ? solids(r, near_sq, gB) : 0u;
            f4 p[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int rsrc = r - CY[i];
                if (rsrc < 0 || rsrc >= ny) {  // wall row: the cell's own opposite population
                    p[i] = *(const f4*)(own + OPP[i] * RING_ROW + RING_CELL0 + 4 * lane);
                    continue;
                }
                const float* srow = ring + (rsrc % RROWS) * 9 * RING_ROW + i * RING_ROW;
                const f4 v = *(const f4*)(srow + RING_CELL0 + 4 * lane);
                if (CX[i] == 1) {
                    const float h = srow[RING_LEFT];
                    const float sh = wave_shr1(v.w);
                    p[i] = f4{lane == 0 ? h : sh, v.x, v.y, v.z};
                } else if (CX[i] == -1) {
                    float h;
                    if (OPEN && right_end) {  // the outlet ghost column of step t+1, row rsrc
                        const OutletVel va = vring[(rsrc > 0 ? rsrc - 1 : 0) & (VROWS - 1)];
                        const OutletVel v0 = vring[rsrc & (VROWS - 1)];
                        const OutletVel vb = vring[(rsrc + 1 < ny ? rsrc + 1 : ny - 1) & (VROWS - 1)];
                        h = outlet_ghost_value(m, CX[i], CY[i], WD[i], rsrc, va, v0, vb, rring[rsrc & (VROWS - 1)]);
                    } else {
                        h = srow[RING_RIGHT];
                    }
                    const float sh = wave_shl1(v.x);
                    p[i] = f4{v.y, v.z, v.w, lane == 63 ? h : sh};
                } else {
                    p[i] = v;
                }
            }
            if (near_b) {
                if (OPEN) {
                    f4 ownb[9];
#pragma unroll
                    for (int i = 1; i < 9; ++i) ownb[i] = *(const f4*)(own + OPP[i] * RING_ROW + RING_CELL0 + 4 * lane);
                    bounce_select(mkb, ny, r, ownb, p);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (solid(mkb, k, r, 1, near_sq)) continue;
#pragma unroll
                        for (int i = 1; i < 9; ++i) {
                            const int rsrc = r - CY[i];
                            if (rsrc < 0 || rsrc >= ny) continue;
                            if (solid(mkb, k - CX[i], rsrc, 1 - CY[i], near_sq))
                                p[i][k] = own[OPP[i] * RING_ROW + RING_CELL0 + 4 * lane + k];
                        }
                    }
                }
            }
            collide_row<MODEL, OPEN>(m, p, part1, near_sq, x0, r, sponge);
            const unsigned rowoff = (unsigned)r * (unsigned)nx;
            unsigned smask = (mkb >> 7) & 0xFu;  // bit k: cell x0 + k is solid
            if (!OPEN && near_b)
#pragma unroll
                for (int k = 0; k < 4; ++k) smask |= (solid(0u, k, r, 1, near_sq) ? 1u : 0u) << k;
            if (smask == 0) {
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    __builtin_amdgcn_raw_buffer_store_b128(p[i], rd, voff, 4u * ((unsigned)i * plane + rowoff), BUFFER_NT);
            } else if (smask != 0xFu) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if ((smask >> k) & 1u) continue;
#pragma unroll
                    for (int i = 0; i < 9; ++i) dst[(unsigned)i * plane + rowoff + (unsigned)(x0 + k)] = p[i][k];
                }
            }
        }
        lds_barrier();
        cur = nxt;
        if (OPEN && grid_cols) {
            gph += NW;
            while (gph >= gper) gph -= gper;
        }
    }
}

template <int NW, bool SPLIT>
static void launch_step2_s(const StepArgs& a, int model, hipStream_t st) {
    const dim3 grid(a.total_blocks), block(64 * NW);
    if (a.ghost) {
        if (model == 2) hipLaunchKernelGGL((step2_kernel<NW, 2, true, SPLIT>), grid, block, 0, st, a);
        else if (model == 1) hipLaunchKernelGGL((step2_kernel<NW, 1, true, SPLIT>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((step2_kernel<NW, 0, true, SPLIT>), grid, block, 0, st, a);
    } else {
        if (model == 2) hipLaunchKernelGGL((step2_kernel<NW, 2, false, SPLIT>), grid, block, 0, st, a);
        else if (model == 1) hipLaunchKernelGGL((step2_kernel<NW, 1, false, SPLIT>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((step2_kernel<NW, 0, false, SPLIT>), grid, block, 0, st, a);
    }
}

template <int NW>
static hipError_t launch_step2_t(const StepArgs& a, int model, hipStream_t st) {
    if (a.split) launch_step2_s<NW, true>(a, model, st);
    else launch_step2_s<NW, false>(a, model, st);
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
