// Device-side building blocks shared by the library's kernels: the D2Q9
// lattice (paper Appendix A), the Philox4x64-10 generator (Salmon et al.,
// SC'11) and the per-member parameter table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// D2Q9 velocities, weights and opposite directions; numbering (0,0), (1,0),
// (0,1), (-1,0), (0,-1), (1,1), (-1,1), (-1,-1), (1,-1).
constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr float WF[9] = {4.0f / 9.0f, 1.0f / 9.0f, 1.0f / 9.0f, 1.0f / 9.0f, 1.0f / 9.0f,
                         1.0f / 36.0f, 1.0f / 36.0f, 1.0f / 36.0f, 1.0f / 36.0f};
constexpr double WD[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// Philox purpose tags (ASCII of the four-letter names), key word 1.
constexpr uint64_t PURPOSE_INIT = 0x494E4954ull;
constexpr uint64_t PURPOSE_GKTS = 0x474B5453ull;
constexpr uint64_t PURPOSE_PRTB = 0x50525442ull;
constexpr uint64_t PURPOSE_AMSP = 0x414D5350ull;

struct U64x4 {
    uint64_t v[4];
};

// Philox4x64-10: ten rounds of two 64x64->128 multiplications with Weyl
// key bumps between rounds.
__host__ __device__ inline U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
#if defined(__HIP_DEVICE_COMPILE__)
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
#else
        const unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        const unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
#endif
        const uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    U64x4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

__host__ __device__ inline double uniform53(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

__device__ inline uint64_t index_below(uint64_t w, uint64_t n) { return __umul64hi(w, n); }

// Per-member parameters as the kernels read them.
struct MemberDev {
    int nx, ny;
    int sx0, sy0, ss;     // square: lower-left cell and side (0 = none)
    int ring;             // cells around the square that own drag partials: 4 s + 4
    double omega;         // 1 / tau
    double half_fx;       // F / 2 (Guo velocity shift)
    double gf3, gf9;      // (1 - omega/2) * 3F and (1 - omega/2) * 9F (Guo source)
    double force;         // F (central-moment collision)
    double sb, s3, s4;    // central-moment rates: trace, third order, fourth order
    int model;            // 0: BGK; 1: central moments; 2: central moments, unit bulk/third/fourth rates
    int open;             // 1: inlet, entrance grid, sponge and outlet instead of periodic x
    long long off;        // first float of the member in a population buffer
    long long part_off;   // first float of the member in the drag-partial buffer
    // open channel (zero otherwise)
    int gx0, bar;         // grid bars: columns gx0 .. gx0 + bar - 1 (bar = 0: no grid)
    int sp_x0;            // last column before the sponge ramp (>= nx - 1: no sponge)
    int out_rho;          // outlet density: 0 held at 1, 1 extrapolated to second order
    double tau;           // relaxation time outside the sponge
    double tau_sp;        // relaxation time at the outlet column
    double sp_inv;        // 1 / (nx - 1 - sp_x0) (0: no sponge)
    double u_c;           // inlet centre-line velocity
    long long ghost_off;  // first float of the member's outlet ghost column [9][ny]
};

// True if (x, y) is a cell of the member's square.
__device__ __forceinline__ bool in_square(const MemberDev& m, int x, int y) {
    return (unsigned)(x - m.sx0) < (unsigned)m.ss && (unsigned)(y - m.sy0) < (unsigned)m.ss;
}

// True if row y, 0 <= y < ny, crosses the bars of the entrance grid: rows
// y >= bar/2 with (y - bar/2) mod (2 bar) < bar (bars and gaps of one height,
// half gaps at the walls).
__device__ __forceinline__ bool grid_row(const MemberDev& m, int y) {
    const int r = y - (m.bar >> 1);
    return m.bar > 0 && r >= 0 && r % (2 * m.bar) < m.bar;
}

// True if (x, y), 0 <= y < ny, is a cell of the entrance grid: bar x bar cells
// in columns gx0 .. gx0 + bar - 1 on the grid's rows.
__device__ __forceinline__ bool in_grid(const MemberDev& m, int x, int y) {
    return (unsigned)(x - m.gx0) < (unsigned)m.bar && grid_row(m, y);
}

// True on every solid cell: the square, and the grid of an open channel.
__device__ __forceinline__ bool in_solid(const MemberDev& m, int x, int y) {
    return in_square(m, x, y) || in_grid(m, x, y);
}

// Index of (x, y) in the ring of cells around the square, or -1.
// Order: bottom row (y0-1, x0-1..x0+s), top row (y0+s, same x), left column
// (x0-1, y0..y0+s-1), right column (x0+s, same y).
__device__ __forceinline__ int ring_index(const MemberDev& m, int x, int y) {
    if (m.ss == 0) return -1;
    const int s = m.ss;
    const int rx = x - (m.sx0 - 1), ry = y - (m.sy0 - 1);
    if ((unsigned)rx > (unsigned)(s + 1) || (unsigned)ry > (unsigned)(s + 1)) return -1;
    if (ry == 0) return rx;
    if (ry == s + 1) return (s + 2) + rx;
    if (rx == 0) return 2 * (s + 2) + (ry - 1);
    if (rx == s + 1) return 2 * (s + 2) + s + (ry - 1);
    return -1;  // inside the square
}

}  // namespace lbm
