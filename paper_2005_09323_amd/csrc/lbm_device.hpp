// Device code shared by the one-step and two-step lattice kernels: the
// BGK + Guo collision of one cell, the obstacle links, the workgroup -> tile
// mapping, and the wave-level primitives of the row kernels.
//
// Paper Appendix A gives the scheme (exact streaming, BGK relaxation to the
// second-order equilibrium); Section 2 the halfway bounce-back on walls and
// obstacle; Section 2.1 the drag.  Populations are FP32 deviations
// d_i = f_i - w_i so that the O(1) rest weights never enter FP32 sums.
#pragma once

#include "kernels.hpp"

namespace lbm {

// BGK relaxation with Guo forcing of one cell, in deviation form:
//   rho = 1 + sum d_i,  J = sum c_i d_i + F/2 = rho u,
//   d_i^eq = w_i [(rho - 1) + 3 c.J + 4.5 (c.J)(c.u) - 1.5 J.u],
//   d_i <- (1 - omega) d_i + omega d_i^eq + w_i (1 - omega/2) [3 (c_ix - u_x) + 9 (c.u) c_ix] F.
// (The w_i of f_i = w_i + d_i cancel exactly between f_i and f_i^eq.)
// Opposite directions i and i' (c_i' = -c_i) share the even part of that
// update and differ in the sign of the odd part, so each pair costs one
// even and one odd term:
//   even = b + 4.5 omega (c.J)(c.u) + g9 c_ix (c.u) c_ix,  odd = 3 omega c.J + g3 c_ix,
//   b = omega ((rho - 1) - 1.5 J.u) - g3 u_x,  g3 = 3 (1 - omega/2) F,  g9 = 9 (1 - omega/2) F,
//   d_i <- (1 - omega) d_i + w_i (even + odd),  d_i' <- (1 - omega) d_i' + w_i (even - odd).
// The populations are stored in FP32 but the update is computed in FP64:
// the flow changes little from one step to the next, so FP32 rounding in
// the update repeats with the same sign step after step and its error grows
// linearly in time, while one rounding on store does not.  The update is
// done in place, one pair at a time, to keep few doubles live.
//
// links: bit i set when x + c_i lies in the square; returns the momentum
// those links hand to the square, sum of 2 c_ix f_i^out (the w_i parts
// cancel over the closed square, so deviations give the same total).
__device__ __forceinline__ double bgk_guo(const MemberDev& m, float d[9], unsigned links) {
    const double d0 = d[0], d1 = d[1], d2 = d[2], d3 = d[3], d4 = d[4];
    const double d5 = d[5], d6 = d[6], d7 = d[7], d8 = d[8];
    const double drho = ((d0 + d1) + (d2 + d3)) + ((d4 + d5) + (d6 + d7)) + d8;
    const double jx = (((d1 - d3) + (d5 - d6)) + (d8 - d7)) + m.half_fx;
    const double jy = ((d2 - d4) + (d5 - d7)) + (d6 - d8);
    const double rho = 1.0 + drho;
    // 1/rho: hardware FP32 reciprocal refined by two Newton steps in FP64
    // (relative error ~1e-14 << the FP32 storage rounding)
    double inv = (double)__builtin_amdgcn_rcpf((float)rho);
    inv = inv * (2.0 - rho * inv);
    inv = inv * (2.0 - rho * inv);
    const double ux = jx * inv;
    const double uy = jy * inv;
    const double om = m.omega;
    const double keep = 1.0 - om;
    const double c3 = 3.0 * om, c45 = 4.5 * om;
    const double b = om * (drho - 1.5 * (jx * ux + jy * uy)) - m.gf3 * ux;
    double drag = 0.0;
    d[0] = (float)(keep * d0 + WD[0] * b);
    // pair (ip, im) with c_ip = -c_im; e = c_ip.J, v = c_ip.u; xmove: c_ip,x = +1 (else 0)
    auto pair = [&](int ip, int im, double dp, double dm, double e, double v, bool xmove) {
        const double even = xmove ? fma(c45 * e, v, fma(m.gf9, v, b)) : fma(c45 * e, v, b);
        const double odd = xmove ? fma(c3, e, m.gf3) : c3 * e;
        const double op = fma(keep, dp, WD[ip] * (even + odd));
        const double on = fma(keep, dm, WD[im] * (even - odd));
        if (xmove) {
            if ((links >> ip) & 1u) drag += 2.0 * op;
            if ((links >> im) & 1u) drag -= 2.0 * on;
        }
        d[ip] = (float)op;
        d[im] = (float)on;
    };
    pair(1, 3, d1, d3, jx, ux, true);
    pair(2, 4, d2, d4, jy, uy, false);
    pair(5, 7, d5, d7, jx + jy, ux + uy, true);
    pair(8, 6, d8, d6, jx - jy, ux - uy, true);
    return drag;
}

// Directions of (x, y) whose next cell lies in the square (x-moving ones only).
__device__ __forceinline__ unsigned square_links(const MemberDev& m, int x, int y) {
    unsigned mask = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i)
        if (CX[i] != 0 && in_square(m, x + CX[i], y + CY[i])) mask |= 1u << i;
    return mask;
}

// Workgroup -> (member, tile): members are grouped in segments of equal
// lattice shape; within a segment tiles run x-fastest, then y, then member.
__device__ __forceinline__ int block_to_member(const StepArgs& a, int b, int& tx, int& ty, int& vec) {
    int s = 0;
#pragma unroll 1
    while (s + 1 < a.nseg && b >= a.seg[s + 1].block_begin) ++s;
    const int local = b - a.seg[s].block_begin;
    const int mloc = local / a.seg[s].tiles_per_member;
    const int tile = local - mloc * a.seg[s].tiles_per_member;
    ty = tile / a.seg[s].tiles_x;
    tx = tile - ty * a.seg[s].tiles_x;
    vec = a.seg[s].vec;
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

typedef float f4 __attribute__((ext_vector_type(4)));

// Word 3 of a raw (untyped) buffer resource on the GFX9/CDNA family, and the
// cache-policy bit that marks an access non-temporal on gfx94x/gfx950.  Every
// population is read once and written once per step, so both the row loads
// and the stores stream past the caches (measured: +2 % over cached loads).
constexpr int BUFFER_RSRC_WORD3 = 0x00020000;
constexpr int BUFFER_NT = 2;

// DPP wave shifts (GFX9 data-parallel primitives): lane l receives the value
// of lane l-1 (shr) or l+1 (shl); the lane without a source is replaced by
// the caller.
__device__ __forceinline__ float wave_shr1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float wave_shl1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}

}  // namespace lbm
