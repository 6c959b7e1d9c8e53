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
//
// Contraction is pinned per source expression (fp contract on: a * b + c
// written in one expression may become one FMA, nothing across statements),
// so that every kernel that inlines this function computes the same bits
// whatever the optimizer does around it.
__device__ __forceinline__ double bgk_guo(const MemberDev& m, float d[9], unsigned links) {
#pragma clang fp contract(on)
    const double d0 = d[0], d1 = d[1], d2 = d[2], d3 = d[3], d4 = d[4];
    const double d5 = d[5], d6 = d[6], d7 = d[7], d8 = d[8];
    const double drho = ((d0 + d1) + (d2 + d3)) + ((d4 + d5) + (d6 + d7)) + d8;
    const double jx = (((d1 - d3) + (d5 - d6)) + (d8 - d7)) + m.half_fx;
    const double jy = ((d2 - d4) + (d5 - d7)) + (d6 - d8);
    const double rho = 1.0 + drho;
    // 1/rho: hardware FP32 reciprocal of rho rounded to FP32 (relative error
    // below 2e-7 together) refined by one Newton step in FP64, which squares
    // it: below 4e-14, far under the FP32 storage rounding
    double inv = (double)__builtin_amdgcn_rcpf((float)rho);
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
#pragma clang fp contract(on)
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

// Central-moment multiple-relaxation-time collision with Guo forcing of one
// cell (the collision the paper uses for its turbulent runs, Appendix A, last
// paragraph), in deviation form and FP64:
//   raw moments m_pq = sum_i c_ix^p c_iy^q f_i of f = w + d (w contributes
//   1, 1/3, 1/3, 1/9 to m00, m20, m02, m22), u = (m10 + F/2, m01) / rho;
//   central moments k_pq by the binomial shift c^p = ((c - u) + u)^p;
//   k* = k - s (k - k^eq) + (1 - s/2) k^F, with k^eq and k^F the central
//   moments of the discrete second-order equilibrium and of Guo's source
//   w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F (F along x):
//     k20^eq = k02^eq = rho/3, k11^eq = 0, k21^eq = -rho ux^2 uy,
//     k12^eq = -rho ux uy^2, k22^eq = rho/9 + 3 rho ux^2 uy^2;
//     k^F: k10 = F, k21 = -2 ux uy F, k12 = F/3 - uy^2 F, k22 = 4 ux uy^2 F;
//   rates: omega for k20 - k02 and k11, sb for k20 + k02, s3 for k21 and k12,
//   s4 for k22 (the conserved k00, k10, k01 end at rho, F/2, 0);
//   the increments k* - k go back to raw moments by the inverse shift and to
//   population increments by the inverse of the D2Q9 raw-moment matrix.
// With every rate equal to omega this is the BGK + Guo update.  Contraction
// is pinned per source expression, as in bgk_guo.
__device__ __forceinline__ double cm_guo(const MemberDev& m, float d[9], unsigned links) {
#pragma clang fp contract(on)
    const double d0 = d[0], d1 = d[1], d2 = d[2], d3 = d[3], d4 = d[4];
    const double d5 = d[5], d6 = d[6], d7 = d[7], d8 = d[8];
    const double dr = ((d0 + d1) + (d2 + d3)) + ((d4 + d5) + (d6 + d7)) + d8;  // rho - 1
    const double diag = (d5 + d6) + (d7 + d8);
    const double rho = 1.0 + dr;
    const double jx = ((d1 - d3) + (d5 - d6)) + (d8 - d7);
    const double jy = ((d2 - d4) + (d5 - d7)) + (d6 - d8);
    const double m20 = (1.0 / 3.0) + ((d1 + d3) + diag);
    const double m02 = (1.0 / 3.0) + ((d2 + d4) + diag);
    const double m11 = (d5 - d6) + (d7 - d8);
    const double m21 = (d5 + d6) - (d7 + d8);
    const double m12 = (d5 - d6) - (d7 - d8);
    const double m22 = (1.0 / 9.0) + diag;
    double inv = (double)__builtin_amdgcn_rcpf((float)rho);
    inv = inv * (2.0 - rho * inv);
    const double F = m.force;
    const double mx = jx + m.half_fx;  // rho u_x
    const double ux = mx * inv, uy = jy * inv;
    const double uxx = ux * ux, uyy = uy * uy, uxy = ux * uy;
    // central moments (k10 = -F/2, k01 = 0)
    const double k20 = m20 - 2.0 * ux * jx + uxx * rho;
    const double k02 = m02 - 2.0 * uy * jy + uyy * rho;
    const double k11 = m11 - ux * jy - uy * jx + uxy * rho;
    const double k21 = m21 - 2.0 * ux * m11 - uy * m20 + uxx * jy + 2.0 * uxy * jx - uxx * uy * rho;
    const double k12 = m12 - 2.0 * uy * m11 - ux * m02 + uyy * jx + 2.0 * uxy * jy - ux * uyy * rho;
    const double k22 = m22 - 2.0 * ux * m12 - 2.0 * uy * m21 + uxx * m02 + uyy * m20 + 4.0 * uxy * m11
                       - 2.0 * ux * uyy * jx - 2.0 * uxx * uy * jy + uxx * uyy * rho;
    // relaxation, as increments dk = -s (k - k^eq) + (1 - s/2) k^F of the
    // central moments (k10 goes from -F/2 to F/2: dk10 = F)
    const double om = m.omega, sb = m.sb, s3 = m.s3, s4 = m.s4;
    const double dks = -sb * ((k20 + k02) - (2.0 / 3.0) * rho);
    const double dkd = -om * (k20 - k02);
    const double e20 = 0.5 * (dks + dkd), e02 = 0.5 * (dks - dkd);
    const double e11 = -om * k11;
    const double e21 = -s3 * (k21 + rho * uxx * uy) + (1.0 - 0.5 * s3) * (-2.0 * uxy * F);
    const double e12 = -s3 * (k12 + rho * ux * uyy) + (1.0 - 0.5 * s3) * (F * (1.0 / 3.0) - uyy * F);
    const double e22 = -s4 * (k22 - rho * (1.0 / 9.0) - 3.0 * rho * uxx * uyy) + (1.0 - 0.5 * s4) * (4.0 * ux * uyy * F);
    // the same increments as raw moments (inverse shift, linear in the increments)
    const double M10 = F;
    const double M20 = e20 + 2.0 * ux * F;
    const double M02 = e02;
    const double M11 = e11 + uy * F;
    const double M21 = e21 + 2.0 * ux * e11 + uy * e20 + 2.0 * uxy * F;
    const double M12 = e12 + 2.0 * uy * e11 + ux * e02 + uyy * F;
    const double M22 = e22 + 2.0 * ux * e12 + 2.0 * uy * e21 + uxx * e02 + uyy * e20 + 4.0 * uxy * e11 + 2.0 * ux * uyy * F;
    // and as populations (inverse of the raw-moment matrix; dM00 = dM01 = 0)
    const double o0 = d0 + ((M22 - M20) - M02);
    const double o1 = d1 + 0.5 * ((M10 + M20) - (M12 + M22));
    const double o3 = d3 + 0.5 * ((M20 - M10) + (M12 - M22));
    const double o2 = d2 + 0.5 * (M02 - (M21 + M22));
    const double o4 = d4 + 0.5 * ((M02 + M21) - M22);
    const double o5 = d5 + 0.25 * ((M11 + M21) + (M12 + M22));
    const double o6 = d6 + 0.25 * ((M21 - M11) + (M22 - M12));
    const double o7 = d7 + 0.25 * ((M11 - M21) + (M22 - M12));
    const double o8 = d8 + 0.25 * ((M12 - M11) + (M22 - M21));
    double drag = 0.0;
    if (links) {
        if ((links >> 1) & 1u) drag += 2.0 * o1;
        if ((links >> 3) & 1u) drag -= 2.0 * o3;
        if ((links >> 5) & 1u) drag += 2.0 * o5;
        if ((links >> 6) & 1u) drag -= 2.0 * o6;
        if ((links >> 7) & 1u) drag -= 2.0 * o7;
        if ((links >> 8) & 1u) drag += 2.0 * o8;
    }
    d[0] = (float)o0; d[1] = (float)o1; d[2] = (float)o2; d[3] = (float)o3; d[4] = (float)o4;
    d[5] = (float)o5; d[6] = (float)o6; d[7] = (float)o7; d[8] = (float)o8;
    return drag;
}

// The central-moment collision above when the bulk, third- and fourth-order
// rates are all 1 (the setting of the paper's turbulent runs): the trace
// k20 + k02 and the third- and fourth-order central moments then leave the
// collision at their equilibrium-plus-forcing values, closed forms of rho, u
// and F, so the pre-collision k21, k12 and k22 are never needed.  The
// post-collision raw moments follow by the binomial shift and the
// populations by the inverse moment matrix, all as deviations from the rest
// state (the weights' moments 1, 1/3, 1/3, 1/9 subtracted analytically, so a
// state at rest stays exactly at rest).  The shift's terms in rho u^n and
// F u^n cancel against those of the third- and fourth-order moments, and the
// pre-collision second moments about u use j_x = rho u_x - F/2, j_y = rho u_y,
// so each raw moment is a short sum.  Equal to cm_guo with those rates up to
// FP64 rounding; contraction pinned as there.
__device__ __forceinline__ double cm1_guo(const MemberDev& m, float d[9], unsigned links) {
#pragma clang fp contract(on)
    const double d0 = d[0], d1 = d[1], d2 = d[2], d3 = d[3], d4 = d[4];
    const double d5 = d[5], d6 = d[6], d7 = d[7], d8 = d[8];
    const double dr = ((d0 + d1) + (d2 + d3)) + ((d4 + d5) + (d6 + d7)) + d8;  // rho - 1
    const double rho = 1.0 + dr;
    const double jx = ((d1 - d3) + (d5 - d6)) + (d8 - d7);
    const double jy = ((d2 - d4) + (d5 - d7)) + (d6 - d8);
    const double m11 = (d5 - d6) + (d7 - d8);
    double inv = (double)__builtin_amdgcn_rcpf((float)rho);
    inv = inv * (2.0 - rho * inv);
    const double F = m.force;
    const double ux = (jx + m.half_fx) * inv, uy = jy * inv;
    const double uxx = ux * ux, uyy = uy * uy, uxy = ux * uy;
    // second order: k20 - k02 and k11 relax at omega, k20 + k02 goes to 2 rho / 3
    // (m20 - m02 = (d1 + d3) - (d2 + d4): the diagonal directions and the weights cancel)
    const double kd = (((d1 + d3) - (d2 + d4)) - rho * (uxx - uyy)) + ux * F;
    const double k11 = (m11 - rho * uxy) + 0.5 * F * uy;
    const double om1 = 1.0 - m.omega;
    const double a = 0.5 * om1 * kd;
    const double k11s = om1 * k11;
    const double k20s = rho * (1.0 / 3.0) + a, k02s = rho * (1.0 / 3.0) - a;
    // post-collision raw moments (k10* = F/2, k01* = 0), as deviations from rest; the third
    // and fourth central moments (equilibrium plus half the source's) enter only through
    // what survives the shift
    const double m10s = jx + F;
    const double dm20s = dr * (1.0 / 3.0) + a + ux * F + uxx * rho;
    const double dm02s = dr * (1.0 / 3.0) - a + uyy * rho;
    const double m11s = k11s + 0.5 * uy * F + uxy * rho;
    const double m21s = 2.0 * ux * k11s + uy * k20s;
    const double m12s = F * (1.0 / 6.0) + 2.0 * uy * k11s + ux * k02s;
    const double dm22s = (dr * (1.0 / 9.0) + ux * F * (1.0 / 3.0)) + (uxx * k02s + uyy * k20s + 4.0 * uxy * k11s);
    // populations (inverse of the raw-moment matrix), opposite directions as sum and
    // difference of shared terms
    const double ax = dm20s - dm22s, bx = m10s - m12s;  // f1 + f3 and f1 - f3 (deviations)
    const double ay = dm02s - dm22s, by = jy - m21s;    // f2 + f4 and f2 - f4
    const double t1 = dm22s + m12s, t2 = dm22s - m12s, t3 = m11s + m21s, t4 = m21s - m11s;
    const double o0 = (dr - dm20s) - ay;
    const double o1 = 0.5 * (ax + bx), o3 = 0.5 * (ax - bx);
    const double o2 = 0.5 * (ay + by), o4 = 0.5 * (ay - by);
    const double o5 = 0.25 * (t1 + t3), o8 = 0.25 * (t1 - t3);
    const double o6 = 0.25 * (t2 + t4), o7 = 0.25 * (t2 - t4);
    double drag = 0.0;
    if (links) {
        if ((links >> 1) & 1u) drag += 2.0 * o1;
        if ((links >> 3) & 1u) drag -= 2.0 * o3;
        if ((links >> 5) & 1u) drag += 2.0 * o5;
        if ((links >> 6) & 1u) drag -= 2.0 * o6;
        if ((links >> 7) & 1u) drag -= 2.0 * o7;
        if ((links >> 8) & 1u) drag += 2.0 * o8;
    }
    d[0] = (float)o0; d[1] = (float)o1; d[2] = (float)o2; d[3] = (float)o3; d[4] = (float)o4;
    d[5] = (float)o5; d[6] = (float)o6; d[7] = (float)o7; d[8] = (float)o8;
    return drag;
}

// The collision of a kernel instantiated for one model (0: BGK, 1: central
// moments, 2: central moments with unit bulk, third- and fourth-order rates);
// the step kernels are compiled once per model so that each keeps its own
// register allocation.
template <int MODEL>
__device__ __forceinline__ double collide_cell(const MemberDev& m, float d[9], unsigned links) {
    if constexpr (MODEL == 2) return cm1_guo(m, d, links);
    else if constexpr (MODEL == 1) return cm_guo(m, d, links);
    else return bgk_guo(m, d, links);
}

// The member's own model, decided at run time (the one-off initial step).
__device__ __forceinline__ double collide_member(const MemberDev& m, float d[9], unsigned links) {
    return m.model == 2 ? cm1_guo(m, d, links) : (m.model ? cm_guo(m, d, links) : bgk_guo(m, d, links));
}

// The nine pulled populations of one cell (x, y) from the state at t, with
// periodic x, wall rows and solid cells bouncing back (per-lane gathers).
// GRID = false: the square is the only obstacle (periodic channels).
template <bool GRID = true>
__device__ __forceinline__ void load_cell(const MemberDev& m, const float* __restrict__ src, int x, int y, float dl[9]) {
    const int nx = m.nx, ny = m.ny;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int xs = x - CX[i];
        xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
        const int ys = y - CY[i];
        const bool bounce = (ys < 0) | (ys >= ny) | (GRID ? in_solid(m, xs, ys) : in_square(m, xs, ys));
        const unsigned idx = bounce ? (unsigned)OPP[i] * plane + (unsigned)y * (unsigned)nx + (unsigned)x
                                    : (unsigned)i * plane + (unsigned)ys * (unsigned)nx + (unsigned)xs;
        dl[i] = src[idx];
    }
}

// Solid test of a kernel instantiated for periodic (square only) or open
// channels (square and grid).
template <bool OPEN>
__device__ __forceinline__ bool solid_at(const MemberDev& m, int x, int y) {
    if constexpr (OPEN) return in_solid(m, x, y);
    else return in_square(m, x, y);
}

// Open channel, paper Section 2: the relaxation rates at column x of the
// sponge zone, tau(x) = tau + (tau_sp - tau) r^2 with
// r = (x - sp_x0) / (nx - 1 - sp_x0) beyond sp_x0 (tau before it), and the
// Guo coefficients that depend on them.  1/tau(x) as for 1/rho: hardware
// FP32 reciprocal refined by two Newton steps in FP64 (relative error
// ~1e-14, far below the FP32 storage rounding).
__device__ __forceinline__ void sponge_at(MemberDev& m, int x) {
    if (x <= m.sp_x0) return;
    const double r = (double)(x - m.sp_x0) * m.sp_inv;
    const double tau = m.tau + ((m.tau_sp - m.tau) * r) * r;
    double om = (double)__builtin_amdgcn_rcpf((float)tau);
    om = om * (2.0 - tau * om);
    om = om * (2.0 - tau * om);
    m.omega = om;
    m.gf3 = (1.0 - 0.5 * om) * 3.0 * m.force;
    m.gf9 = (1.0 - 0.5 * om) * 9.0 * m.force;
}

// Open channel inlet: the ghost column x = -1 holds the equilibrium of
// rho = 1, u = (u_in(y), 0), u_in(y) = 4 u_c (y + 1/2)(ny - y - 1/2) / ny^2
// (zero on the halfway walls).  Its populations with c_ix = +1, the only
// ones pulled from it, deviate from their rest weights by w_i (3 u + 3 u^2).
__device__ __forceinline__ float inlet_dev(const MemberDev& m, int i, int y) {
    const double yc = (double)y + 0.5;
    const double u = 4.0 * m.u_c * yc * ((double)m.ny - yc) / ((double)m.ny * (double)m.ny);
    return (float)(WD[i] * (3.0 * u + 3.0 * (u * u)));
}

// Open channel outlet (paper Section 2): the velocity sum c_i f_i / sum f_i of
// one stored (post-collision) cell from its FP32 deviations.
__device__ __forceinline__ void stored_velocity(const float dl[9], double& ux, double& uy) {
    double d[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) d[i] = (double)dl[i];
    const double rho = 1.0 + (((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8]);
    const double inv = 1.0 / rho;
    ux = (((d[1] - d[3]) + (d[5] - d[6])) + (d[8] - d[7])) * inv;
    uy = (((d[2] - d[4]) + (d[5] - d[7])) + (d[6] - d[8])) * inv;
}

// Open channel outlet, density extrapolated to second order (paper Section 2):
// rho_g = 2 rho(nx-1) - rho(nx-2) of one row from the two stored cells, as
// 1 + (2 sum d(nx-1) - sum d(nx-2)) so that the O(1) weights never enter the
// sums; 1 when the member's outlet holds its density.
__device__ __forceinline__ double outlet_density(const MemberDev& m, const float d1[9], const float d2[9]) {
#pragma clang fp contract(off)
    if (!m.out_rho) return 1.0;
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        s1 += (double)d1[i];
        s2 += (double)d2[i];
    }
    return 1.0 + (2.0 * s1 - s2);
}

// The velocities of the last two columns of one row: (ux1, uy1) at nx - 1,
// (ux2, uy2) at nx - 2.
struct OutletVel {
    double ux1, uy1, ux2, uy2;
};

// Outlet ghost population of a direction with c_x = -1 at row y, as a
// deviation from its weight w:
//   rho_g = 1 or the extrapolated density (outlet_density),
//   u_g = 2 u(nx-1) - u(nx-2),
//   S_xx = ux(nx-1) - ux(nx-2),  S_yy = d_y uy_g,
//   S_xy = (d_y ux_g + uy(nx-1) - uy(nx-2)) / 2
//   (d_y centred over rows ya = y - 1 and yb = y + 1, one-sided in the first
//   and last row, where the caller passes ya = y or yb = y),
//   Pi = -2 rho_g c_s^2 (tau(nx-1) - 1) S,
//   g_i = f_i^eq(rho_g, u_g) + w_i / (2 c_s^4) (c_i c_i - c_s^2 I) : Pi,
//   i.e. g_i - w_i = w_i [(rho_g - 1) + rho_g X] with X the bracket for rho_g = 1.
// The ghost kernel and the two-step kernel both build the ghost column with
// this function; contraction into FMAs is off so that both give the same bits
// wherever they are inlined.
// (cx, cy, w: the direction's velocity and weight, passed as values so that
// lanes can build different directions at once.)
__device__ __forceinline__ float outlet_ghost_value(const MemberDev& m, double cx, double cy, double w, int y,
                                                    const OutletVel& va, const OutletVel& v0, const OutletVel& vb,
                                                    double rho_g) {
#pragma clang fp contract(off)
    const double h = (y > 0 && y + 1 < m.ny) ? 0.5 : 1.0;  // centred or one-sided
    const double ux = 2.0 * v0.ux1 - v0.ux2, uy = 2.0 * v0.uy1 - v0.uy2;
    const double uxa = 2.0 * va.ux1 - va.ux2, uya = 2.0 * va.uy1 - va.uy2;
    const double uxb = 2.0 * vb.ux1 - vb.ux2, uyb = 2.0 * vb.uy1 - vb.uy2;
    const double sxx = v0.ux1 - v0.ux2;
    const double syy = h * (uyb - uya);
    const double sxy = 0.5 * (h * (uxb - uxa) + (v0.uy1 - v0.uy2));
    const double tau_out = m.sp_x0 < m.nx - 1 ? m.tau + (m.tau_sp - m.tau) : m.tau;  // tau(nx - 1), r = 1
    const double cpi = -2.0 * (1.0 / 3.0) * (tau_out - 1.0);                        // Pi = cpi * S (rho_g = 1)
    const double pxx = cpi * sxx, pyy = cpi * syy, pxy = cpi * sxy;
    const double usq = ux * ux + uy * uy;
    const double cu = cx * ux + cy * uy;
    const double q = (cx * cx - 1.0 / 3.0) * pxx + 2.0 * cx * cy * pxy + (cy * cy - 1.0 / 3.0) * pyy;
    const double x = (3.0 * cu + 4.5 * cu * cu - 1.5 * usq) + 4.5 * q;
    if (!m.out_rho) return (float)(w * x);
    return (float)(w * ((rho_g - 1.0) + rho_g * x));
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
__device__ __forceinline__ int block_to_member(const StepArgs& a, int b, int& tx, int& ty, int& vec, int& rows) {
    if (a.active_list) {  // a subset of members of one lattice shape
        const int k = b / a.seg[0].tiles_per_member;
        const int tile = b - k * a.seg[0].tiles_per_member;
        ty = tile / a.seg[0].tiles_x;
        tx = tile - ty * a.seg[0].tiles_x;
        vec = a.seg[0].vec;
        rows = a.seg[0].rows;
        return a.active_list[k];
    }
    int s = 0;
#pragma unroll 1
    while (s + 1 < a.nseg && b >= a.seg[s + 1].block_begin) ++s;
    const int local = b - a.seg[s].block_begin;
    const int mloc = local / a.seg[s].tiles_per_member;
    const int tile = local - mloc * a.seg[s].tiles_per_member;
    ty = tile / a.seg[s].tiles_x;
    tx = tile - ty * a.seg[s].tiles_x;
    vec = a.seg[s].vec;
    rows = a.seg[s].rows;
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
