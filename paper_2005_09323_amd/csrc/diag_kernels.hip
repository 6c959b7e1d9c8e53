// Pressure, stress-integral drag and mean shear on the square's faces.
//
// The paper defines the drag as the surface integral of the stress over the
// obstacle (Section 2.1, drag definition; stress of Appendix A), approximates
// it by forebody minus base pressure (Section 2.1), and follows the mean shear
// along the top or bottom face as a precursor of extreme drag (Section 3.2.2).
// On the lattice the faces lie half a cell from the adjacent fluid cells; the
// quantities are taken from those cells' pulled populations (what the next
// step collides):
//   p_fb = sum_front c_s^2 rho,  p_base = sum_base c_s^2 rho,
//   stress drag = sum_front(-tau_xx) + sum_base(tau_xx) + sum_top(tau_xy) - sum_bottom(tau_xy),
//     tau_ab = -c_s^2 rho delta_ab - (1 - 1/(2 tau)) sum_i c_ia c_ib (f_i - f_i^eq),
//   shear_top = (1/s) sum_top u_x / (1/2),  shear_bottom = (1/s) sum_bottom (-u_x) / (1/2),
// with u the Guo-shifted velocity and f^eq the equilibrium of (rho, u).
#include "api_internal.hpp"
#include "lbm_device.hpp"

namespace lbm {

constexpr int DIAG_FIELDS = 5;

struct DiagArgs {
    const MemberDev* members;
    const int* parity;
    const float* pop0;
    const float* pop1;
    double* out;  // [member][DIAG_FIELDS]
};

// One workgroup per member; thread t takes face cells t, t + 256, ... and
// the partial sums meet in a fixed-order tree, so the result is reproducible.
__global__ __launch_bounds__(256) void face_diagnostics_kernel(DiagArgs a) {
    const int mi = (int)blockIdx.x;
    const MemberDev m = a.members[mi];
    __shared__ double red[DIAG_FIELDS][256];
    const int t = (int)threadIdx.x;
    double acc[DIAG_FIELDS] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (m.ss > 0) {
        const float* src = (a.parity[mi] ? a.pop1 : a.pop0) + m.off;
        const int s = m.ss;
        const double visc = 1.0 - 0.5 * m.omega;
        for (int c = t; c < 4 * s; c += 256) {
            const int face = c / s, k = c - face * s;  // 0 front, 1 base, 2 top, 3 bottom
            const int x = face == 0 ? m.sx0 - 1 : (face == 1 ? m.sx0 + s : m.sx0 + k);
            const int y = face < 2 ? m.sy0 + k : (face == 2 ? m.sy0 + s : m.sy0 - 1);
            float dl[9];
            load_cell(m, src, x, y, dl);
            double f[9], rho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                f[i] = WD[i] + (double)dl[i];
                rho += f[i];
                jx += CX[i] * f[i];
                jy += CY[i] * f[i];
            }
            const double ux = (jx + m.half_fx) / rho, uy = jy / rho;
            const double usq = ux * ux + uy * uy;
            double pxx = 0.0, pxy = 0.0;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const double cu = CX[i] * ux + CY[i] * uy;
                const double neq = f[i] - WD[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
                pxx += (double)(CX[i] * CX[i]) * neq;
                pxy += (double)(CX[i] * CY[i]) * neq;
            }
            const double txx = -rho / 3.0 - visc * pxx;
            const double txy = -visc * pxy;
            if (face == 0) {
                acc[0] += rho / 3.0;
                acc[2] -= txx;
            } else if (face == 1) {
                acc[1] += rho / 3.0;
                acc[2] += txx;
            } else if (face == 2) {
                acc[2] += txy;
                acc[3] += ux / (0.5 * s);
            } else {
                acc[2] -= txy;
                acc[4] -= ux / (0.5 * s);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < DIAG_FIELDS; ++q) red[q][t] = acc[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < DIAG_FIELDS; ++q) red[q][t] += red[q][t + w];
        __syncthreads();
    }
    if (t < DIAG_FIELDS) a.out[(long long)mi * DIAG_FIELDS + t] = red[t][0];
}

}  // namespace lbm

using namespace lbm;

extern "C" int lbm_face_diagnostics(const lbm_ctx* c, double* out_dev) {
    if (!c || !out_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
    DiagArgs a;
    a.members = c->d_members;
    a.parity = c->d_parity;
    a.pop0 = c->pop[0];
    a.pop1 = c->pop[1];
    a.out = out_dev;
    hipLaunchKernelGGL(face_diagnostics_kernel, dim3(c->n), dim3(256), 0, c->stream, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : lbm_hip_fail(e, "face diagnostics");
}
