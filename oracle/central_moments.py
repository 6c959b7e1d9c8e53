"""Central-moment multiple-relaxation-time collision with Guo forcing, FP64.

Test infrastructure (see ``oracle/__init__``).

For its turbulent runs the paper swaps the single-relaxation-time BGK collision
for a multiple-relaxation-time collision in central moments, for stability,
and cites the scheme without printing it (Appendix A, last paragraph).  The
reading used here (its equations are this module's):

* central moments k_pq = sum_i (c_ix - u_x)^p (c_iy - u_y)^q f_i for the nine
  exponent pairs of D2Q9, (0,0) (1,0) (0,1) (2,0) (0,2) (1,1) (2,1) (1,2)
  (2,2), with u the Guo-shifted velocity (sum_i c_i f_i + F/2) / rho;
* every moment relaxes towards the same central moment of the discrete
  second-order equilibrium f^eq(rho, u) of Appendix A, and receives its
  central moment of Guo's source w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F
  weighted by (1 - s/2):
      k* = k - s (k - k^eq) + (1 - s/2) k^F;
* rates: 1/tau for the shear moments k20 - k02 and k11 (so nu = (tau - 1/2)
  c_s^2 as for BGK), s_b for the trace k20 + k02 (bulk viscosity), s_3 for
  k21 and k12, s_4 for k22.  Mass and momentum come out the same for any
  rate (k00 = rho is left alone; k10 goes from -F/2 to +F/2).

Moments are a linear, invertible map of the populations, so with every rate
equal to 1/tau the update is exactly the BGK + Guo update of ``oracle.lbm``.
Central moments are computed here by their definition; the way back uses the
binomial expansion c^p = ((c - u) + u)^p to raw moments and the inverse of
the (constant) raw-moment matrix.
"""
from __future__ import annotations

from math import comb

import numpy as np

BASIS = ((0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2))
_K20, _K02, _K11, _K21, _K12, _K22 = 3, 4, 5, 6, 7, 8


def _lattice():
    from .lbm import C
    return C


def central_moments(g: np.ndarray, ux, uy) -> np.ndarray:
    """k[n] = sum_i (c_ix - u_x)^p (c_iy - u_y)^q g_i for (p, q) = BASIS[n]; g is [9, ...]."""
    C = _lattice()
    k = np.zeros((9,) + np.shape(g)[1:])
    for n, (p, q) in enumerate(BASIS):
        for i in range(9):
            k[n] = k[n] + (C[i, 0] - ux) ** p * (C[i, 1] - uy) ** q * g[i]
    return k


def raw_moment_matrix() -> np.ndarray:
    """M[n, i] = c_ix^p c_iy^q for (p, q) = BASIS[n]."""
    C = _lattice()
    return np.array([[float(C[i, 0] ** p * C[i, 1] ** q) for i in range(9)] for (p, q) in BASIS])


def populations(k: np.ndarray, ux, uy) -> np.ndarray:
    """The populations whose central moments (about u) are k."""
    index = {pq: n for n, pq in enumerate(BASIS)}
    raw = np.zeros_like(k)
    for n, (p, q) in enumerate(BASIS):
        for a in range(p + 1):
            for b in range(q + 1):
                raw[n] = raw[n] + comb(p, a) * comb(q, b) * ux ** (p - a) * uy ** (q - b) * k[index[(a, b)]]
    minv = np.linalg.inv(raw_moment_matrix())
    return np.tensordot(minv, raw, axes=(1, 0))


def relax(k: np.ndarray, keq: np.ndarray, kf: np.ndarray, omega: float, s_b: float, s_3: float,
          s_4: float) -> np.ndarray:
    """k* = k - s (k - k^eq) + (1 - s/2) k^F per moment; the second order in trace / difference form."""
    def one(s, a, e, f):
        return a - s * (a - e) + (1.0 - 0.5 * s) * f

    out = np.empty_like(k)
    for n in (0, 1, 2):  # conserved: any rate gives the same result
        out[n] = one(omega, k[n], keq[n], kf[n])
    trace = one(s_b, k[_K20] + k[_K02], keq[_K20] + keq[_K02], kf[_K20] + kf[_K02])
    diff = one(omega, k[_K20] - k[_K02], keq[_K20] - keq[_K02], kf[_K20] - kf[_K02])
    out[_K20] = 0.5 * (trace + diff)
    out[_K02] = 0.5 * (trace - diff)
    out[_K11] = one(omega, k[_K11], keq[_K11], kf[_K11])
    out[_K21] = one(s_3, k[_K21], keq[_K21], kf[_K21])
    out[_K12] = one(s_3, k[_K12], keq[_K12], kf[_K12])
    out[_K22] = one(s_4, k[_K22], keq[_K22], kf[_K22])
    return out


def guo_term(ux, uy, fx, fy) -> np.ndarray:
    """Guo's source without its (1 - omega/2) factor: w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F."""
    from .lbm import CS2, W
    C = _lattice()
    out = np.empty((9,) + np.shape(ux))
    for i in range(9):
        cx, cy = C[i]
        cu = cx * ux + cy * uy
        out[i] = W[i] * (((cx - ux) / CS2 + cu * cx / (CS2 * CS2)) * fx
                         + ((cy - uy) / CS2 + cu * cy / (CS2 * CS2)) * fy)
    return out


def collide(ch, f: np.ndarray) -> np.ndarray:
    """Central-moment relaxation with Guo forcing on the fluid cells; solid cells stay zero.

    ch.collision = (s_b, s_3, s_4); the shear rate is 1/ch.tau."""
    from .lbm import density, equilibrium, momentum, relaxation_time, solid_mask
    s_b, s_3, s_4 = ch.collision
    solid = solid_mask(ch)
    rho = density(f)
    rho_safe = np.where(solid, 1.0, rho)
    jx, jy = momentum(f)
    ux = (jx + 0.5 * ch.force_x) / rho_safe
    uy = jy / rho_safe
    k = central_moments(f, ux, uy)
    keq = central_moments(equilibrium(rho_safe, ux, uy), ux, uy)
    kf = central_moments(guo_term(ux, uy, ch.force_x, 0.0), ux, uy)  # weighted per rate in relax
    fout = populations(relax(k, keq, kf, 1.0 / relaxation_time(ch), s_b, s_3, s_4), ux, uy)
    fout[:, solid] = 0.0
    return fout
