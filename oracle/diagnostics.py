"""Pressure, stress and shear on the square's faces, FP64.

Test infrastructure (see ``oracle/__init__``).

The paper defines the drag as the surface integral of the stress tensor over
the obstacle (Section 2.1, drag definition), with the stress of Appendix A
(total stress: -c_s^2 rho delta_ab minus (nu / (tau c_s^2)) sum_i c_ia c_ib
(f_i - f_i^eq), i.e. (1 - 1/(2 tau)) times the non-equilibrium second
moment); it approximates the drag by forebody minus base pressure (Section
2.1, drag approximation), and follows the mean shear du/dy along the top or
bottom face as a precursor of extreme drag (Section 3.2.2, mean shear
definition).  Reading used here (the lattice puts the faces half a cell from
the adjacent fluid cells):

* everything is evaluated on the populations f that the next step collides
  (the pulled populations of the stored state), with u the Guo-shifted
  velocity (sum c_i f_i + F/2) / rho and f^eq the equilibrium of (rho, u);
* a face's value is the sum over the s fluid cells adjacent to it (unit
  length each): front x0 - 1, base x0 + s (rows y0 .. y0+s-1), bottom y0 - 1,
  top y0 + s (columns x0 .. x0+s-1);
* p_fb = sum_front c_s^2 rho, p_base = sum_base c_s^2 rho;
* stress drag = sum over the four faces of tau_xb n_b with n the outward
  normal of the square: sum_front(-tau_xx) + sum_base(tau_xx)
  + sum_top(tau_xy) - sum_bottom(tau_xy);
* mean shear: the velocity vanishes on the face (halfway bounce-back), the
  adjacent cell centre is half a cell away: gamma_top = (1/s) sum_top
  u_x / (1/2), gamma_bottom = (1/s) sum_bottom (-u_x) / (1/2).
"""
from __future__ import annotations

import numpy as np

from . import lbm

FIELDS = ("p_forebody", "p_base", "stress_drag", "shear_top", "shear_bottom")


def face_cells(ch):
    """(front, base, top, bottom) lists of (y, x) cells adjacent to the square's faces."""
    x0, y0, s = ch.square
    front = [(y, x0 - 1) for y in range(y0, y0 + s)]
    base = [(y, x0 + s) for y in range(y0, y0 + s)]
    top = [(y0 + s, x) for x in range(x0, x0 + s)]
    bottom = [(y0 - 1, x) for x in range(x0, x0 + s)]
    return front, base, top, bottom


def cell_fields(ch, f: np.ndarray, y: int, x: int):
    """(rho, u_x, tau_xx, tau_xy) of one cell from its populations f[:, y, x]."""
    g = f[:, y, x]
    rho = float(g.sum())
    jx = float((lbm.C[:, 0] * g).sum())
    jy = float((lbm.C[:, 1] * g).sum())
    ux = (jx + 0.5 * ch.force_x) / rho
    uy = jy / rho
    feq = lbm.equilibrium(np.array(rho), np.array(ux), np.array(uy))
    neq = g - feq
    pxx = float((lbm.C[:, 0] * lbm.C[:, 0] * neq).sum())
    pxy = float((lbm.C[:, 0] * lbm.C[:, 1] * neq).sum())
    visc = 1.0 - 1.0 / (2.0 * ch.tau)
    tau_xx = -lbm.CS2 * rho - visc * pxx
    tau_xy = -visc * pxy
    return rho, ux, tau_xx, tau_xy


def diagnostics(ch, f: np.ndarray) -> np.ndarray:
    """The five face quantities (FIELDS) of the pre-collision populations f [9, ny, nx]."""
    if ch.square is None:
        return np.zeros(len(FIELDS))
    s = ch.square[2]
    front, base, top, bottom = face_cells(ch)
    fr = [cell_fields(ch, f, y, x) for y, x in front]
    ba = [cell_fields(ch, f, y, x) for y, x in base]
    to = [cell_fields(ch, f, y, x) for y, x in top]
    bo = [cell_fields(ch, f, y, x) for y, x in bottom]
    p_fb = sum(lbm.CS2 * c[0] for c in fr)
    p_base = sum(lbm.CS2 * c[0] for c in ba)
    stress = sum(-c[2] for c in fr) + sum(c[2] for c in ba) + sum(c[3] for c in to) - sum(c[3] for c in bo)
    shear_top = sum(c[1] for c in to) / (0.5 * s)
    shear_bottom = sum(-c[1] for c in bo) / (0.5 * s)
    return np.array([p_fb, p_base, stress, shear_top, shear_bottom])
