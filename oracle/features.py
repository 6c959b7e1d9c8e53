"""Near-wake feature patch for the learned score, FP64.

Test infrastructure (see ``oracle/__init__``).

The learned score sees a coarse picture of the flow just behind the square,
where the paper locates the vortex responsible for extreme drag (Section 3.2):
the fields (u_x, u_y, rho - 1) on a P x P cell patch whose lower-left cell is
(px0, py0), averaged over non-overlapping pool x pool blocks and multiplied
by the given scales.  Density and velocity are those of the step the
post-collision populations belong to (see
``lbm.velocity_from_post_collision``).  Output [3, P/pool, P/pool], channel
order (u_x, u_y, rho - 1), row = y.
"""
from __future__ import annotations

import numpy as np

from . import lbm


def near_wake(ch: lbm.Channel, fout: np.ndarray, px0: int, py0: int, patch: int, pool: int,
              u_scale: float, rho_scale: float) -> np.ndarray:
    rho, ux, uy = lbm.velocity_from_post_collision(ch, fout)
    sl = (slice(py0, py0 + patch), slice(px0, px0 + patch))
    fields = [ux[sl] * u_scale, uy[sl] * u_scale, (rho[sl] - 1.0) * rho_scale]
    n = patch // pool
    out = np.empty((3, n, n))
    for c, fld in enumerate(fields):
        out[c] = fld.reshape(n, pool, n, pool).mean(axis=(1, 3))
    return out
