"""Perturbation of a branched trajectory (paper Appendix D), FP64.

Test infrastructure (see ``oracle/__init__``).

The populations of the new trajectory are shifted by a random positive
combination of N_s snapshots of the flow,
    f_i(x) -> f_i(x) + eps * sum_n alpha_n f_i^(n)(x),   alpha_n ~ U[0, 1],
and then multiplied by one scalar so that the total mass of the trajectory is
what it was before the shift (Appendix D; eps = 0.002 and N_s = 10 there).
The mass is the sum of f_i over every fluid cell and direction.

The alpha_n come from the PRTB Philox stream at counter (slot, period, n // 4),
word n % 4 (see ``oracle.philox``).
"""
from __future__ import annotations

import math

import numpy as np

from . import philox


def alphas(key: int, slot: int, period: int, n_snap: int) -> np.ndarray:
    """alpha_1..alpha_Ns in [0, 1) for one branched trajectory."""
    out = np.empty(n_snap)
    for n in range(n_snap):
        w = philox.philox4x64_10((slot, period, n // 4, 0), (key, philox.PRTB))[n % 4]
        out[n] = philox.uniform53(w)
    return out


def total_mass(f: np.ndarray, fluid: np.ndarray) -> float:
    """Sum of all populations over fluid cells, correctly rounded."""
    return math.fsum(f[:, fluid].ravel().tolist())


def perturb(f: np.ndarray, snapshots: np.ndarray, alpha: np.ndarray, eps: float,
            fluid: np.ndarray) -> np.ndarray:
    """Shift f by eps * sum_n alpha_n snapshots[n], then rescale to the old mass.

    f: [9, ny, nx] full populations; snapshots: [N_s, 9, ny, nx] full
    populations; fluid: bool [ny, nx].
    """
    m_before = total_mass(f, fluid)
    g = f.copy()
    for n in range(len(alpha)):
        g = g + eps * alpha[n] * snapshots[n]
    m_after = total_mass(g, fluid)
    g = g * (m_before / m_after)
    g[:, ~fluid] = 0.0
    return g
