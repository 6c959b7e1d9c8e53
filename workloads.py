"""Workload definitions and seeded synthetic inputs shared by tests, bench and smoke.

This module holds no arithmetic of the method: only geometry and parameter
tables of the channel-flow ensembles, and seeded generators for inputs that
the method does not draw itself (random log-weights, score series, network
parameters, feature batches).  Both the HIP path and the oracle receive
these values from here; neither imports the other.

Geometry readings (the paper's flow uses an inlet; these workloads use a
periodic channel driven by a body force):
* ny rows of fluid between halfway walls at y = 0 and y = ny, periodic x;
* an s x s square "centred at (cx, cy)" occupies cells cx - s/2 .. cx + s/2 - 1
  in x and likewise in y;
* where no body force is given, F = 8 nu u_c / ny^2 with u_c = 0.05 (the
  paper's inlet centre-line velocity), the force that would drive a plane
  Poiseuille flow with that centre-line speed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class Member:
    nx: int
    ny: int
    tau: float
    force_x: float
    square: Optional[Tuple[int, int, int]]  # (x0, y0, side) lower-left solid cell and side

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    @property
    def fluid_cells(self) -> int:
        s = self.square[2] if self.square else 0
        return self.nx * self.ny - s * s


def centred_square(cx: int, cy: int, side: int) -> Tuple[int, int, int]:
    return (cx - side // 2, cy - side // 2, side)


def poiseuille_force(tau: float, ny: int, u_c: float = 0.05) -> float:
    nu = (tau - 0.5) / 3.0
    return 8.0 * nu * u_c / (ny * ny)


@dataclass
class Workload:
    name: str
    members: List[Member]
    steps: int
    seed: int
    noise_amp: float = 1e-3
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return sum(m.cells for m in self.members)


def single_channel() -> Workload:
    """One trajectory, 256 x 64, square 8 centred at (64, 32), tau 0.55, g_x 1e-6, 2000 steps."""
    m = Member(256, 64, 0.55, 1e-6, centred_square(64, 32, 8))
    return Workload("single 256x64 tau0.55", [m], 2000, seed=1)


def ensemble_1024(n_members: int = 128, steps: int = 10_000) -> Workload:
    """128 trajectories of 1024 x 256, square 32 centred at (256, 128), tau 0.5015, g_x 3e-6."""
    m = Member(1024, 256, 0.5015, 3e-6, centred_square(256, 128, 32))
    return Workload(f"ensemble {n_members}x1024x256 tau0.5015", [m] * n_members, steps, seed=2)


def gktl_ensemble(n_members: int = 256) -> Workload:
    """GKTL: 256 clones on the 1024 x 256 channel; period 256 steps, window 2048, T_a 6144."""
    m = Member(1024, 256, 0.5015, 3e-6, centred_square(256, 128, 32))
    return Workload(f"gktl {n_members}x1024x256", [m] * n_members, 6144, seed=100,
                    extra=dict(period=256, window=2048, t_a=6144, ks=(0.5, 1.0, 2.0),
                               dt=1.0 / 512.0, eps=0.002, n_snap=10))


def ams_ensemble(n_members: int = 512) -> Workload:
    """AMS: 512 members on 512 x 128, square 16 centred at (128, 64), tau 0.502."""
    tau = 0.502
    m = Member(512, 128, tau, poiseuille_force(tau, 128), centred_square(128, 64, 16))
    return Workload(f"ams {n_members}x512x128", [m] * n_members, 2560, seed=200,
                    extra=dict(window=512, patch=64, pool=4, eps=0.002, n_snap=10))


def mixed_sizes(per_size: int = 64, steps: int = 20_000, seed: int = 5) -> Workload:
    """64 trajectories each on 256x64, 512x128, 1024x256; side ny/8 at (nx/4, ny/2);
    tau uniform in [0.501, 0.52] per member (seeded); g_x from the Poiseuille rule."""
    rng = np.random.default_rng(seed)
    members = []
    for nx in (256, 512, 1024):
        ny = nx // 4
        for _ in range(per_size):
            tau = float(rng.uniform(0.501, 0.52))
            members.append(Member(nx, ny, tau, poiseuille_force(tau, ny),
                                  centred_square(nx // 4, ny // 2, ny // 8)))
    return Workload(f"mixed {per_size}x(256x64,512x128,1024x256)", members, steps, seed=seed)


@dataclass(frozen=True)
class OpenParams:
    """Open channel: inlet centre-line velocity, grid bars (first column, size; 0 = none),
    sponge (last column before the ramp, relaxation time at the outlet)."""
    u_c: float
    grid_x0: int
    bar: int
    sponge_x0: int
    sponge_tau: float
    outlet_rho: int = 0  # outlet density: 0 held at 1, 1 extrapolated to second order


def open_channel(n_members: int = 1024) -> Workload:
    """The paper's flow (Section 2): 512 x 128 cells (513 x 129 mesh points), square R = 16 at
    the centre, entrance grid of bars R/2 from x = 32, inlet centre-line velocity 0.05, sponge over
    the last 64 columns rising to tau 1; tau 0.501 (Re_grid = u_c R/2 / nu = 1200), no body
    force; meant for the central-moment collision with unit higher-order rates."""
    m = Member(512, 128, 0.501, 0.0, centred_square(256, 64, 16))
    return Workload(f"open channel {n_members}x512x128", [m] * n_members, 2000, seed=300,
                    extra=dict(open=OpenParams(0.05, 32, 8, 447, 1.0), rates=(1.0, 1.0, 1.0)))


# ----------------------------------------------------------------------------
# seeded inputs the method does not draw itself

def log_weights(n: int, seed: int, scale: float = 3.0, n_bad: int = 0) -> np.ndarray:
    """Random GKTL period log-weights s_n; the first n_bad entries set to NaN."""
    rng = np.random.default_rng(seed)
    s = rng.standard_normal(n) * scale
    s[:n_bad] = np.nan
    return s


def score_series(n: int, t_len: int, seed: int) -> np.ndarray:
    """Random-walk score series [n, t_len] (float32), distinct maxima almost surely."""
    rng = np.random.default_rng(seed)
    steps = rng.standard_normal((n, t_len)).astype(np.float32)
    return np.cumsum(steps, axis=1, dtype=np.float32) * np.float32(0.1)


def cnn_params(seed: int, c_in: int = 3, ch: int = 32) -> dict:
    """He-style random parameters of the score network (FP64)."""
    rng = np.random.default_rng(seed)
    shp = {"w1": (ch, c_in, 3, 3), "b1": (ch,), "w2": (ch, ch, 3, 3), "b2": (ch,),
           "w3": (ch, ch, 3, 3), "b3": (ch,), "w4": (ch,), "b4": ()}
    p = {}
    for name, s in shp.items():
        if name.startswith("w"):
            fan_in = int(np.prod(s[1:])) if len(s) > 1 else s[0]
            p[name] = rng.standard_normal(s) * np.sqrt(2.0 / fan_in)
        else:
            p[name] = rng.standard_normal(s) * 0.05
    return p


def cnn_batch(batch: int, seed: int, c_in: int = 3, hw: int = 16):
    """Random feature batch [B, c_in, hw, hw] and labels [B]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((batch, c_in, hw, hw)), rng.standard_normal(batch)


def snapshot_states(n_snap: int, member: Member, seed: int) -> np.ndarray:
    """Arbitrary flow-like snapshots as FP32 deviations [n_snap, 9, ny, nx] (zero in the square):
    d_i = w_i * 1e-3 * (density + 3 c_i.u) with smooth random fields."""
    rng = np.random.default_rng(seed)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
    cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
    out = np.empty((n_snap, 9, member.ny, member.nx), dtype=np.float32)
    yy, xx = np.meshgrid(np.arange(member.ny), np.arange(member.nx), indexing="ij")
    for q in range(n_snap):
        k1, k2, ph = rng.integers(1, 5), rng.integers(1, 5), rng.uniform(0, 2 * np.pi, 3)
        rho = np.sin(2 * np.pi * k1 * xx / member.nx + ph[0]) * np.cos(np.pi * k2 * yy / member.ny + ph[1])
        ux = np.cos(2 * np.pi * k2 * xx / member.nx + ph[2])
        uy = 0.3 * rho
        for i in range(9):
            out[q, i] = (w[i] * 1e-3 * (rho + 3 * (cx[i] * ux + cy[i] * uy))).astype(np.float32)
        if member.square is not None:
            x0, y0, s = member.square
            out[q, :, y0:y0 + s, x0:x0 + s] = 0.0
    return out
