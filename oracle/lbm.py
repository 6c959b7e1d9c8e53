"""D2Q9 lattice-BGK channel flow past a square, in FP64 with full populations.

Test infrastructure (see ``oracle/__init__``).

What is computed, and where the paper states it:

* lattice, moments rho = sum f_i, rho u = sum f_i c_i, c_s^2 = 1/3
  (Appendix A, moment definitions and the D2Q9 figure caption);
* exact streaming f_i(x + c_i, t + 1) = f_i^out(x, t) (Appendix A, streaming
  equation), written here in pull form;
* BGK relaxation towards the second-order equilibrium with weights 4/9, 1/9,
  1/36 (Appendix A, collision and equilibrium equations).  The printed
  collision equation lacks the leading f_i term; the reading used is
  f_i^out = f_i - (f_i - f_i^eq)/tau, the standard BGK form the viscosity
  relation nu = (tau - 1/2) c_s^2 belongs to;
* halfway bounce-back no-slip on the channel walls and on the square
  (Section 2, boundary conditions);
* a uniform body force density F = (g_x, 0) replaces the paper's inlet (the
  periodic, force-driven channel is the benchmark workload).  It enters
  by Guo's scheme: u = (sum f_i c_i + F/2)/rho in the equilibrium, and the
  source term (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F is
  added after relaxation;
* drag = x-force on the square.  The paper defines it as the surface
  integral of the stress (Section 2.1, drag definition); with halfway
  bounce-back the exact momentum handed to the square per step is the
  momentum-exchange sum over cut links, 2 c_ix f_i^out(x) for every fluid
  cell x and direction i with x + c_i inside the square.

Conventions (the paper's D2Q9 figure is missing, so the numbering is ours):
directions c_0..c_8 = (0,0), (1,0), (0,1), (-1,0), (0,-1), (1,1), (-1,1),
(-1,-1), (1,-1).  Arrays are indexed [i, y, x].  Cell (x, y) is the unit
square [x, x+1) x [y, y+1); the walls sit half way between the first/last
row and the ghost rows y = -1 and y = ny; x is periodic.  The square with
side s and lower-left cell (x0, y0) occupies cells x0..x0+s-1, y0..y0+s-1.
Solid cells carry no populations (zeros) and are excluded from every sum.

Step indexing: the state at time 0 is the equilibrium at rest with the
seeded density; step t is collide(t) -> drag(t) -> stream -> state(t+1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from functools import lru_cache
from typing import Optional, Tuple

import numpy as np

from . import philox

# D2Q9 velocity set, weights, opposite directions (Appendix A)
C = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
              (1, 1), (-1, 1), (-1, -1), (1, -1)], dtype=np.int64)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6], dtype=np.int64)
CS2 = 1.0 / 3.0


@dataclass(frozen=True)
class Channel:
    """One trajectory's geometry and parameters (lattice units)."""
    nx: int
    ny: int
    tau: float
    force_x: float
    square: Optional[Tuple[int, int, int]] = None  # (x0, y0, side) of the solid block
    # None: BGK.  (s_b, s_3, s_4): central-moment relaxation (``oracle.central_moments``)
    collision: Optional[Tuple[float, float, float]] = None
    # None: periodic x.  An ``oracle.open_channel.OpenChannel``: inlet, grid, sponge, outlet
    open: Optional[object] = None

    @property
    def nu(self) -> float:
        """Kinematic viscosity nu = (tau - 1/2) c_s^2 (Appendix A)."""
        return (self.tau - 0.5) * CS2


@lru_cache(maxsize=32)
def _square(ch: Channel) -> np.ndarray:
    m = np.zeros((ch.ny, ch.nx), dtype=bool)
    if ch.square is not None and ch.square[2] > 0:
        x0, y0, s = ch.square
        m[y0:y0 + s, x0:x0 + s] = True
    m.setflags(write=False)
    return m


@lru_cache(maxsize=32)
def _solid(ch: Channel) -> np.ndarray:
    m = _square(ch).copy()
    if ch.open is not None:
        from .open_channel import grid_mask
        m |= grid_mask(ch.ny, ch.nx, ch.open)
    m.setflags(write=False)
    return m


def square_mask(ch: Channel) -> np.ndarray:
    """Boolean [ny, nx]: True on the cells of the square, the body whose drag is measured."""
    return _square(ch)


def solid_mask(ch: Channel) -> np.ndarray:
    """Boolean [ny, nx]: True on every solid cell (the square and, in an open channel, the
    entrance grid's bars); read-only, cached."""
    return _solid(ch)


def relaxation_time(ch: Channel):
    """tau, or the [ny, nx] field of an open channel's sponge zone."""
    if ch.open is None:
        return ch.tau
    from .open_channel import tau_field
    return tau_field(ch)


def equilibrium(rho, ux, uy):
    """Second-order equilibrium f_i^eq(rho, u) on any array shape (Appendix A)."""
    usq = ux * ux + uy * uy
    feq = np.empty((9,) + np.shape(rho))
    for i in range(9):
        cu = C[i, 0] * ux + C[i, 1] * uy
        feq[i] = W[i] * rho * (1.0 + cu / CS2 + cu * cu / (2 * CS2 * CS2) - usq / (2 * CS2))
    return feq


def guo_source(ux, uy, fx, fy, tau):
    """Guo forcing term F_i added after relaxation (second-order body force)."""
    src = np.empty((9,) + np.shape(ux))
    for i in range(9):
        cx, cy = C[i]
        cu = cx * ux + cy * uy
        term = ((cx - ux) / CS2 + cu * cx / (CS2 * CS2)) * fx \
            + ((cy - uy) / CS2 + cu * cy / (CS2 * CS2)) * fy
        src[i] = (1.0 - 1.0 / (2.0 * tau)) * W[i] * term
    return src


def density(f):
    return f.sum(axis=0)


def momentum(f):
    jx = np.tensordot(C[:, 0].astype(np.float64), f, axes=(0, 0))
    jy = np.tensordot(C[:, 1].astype(np.float64), f, axes=(0, 0))
    return jx, jy


def collide(ch: Channel, f: np.ndarray) -> np.ndarray:
    """BGK relaxation with Guo forcing on the fluid cells; solid cells stay zero.

    A channel with ``collision`` set relaxes in central moments instead."""
    if ch.collision is not None:
        from . import central_moments
        return central_moments.collide(ch, f)
    solid = solid_mask(ch)
    rho = density(f)
    rho_safe = np.where(solid, 1.0, rho)
    jx, jy = momentum(f)
    ux = (jx + 0.5 * ch.force_x) / rho_safe
    uy = (jy + 0.0) / rho_safe
    feq = equilibrium(rho_safe, ux, uy)
    tau = relaxation_time(ch)
    src = guo_source(ux, uy, ch.force_x, 0.0, tau)
    fout = f - (f - feq) / tau + src
    fout[:, solid] = 0.0
    return fout


@lru_cache(maxsize=32)
def square_links(ch: Channel):
    """Tuple of (i, mask[ny, nx]) with mask True where fluid x has x + c_i in the square."""
    solid = square_mask(ch)
    links = []
    for i in range(1, 9):
        cx, cy = C[i]
        target = np.zeros_like(solid)
        # target[y, x] = solid[y + cy, x + cx], with y out of range meaning "not square"
        ys = np.arange(ch.ny) + cy
        valid = (ys >= 0) & (ys < ch.ny)
        xs = (np.arange(ch.nx) + cx) % ch.nx
        target[valid, :] = solid[ys[valid]][:, xs]
        links.append((i, target & ~solid))
    return tuple(links)


def drag(ch: Channel, fout: np.ndarray) -> float:
    """Momentum-exchange x-force on the square from post-collision populations.

    Each population leaving a fluid cell towards the square comes back reversed,
    handing the square 2 c_ix f_i^out.  Summed with ``math.fsum`` (correctly
    rounded, hence independent of the order of the links).
    """
    terms = []
    for i, mask in square_links(ch):
        if C[i, 0] != 0:
            terms.extend((2.0 * C[i, 0] * fout[i][mask]).tolist())
    return math.fsum(terms)


@lru_cache(maxsize=32)
def stream_sources(ch: Channel):
    """For every direction i: (direction, flat cell) each f_i(x, t+1) is pulled from.

    f_i(x, t+1) = f_i^out(x - c_i, t) when x - c_i is a fluid cell inside the
    channel; otherwise the population that left x towards the wall comes
    back: f_i(x, t+1) = f_{opp(i)}^out(x, t).
    """
    solid = solid_mask(ch)
    ny, nx = ch.ny, ch.nx
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    own = (yy * nx + xx).ravel()
    out = []
    for i in range(9):
        cx, cy = C[i]
        xs = (xx - cx) % nx
        ys = yy - cy
        inside = (ys >= 0) & (ys < ny)
        ys_c = np.clip(ys, 0, ny - 1)
        bounce = (~inside | solid[ys_c, xs]).ravel()
        src_dir = np.where(bounce, OPP[i], i)
        src_cell = np.where(bounce, own, (ys_c * nx + xs).ravel())
        out.append((src_dir, src_cell))
    return tuple(out)


def stream(ch: Channel, fout: np.ndarray) -> np.ndarray:
    """Pull streaming with periodic x and halfway bounce-back at walls and square
    (an open channel streams through its inlet and outlet instead)."""
    if ch.open is not None:
        from . import open_channel
        return open_channel.stream(ch, fout)
    flat = fout.reshape(9, -1)
    fnew = np.empty_like(fout)
    for i, (src_dir, src_cell) in enumerate(stream_sources(ch)):
        fnew[i] = flat[src_dir, src_cell].reshape(ch.ny, ch.nx)
    fnew[:, solid_mask(ch)] = 0.0
    return fnew


def init_density(ch: Channel, seed: int, member: int, amp: float) -> np.ndarray:
    """rho(x) = 1 + amp (2u - 1) with u from the INIT Philox stream; 1 on solid cells.

    The counter is (y*nx + x, member); the seeded +-amp noise is the
    workload's initial perturbation (the paper starts from equilibrium).
    """
    rho = np.ones((ch.ny, ch.nx))
    if amp == 0.0:
        return rho
    for y in range(ch.ny):
        for x in range(ch.nx):
            w = philox.philox4x64_10((y * ch.nx + x, member, 0, 0), (seed, philox.INIT))[0]
            rho[y, x] = 1.0 + amp * (2.0 * philox.uniform53(w) - 1.0)
    return rho


def init_populations(ch: Channel, rho: np.ndarray, ux0: float = 0.0) -> np.ndarray:
    """Equilibrium with density rho and uniform velocity (ux0, 0): f_i = f_i^eq(rho, u0)
    (w_i rho at rest); zeros on solid cells."""
    if ux0 == 0.0:
        f = (W[:, None, None] * rho[None, :, :]).copy()
    else:
        f = equilibrium(rho, np.full_like(rho, ux0), np.zeros_like(rho))
    f[:, solid_mask(ch)] = 0.0
    return f


def run(ch: Channel, f0: np.ndarray, n_steps: int):
    """Run n_steps steps from pre-collision state f0.

    Returns (fout, drags): the post-collision populations of the last step and
    the drag of each step t = 0..n_steps-1.
    """
    f = f0
    drags = np.empty(n_steps)
    fout = None
    for t in range(n_steps):
        fout = collide(ch, f)
        drags[t] = drag(ch, fout)
        if t + 1 < n_steps:
            f = stream(ch, fout)
    return fout, drags


def velocity_from_post_collision(ch: Channel, fout: np.ndarray):
    """Physical (rho, u_x, u_y) of a step, recovered from its post-collision populations.

    Relaxation conserves mass and adds F to the momentum, so
    rho = sum f_i^out and u = (sum c_i f_i^out - F/2) / rho equal the
    pre-collision density and the Guo-shifted velocity of that step.
    """
    solid = solid_mask(ch)
    rho = density(fout)
    rho_safe = np.where(solid, 1.0, rho)
    jx, jy = momentum(fout)
    ux = (jx - 0.5 * ch.force_x) / rho_safe
    uy = jy / rho_safe
    ux[solid] = 0.0
    uy[solid] = 0.0
    return rho_safe, ux, uy
