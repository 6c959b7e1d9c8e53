"""Pins for the open channel of the oracle (``oracle.open_channel``): exact mass
accounting of streaming through the inlet and outlet, the developed pressure-driven
channel flow, the moments of the two ghost columns, the grid's geometry and the
sponge ramp."""
import math

import numpy as np

from oracle import lbm
from oracle.open_channel import OpenChannel, grid_mask, inlet_ghost, inlet_velocity, outlet_ghost, tau_field


def _start(ch):
    u0 = inlet_velocity(ch)
    f = lbm.equilibrium(np.ones((ch.ny, ch.nx)), np.repeat(u0[:, None], ch.nx, 1), np.zeros((ch.ny, ch.nx)))
    f[:, lbm.solid_mask(ch)] = 0.0
    return f


def _ghost_mass_balance(ch, fout):
    """Mass gained by one stream: ghost populations pulled in minus populations leaving the
    channel, counted cell by cell from the lattice rules (not from the streaming code)."""
    solid = lbm.solid_mask(ch)
    gin, gout = inlet_ghost(ch), outlet_ghost(ch, fout)
    gained = []
    for y in range(ch.ny):
        for i in range(9):
            cx, cy = lbm.C[i]
            ys = y - cy  # the row a population arriving at (x, y) comes from
            if 0 <= ys < ch.ny:  # (from beyond a wall: the cell's own population bounces back)
                if cx == 1 and not solid[y, 0]:
                    gained.append(gin[i, ys])            # enters at x = 0 from the inlet
                if cx == -1 and not solid[y, ch.nx - 1]:
                    gained.append(gout[i, ys])           # enters at x = nx - 1 from the outlet
            yd = y + cy  # the row a population leaving (x, y) heads for
            if 0 <= yd < ch.ny:  # (into a wall: it comes back and stays inside)
                if cx == -1 and not solid[y, 0]:
                    gained.append(-fout[i, y, 0])        # leaves through the inlet face
                if cx == 1 and not solid[y, ch.nx - 1]:
                    gained.append(-fout[i, y, ch.nx - 1])  # leaves through the outlet face
    return math.fsum(gained)


def test_streaming_mass_accounting():
    ch = lbm.Channel(40, 16, 0.7, 0.0, (20, 5, 4), open=OpenChannel(0.03, 6, 4, 30, 0.9))
    f = _start(ch)
    rng = np.random.default_rng(3)
    f = f * (1 + 0.01 * rng.standard_normal(f.shape))  # any state, not only steady ones
    f[:, lbm.solid_mask(ch)] = 0.0
    fl = ~lbm.solid_mask(ch)
    for _ in range(5):
        fo = lbm.collide(ch, f)
        m_out = math.fsum(fo[:, fl].ravel())
        f = lbm.stream(ch, fo)
        m_new = math.fsum(f[:, fl].ravel())
        assert abs(m_new - (m_out + _ghost_mass_balance(ch, fo))) < 1e-13


def test_developed_channel_flow():
    """No obstacle: the steady flow has one mass flux at every x, the plane-Poiseuille pressure
    gradient dp/dx = -12 nu rho u_mean / H^2 and a parabolic profile."""
    ny, nx, tau, uc = 16, 64, 0.8, 0.02
    ch = lbm.Channel(nx, ny, tau, 0.0, None, open=OpenChannel(uc, 0, 0, nx, tau))
    f = _start(ch)
    for _ in range(5000):
        fo = lbm.collide(ch, f)
        f = lbm.stream(ch, fo)
    rho, ux, uy = lbm.velocity_from_post_collision(ch, fo)
    q = (rho * ux).sum(axis=0)
    assert (q.max() - q.min()) / q.mean() < 1e-7
    nu = (tau - 0.5) / 3
    mid = slice(16, 48)
    slope = np.polyfit(np.arange(nx)[mid], rho.mean(axis=0)[mid], 1)[0] / 3  # dp/dx, p = rho c_s^2
    expect = -12 * nu * (q.mean() / ny) / ny ** 2
    assert abs(slope - expect) < 0.01 * abs(expect)
    y = np.arange(ny) + 0.5
    par = y * (ny - y)
    assert np.abs(ux[:, nx // 2] / ux[:, nx // 2].max() - par / par.max()).max() < 0.005
    assert np.abs(rho[:, -1] - 1).max() < 1e-3  # the outlet holds the density near 1


def test_inlet_ghost_moments():
    ch = lbm.Channel(32, 12, 0.6, 0.0, None, open=OpenChannel(0.05, 0, 0, 32, 0.6))
    g = inlet_ghost(ch)
    y = np.arange(12) + 0.5
    assert np.abs(g.sum(axis=0) - 1).max() < 1e-15
    assert np.abs((lbm.C[:, 0][:, None] * g).sum(axis=0) - 4 * 0.05 * y * (12 - y) / 144).max() < 1e-16
    assert np.abs((lbm.C[:, 1][:, None] * g).sum(axis=0)).max() < 1e-16


def test_outlet_ghost_moments():
    """Last two columns at equilibrium with u_x = U and U - d: the ghost has density 1, velocity
    U + d, and a non-equilibrium xx moment of -2 c_s^2 (tau - 1) d, nothing else."""
    ny, nx, tau, U, d = 8, 20, 0.7, 0.04, 0.002
    ch = lbm.Channel(nx, ny, tau, 0.0, None, open=OpenChannel(0.05, 0, 0, nx, tau))
    fo = np.zeros((9, ny, nx))
    fo[:, :, nx - 1] = lbm.equilibrium(np.full(ny, 1.02), np.full(ny, U), np.zeros(ny))
    fo[:, :, nx - 2] = lbm.equilibrium(np.full(ny, 1.03), np.full(ny, U - d), np.zeros(ny))
    g = outlet_ghost(ch, fo)
    neq = g - lbm.equilibrium(np.ones(ny), np.full(ny, U + d), np.zeros(ny))
    cx, cy = lbm.C[:, 0][:, None], lbm.C[:, 1][:, None]
    assert np.abs(neq.sum(axis=0)).max() < 1e-16
    assert np.abs((cx * neq).sum(axis=0)).max() < 1e-15 and np.abs((cy * neq).sum(axis=0)).max() < 1e-15  # ulps of ~0.4
    assert np.abs((cx * cx * neq).sum(axis=0) - (-2 / 3 * (tau - 1) * d)).max() < 1e-16  # value ~3e-4
    assert np.abs((cx * cy * neq).sum(axis=0)).max() < 1e-16
    assert np.abs((cy * cy * neq).sum(axis=0)).max() < 1e-16


def test_grid_geometry():
    m = grid_mask(128, 64, OpenChannel(0.05, 10, 8, 64, 0.6))
    col = m[:, 10]
    assert m[:, 10:18].all(axis=1).tolist() == col.tolist() and not m[:, 9].any() and not m[:, 18].any()
    assert col.sum() == 64 and not col[:4].any() and not col[124:].any()
    assert (col == col[::-1]).all()  # symmetric about the centre line
    runs = np.diff(np.flatnonzero(np.diff(col.astype(int)))).tolist()
    assert set(runs) == {8}  # bars and gaps of height 8


def test_sponge():
    ch = lbm.Channel(50, 8, 0.55, 0.0, None, open=OpenChannel(0.05, 0, 0, 30, 0.95))
    t = tau_field(ch)[0]
    assert np.all(t[:31] == 0.55) and abs(t[49] - 0.95) < 1e-15 and np.all(np.diff(t[30:]) > 0)
    f = _start(ch)
    same = lbm.Channel(50, 8, 0.55, 0.0, None, open=OpenChannel(0.05, 0, 0, 30, 0.55))
    plain = lbm.Channel(50, 8, 0.55, 0.0, None, open=OpenChannel(0.05, 0, 0, 50, 0.55))
    assert np.array_equal(lbm.collide(same, f), lbm.collide(plain, f))
