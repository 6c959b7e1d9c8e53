"""Pins for the central-moment collision of the oracle (``oracle.central_moments``).

Each checks a property fixed by the mathematics rather than re-typing the
module: moments are a linear invertible map of the populations, so uniform
rates must give BGK exactly; mass and momentum must not depend on the rates;
the shear rate alone must set the viscosity; and the momentum balance must
still account for the drag exactly.
"""
import math

import numpy as np
import pytest

from oracle import central_moments as cm
from oracle import lbm


def _random_state(n, seed, amp=0.03):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((9, 1, n)) * amp * lbm.W[:, None, None]
    return d + lbm.W[:, None, None]


@pytest.mark.parametrize("tau,force", [(0.53, 2e-5), (0.9, 0.0), (0.5015, 3e-6)])
def test_uniform_rates_are_bgk(tau, force):
    f = _random_state(400, 1)
    bgk = lbm.collide(lbm.Channel(400, 1, tau, force), f)
    cmr = lbm.collide(lbm.Channel(400, 1, tau, force, collision=(1 / tau,) * 3), f)
    assert np.abs(cmr - bgk).max() <= 4e-15


def test_round_trip_moments_populations():
    f = _random_state(50, 2)[:, 0, :]
    ux = np.linspace(-0.1, 0.1, 50)
    uy = np.linspace(0.05, -0.08, 50)
    back = cm.populations(cm.central_moments(f, ux, uy), ux, uy)
    assert np.abs(back - f).max() <= 1e-15


@pytest.mark.parametrize("rates", [(1.0, 1.0, 1.0), (1.4, 0.7, 1.2), (0.3, 1.9, 1.6)])
def test_mass_and_momentum_for_any_rates(rates):
    force = 2e-5
    f = _random_state(300, 3)
    out = lbm.collide(lbm.Channel(300, 1, 0.53, force, collision=rates), f)
    assert np.abs(out.sum(axis=0) - f.sum(axis=0)).max() <= 4e-15  # a few ulps of rho ~ 1
    jx0, jy0 = lbm.momentum(f)
    jx1, jy1 = lbm.momentum(out)
    assert np.abs(jx1 - jx0 - force).max() <= 1e-15  # relaxation hands over exactly F
    assert np.abs(jy1 - jy0).max() <= 1e-15


def test_equilibrium_is_fixed_point():
    """Without force, the equilibrium of its own (rho, u) is left unchanged for any rates."""
    n = 100
    rng = np.random.default_rng(4)
    rho = 1 + 0.01 * rng.standard_normal((1, n))
    ux = 0.05 * rng.standard_normal((1, n))
    uy = 0.05 * rng.standard_normal((1, n))
    feq = lbm.equilibrium(rho, ux, uy)
    out = lbm.collide(lbm.Channel(n, 1, 0.6, 0.0, collision=(1.3, 0.8, 1.7)), feq)
    assert np.abs(out - feq).max() <= 2e-15  # a few ulps of populations ~ 0.45


def test_equilibrium_and_force_central_moments_closed_forms():
    """The central moments of the discrete equilibrium and of Guo's term, in closed form
    (the forms the device collision evaluates)."""
    n = 200
    rng = np.random.default_rng(5)
    rho = 1 + 0.02 * rng.standard_normal(n)
    ux = 0.08 * rng.standard_normal(n)
    uy = 0.08 * rng.standard_normal(n)
    keq = cm.central_moments(lbm.equilibrium(rho, ux, uy), ux, uy)
    z = 0 * rho
    closed = np.array([rho, z, z, rho / 3, rho / 3, z, -rho * ux ** 2 * uy, -rho * ux * uy ** 2,
                       rho / 9 + 3 * rho * ux ** 2 * uy ** 2])
    assert np.abs(keq - closed).max() <= 1e-15
    fx = 3e-5
    kf = cm.central_moments(cm.guo_term(ux, uy, fx, 0.0), ux, uy)
    closed_f = np.array([z, z + fx, z, z, z, z, -2 * ux * uy * fx, fx / 3 - uy ** 2 * fx, 4 * ux * uy ** 2 * fx])
    assert np.abs(kf - closed_f).max() <= 1e-19


@pytest.mark.parametrize("rates", [(1.0, 1.0, 1.0), (1.4, 0.7, 1.2)])
def test_poiseuille_curvature_set_by_shear_rate(rates):
    """Steady forced channel: the second difference of u is -F/nu with nu from tau alone."""
    h, tau, force = 8, 0.8, 1e-5
    ch = lbm.Channel(4, h, tau, force, collision=rates)
    f = lbm.init_populations(ch, np.ones((h, 4)))
    n_steps = int(30 * h * h / (math.pi ** 2 * ch.nu))
    fo = None
    for _ in range(n_steps):
        fo = lbm.collide(ch, f)
        f = lbm.stream(ch, fo)
    rho, u, v = lbm.velocity_from_post_collision(ch, fo)
    col = u[:, 0]
    d2 = col[2:] - 2 * col[1:-1] + col[:-2]
    assert np.abs(d2 + force / ch.nu).max() <= 1e-8 * force / ch.nu
    assert np.abs(v).max() <= 1e-14  # round-off of O(1) populations; an asymmetry would show at O(u)


def test_momentum_balance_pins_drag_central_moments():
    """P_x(t+1) = P_x(t) + N_fluid F - drag(t) - wall(t) with the central-moment collision."""
    ch = lbm.Channel(64, 16, 0.52, 2e-5, (20, 5, 4), collision=(1.0, 1.0, 1.0))
    f = lbm.init_populations(ch, lbm.init_density(ch, 3, 0, 1e-2))
    fl = ~lbm.solid_mask(ch)
    nf = int(fl.sum())
    c = lbm.C[:, 0].astype(float)
    for _ in range(60):
        px0 = math.fsum((c[:, None] * f[:, fl]).ravel())
        fo = lbm.collide(ch, f)
        d = lbm.drag(ch, fo)
        wall = []
        for i in range(1, 9):
            cx, cy = lbm.C[i]
            if cy == 0 or cx == 0:
                continue
            row = 0 if cy < 0 else ch.ny - 1
            wall.extend((2.0 * cx * fo[i, row, :][fl[row, :]]).tolist())
        f = lbm.stream(ch, fo)
        px1 = math.fsum((c[:, None] * f[:, fl]).ravel())
        assert abs(px1 - (px0 + nf * ch.force_x - d - math.fsum(wall))) < 1e-14


def test_central_moments_stay_finite_where_bgk_blows_up():
    """tau close to 1/2 with a sharp start (uniform flow impulsively started around the square):
    BGK turns non-finite within the run, unit higher-order rates keep the flow bounded."""
    kw = dict(nx=128, ny=32, tau=0.5005, force_x=0.0, square=(30, 13, 6))
    rho = np.ones((32, 128))

    def run(ch, steps=600):
        f = lbm.init_populations(ch, rho, ux0=0.08)
        for _ in range(steps):
            f = lbm.stream(ch, lbm.collide(ch, f))
            if not np.all(np.isfinite(f)) or np.abs(f).max() > 1e3:
                return False
        return True

    assert not run(lbm.Channel(**kw))
    assert run(lbm.Channel(**kw, collision=(1.0, 1.0, 1.0)))
