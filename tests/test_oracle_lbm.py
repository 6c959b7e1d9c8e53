"""Pins for the LBM oracle: closed forms, conservation laws and symmetries.

None of these re-types an oracle formula: each checks a property the paper's
scheme (Appendix A) or the mathematics fixes, chosen so that a plausible slip
(a dropped term, a wrong sign or index, a transposed direction) fails one.
"""
import math

import numpy as np
import pytest

from oracle import lbm


def _fluid(ch):
    return ~lbm.solid_mask(ch)


def test_lattice_isotropy():
    # D2Q9 moments: sum w = 1, sum w c = 0, sum w c c = cs^2 I, 4th moment isotropic
    c, w = lbm.C.astype(float), lbm.W
    assert math.isclose(w.sum(), 1.0, rel_tol=0, abs_tol=1e-15)
    assert np.allclose(w @ c, 0.0, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(2) / 3, atol=1e-15)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(2)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(m4, iso, atol=1e-15)
    assert all(np.array_equal(lbm.C[lbm.OPP[i]], -lbm.C[i]) for i in range(9))


def test_equilibrium_moments():
    rng = np.random.default_rng(1)
    rho = 1 + 0.01 * rng.standard_normal(50)
    ux, uy = 0.05 * rng.standard_normal(50), 0.05 * rng.standard_normal(50)
    feq = lbm.equilibrium(rho, ux, uy)
    c = lbm.C.astype(float)
    assert np.allclose(feq.sum(0), rho, rtol=0, atol=1e-15)
    assert np.allclose(np.einsum("i,in->n", c[:, 0], feq), rho * ux, atol=1e-15)
    assert np.allclose(np.einsum("i,in->n", c[:, 1], feq), rho * uy, atol=1e-15)
    pxx = np.einsum("i,i,in->n", c[:, 0], c[:, 0], feq)
    pxy = np.einsum("i,i,in->n", c[:, 0], c[:, 1], feq)
    pyy = np.einsum("i,i,in->n", c[:, 1], c[:, 1], feq)
    assert np.allclose(pxx, rho / 3 + rho * ux * ux, atol=1e-15)
    assert np.allclose(pxy, rho * ux * uy, atol=1e-15)
    assert np.allclose(pyy, rho / 3 + rho * uy * uy, atol=1e-15)


def test_guo_source_moments():
    rng = np.random.default_rng(2)
    ux, uy = 0.05 * rng.standard_normal(20), 0.05 * rng.standard_normal(20)
    fx, fy, tau = 3e-6, -2e-6, 0.53
    src = lbm.guo_source(ux, uy, fx, fy, tau)
    c = lbm.C.astype(float)
    g = 1 - 1 / (2 * tau)
    assert np.allclose(src.sum(0), 0.0, atol=1e-20)
    assert np.allclose(np.einsum("i,in->n", c[:, 0], src), g * fx, rtol=1e-12, atol=0)
    assert np.allclose(np.einsum("i,in->n", c[:, 1], src), g * fy, rtol=1e-12, atol=0)
    # second moment: (1 - 1/2tau)(u F + F u)
    pxy = np.einsum("i,i,in->n", c[:, 0], c[:, 1], src)
    assert np.allclose(pxy, g * (ux * fy + uy * fx), rtol=1e-10, atol=1e-22)


def _noisy_channel(nx=64, ny=16, square=(20, 5, 4), tau=0.56, force=2e-5, seed=3):
    ch = lbm.Channel(nx, ny, tau, force, square)
    rho = lbm.init_density(ch, seed, 0, 1e-2)
    return ch, lbm.init_populations(ch, rho)


def test_mass_conserved():
    ch, f = _noisy_channel()
    fl = _fluid(ch)
    m0 = math.fsum(f[:, fl].ravel())
    for _ in range(200):
        f = lbm.stream(ch, lbm.collide(ch, f))
    m1 = math.fsum(f[:, fl].ravel())
    assert abs(m1 - m0) <= 2e-13 * m0


def _wall_force(ch, fout):
    # x-momentum handed to the top/bottom walls: every population leaving the
    # channel through y = 0 or y = ny carries 2 c_x f back
    tot = []
    for i in range(1, 9):
        cx, cy = lbm.C[i]
        if cy == 0 or cx == 0:
            continue
        row = 0 if cy < 0 else ch.ny - 1
        vals = fout[i, row, :][_fluid(ch)[row, :]]
        tot.extend((2.0 * cx * vals).tolist())
    return math.fsum(tot)


def test_momentum_balance_pins_drag():
    """P_x(t+1) = P_x(t) + N_fluid F - drag(t) - wall(t): fixes the drag's sign, links and timing."""
    ch, f = _noisy_channel()
    fl = _fluid(ch)
    nf = int(fl.sum())
    c = lbm.C[:, 0].astype(float)
    for _ in range(100):
        px0 = math.fsum((c[:, None] * f[:, fl]).ravel())
        fo = lbm.collide(ch, f)
        d = lbm.drag(ch, fo)
        fw = _wall_force(ch, fo)
        f = lbm.stream(ch, fo)
        px1 = math.fsum((c[:, None] * f[:, fl]).ravel())
        assert abs(px1 - (px0 + nf * ch.force_x - d - fw)) < 1e-14


def _poiseuille(h, tau, force):
    nu = (tau - 0.5) / 3
    j = np.arange(h)
    return force / (2 * nu) * (j + 0.5) * (h - j - 0.5) + force * (16 * (tau - 0.5) ** 2 - 3) / (8 * (tau - 0.5))


@pytest.mark.parametrize("tau", [0.6, 0.5 + math.sqrt(3 / 16), 1.0])
def test_poiseuille_exact_steady_state(tau):
    """Obstacle-free channel: the discrete steady state is the parabola plus the BGK slip."""
    h, force = 16, 1e-5
    ch = lbm.Channel(2, h, tau, force, None)
    ua = _poiseuille(h, tau, force)
    ones = np.ones((h, 2))
    f = lbm.equilibrium(ones, np.repeat(ua[:, None], 2, 1) - 0.5 * force, 0 * ones)
    # the start lacks the non-equilibrium part; its transient decays on the
    # slowest viscous mode, exp(-pi^2 nu t / h^2): run 18 e-folds
    n_steps = int(18 * h * h / (math.pi ** 2 * ch.nu))
    for _ in range(n_steps):
        f = lbm.stream(ch, lbm.collide(ch, f))
    rho, u, v = lbm.velocity_from_post_collision(ch, lbm.collide(ch, f))
    assert np.abs(u[:, 0] - ua).max() < 1e-8 * ua.max()
    assert np.abs(v).max() < 1e-11 * ua.max()  # round-off only
    assert np.abs(rho - 1).max() < 1e-11  # mass round-off over ~1e4 steps


def test_poiseuille_without_slip_term_drifts():
    """Sensitivity of the pin above: the plain parabola (no slip) is not a fixed point."""
    h, force, tau = 16, 1e-5, 0.6
    ch = lbm.Channel(2, h, tau, force, None)
    nu = (tau - 0.5) / 3
    j = np.arange(h)
    ua = force / (2 * nu) * (j + 0.5) * (h - j - 0.5)
    ones = np.ones((h, 2))
    f = lbm.equilibrium(ones, np.repeat(ua[:, None], 2, 1) - 0.5 * force, 0 * ones)
    for _ in range(3000):
        f = lbm.stream(ch, lbm.collide(ch, f))
    _, u, _ = lbm.velocity_from_post_collision(ch, lbm.collide(ch, f))
    assert np.abs(u[:, 0] - ua).max() > 1e-4 * ua.max()


def test_rest_state_invariant():
    # full populations: sum w_i rounds in FP64, so rest holds to round-off only
    ch = lbm.Channel(32, 12, 0.51, 0.0, (10, 4, 4))
    f0 = lbm.init_populations(ch, np.ones((12, 32)))
    f = f0
    for _ in range(50):
        fo = lbm.collide(ch, f)
        assert abs(lbm.drag(ch, fo)) < 1e-15
        f = lbm.stream(ch, fo)
    assert np.allclose(f, f0, rtol=0, atol=1e-15)


def test_mirror_symmetry_no_lift():
    """No noise, square centred in y: the flow stays mirror-symmetric about the mid-plane."""
    ch = lbm.Channel(48, 20, 0.6, 1e-4, (12, 8, 4))
    f = lbm.init_populations(ch, np.ones((20, 48)))
    mirror = [0, 1, 4, 3, 2, 8, 7, 6, 5]  # c_y -> -c_y
    for _ in range(150):
        fo = lbm.collide(ch, f)
        f = lbm.stream(ch, fo)
    assert np.allclose(f[mirror][:, ::-1, :], f, rtol=0, atol=1e-15)
    # lift (y-force) by momentum exchange vanishes
    lift = math.fsum(2.0 * lbm.C[i, 1] * v for i, m in lbm.square_links(ch) for v in fo[i][m])
    assert abs(lift) < 1e-15


def test_translation_invariance_bitexact():
    """Shifting square and initial density along periodic x gives the same drag series."""
    ch_a, f_a = _noisy_channel(square=(20, 5, 4))
    shift = 13
    ch_b = lbm.Channel(ch_a.nx, ch_a.ny, ch_a.tau, ch_a.force_x, (20 + shift, 5, 4))
    f_b = np.roll(f_a, shift, axis=2)
    _, da = lbm.run(ch_a, f_a, 60)
    _, db = lbm.run(ch_b, f_b, 60)
    assert np.array_equal(da, db)


def test_drag_positive_in_forced_flow():
    ch = lbm.Channel(64, 16, 0.6, 1e-5, (20, 6, 4))
    f = lbm.init_populations(ch, np.ones((16, 64)))
    _, d = lbm.run(ch, f, 400)
    assert np.all(d > 0)
    assert d[-1] > d[100]


def test_init_noise_statistics():
    ch = lbm.Channel(64, 32, 0.6, 0.0, (10, 10, 4))
    rho = lbm.init_density(ch, seed=9, member=2, amp=1e-3)
    fl = _fluid(ch)
    v = (rho[fl] - 1) / 1e-3
    assert v.min() >= -1 and v.max() < 1
    assert abs(v.mean()) < 0.06  # uniform on [-1, 1): sd of mean ~ 0.58/sqrt(2032)
    assert abs((v ** 2).mean() - 1 / 3) < 0.03
    other = lbm.init_density(ch, seed=9, member=3, amp=1e-3)
    assert not np.array_equal(rho, other)
    f = lbm.init_populations(ch, rho)
    assert np.allclose(f.sum(0)[fl], rho[fl], atol=1e-15)
    assert np.all(f[:, ~fl] == 0)


def test_uniform_flow_start_moments():
    ch = lbm.Channel(32, 8, 0.6, 0.0, (10, 2, 3))
    rho = 1 + 0.01 * np.random.default_rng(0).random((8, 32))
    f = lbm.init_populations(ch, rho, ux0=0.07)
    fl = ~lbm.solid_mask(ch)
    jx, jy = lbm.momentum(f)
    assert np.allclose(f.sum(0)[fl], rho[fl], atol=1e-15)
    assert np.allclose(jx[fl], 0.07 * rho[fl], atol=1e-15)
    assert np.allclose(jy[fl], 0.0, atol=1e-16)
