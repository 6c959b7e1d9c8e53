"""Pins for the near-wake feature patch: block means of known fields."""
import numpy as np

from oracle import features, lbm


def test_uniform_flow_features():
    ch = lbm.Channel(64, 32, 0.6, 2e-5, (4, 12, 4))
    rho, ux, uy = 1.003, 0.04, -0.01
    f = lbm.equilibrium(np.full((32, 64), rho), np.full((32, 64), ux), np.full((32, 64), uy))
    # post-collision momentum carries the force on top of rho u - F/2 ... build it directly
    f_out = lbm.collide(ch, lbm.equilibrium(np.full((32, 64), rho), np.full((32, 64), ux - 0.5 * 2e-5 / rho),
                                            np.full((32, 64), uy)))
    feat = features.near_wake(ch, f_out, px0=16, py0=0, patch=32, pool=4, u_scale=10.0, rho_scale=100.0)
    assert feat.shape == (3, 8, 8)
    assert np.allclose(feat[0], ux * 10, rtol=1e-12)
    assert np.allclose(feat[1], uy * 10, rtol=1e-12)
    assert np.allclose(feat[2], (rho - 1) * 100, rtol=1e-9)
    assert f.shape == (9, 32, 64)


def test_pooling_is_block_mean():
    ch = lbm.Channel(16, 16, 0.6, 0.0, None)
    rng = np.random.default_rng(0)
    rho = 1 + 0.01 * rng.standard_normal((16, 16))
    ux = 0.01 * rng.standard_normal((16, 16))
    f = lbm.equilibrium(rho, ux, 0 * ux)
    feat = features.near_wake(ch, f, 0, 0, 16, 4, 1.0, 1.0)
    assert np.isclose(feat[0, 1, 2], ux[4:8, 8:12].mean(), rtol=1e-12)
    assert np.isclose(feat[2].mean(), (rho - 1).mean(), rtol=1e-10)
