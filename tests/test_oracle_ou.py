"""Pins for the OU helpers: exact AR(1) moments against Monte Carlo and the continuum."""
import math

import numpy as np

from oracle import ou


def test_stationary_variance_and_autocorrelation():
    rng = np.random.default_rng(1)
    p = ou.paths(ou.stationary(20000, rng), 50, 0.1, rng)
    assert abs(p[:, -1].var() - 0.5) < 0.02
    c = np.mean(p[:, -1] * p[:, -11]) / 0.5
    assert abs(c - math.exp(-1.0)) < 0.03


def test_sum_variance_monte_carlo_and_continuum_limit():
    rng = np.random.default_rng(2)
    dt, m = 0.05, 60
    p = ou.paths(ou.stationary(40000, rng), m, dt, rng)
    mc = (p.sum(axis=1) * dt).var()
    assert abs(mc / ou.sum_variance(m, dt) - 1) < 0.03
    t = 3.0
    fine = ou.sum_variance(int(t / 1e-3), 1e-3)
    assert abs(fine / ou.integral_variance(t) - 1) < 2e-3
