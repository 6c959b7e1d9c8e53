"""Ornstein-Uhlenbeck test process of Appendix B.2 and its closed forms, FP64.

Test infrastructure (see ``oracle/__init__``).

dx/dt = -x + eta(t) with <eta(t) eta(t')> = delta(t - t'): unit relaxation
rate, stationary variance 1/2, autocovariance C(s) = exp(-|s|)/2.  Sampled
exactly on a grid of step dt (AR(1) recursion)
    x_{n+1} = rho x_n + sqrt((1 - rho^2)/2) xi_n,   rho = exp(-dt),
so every closed form below holds for the sampled chain, not only in the
dt -> 0 limit.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.signal import lfilter


def ar1_coeffs(dt: float):
    rho = math.exp(-dt)
    return rho, math.sqrt((1.0 - rho * rho) / 2.0)


def paths(x0: np.ndarray, n_steps: int, dt: float, rng: np.random.Generator) -> np.ndarray:
    """[N, n_steps] samples x_1..x_n of N independent chains started at x0."""
    rho, sig = ar1_coeffs(dt)
    x0 = np.asarray(x0, dtype=np.float64)
    if n_steps == 0:
        return np.zeros((len(x0), 0))
    noise = sig * rng.standard_normal((len(x0), n_steps))
    # x_n = rho x_{n-1} + e_n, with the initial condition folded into e_1
    noise[:, 0] += rho * x0
    return lfilter([1.0], [1.0, -rho], noise, axis=1)


def stationary(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.standard_normal(n) * math.sqrt(0.5)


def sum_variance(m: int, dt: float) -> float:
    """Var(dt * sum_{n=1}^{m} x_n) for a stationary start (exact for the chain)."""
    rho = math.exp(-dt)
    tot = float(m)
    for d in range(1, m):
        tot += 2.0 * (m - d) * rho ** d
    return dt * dt * 0.5 * tot


def integral_variance(t: float) -> float:
    """Var(int_0^T x dt) = T - 1 + exp(-T) for the continuous process."""
    return t - 1.0 + math.exp(-t)


def log_mgf_sum(k: float, m: int, dt: float) -> float:
    """ln E[exp(k dt sum_{n=1}^m x_n)] = k^2 Var / 2 (the sum is Gaussian)."""
    return 0.5 * k * k * sum_variance(m, dt)


def window_mean_sd(window: int, dt: float) -> float:
    """Standard deviation of the mean of `window` consecutive stationary samples."""
    return math.sqrt(sum_variance(window, dt)) / (window * dt)
