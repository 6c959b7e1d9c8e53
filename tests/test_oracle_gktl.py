"""Pins for the GKTL oracle: normalisation, multinomial law, OU closed forms, lineage."""
import math

import numpy as np
import pytest
from scipy.special import erfc, logsumexp

from oracle import gktl, ou


def test_weights_sum_to_n_and_log_normaliser():
    rng = np.random.default_rng(0)
    for n in (1, 5, 256):
        s = rng.standard_normal(n) * 40
        w = gktl.weights(s)
        assert math.isclose(math.fsum(w), n, rel_tol=1e-13)
        assert math.isclose(gktl.log_normaliser(s), logsumexp(s) - math.log(n), rel_tol=1e-14, abs_tol=1e-13)


def test_non_finite_member_has_zero_weight_and_is_never_chosen():
    s = np.array([np.nan, 0.3, -np.inf, 1.0, np.nan])
    w = gktl.weights(s)
    assert w[0] == 0 and w[2] == 0 and w[4] == 0
    assert math.isclose(w.sum(), 5.0, rel_tol=1e-14)
    for period in range(200):
        a = gktl.select(s, key=4, period=period)
        assert set(a.tolist()) <= {1, 3}
    with pytest.raises(ValueError):
        gktl.select(np.array([np.nan, np.nan]), 1, 0)


def test_selection_is_multinomial():
    """Ancestor frequencies follow W_n / N (chi-square over many periods)."""
    s = np.log(np.array([1.0, 2.0, 3.0, 4.0, 0.5]))
    p = np.exp(s) / np.exp(s).sum()
    counts = np.zeros(5)
    periods = 800
    for period in range(periods):
        counts += np.bincount(gktl.select(s, key=11, period=period), minlength=5)
    expect = p * 5 * periods
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert chi2 < 20  # 4 dof: p ~ 5e-4
    # and each slot's marginal is the same law: slot 0 alone over the periods
    slot0 = np.bincount([gktl.select(s, 11, q)[0] for q in range(periods)], minlength=5)
    chi2 = ((slot0 - p * periods) ** 2 / (p * periods)).sum()
    assert chi2 < 20


def test_k_zero_selection_is_uniform():
    s = np.zeros(8)
    counts = np.zeros(8)
    for period in range(500):
        counts += np.bincount(gktl.select(s, 3, period), minlength=8)
    chi2 = ((counts - 500) ** 2 / 500).sum()
    assert chi2 < 25


def test_first_copy_flags():
    a = np.array([3, 3, 0, 1, 0, 3])
    assert gktl.first_copy(a).tolist() == [True, False, True, True, False, False]


def _ou_advance(rng, steps, dt):
    def advance(x, period):
        path = ou.paths(x, steps, dt, rng)
        return path[:, -1], path, path.sum(axis=1) * dt
    return advance


def test_scgf_matches_ou_closed_form():
    """lambda_hat(k) -> ln E[exp(k int x)] / T_a; Gaussian integral makes it exact."""
    dt, steps, n_per, n = 0.05, 10, 10, 512
    k = 1.0
    t_a = dt * steps * n_per
    exact = ou.log_mgf_sum(k, steps * n_per, dt) / t_a
    est = []
    for rep in range(6):
        rng = np.random.default_rng(100 + rep)
        res = gktl.run(ou.stationary(n, rng), _ou_advance(rng, steps, dt), n_per, k, key=rep)
        est.append(gktl.scgf(res["ln_r"], t_a))
    mean, se = np.mean(est), np.std(est, ddof=1) / math.sqrt(len(est))
    assert abs(mean - exact) < 4 * se + 0.02 * exact, (mean, exact, se)
    # sign sensitivity: k -> -k gives the same closed form (symmetric process)
    assert exact > 0


def test_lineage_reconstructs_histories():
    """Carry each slot's full history with the state; it must equal the reconstruction."""
    rng = np.random.default_rng(5)
    n, steps, n_per, dt = 16, 4, 5, 0.1
    x = ou.stationary(n, rng)
    hist = np.zeros((n, 0))
    segs, ancs = [], []
    for i in range(n_per):
        path = ou.paths(x, steps, dt, rng)
        hist = np.concatenate([hist, path], axis=1)
        s = 2.0 * path.sum(axis=1) * dt
        a = gktl.select(s, 9, i)
        segs.append(path)
        ancs.append(a)
        x, hist = path[a, -1], hist[a]
    assert np.array_equal(gktl.reconstruct_series(segs, ancs), hist)
    # without the final selection the last column of the lineage is the slot itself
    assert np.array_equal(gktl.reconstruct_series(segs, ancs[:-1]), hist_without_last(segs, ancs))


def hist_without_last(segs, ancs):
    n = segs[0].shape[0]
    hist = np.zeros((n, 0))
    for i, path in enumerate(segs):
        hist = np.concatenate([hist, path], axis=1)
        if i < len(segs) - 1:
            hist = hist[ancs[i]]
    return hist


def test_window_mean_max_brute_force():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((3, 20))
    got = gktl.window_mean_max(x, 5)
    ref = [max(x[j, t - 5:t].mean() for t in range(5, 21)) for j in range(3)]
    assert np.allclose(got, ref, rtol=1e-14)


@pytest.mark.parametrize("k", [0.0, 2.0])
def test_return_time_tail_on_ou(k):
    """T_a = T: F_T is the mean over the whole trajectory, Gaussian with known sd.

    The reweighted GKTL estimate of P(F_T >= a) must match the Gaussian tail;
    at k = 2 it reaches levels direct sampling with the same N cannot.
    """
    dt, steps, n_per, n = 0.05, 10, 8, 1000
    m = steps * n_per
    t_a = m * dt
    sd = ou.window_mean_sd(m, dt)
    levels = np.array([0.5, 1.0, 1.5, 2.0]) * sd if k == 0 else np.array([2.0, 2.5, 3.0]) * sd
    probs = []
    for rep in range(4):
        rng = np.random.default_rng(300 + rep)
        res = gktl.run(ou.stationary(n, rng), _ou_advance(rng, steps, dt), n_per, k, key=50 + rep)
        series = gktl.reconstruct_series(res["samples"], res["ancestors"])
        lin = gktl.lineage(res["ancestors"])
        integ = sum(res["integrals"][i][lin[:, i]] for i in range(n_per))
        assert np.allclose(integ, series.sum(axis=1) * dt, rtol=1e-12, atol=1e-12)
        fmax = gktl.window_mean_max(series, m)
        lw = gktl.unbias_log_weights(res["ln_r"], k, integ)
        probs.append(gktl.tail_probability(fmax, lw, levels))
    est = np.mean(probs, axis=0)
    exact = 0.5 * erfc(levels / (math.sqrt(2) * sd))
    assert np.all(np.abs(est / exact - 1) < 0.25), (est, exact)


def test_return_time_poisson_limits():
    """r = -(T_a - T)/ln(1 - P): Poisson waiting time; r P/(T_a - T) -> 1 as P -> 0."""
    p = np.array([0.0, 1e-9, 1e-3, 0.5])
    r = gktl.return_time(p, 10.0, 4.0)
    assert r[0] == math.inf
    assert math.isclose(r[1] * p[1] / 6.0, 1.0, rel_tol=1e-8)
    assert math.isclose(r[3], 6.0 / math.log(2.0), rel_tol=1e-14)
    assert np.all(np.diff(r[1:]) < 0)


def test_window_means_consistent_with_max():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((2, 30))
    wm = gktl.window_means(x, 7)
    assert np.all(np.isneginf(wm[:, :6]))
    assert np.allclose(wm[:, 6:].max(axis=1), gktl.window_mean_max(x, 7), rtol=1e-15)
    assert np.isclose(wm[1, 12], x[1, 6:13].mean(), rtol=1e-14)
