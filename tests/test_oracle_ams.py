"""Pins for the AMS oracle: selection rules by construction, unbiasedness on OU."""
import math

import numpy as np

from oracle import ams, ou


def test_kill_branch_rules():
    series = np.array([[0.0, 1.0, 0.5],    # max 1.0
                       [0.0, 0.2, 0.1],    # max 0.2  <- lowest
                       [0.3, 0.9, 2.0],    # max 2.0
                       [0.2, 0.2, 0.0],    # max 0.2  <- tie with slot 1
                       [np.nan, 5.0, 5.0]])  # non-finite -> -inf, killed first
    kb = ams.kill_branch(series, n_kill=2, key=1, iteration=0)
    assert kb.level == 0.2 and not kb.extinct
    assert kb.killed.tolist() == [1, 3, 4]
    for p, tb in zip(kb.parents, kb.branch_t):
        assert p in (0, 2)
        row = series[p]
        assert row[tb] > 0.2 and np.all(row[:tb] <= 0.2)


def test_extinction_when_all_equal():
    kb = ams.kill_branch(np.ones((4, 3)), 1, 0, 0)
    assert kb.extinct and len(kb.killed) == 4


def test_parent_choice_uniform_over_survivors():
    series = np.array([[float(i)] * 2 for i in range(6)])
    counts = np.zeros(6)
    for it in range(600):
        kb = ams.kill_branch(series, 2, 7, it)
        counts += np.bincount(kb.parents, minlength=6)
    assert counts[0] == 0 and counts[1] == 0
    exp = counts.sum() / 4
    assert ((counts[2:] - exp) ** 2 / exp).sum() < 20


def test_estimator_without_iterations_is_direct_sampling():
    q = np.array([0.1, 0.5, 0.7, 2.0])
    assert np.allclose(ams.estimate([], 4, q, np.array([0.5, 1.0])), [0.75, 0.25])
    assert np.allclose(ams.estimate([1, 2], 4, q, np.array([0.0])), [0.75 * 0.5])


def test_ams_unbiased_on_ou():
    """Mean AMS estimate of P(max_[0,T_a] x >= a) equals brute-force Monte Carlo."""
    dt, n_steps, a = 0.02, 100, 1.2
    t_a = n_steps * dt
    rng = np.random.default_rng(0)
    x0 = ou.stationary(200_000, rng)
    brute = (ou.paths(x0, n_steps, dt, rng).max(axis=1) >= a).mean()

    def make_resim(rng):
        def resim(parent, tb, slot, it):
            tail = ou.paths(np.array([parent[tb]]), n_steps - tb - 1, dt, rng)[0]
            return np.concatenate([parent[:tb + 1], tail])
        return resim

    est = []
    for rep in range(120):
        rng = np.random.default_rng(1000 + rep)
        paths = ou.paths(ou.stationary(16, rng), n_steps, dt, rng)
        res = ams.run(paths, make_resim(rng), n_kill=1, key=rep, max_iter=400, threshold=a)
        assert not res["extinct"]
        est.append(ams.estimate(res["k_history"], 16, ams.clean_maxima(res["paths"]), np.array([a]))[0])
    mean, se = np.mean(est), np.std(est, ddof=1) / math.sqrt(len(est))
    assert abs(mean - brute) < 4 * se + 0.003, (mean, brute, se)
    assert brute < 0.3  # the level is not typical


def test_return_time_formula_limits():
    r = ams.return_time(np.array([0.0, 1e-9]), 5.0)
    assert r[0] == math.inf and math.isclose(r[1] * 1e-9 / 5.0, 1.0, rel_tol=1e-8)


def test_minus_inf_entries_are_ordinary_scores():
    series = np.array([[-np.inf, 0.5, 0.7], [-np.inf, -np.inf, 0.2], [np.inf, 0.1, 0.1], [0.3, np.nan, 0.0]])
    q = ams.clean_maxima(series)
    assert q.tolist() == [0.7, 0.2, -np.inf, -np.inf]
    kb = ams.kill_branch(series, 3, 0, 0)
    assert kb.level == 0.2 and kb.killed.tolist() == [1, 2, 3] and kb.parents.tolist() == [0, 0, 0]
    assert kb.branch_t.tolist() == [1, 1, 1]


def test_learned_score_against_the_hard_clamp_and_the_logistic_slope():
    """The learned-score map is within width*ln 2 of min(ghat, level) everywhere, equal to
    level - width*ln 2 at ghat = level, strictly below the level, and its slope is the logistic
    function of (level - ghat)/width (scipy's expit), so it is strictly increasing."""
    from scipy.special import expit
    level, width = 1.3, 0.05
    g = np.linspace(level - 40 * width, level + 30 * width, 7001)
    s = ams.learned_score(g, np.full(g.shape, -np.inf), level, width)
    assert np.all(np.abs(s - np.minimum(g, level)) <= width * math.log(2) * (1 + 1e-12))
    assert math.isclose(ams.learned_score(np.array([level]), np.array([0.0]), level, width)[0],
                        level - width * math.log(2), rel_tol=1e-15)
    assert np.all(s < level)
    near = g <= level + 10 * width            # past that FP64 no longer resolves the approach
    assert np.all(np.diff(s[near]) > 0)
    h = 1e-6
    slope = (ams.learned_score(g + h, np.full(g.shape, -np.inf), level, width)
             - ams.learned_score(g - h, np.full(g.shape, -np.inf), level, width)) / (2 * h)
    assert np.allclose(slope, expit((level - g) / width), atol=1e-7)
    # far below the level the map is the prediction itself
    assert abs(ams.learned_score(np.array([level - 40 * width]), np.array([0.0]), level, width)[0]
               - (level - 40 * width)) < width * 1e-17 + 1e-15


def test_learned_score_reaches_the_level_exactly_with_the_event():
    rng = np.random.default_rng(3)
    level, width = 0.0, 0.3
    ghat = rng.standard_normal((50, 40)) + 2.0            # predictions that over-shoot
    ghat[3, 5] = np.nan
    ev = rng.standard_normal((50, 40)) * 0.4 - 0.5
    s = ams.learned_score(ghat, ev, level, width)
    assert np.array_equal(s.max(axis=1) >= level, ev.max(axis=1) >= level)
    assert np.all(s[ev >= level] == level) and s[3, 5] == -np.inf or ev[3, 5] >= level


def test_learned_score_ams_unbiased_on_ou_where_the_hard_clamp_ties():
    """OU with a prediction that over-shoots by 0.8.  The smooth map is an increasing function of
    the state below the level, so AMS on it takes the very same decisions as AMS on the state
    itself (same discards, same estimate), which matches brute force.  Clamping the same
    prediction at the float below the level makes the maxima tie there, so whole groups are
    discarded at once."""
    dt, n_steps, a, bias, width = 0.02, 100, 1.2, 0.8, 0.1
    rng = np.random.default_rng(0)
    brute = (ou.paths(ou.stationary(200_000, rng), n_steps, dt, rng).max(axis=1) >= a).mean()
    below = float(np.nextafter(a, -np.inf))

    def smooth(p):
        return ams.learned_score(p + bias, p, a, width)

    def hard(p):
        return np.where(p >= a, a, np.minimum(p + bias, below))

    def make_resim(rng):
        def resim(parent, tb, slot, it):
            tail = ou.paths(np.array([parent[tb]]), n_steps - tb - 1, dt, rng)[0]
            return np.concatenate([parent[:tb + 1], tail])
        return resim

    est, k_hard = [], []
    for rep in range(60):
        rng = np.random.default_rng(5000 + rep)
        paths = ou.paths(ou.stationary(16, rng), n_steps, dt, rng)
        runs = {name: ams.run(paths, make_resim(np.random.default_rng(rep)), n_kill=1, key=rep, max_iter=400,
                              threshold=a, score=f) for name, f in (("plain", None), ("smooth", smooth),
                                                                     ("hard", hard))}
        assert not runs["smooth"]["extinct"]
        assert runs["smooth"]["k_history"] == runs["plain"]["k_history"]
        assert np.array_equal(runs["smooth"]["paths"], runs["plain"]["paths"])
        est.append(ams.estimate(runs["smooth"]["k_history"], 16, ams.clean_maxima(runs["smooth"]["scores"]),
                                np.array([a]))[0])
        k_hard += runs["hard"]["k_history"]
    mean, se = np.mean(est), np.std(est, ddof=1) / math.sqrt(len(est))
    assert abs(mean - brute) < 4 * se + 0.004, (mean, brute, se)
    assert np.mean(k_hard) > 2.0 and max(k_hard) >= 8, (np.mean(k_hard), max(k_hard))


def test_ams_stops_when_the_level_reaches_the_threshold():
    """n_kill = 4 on OU with the learned-score map (which stays at the threshold once the event
    has happened): AMS stops once the 4th lowest maximum reaches the threshold; the estimate
    matches brute force and no run goes extinct.  Where a run stops that way, one more
    selection would have discarded every trajectory (all maxima at or below a level equal to the
    threshold), which is what happened before the stop existed."""
    dt, n_steps, a, width, n_kill = 0.02, 100, 1.2, 0.1, 4
    rng = np.random.default_rng(1)
    brute = (ou.paths(ou.stationary(200_000, rng), n_steps, dt, rng).max(axis=1) >= a).mean()

    def score(p):
        return ams.learned_score(p + 0.3, p, a, width)

    def make_resim(rng):
        def resim(parent, tb, slot, it):
            tail = ou.paths(np.array([parent[tb]]), n_steps - tb - 1, dt, rng)[0]
            return np.concatenate([parent[:tb + 1], tail])
        return resim

    est, by_level = [], 0
    for rep in range(80):
        rng = np.random.default_rng(7000 + rep)
        paths = ou.paths(ou.stationary(16, rng), n_steps, dt, rng)
        res = ams.run(paths, make_resim(rng), n_kill=n_kill, key=rep, max_iter=400, threshold=a, score=score)
        assert not res["extinct"]
        q = ams.clean_maxima(res["scores"])
        est.append(ams.estimate(res["k_history"], 16, q, np.array([a]))[0])
        if q.min() < a:  # stopped by the level, not because every trajectory reached the event
            by_level += 1
            assert ams.kill_branch(res["scores"], n_kill, rep, len(res["k_history"])).extinct
    mean, se = np.mean(est), np.std(est, ddof=1) / math.sqrt(len(est))
    assert abs(mean - brute) < 4 * se + 0.004, (mean, brute, se)
    assert by_level >= 20, by_level
