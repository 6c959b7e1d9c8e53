"""Trajectory-adaptive multilevel splitting (paper Section 4.1, Appendix B), FP64.

Test infrastructure (see ``oracle/__init__``).

Each of N trajectories of fixed duration T_a carries a score series xi(t) and
its maximum Q over [0, T_a].  One iteration (Appendix B.1):

* level: the n_kill-th lowest maximum; every trajectory whose maximum is at
  or below it is discarded (ties go together), so K_j >= n_kill.  The paper
  discards one per iteration in its OU example and "the trajectories with the
  lowest maxima" in the drag runs; n_kill covers both.  A trajectory whose
  score series holds NaN or +inf (blown up) counts as -inf.  If every trajectory is at the level the run is extinct.
* branching: each discarded slot picks a parent uniformly among the
  survivors (AMSP Philox stream at (kill index, iteration)), copies it up to
  its first time t_b with xi(t_b) > level (strictly above, so the copy
  already beats the level), and is re-simulated from there (with a
  perturbation for deterministic dynamics).
* stopping: after J iterations, once every maximum reaches the target
  threshold, or once the level itself reaches it (with n_kill > 1 the
  n_kill-th lowest maximum can reach the threshold before the lowest one
  does; discarding at such a level would discard trajectories that reached
  the event, and a score that stops at the threshold once the event has
  happened would discard all of them).

Estimator (the paper cites it without printing it): the standard unbiased
generalised-AMS estimate of p(a) = P(max_{[0, T_a]} xi >= a) is
prod_j (1 - K_j / N) * (1/N) sum_n 1[Q_n >= a], and the return time is
r(a) = -T_a / ln(1 - p(a)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np

from . import philox


@dataclass
class KillBranch:
    level: float
    killed: np.ndarray     # slots discarded this iteration, increasing
    parents: np.ndarray    # parent slot for each killed slot
    branch_t: np.ndarray   # first index where the parent's score > level
    extinct: bool


def clean_maxima(series: np.ndarray) -> np.ndarray:
    """Maximum of each row.  A row holding NaN or +inf (a blown-up trajectory)
    counts as -inf; -inf entries are ordinary lowest scores (no score yet)."""
    series = np.asarray(series, dtype=np.float64)
    out = np.empty(series.shape[0])
    for n in range(series.shape[0]):
        row = series[n]
        bad = np.isnan(row).any() or np.isposinf(row).any()
        out[n] = -math.inf if bad else float(row.max())
    return out


def kill_branch(series: np.ndarray, n_kill: int, key: int, iteration: int) -> KillBranch:
    """One AMS selection on score series [N, T] (values compared as given)."""
    series = np.asarray(series)
    n = series.shape[0]
    q = clean_maxima(series)
    level = float(sorted(q.tolist())[n_kill - 1])
    killed = np.array([m for m in range(n) if q[m] <= level], dtype=np.int64)
    survivors = [m for m in range(n) if q[m] > level]
    if not survivors:
        return KillBranch(level, killed, np.full(len(killed), -1), np.full(len(killed), -1), True)
    parents = np.empty(len(killed), dtype=np.int64)
    branch_t = np.empty(len(killed), dtype=np.int64)
    for j in range(len(killed)):
        w = philox.philox4x64_10((j, iteration, 0, 0), (key, philox.AMSP))[0]
        p = survivors[philox.index_below(w, len(survivors))]
        parents[j] = p
        row = series[p]
        tb = -1
        for t in range(series.shape[1]):
            if row[t] > level:
                tb = t
                break
        branch_t[j] = tb
    return KillBranch(level, killed, parents, branch_t, False)


def learned_score(ghat: np.ndarray, event: np.ndarray, level: float, width: float) -> np.ndarray:
    """AMS score built on a learned prediction ghat of the target observable, for the event
    {max_t event(t) >= level} (the score may be any function of the state as long as it reaches
    the level exactly when the event happens, which keeps the estimate unbiased, Section 4.1).

    Where event(t) >= level the score is the level.  Elsewhere it is a smooth, strictly
    increasing map of the prediction into (-inf, level):
        level - width * ln(1 + exp((level - ghat) / width)),
    which follows ghat far below the level and approaches the level from below as ghat grows past
    it, so over-predictions keep their order instead of all landing on one value.  A non-finite
    prediction gives -inf.  FP64, element by element; `level` and `width` > 0 as given.
    """
    g = np.asarray(ghat, dtype=np.float64).ravel()
    e = np.asarray(event, dtype=np.float64).ravel()
    out = np.empty(g.shape)
    for i in range(g.size):
        if e[i] >= level:
            out[i] = level
        elif not math.isfinite(g[i]):
            out[i] = -math.inf
        else:
            x = (level - g[i]) / width
            # the same quantity written so that exp never overflows
            if x > 0.0:
                out[i] = g[i] - width * math.log1p(math.exp(-x))
            else:
                out[i] = level - width * math.log1p(math.exp(x))
    return out.reshape(np.shape(ghat))


def estimate(k_history: List[int], n: int, final_maxima: np.ndarray, levels: np.ndarray) -> np.ndarray:
    """Unbiased AMS estimate of P(max >= a) for each level a."""
    factor = 1.0
    for kj in k_history:
        factor *= (1.0 - kj / n)
    q = np.asarray(final_maxima, dtype=np.float64)
    return np.array([factor * float(np.count_nonzero(q >= a)) / n for a in levels])


def return_time(prob: np.ndarray, t_a: float) -> np.ndarray:
    """r(a) = -T_a / ln(1 - p(a)); inf where p = 0."""
    prob = np.asarray(prob, dtype=np.float64)
    out = np.full(prob.shape, math.inf)
    pos = prob > 0
    out[pos] = -t_a / np.log1p(-np.minimum(prob[pos], 1.0 - 1e-300))
    return out


def run(init_paths: np.ndarray, resimulate: Callable, n_kill: int, key: int,
        max_iter: int, threshold: float, score: Optional[Callable] = None):
    """Generic AMS loop for a toy dynamics given by whole paths.

    init_paths: [N, T] state paths.  score(paths) -> [N, T] score series
    (default: the state itself, as for OU).  resimulate(parent_path, t_b, slot,
    iteration) -> new path equal to the parent on [0, t_b] and freshly
    simulated after.  Returns dict(paths, scores, k_history, levels, extinct).
    """
    score = (lambda p: p) if score is None else score
    paths = np.array(init_paths, dtype=np.float64)
    n = paths.shape[0]
    k_hist, levels = [], []
    extinct = False
    for it in range(max_iter):
        xi = score(paths)
        if clean_maxima(xi).min() >= threshold:
            break
        kb = kill_branch(xi, n_kill, key, it)
        if kb.level >= threshold:
            break
        if kb.extinct:
            extinct = True
            break
        k_hist.append(len(kb.killed))
        levels.append(kb.level)
        new_paths = paths.copy()
        for slot, parent, tb in zip(kb.killed, kb.parents, kb.branch_t):
            new_paths[slot] = resimulate(paths[parent], int(tb), int(slot), it)
        paths = new_paths
    return dict(paths=paths, scores=score(paths), k_history=k_hist, levels=levels, extinct=extinct)
