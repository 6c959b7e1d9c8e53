"""GKTL cloning algorithm and its estimators (paper Section 4.2, Appendix C), FP64.

Test infrastructure (see ``oracle/__init__``).

* weights: at each cloning time t_i = i*tau, trajectory n gets
  W_n = exp(s_n) / R_i with s_n = k * int_{t_{i-1}}^{t_i} A(x_n(t)) dt and
  R_i = (1/N) sum_n exp(s_n), so that sum_n W_n = N (Appendix C.1, weight
  equation).  ln R_i is formed with the largest s_n factored out.
* selection: the weights set how many copies each trajectory gets; the
  implementation is left to the paper's references.  The reading used here is
  multinomial resampling: new slot m takes ancestor a_m = the first n whose
  running sum C_n = sum_{l<=n} exp(s_l - s_max), taken in index order, exceeds
  u_m * C_{N-1}, with u_m from the GKTS Philox stream at (m, period).  A
  trajectory whose s_n is not finite (a blown-up simulation) has weight 0 and
  is never chosen.
* SCGF: Z(k, T_a) = prod_i R_i (Appendix C.1), lambda(k) = ln Z / T_a.
* return times (Appendix C.2): every trajectory j of the final ensemble,
  traced back through the ancestors, carries its whole drag series; its
  time-averaged drag F_T^(j)(t), t in [T, T_a], is the window mean (the
  definition of Section 3.2 -- the appendix drops the 1/T).  The probability
  P(max F_T >= a) is the sum of s_j(a) = 1[max_t F_T^(j)(t) >= a] with weights
  exp(T_a lambda(k)) exp(-k int_0^{T_a} A_j dt) / N, which inverts the biased
  path law; the printed formula has the sign of the exponent flipped and the
  average in place of the integral, and that reading is corrected here.  Then
  r(a) = -(T_a - T) / ln(1 - P).
"""
from __future__ import annotations

import math
from typing import Callable, List, Sequence

import numpy as np

from . import philox


def log_normaliser(s: np.ndarray) -> float:
    """ln R = ln((1/N) sum_n exp(s_n)), non-finite s_n counting as weight 0."""
    s = np.asarray(s, dtype=np.float64)
    finite = np.isfinite(s)
    if not finite.any():
        raise ValueError("every trajectory has a non-finite weight")
    smax = float(s[finite].max())
    total = math.fsum(math.exp(float(v) - smax) for v in s[finite])
    return smax + math.log(total) - math.log(len(s))


def weights(s: np.ndarray) -> np.ndarray:
    """W_n = exp(s_n) / R; sums to N."""
    lnr = log_normaliser(s)
    s = np.asarray(s, dtype=np.float64)
    return np.array([math.exp(float(v) - lnr) if math.isfinite(v) else 0.0 for v in s])


def select(s: np.ndarray, key: int, period: int) -> np.ndarray:
    """Multinomial ancestors a_m (int array of length N) for one cloning time."""
    s = np.asarray(s, dtype=np.float64)
    n_tot = len(s)
    finite = np.isfinite(s)
    if not finite.any():
        raise ValueError("every trajectory has a non-finite weight")
    smax = float(s[finite].max())
    prefix = []
    acc = 0.0
    for n in range(n_tot):
        acc += math.exp(float(s[n]) - smax) if finite[n] else 0.0
        prefix.append(acc)
    last_live = int(np.nonzero(finite)[0][-1])
    out = np.empty(n_tot, dtype=np.int64)
    for m in range(n_tot):
        u = philox.uniform53(philox.philox4x64_10((m, period, 0, 0), (key, philox.GKTS))[0])
        target = u * acc
        a = last_live
        for n in range(n_tot):
            if prefix[n] > target:
                a = n
                break
        out[m] = a
    return out


def first_copy(ancestors: Sequence[int]) -> np.ndarray:
    """True for the lowest slot index taking each ancestor (that copy is not perturbed)."""
    seen = set()
    flags = np.zeros(len(ancestors), dtype=bool)
    for m, a in enumerate(ancestors):
        if int(a) not in seen:
            seen.add(int(a))
            flags[m] = True
    return flags


def scgf(ln_r: Sequence[float], t_a: float) -> float:
    """lambda(k) = (1/T_a) sum_i ln R_i."""
    return math.fsum(ln_r) / t_a


def lineage(ancestors: List[np.ndarray]) -> np.ndarray:
    """Slot occupied in each period by the ancestors of every final trajectory.

    ``ancestors[i][m]`` is the slot (in the ensemble of period i) whose state
    slot m continues with in period i+1.  Returns L[j, i] = slot that final
    trajectory j occupied during period i (i = 0 .. len(ancestors)), where the
    last column is j itself.
    """
    n_p = len(ancestors)
    n = len(ancestors[0]) if n_p else 0
    out = np.empty((n, n_p + 1), dtype=np.int64)
    out[:, n_p] = np.arange(n)
    for i in range(n_p - 1, -1, -1):
        out[:, i] = np.asarray(ancestors[i])[out[:, i + 1]]
    return out


def reconstruct_series(period_series: List[np.ndarray], ancestors: List[np.ndarray]) -> np.ndarray:
    """Full series of every final trajectory from per-period segments.

    period_series[i] is [N, tau] (the samples produced during period i by each
    slot); ancestors[i] maps the slots after cloning time i+1 to slots of
    period i.  len(period_series) == len(ancestors) + 1 or == len(ancestors)
    (when the last cloning happens at T_a, its ancestors also apply).
    """
    n_per = len(period_series)
    anc = list(ancestors)
    if len(anc) == n_per:  # selection also at T_a: final slots are post-selection
        lin = lineage(anc)[:, :n_per]
    else:
        lin = lineage(anc)
    segs = [period_series[i][lin[:, i]] for i in range(n_per)]
    return np.concatenate(segs, axis=1)


def window_means(series: np.ndarray, window: int) -> np.ndarray:
    """[N, T] -> [N, T]: mean of the last `window` samples ending at t (-inf before the first full window)."""
    series = np.asarray(series, dtype=np.float64)
    n, t_len = series.shape
    out = np.full((n, t_len), -math.inf)
    for j in range(n):
        for t in range(window - 1, t_len):
            out[j, t] = math.fsum(series[j, t - window + 1:t + 1].tolist()) / window
    return out


def window_mean_max(series: np.ndarray, window: int) -> np.ndarray:
    """max over t of the window mean (1/T) sum of the last T samples; one per row."""
    series = np.asarray(series, dtype=np.float64)
    n, t_len = series.shape
    out = np.empty(n)
    for j in range(n):
        best = -math.inf
        for t in range(window, t_len + 1):
            v = math.fsum(series[j, t - window:t].tolist()) / window
            if v > best:
                best = v
        out[j] = best
    return out


def tail_probability(maxima: np.ndarray, log_weights: np.ndarray, levels: np.ndarray) -> np.ndarray:
    """P(max >= a) = (1/N) sum_j exp(log_weight_j) 1[max_j >= a], for each a."""
    n = len(maxima)
    out = np.empty(len(levels))
    for q, a in enumerate(levels):
        out[q] = math.fsum(math.exp(lw) for mx, lw in zip(maxima, log_weights) if mx >= a) / n
    return out


def return_time(prob: np.ndarray, t_a: float, window: float) -> np.ndarray:
    """r(a) = -(T_a - T) / ln(1 - P(a)); inf where P = 0."""
    prob = np.asarray(prob, dtype=np.float64)
    out = np.full(prob.shape, math.inf)
    pos = prob > 0
    out[pos] = -(t_a - window) / np.log1p(-np.minimum(prob[pos], 1.0 - 1e-300))
    return out


def unbias_log_weights(ln_r: Sequence[float], k: float, integrals: np.ndarray) -> np.ndarray:
    """ln of exp(T_a lambda) exp(-k int_0^{T_a} A_j dt) for each final trajectory."""
    lz = math.fsum(ln_r)
    return lz - k * np.asarray(integrals, dtype=np.float64)


def run(x0: np.ndarray, advance: Callable, n_periods: int, k: float, key: int):
    """Generic GKTL driver for a stochastic toy dynamics (used with the OU process).

    advance(x, period) -> (x_end, samples[N, tau], integral[N]) evolves every
    slot over one cloning period and returns its samples and int A dt.
    Selection happens at every t_i = i*tau, i = 1..n_periods (the last one at
    T_a included).  Returns dict(ln_r, ancestors, samples, integrals).
    """
    x = np.array(x0, dtype=np.float64)
    ln_r, ancs, segs, ints = [], [], [], []
    for i in range(n_periods):
        x, samples, integral = advance(x, i)
        s = k * integral
        ln_r.append(log_normaliser(s))
        a = select(s, key, i)
        ancs.append(a)
        segs.append(samples)
        ints.append(integral)
        x = x[a]
    return dict(ln_r=ln_r, ancestors=ancs, samples=segs, integrals=ints)
