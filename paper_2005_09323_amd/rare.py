"""GKTL and trajectory-AMS drivers over the device kernels.

The drivers only order the library calls (stepping, selection, cloning,
checkpoint copies, estimators); every computation runs on the GPU.  Paper
references: GKTL, Section 4.2 and Appendix C; AMS, Section 4.1 and Appendix B;
perturbation at branching, Appendix D.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import native
from .ensemble import Ensemble, _ptr, _stream_handle, ams_score_kill_branch, window_mean


@dataclass
class GktlRun:
    """Record of one GKTL run: what the estimators need."""
    k: float
    tau: int
    n_periods: int
    col0: int                 # first drag column of period 0
    ancestors: torch.Tensor   # int32 [P, N]
    integrals: torch.Tensor   # float64 [P, N]: int A dt of each slot over each period
    ln_r: torch.Tensor        # float64 [P]

    @property
    def t_a(self) -> int:
        return self.tau * self.n_periods

    def scgf(self, dt: float) -> float:
        """lambda(k) = (1/T_a) sum_i ln R_i, T_a in the units of dt."""
        return float(self.ln_r.double().sum().item()) / (self.t_a * dt)


def run_gktl(ens: Ensemble, k: float, n_periods: int, tau: int, key: int, eps: float = 0.0,
             snapshots: Optional[torch.Tensor] = None) -> GktlRun:
    """GKTL over n_periods cloning periods of tau steps, selecting at every t_i = i tau (T_a included).

    The ensemble must be initialised and its observable set (lbm_set_observable);
    its drag series needs tau * n_periods free columns.
    """
    n = ens.n
    dev = ens.device
    anc = torch.empty((n_periods, n), dtype=torch.int32, device=dev)
    ints = torch.empty((n_periods, n), dtype=torch.float64, device=dev)
    lnr = torch.empty(n_periods, dtype=torch.float64, device=dev)
    col0 = ens.time(0)
    n_snap = 0 if snapshots is None else int(snapshots.shape[0])
    lib = native.lib()
    for i in range(n_periods):
        ens.step(tau)
        ints[i].copy_(ens.accum)  # the period integrals, before the selection resets them
        native.check(lib.gktl_select_clone(ens._ctx, k, key, i, eps, _ptr(snapshots), n_snap,
                                           ctypes.c_void_p(anc[i].data_ptr()), ctypes.c_void_p(lnr[i:].data_ptr())))
    return GktlRun(k, tau, n_periods, col0, anc, ints, lnr)


@dataclass
class Trajectories:
    series: torch.Tensor      # float32 [N, T_a] drag of each final trajectory
    log_weight: torch.Tensor  # float64 [N]
    integral: torch.Tensor    # float64 [N]


def rebuild(run: GktlRun, ens: Ensemble) -> Trajectories:
    """Trace every final trajectory back through the ancestors (device kernel)."""
    n, p, tau = ens.n, run.n_periods, run.tau
    traj = torch.empty((n, p * tau), dtype=torch.float32, device=ens.device)
    lw = torch.empty(n, dtype=torch.float64, device=ens.device)
    integ = torch.empty(n, dtype=torch.float64, device=ens.device)
    native.check(native.lib().gktl_rebuild(_ptr(run.ancestors), _ptr(run.integrals), _ptr(run.ln_r),
                                           _ptr(ens.series), ens.capacity, run.col0, n, p, tau, run.k,
                                           _ptr(traj), _ptr(lw), _ptr(integ), _stream_handle(None)))
    return Trajectories(traj, lw, integ)


def window_maxima(series: torch.Tensor, window: int) -> torch.Tensor:
    """Largest window mean of each row (device, FP64)."""
    rows, length = series.shape
    series = series.contiguous()
    pre = torch.empty((rows, length + 1), dtype=torch.float64, device=series.device)
    fmax = torch.empty(rows, dtype=torch.float64, device=series.device)
    native.check(native.lib().window_mean_max(_ptr(series), rows, length, window, _ptr(pre), _ptr(fmax),
                                              _stream_handle(None)))
    return fmax


def tail_probability(fmax: torch.Tensor, log_weight: torch.Tensor, levels: Sequence[float]) -> np.ndarray:
    """(1/N) sum_j exp(log_weight_j) [fmax_j >= a] for each level (device, FP64)."""
    lev = torch.tensor(list(levels), dtype=torch.float64, device=fmax.device)
    prob = torch.empty(len(lev), dtype=torch.float64, device=fmax.device)
    native.check(native.lib().tail_probability(_ptr(fmax), _ptr(log_weight.contiguous()), int(fmax.numel()),
                                               _ptr(lev), len(lev), _ptr(prob), _stream_handle(None)))
    return prob.cpu().numpy()


def return_time(prob: np.ndarray, block: float, window: float) -> np.ndarray:
    """r(a) = -(T_a - T) / ln(1 - P(a)) (paper Appendix C.2); inf where P = 0."""
    prob = np.asarray(prob, dtype=np.float64)
    out = np.full(prob.shape, math.inf)
    pos = prob > 0
    out[pos] = -(block - window) / np.log1p(-np.minimum(prob[pos], 1 - 1e-16))
    return out


def gktl_return_times(run: GktlRun, ens: Ensemble, window: int, levels: Sequence[float]):
    """Reweighted tail probability of the time-averaged drag and its return time (steps)."""
    tr = rebuild(run, ens)
    fmax = window_maxima(tr.series, window)
    prob = tail_probability(fmax, tr.log_weight, levels)
    return prob, return_time(prob, run.t_a, window), tr, fmax


def direct_return_times(series: torch.Tensor, block: int, window: int, levels: Sequence[float]):
    """Direct sampling: cut every row into blocks of `block` steps; fraction of blocks whose
    largest window mean reaches each level; r(a) = -(block - T)/ln(1 - P)."""
    rows, length = series.shape
    nb = length // block
    blocks = series[:, :nb * block].reshape(rows * nb, block)
    fmax = window_maxima(blocks, window)
    prob = tail_probability(fmax, torch.zeros_like(fmax), levels)
    return prob, return_time(prob, block, window), fmax
