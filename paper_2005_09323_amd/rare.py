"""GKTL and trajectory-AMS drivers over the device kernels.

The drivers only order the library calls (stepping, selection, cloning,
checkpoint copies, estimators); every computation runs on the GPU.  Paper
references: GKTL, Section 4.2 and Appendix C; AMS, Section 4.1 and Appendix B;
perturbation at branching, Appendix D.
"""
from __future__ import annotations

import ctypes
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
        """lambda(k) = (1/T_a) sum_i ln R_i, T_a in the units of dt (device, FP64)."""
        ln_r = self.ln_r.to(device="cuda", dtype=torch.float64).contiguous()
        out = torch.empty(1, dtype=torch.float64, device=ln_r.device)
        native.check(native.lib().gktl_scgf(_ptr(ln_r), int(ln_r.numel()), float(self.t_a * dt), _ptr(out),
                                            _stream_handle(None)))
        return float(out.item())

    def then(self, later: "GktlRun") -> "GktlRun":
        """This run followed by `later`, its continuation (same k and tau, its periods numbered on
        from this run's, its drag columns right after this run's): one record of the whole run."""
        if later.k != self.k or later.tau != self.tau:
            raise ValueError("a continuation needs the same k and tau")
        if later.col0 != self.col0 + self.t_a:
            raise ValueError("the continuation must start at the column this run ended on")
        return GktlRun(self.k, self.tau, self.n_periods + later.n_periods, self.col0,
                       torch.cat([self.ancestors, later.ancestors]), torch.cat([self.integrals, later.integrals]),
                       torch.cat([self.ln_r, later.ln_r]))


def run_gktl(ens: Ensemble, k: float, n_periods: int, tau: int, key: int, eps: float = 0.0,
             snapshots: Optional[torch.Tensor] = None, first_period: int = 0) -> GktlRun:
    """GKTL over n_periods cloning periods of tau steps, selecting at every t_i = i tau (T_a included).

    The ensemble must be initialised and its observable set (lbm_set_observable);
    its drag series needs tau * n_periods free columns.  first_period numbers the
    periods (the selection and perturbation draws are keyed by it): a run resumed
    from a checkpoint taken after p periods continues with first_period = p, and
    `GktlRun.then` joins the two records.
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
        native.check(lib.gktl_select_clone(ens._ctx, k, key, first_period + i, eps, _ptr(snapshots), n_snap,
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
    """r(a) = -(T_a - T) / ln(1 - P(a)) (paper Appendix C.2); inf where P = 0 (device, FP64)."""
    p = torch.as_tensor(np.asarray(prob, dtype=np.float64)).reshape(-1).to("cuda").contiguous()
    r = torch.empty_like(p)
    native.check(native.lib().return_times(_ptr(p), int(p.numel()), float(block), float(window), _ptr(r),
                                           _stream_handle(None)))
    return r.cpu().numpy().reshape(np.shape(prob))


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


# ---------------------------------------------------------------------------
# trajectory AMS on the lattice-Boltzmann ensemble


@dataclass
class AmsResult:
    n: int
    k_history: List[int] = field(default_factory=list)
    levels: List[float] = field(default_factory=list)
    extinct: bool = False
    member_steps: int = 0          # simulated member-steps, re-simulation and replay included
    score_max: Optional[np.ndarray] = None   # final maxima of the score, per member
    event_max: Optional[np.ndarray] = None   # final maxima of F_T on the score grid, per member

    def probability(self, levels: Sequence[float]) -> np.ndarray:
        """prod_j (1 - K_j / N) * (1/N) #{n : max F_T >= a}: the unbiased AMS estimate for levels at
        or above the one every trajectory reached when the run stopped (below it, the final ensemble
        no longer holds the trajectories that were discarded on the way)."""
        kh = torch.tensor(list(self.k_history), dtype=torch.int32, device="cuda")
        q = torch.as_tensor(np.asarray(self.event_max, dtype=np.float64)).to("cuda").contiguous()
        lev = torch.tensor(list(levels), dtype=torch.float64, device="cuda")
        prob = torch.empty_like(lev)
        native.check(native.lib().ams_probability(_ptr(kh) if kh.numel() else None, int(kh.numel()), self.n,
                                                  _ptr(q), _ptr(lev), int(lev.numel()), _ptr(prob),
                                                  _stream_handle(None)))
        return prob.cpu().numpy()


class AmsRunner:
    """Trajectory AMS with branching from checkpoints (paper Section 4.1, Appendix B.1).

    Every member runs t_a steps from its current state.  The score lives on a
    grid of `stride` steps: the time-averaged drag F_T(t) over the last `window`
    steps (plain) or, with a score network, the network's prediction mapped
    strictly increasingly below the target level until the event has happened
    (learned; `width` sets how soon the map bends towards the level).  A killed member restarts from its parent's
    last checkpoint before the branching time, replays the parent's dynamics
    exactly (the kernels are deterministic) up to the branching time, is
    perturbed there (Appendix D) and runs on to t_a.
    """

    def __init__(self, ens: Ensemble, t_a: int, window: int, stride: int, ckpt_every: int, key: int,
                 eps: float, snapshots: torch.Tensor, net=None, feature_args: Optional[dict] = None,
                 target: Optional[float] = None, width: Optional[float] = None):
        if t_a % ckpt_every or ckpt_every % stride:
            raise ValueError("t_a must be a multiple of ckpt_every, itself a multiple of stride")
        if net is not None and (feature_args is None or target is None or width is None):
            raise ValueError("a learned score needs feature_args, the target level and the map's width")
        if ens.capacity < t_a + 1:
            raise ValueError("the drag series needs t_a + 1 columns")
        self.ens, self.t_a, self.window, self.stride, self.ckpt = ens, t_a, window, stride, ckpt_every
        self.key, self.eps, self.snaps = key, eps, snapshots
        # scores are FP32: the clamp level and the stopping level are taken at FP32 so that a
        # trajectory whose score reached the level also compares as having reached it here
        self.net, self.fargs = net, feature_args
        self.target = None if target is None else float(np.float32(target))
        self.width = None if width is None else float(width)
        m = ens.members[0]
        self.state_floats = 9 * m.nx * m.ny
        n = ens.n
        self.n_score = t_a // stride
        self.ckpts = torch.empty((n, t_a // ckpt_every + 1, self.state_floats), dtype=torch.float32, device=ens.device)
        self.ghat = torch.full((n, self.n_score), float("-inf"), dtype=torch.float32, device=ens.device)
        self.time = np.zeros(n, dtype=np.int64)
        self._fcache = None  # (members, their grid columns, their flat grid positions on the device)

    # -- stepping ----------------------------------------------------------
    def _features(self, members: Sequence[int], times: np.ndarray) -> None:
        """Network scores of `members` (the active members) at their current times: one feature
        pass and one forward pass over the active members only, one scatter into the score grid.

        The scatter's row and column indices stay on the device while the active set is the same
        (its members step together, so every column moves by the same count): a stride copies
        nothing from the host and never waits for the device."""
        if self.net is None:
            return
        order = sorted(members)
        cols = times[order] // self.stride - 1
        c = self._fcache
        if (c is None or c[0] != tuple(order) or cols[0] < c[1][0]
                or np.any(cols - c[1] != cols[0] - c[1][0])):
            # flat positions in the score grid at the columns of this moment
            flat = np.asarray(order, dtype=np.int64) * self.n_score + cols
            pos = torch.as_tensor(flat).pin_memory().to(self.ghat.device, non_blocking=True)
            self._fcache = c = (tuple(order), cols.copy(), pos)
        f = self.ens.features_active(**self.fargs)  # rows in ascending member order
        if f.shape[0] != len(order):
            raise RuntimeError("the ensemble's active members differ from the members being scored")
        step = self.net.max_batch
        y = (self.net.forward(f) if f.shape[0] <= step else
             torch.cat([self.net.forward(f[b:b + step]) for b in range(0, f.shape[0], step)]))
        # every column has moved on by the same count since the positions were made: index the
        # flat grid from that offset (a view, no kernel) rather than adding it to the positions
        self.ghat.view(-1)[int(cols[0] - c[1][0]):].index_put_((c[2],), y)

    def _advance(self, members: Sequence[int], perturb_at: dict, period: int) -> int:
        """Run `members` from their times to t_a on the stride grid; returns member-steps.

        The active members step together up to the next time at which one of them has something
        to do: a checkpoint, its branching perturbation, the end of its trajectory, and, with a
        learned score, every point of the score grid (the network's score needs the state)."""
        ens = self.ens
        n = ens.n
        active = [m for m in members if self.time[m] < self.t_a]
        steps = 0
        mask_now = None
        while active:
            mask = np.zeros(n, dtype=np.int32)
            mask[active] = 1
            if mask_now is None or not np.array_equal(mask, mask_now):
                ens.set_active(mask.tolist())
                mask_now = mask
            if self.net is not None:
                delta = self.stride
            else:
                delta = self.t_a
                for m in active:  # no member may step past its own next event
                    t = int(self.time[m])
                    nxt = min((t // self.ckpt + 1) * self.ckpt, self.t_a)
                    tb = perturb_at.get(m, -1)
                    if tb > t:
                        nxt = min(nxt, tb)
                    delta = min(delta, nxt - t)
            ens.step(delta)
            steps += delta * len(active)
            self.time[active] += delta
            self._features(active, self.time)  # before any perturbation: the child still equals its parent
            pert = [m for m in active if perturb_at.get(m, -1) == self.time[m]]
            if pert and self.eps != 0.0:
                pmask = np.zeros(n, dtype=np.int32)
                pmask[pert] = 1
                ens.perturb(pmask.tolist(), self.key, period, self.eps, self.snaps)
            for m in active:
                if self.time[m] % self.ckpt == 0:
                    ens.copy_state_out(m, self.ckpts[m, self.time[m] // self.ckpt])
            active = [m for m in active if self.time[m] < self.t_a]
        ens.set_active(None)
        return steps

    # -- scores ---------------------------------------------------------------
    def event_series(self) -> torch.Tensor:
        """F_T on the score grid: [N, t_a / stride] (-inf before the first full window)."""
        ft = window_mean(self.ens.series[:, 1:self.t_a + 1].contiguous(), self.window)
        return ft[:, self.stride - 1::self.stride].contiguous()

    def score_series(self) -> torch.Tensor:
        ft = self.event_series()
        if self.net is None:
            return ft
        out = torch.empty_like(ft)
        native.check(native.lib().ams_learned_score(_ptr(self.ghat), _ptr(ft), ft.numel(), float(self.target),
                                                    self.width, _ptr(out), _stream_handle(None)))
        return out

    # -- the algorithm --------------------------------------------------------
    def run(self, n_kill: int, max_iter: int, threshold: float) -> AmsResult:
        threshold = float(np.float32(threshold))
        ens = self.ens
        n = ens.n
        res = AmsResult(n=n)
        ens.set_time(1)
        for m in range(n):
            ens.copy_state_out(m, self.ckpts[m, 0])
        self.time[:] = 0
        res.member_steps += self._advance(range(n), {}, 0)
        for it in range(max_iter):
            score = self.score_series()
            sel = ams_score_kill_branch(score, n_kill, self.key, it)
            maxima = sel["maxima"].double().cpu().numpy()
            if maxima.min() >= threshold or sel["level"] >= threshold:
                break  # every trajectory reached the target, or the level did (killing would discard hits)
            if sel["parents"].numel() and int(sel["parents"][0].item()) < 0:
                res.extinct = True
                break
            killed = sel["killed"].cpu().tolist()
            parents = sel["parents"].cpu().tolist()
            branch = sel["branch_t"].cpu().tolist()
            res.k_history.append(len(killed))
            res.levels.append(sel["level"])
            perturb_at = {}
            for k, p, tb in zip(killed, parents, branch):
                t_b = (tb + 1) * self.stride              # score index -> trajectory time
                c = t_b // self.ckpt
                start = c * self.ckpt
                ens.copy_state_in(k, self.ckpts[p, c], start + 1)
                self.ckpts[k, :c + 1].copy_(self.ckpts[p, :c + 1])
                ens.series[k, 1:start + 1].copy_(ens.series[p, 1:start + 1])
                self.ghat[k, :start // self.stride].copy_(self.ghat[p, :start // self.stride])
                self.time[k] = start
                if start == t_b:
                    # branching exactly on a checkpoint: perturb the restored state now
                    mask = np.zeros(n, dtype=np.int32)
                    mask[k] = 1
                    if self.eps != 0.0:
                        ens.perturb(mask.tolist(), self.key, it + 1, self.eps, self.snaps)
                    ens.copy_state_out(k, self.ckpts[k, c])
                else:
                    perturb_at[k] = t_b
            res.member_steps += self._advance(killed, perturb_at, it + 1)
        score = self.score_series()
        res.score_max = torch.max(score, dim=1).values.double().cpu().numpy()
        res.event_max = torch.max(self.event_series(), dim=1).values.double().cpu().numpy()
        return res
