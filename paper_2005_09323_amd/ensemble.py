"""Python face of the C ABI: an ensemble of channel-flow trajectories on one GPU.

PyTorch provides the device memory (population buffers, drag series,
accumulators) and the stream; every computation runs in the HIP library
through ``native``.  Calls are asynchronous on the current torch stream
unless stated otherwise.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import torch

from . import native


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclass(frozen=True)
class MemberSpec:
    """One trajectory's lattice: nx x ny cells, BGK time tau, body force along x, and the
    square obstacle as (x0, y0, side) of its lower-left solid cell (None: no obstacle)."""
    nx: int
    ny: int
    tau: float
    force_x: float
    square: Optional[Tuple[int, int, int]]


CHECKPOINT_VERSION = 1


class Ensemble:
    """Members (objects with nx, ny, tau, force_x, square) advanced together.

    series_capacity: drag columns kept per member (step 0 included).
    """

    def __init__(self, members: Sequence, series_capacity: int, device: str = "cuda",
                 stream: Optional[torch.cuda.Stream] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("the ensemble needs a GPU (HIP device)")
        self.lib = native.lib()
        self.members = list(members)
        self.n = len(self.members)
        self.device = torch.device(device)
        self._descs = native.desc_array(self.members)
        floats = self.lib.lbm_state_floats(self._descs, self.n)
        self.pop_a = torch.empty(floats, dtype=torch.float32, device=self.device)
        self.pop_b = torch.empty(floats, dtype=torch.float32, device=self.device)
        self.series = torch.zeros((self.n, series_capacity), dtype=torch.float32, device=self.device)
        self.accum = torch.zeros(self.n, dtype=torch.float64, device=self.device)
        self.capacity = series_capacity
        self.stream = stream
        self._ctx = ctypes.c_void_p()
        native.check(self.lib.lbm_create(ctypes.byref(self._ctx), self._descs, self.n, _ptr(self.pop_a),
                                         _ptr(self.pop_b), floats, _ptr(self.series), series_capacity,
                                         _ptr(self.accum), _stream_handle(stream)))
        self.offsets = []
        off = 0
        for m in self.members:
            self.offsets.append(off)
            off += 9 * m.nx * m.ny
        # the settings a checkpoint must carry to resume the same dynamics
        self._collision = ("bgk", 1.0, 1.0, 1.0)
        self._open = None
        self._observable = (0.0, 1.0, 1.0)
        self._active = None

    # -- lifetime -----------------------------------------------------------
    def close(self) -> None:
        if self._ctx:
            native.check(self.lib.lbm_destroy(self._ctx))
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping -----------------------------------------------------------
    def init(self, seed: int, noise_amp: float, ux0: float = 0.0) -> None:
        if ux0 == 0.0:
            native.check(self.lib.lbm_init(self._ctx, seed, noise_amp))
        else:
            native.check(self.lib.lbm_init_flow(self._ctx, seed, noise_amp, ux0))
        self._active = None  # the library makes every member active again

    def step(self, n_steps: int) -> None:
        native.check(self.lib.lbm_step_batch(self._ctx, n_steps))

    def set_observable(self, mu: float, sigma: float, dt: float) -> None:
        native.check(self.lib.lbm_set_observable(self._ctx, mu, sigma, dt))
        self._observable = (float(mu), float(sigma), float(dt))

    def set_active(self, active: Optional[Sequence[int]]) -> None:
        if active is None:
            native.check(self.lib.lbm_set_active(self._ctx, None))
            self._active = None
            return
        flags = [int(bool(a)) for a in active]
        arr = (ctypes.c_int32 * self.n)(*flags)
        native.check(self.lib.lbm_set_active(self._ctx, arr))
        self._active = flags

    def set_tile(self, tile_id: int) -> None:
        native.check(self.lib.lbm_set_tile(self._ctx, tile_id))

    def face_diagnostics(self) -> torch.Tensor:
        """[N, 5] FP64 on the device: forebody pressure, base pressure, drag from the stress
        integral, mean shear on the top and on the bottom face (next step's populations)."""
        out = torch.empty((self.n, 5), dtype=torch.float64, device=self.device)
        native.check(self.lib.lbm_face_diagnostics(self._ctx, _ptr(out)))
        return out

    def set_collision(self, model: str = "bgk", s_bulk: float = 1.0, s_third: float = 1.0,
                      s_fourth: float = 1.0) -> None:
        """'bgk' (default) or 'central' (central-moment relaxation with the given rates); before init."""
        code = {"bgk": 0, "central": 1}[model]
        native.check(self.lib.lbm_set_collision(self._ctx, code, s_bulk, s_third, s_fourth))
        self._collision = (model, float(s_bulk), float(s_third), float(s_fourth))

    def set_open_channel(self, u_c: Optional[float], grid_x0: int = 0, grid_bar: int = 0,
                         sponge_x0: int = 1 << 30, sponge_tau: float = 1.0, outlet_density: int = 0) -> None:
        """Inlet, entrance grid, sponge and outlet instead of periodic x (None: periodic); before init.
        outlet_density: 0 holds the outlet's density at 1, 1 extrapolates it to second order."""
        if u_c is None:
            native.check(self.lib.lbm_set_open_channel(self._ctx, None))
            self._open = None
            return
        oc = native.OpenChannelDesc(u_c, grid_x0, grid_bar, sponge_x0, outlet_density, sponge_tau)
        native.check(self.lib.lbm_set_open_channel(self._ctx, ctypes.byref(oc)))
        self._open = (float(u_c), int(grid_x0), int(grid_bar), int(sponge_x0), float(sponge_tau),
                      int(outlet_density))

    def set_cloning(self, relabel: bool) -> None:
        """GKTL copies by relabelling member blocks (default: only copies beyond the first of each
        ancestor move data) or by gathering every copy into the other buffer; same results."""
        native.check(self.lib.lbm_set_cloning(self._ctx, 1 if relabel else 0))

    def set_graphs(self, on: bool) -> None:
        """Replay full 64-step chunks from a captured HIP graph (default) or launch every kernel."""
        native.check(self.lib.lbm_set_graphs(self._ctx, 1 if on else 0))

    def launch_steps(self) -> int:
        """Lattice steps per launch of the shape in use (2 for the two-step kernel)."""
        n = ctypes.c_int32()
        native.check(self.lib.lbm_launch_steps(self._ctx, ctypes.byref(n)))
        return n.value

    def autotune(self, n_steps: int = 20, table: Optional[str] = None) -> int:
        """Time every launch shape and keep the fastest; with `table`, reuse or extend a persisted table."""
        best = ctypes.c_int32()
        if table is None:
            native.check(self.lib.lbm_autotune(self._ctx, n_steps, ctypes.byref(best)))
        else:
            native.check(self.lib.lbm_autotune_cached(self._ctx, n_steps, table.encode(), ctypes.byref(best)))
        return best.value

    def run_count(self) -> int:
        """Runs of consecutive members with one lattice shape."""
        n = ctypes.c_int32()
        native.check(self.lib.lbm_run_count(self._ctx, ctypes.byref(n)))
        return n.value

    def set_run_rows(self, rows: Optional[Sequence[int]]) -> None:
        """Rows per workgroup of each run in two-step launches (-1: as the shape says, 0: whole
        strips); None drops every choice."""
        if rows is None:
            native.check(self.lib.lbm_set_run_rows(self._ctx, None, 0))
            return
        arr = (ctypes.c_int32 * len(rows))(*[int(r) for r in rows])
        native.check(self.lib.lbm_set_run_rows(self._ctx, arr, len(rows)))

    def run_rows(self) -> list:
        """The rows per workgroup each run uses now (0: whole strips; -1: one-step launches)."""
        n = ctypes.c_int32()
        native.check(self.lib.lbm_get_run_rows(self._ctx, None, 0, ctypes.byref(n)))
        arr = (ctypes.c_int32 * max(n.value, 1))()
        native.check(self.lib.lbm_get_run_rows(self._ctx, arr, n.value, ctypes.byref(n)))
        return [int(arr[i]) for i in range(n.value)]

    def set_time(self, t: int) -> None:
        native.check(self.lib.lbm_set_time(self._ctx, t))

    # -- results ------------------------------------------------------------
    def time(self, m: int = 0) -> int:
        t = ctypes.c_int32()
        native.check(self.lib.lbm_member_time(self._ctx, m, ctypes.byref(t)))
        return t.value

    def drag(self, t0: int = 0, t1: Optional[int] = None) -> torch.Tensor:
        t1 = self.time(0) if t1 is None else t1
        out = torch.empty((self.n, t1 - t0), dtype=torch.float32, device=self.device)
        native.check(self.lib.lbm_drag(self._ctx, t0, t1, _ptr(out)))
        return out

    def state(self, m: int) -> torch.Tensor:
        """View [9, ny, nx] of member m's current state (deviations f_i - w_i)."""
        p = ctypes.c_void_p()
        native.check(self.lib.lbm_member_state(self._ctx, m, ctypes.byref(p)))
        mm = self.members[m]
        base = self.pop_a if p.value - self.pop_a.data_ptr() in range(0, self.pop_a.numel() * 4) else self.pop_b
        start = (p.value - base.data_ptr()) // 4
        return base[start:start + 9 * mm.nx * mm.ny].view(9, mm.ny, mm.nx)

    def flags(self) -> torch.Tensor:
        """int32[N] on the device: 1 where a member's drag became non-finite."""
        out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        native.check(self.lib.lbm_flags(self._ctx, _ptr(out)))
        return out

    def copy_state_out(self, m: int, dst: torch.Tensor) -> None:
        native.check(self.lib.lbm_copy_state_out(self._ctx, m, _ptr(dst)))

    def copy_state_in(self, m: int, src: torch.Tensor, t: int) -> None:
        native.check(self.lib.lbm_copy_state_in(self._ctx, m, _ptr(src), t))

    # -- checkpoint / resume -----------------------------------------------
    def checkpoint(self) -> dict:
        """Everything that decides the ensemble's future, as host tensors and plain values
        (synchronises): each member's state and time, the drag series, the FP64 observable
        integrals, the non-finite flags, the active mask, and the settings (collision, open channel, observable).
        The selection and perturbation draws need no saved state: they are counter-based,
        keyed by (key, period)."""
        torch.cuda.synchronize(self.device)
        states = torch.cat([self.state(m).reshape(-1) for m in range(self.n)]).cpu()
        return {
            "version": CHECKPOINT_VERSION,
            "members": [(int(m.nx), int(m.ny), float(m.tau), float(m.force_x),
                         None if m.square is None else tuple(int(v) for v in m.square)) for m in self.members],
            "capacity": int(self.capacity),
            "states": states,
            "times": torch.tensor([self.time(m) for m in range(self.n)], dtype=torch.int32),
            "series": self.series.cpu(),
            "accum": self.accum.cpu(),
            "flags": self.flags().cpu(),
            "active": None if self._active is None else list(self._active),
            "collision": self._collision,
            "open": self._open,
            "observable": self._observable,
        }

    @classmethod
    def restore(cls, ckpt: dict, device: str = "cuda", stream: Optional[torch.cuda.Stream] = None) -> "Ensemble":
        """A new ensemble that continues exactly where `ckpt` (from `checkpoint`) left off."""
        if ckpt.get("version") != CHECKPOINT_VERSION:
            raise ValueError(f"checkpoint version {ckpt.get('version')} (expected {CHECKPOINT_VERSION})")
        members = [MemberSpec(nx, ny, tau, fx, None if sq is None else tuple(sq))
                   for nx, ny, tau, fx, sq in ckpt["members"]]
        ens = cls(members, ckpt["capacity"], device=device, stream=stream)
        model, sb, s3, s4 = ckpt["collision"]
        ens.set_collision(model, sb, s3, s4)
        if ckpt["open"] is not None:
            ens.set_open_channel(*ckpt["open"])
        ens.set_observable(*ckpt["observable"])
        ens.set_active(ckpt["active"])
        states = ckpt["states"].to(ens.device)
        times = ckpt["times"].tolist()
        for m in range(ens.n):
            o, mm = ens.offsets[m], ens.members[m]
            ens.copy_state_in(m, states[o:o + 9 * mm.nx * mm.ny], times[m])
        ens.series.copy_(ckpt["series"])
        ens.accum.copy_(ckpt["accum"])
        flags = ckpt["flags"].to(device=ens.device, dtype=torch.int32).contiguous()
        native.check(ens.lib.lbm_set_flags(ens._ctx, _ptr(flags)))
        torch.cuda.synchronize(ens.device)  # the staging copy of the states must outlive the copies
        return ens

    def save(self, path: str) -> None:
        torch.save(self.checkpoint(), path)

    @classmethod
    def load(cls, path: str, device: str = "cuda", stream: Optional[torch.cuda.Stream] = None) -> "Ensemble":
        """Read a checkpoint written by `save` (plain tensors and values only) and restore it."""
        return cls.restore(torch.load(path, map_location="cpu", weights_only=True), device=device, stream=stream)

    # -- rare-event selection ----------------------------------------------
    def gktl_select_clone(self, k: float, key: int, period: int, eps: float = 0.0,
                          snapshots: Optional[torch.Tensor] = None):
        """Returns (ancestors int32[N] device, ln R float64[1] device)."""
        anc = torch.empty(self.n, dtype=torch.int32, device=self.device)
        lnr = torch.empty(1, dtype=torch.float64, device=self.device)
        n_snap = 0 if snapshots is None else int(snapshots.shape[0])
        native.check(self.lib.gktl_select_clone(self._ctx, k, key, period, eps, _ptr(snapshots), n_snap,
                                                _ptr(anc), _ptr(lnr)))
        return anc, lnr

    def features(self, m0: int, n: int, px0: int, py0: int, patch: int, pool: int,
                 u_scale: float, rho_scale: float) -> torch.Tensor:
        """Near-wake feature pictures [n, 3, patch/pool, patch/pool] of members m0 .. m0+n-1."""
        side = patch // pool
        out = torch.empty((n, 3, side, side), dtype=torch.float32, device=self.device)
        native.check(self.lib.score_features(self._ctx, m0, n, px0, py0, patch, pool, u_scale, rho_scale,
                                             _ptr(out)))
        return out

    def features_active(self, px0: int, py0: int, patch: int, pool: int, u_scale: float,
                        rho_scale: float) -> torch.Tensor:
        """Feature pictures of the active members, in ascending member order:
        [n_active, 3, patch/pool, patch/pool]."""
        side = patch // pool
        n_act = self.n if self._active is None else sum(self._active)
        out = torch.empty((n_act, 3, side, side), dtype=torch.float32, device=self.device)
        rows = ctypes.c_int32()
        native.check(self.lib.score_features_active(self._ctx, px0, py0, patch, pool, u_scale, rho_scale,
                                                    _ptr(out), n_act, ctypes.byref(rows)))
        if rows.value != n_act:
            raise RuntimeError(f"the library has {rows.value} active members, the ensemble {n_act}")
        return out

    def perturb(self, mask: Sequence[int], key: int, period: int, eps: float, snapshots: torch.Tensor) -> None:
        arr = (ctypes.c_int32 * self.n)(*[int(bool(a)) for a in mask])
        native.check(self.lib.lbm_perturb(self._ctx, arr, key, period, eps, _ptr(snapshots),
                                          int(snapshots.shape[0])))


def window_mean(series: torch.Tensor, window: int, t_len: Optional[int] = None) -> torch.Tensor:
    """out[m, t] = mean of series[m, t-window+1 .. t] (FP64 sums), -inf before the first full window."""
    n, ld = series.shape
    t_len = ld if t_len is None else t_len
    out = torch.empty((n, t_len), dtype=torch.float32, device=series.device)
    native.check(native.lib().lbm_window_mean(_ptr(series), n, ld, t_len, window, _ptr(out),
                                              _stream_handle(None)))
    return out


def ams_score_kill_branch(series: torch.Tensor, n_kill: int, key: int, iteration: int):
    """AMS selection on score series [N, T]; returns a dict of device tensors and host values (synchronises)."""
    n, t_len = series.shape
    dev = series.device
    killed = torch.empty(n, dtype=torch.int32, device=dev)
    parent = torch.empty(n, dtype=torch.int32, device=dev)
    branch_t = torch.empty(n, dtype=torch.int32, device=dev)
    n_killed = torch.empty(1, dtype=torch.int32, device=dev)
    level = torch.empty(1, dtype=torch.float32, device=dev)
    maxima = torch.empty(n, dtype=torch.float32, device=dev)
    native.check(native.lib().ams_score_kill_branch(_ptr(series), n, t_len, n_kill, key, iteration,
                                                    _ptr(killed), _ptr(parent), _ptr(branch_t),
                                                    _ptr(n_killed), _ptr(level), _ptr(maxima),
                                                    _stream_handle(None)))
    k = int(n_killed.item())
    return dict(killed=killed[:k], parents=parent[:k], branch_t=branch_t[:k], level=float(level.item()),
                maxima=maxima, n_killed=k)


class ScoreNet:
    """The learned AMS score network: FP32 master parameters on the device, BF16 matrix-core kernels."""

    def __init__(self, params: torch.Tensor, max_batch: int, device: str = "cuda"):
        self.lib = native.lib()
        self.n_params = self.lib.score_net_params()
        if params.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {params.numel()}")
        self.params = params.detach().to(device=device, dtype=torch.float32).contiguous().clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.step_count = 0
        self.max_batch = max_batch
        nbytes = self.lib.score_net_workspace_bytes(max_batch)
        self.workspace = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=device)
        self._ws_bytes = nbytes

    def _check(self, x: torch.Tensor) -> int:
        if x.dim() != 4 or tuple(x.shape[1:]) != (3, 16, 16) or x.dtype != torch.float32 or not x.is_contiguous():
            raise ValueError("x must be a contiguous float32 [B, 3, 16, 16] tensor")
        if x.shape[0] > self.max_batch:
            raise ValueError("batch larger than max_batch")
        return int(x.shape[0])

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        b = self._check(x)
        y = torch.empty(b, dtype=torch.float32, device=x.device)
        native.check(self.lib.score_net_forward(_ptr(self.params), _ptr(x), b, _ptr(y), _ptr(self.workspace),
                                                self._ws_bytes, _stream_handle(None)))
        return y

    def grad(self, x: torch.Tensor, labels: torch.Tensor) -> torch.Tensor:
        """Gradient of the mean squared error into self.grads (returned); the loss into self.loss."""
        b = self._check(x)
        native.check(self.lib.score_net_grad(_ptr(self.params), _ptr(x), _ptr(labels.contiguous()), b,
                                             _ptr(self.grads), _ptr(self.loss), _ptr(self.workspace),
                                             self._ws_bytes, _stream_handle(None)))
        return self.grads

    def adam(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        self.step_count += 1
        native.check(self.lib.score_net_adam(_ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(self.grads),
                                             self.step_count, lr, beta1, beta2, eps, _stream_handle(None)))

    def train_step(self, x: torch.Tensor, labels: torch.Tensor, lr: float = 1e-3) -> torch.Tensor:
        self.grad(x, labels)
        self.adam(lr)
        return self.loss
