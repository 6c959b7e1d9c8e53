"""Benchmark: ensemble lattice-Boltzmann throughput on one MI355X.

Workload (default): 128 independent trajectories of the 1024 x 256 channel
with a 32 x 32 square (tau 0.5015, g_x 3e-6), advanced together by the fused
pull-stream/collide kernel with per-step momentum-exchange drag and the FP64
observable integral.  One timed step = one lattice step of the whole
ensemble (every member: stream, collide, drag; the drag reduction and FP64
accumulation run once per 64-step chunk inside the timed region).

Prints one JSON line.  ``value`` is ensemble MLUPS (all cells of all members
times steps per second); ``roofline`` prices the step kernel against HBM at
72 algorithmic bytes per fluid-cell update (9 FP32 loads + 9 FP32 stores).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ensemble MLUPS + % HBM roofline; GKTL/AMS wall time to 10% return-time error"
HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = 72


def _workload(name):
    import workloads
    if name == "ensemble":
        return workloads.ensemble_1024()
    if name == "mixed":
        return workloads.mixed_sizes()
    if name == "single":
        return workloads.single_channel()
    if name == "open":
        return workloads.open_channel()
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(wl, steps: int):
    """Time the FP64 oracle on member 0 of the workload (single thread)."""
    from threadpoolctl import threadpool_limits

    from oracle import lbm as olbm
    m = wl.members[0]
    op = wl.extra.get("open")
    if op is None:
        ch = olbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square)
        f = olbm.init_populations(ch, olbm.init_density(ch, wl.seed, 0, wl.noise_amp))
    else:
        import numpy as np

        from oracle.open_channel import OpenChannel, inlet_velocity
        ch = olbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square, wl.extra.get("rates"),
                          open=OpenChannel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau))
        u = np.repeat(inlet_velocity(ch)[:, None], ch.nx, axis=1)
        f = olbm.equilibrium(olbm.init_density(ch, wl.seed, 0, wl.noise_amp), u, np.zeros_like(u))
        f[:, olbm.solid_mask(ch)] = 0.0
    with threadpool_limits(limits=1):
        olbm.run(ch, f, 2)  # warm caches of the geometry tables
        t0 = time.perf_counter()
        olbm.run(ch, f, steps)
        dt = time.perf_counter() - t0
        single = _oracle_single_channel()
    host = f"{cpu_model()}, os.cpu_count()={os.cpu_count()}"
    return {"value": round(m.cells * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"member 0 ({m.nx}x{m.ny}) of the same workload, {steps} steps, FP64 numpy, 1 thread; "
                      f"host {host}",
            "host_cpu": host, "single_channel_full": single}


def _oracle_single_channel():
    """The FP64 oracle on the whole single-channel workload (1 x 256 x 64, 2000 steps), one thread."""
    import workloads
    from oracle import lbm as olbm
    wl = workloads.single_channel()
    m = wl.members[0]
    ch = olbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square)
    f = olbm.init_populations(ch, olbm.init_density(ch, wl.seed, 0, wl.noise_amp))
    t0 = time.perf_counter()
    olbm.run(ch, f, wl.steps)
    dt = time.perf_counter() - t0
    return {"workload": wl.name, "steps": wl.steps, "seconds": round(dt, 3),
            "MLUPS": round(m.cells * wl.steps / dt / 1e6, 4), "cores": 1}


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo where there is one)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def copy_calibration(mib: int, reps: int) -> None:
    """Plain device-to-device copy of known size: reference for HBM byte counters and bandwidth."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    print(json.dumps({"mode": "copy", "bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n,
                      "ms_per_copy": round(sec * 1e3, 4), "GBps_read_plus_write": round(8 * n / sec / 1e9, 1)}),
          flush=True)


def copy_bandwidth(mib: int = 1024, reps: int = 5) -> float:
    """Read + write GB/s of a plain device-to-device copy of `mib` MiB (the box's practical ceiling)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ms = _timed(lambda: dst.copy_(src), reps)
    del src, dst
    torch.cuda.empty_cache()
    return 8 * n / (ms / 1e3) / 1e9


def _timed(fn, reps=1):
    """Milliseconds per call of fn on the current stream (HIP events)."""
    import torch
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


KERNEL_SOURCES = ("common.hpp", "kernels.hpp", "lbm_device.hpp", "lbm_kernels.hip", "lbm_step2.hip")


def kernel_sources_sha256() -> str:
    """Hash of the lattice kernels' code (the counters in the traffic record belong to one version).

    Line comments, trailing blanks and empty lines are left out, so that a change of wording
    does not retire the record; any change of code does."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, "paper_2005_09323_amd", "csrc", name)).read()
        for line in text.splitlines():
            code = re.sub(r"//.*$", "", line).rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()


def legs():
    """Secondary measurements of the other rows of the path (one short run each)."""
    import numpy as np
    import torch

    import workloads
    from paper_2005_09323_amd.ensemble import Ensemble, ScoreNet, ams_score_kill_branch, window_mean
    out = {}
    # GKTL: one cloning period of 256 steps on 256 x 1024 x 256, then device selection + clone/perturb
    wl = workloads.gktl_ensemble()
    x = wl.extra
    ens = Ensemble(wl.members, series_capacity=2 * x["period"] + 2)
    ens.init(wl.seed, wl.noise_amp)
    ens.set_observable(0.0, 1e-3, x["dt"])
    snaps = torch.from_numpy(workloads.snapshot_states(x["n_snap"], wl.members[0], 1)).cuda()
    ens.step(x["period"])
    torch.cuda.synchronize()
    t_steps = _timed(lambda: ens.step(x["period"]))
    # the first clone allocates the selection scratch (pinned host mirrors included): untimed
    ens.gktl_select_clone(1.0, 1, 0, x["eps"], snaps)
    torch.cuda.synchronize()
    t_clone = _timed(lambda: ens.gktl_select_clone(1.0, 1, 1, x["eps"], snaps), 5)
    cells = wl.cells
    out["gktl_period"] = {"workload": wl.name, "period_steps": x["period"], "ms_steps": round(t_steps, 3),
                          "ms_select_clone": round(t_clone, 3),
                          "clone_overhead": round(t_clone / t_steps, 5),
                          "MLUPS_with_cloning": round(cells * x["period"] / ((t_steps + t_clone) / 1e3) / 1e6, 1)}
    ens.close()
    del ens
    torch.cuda.empty_cache()
    # AMS: selection over 512 members' window-mean scores of 2560-step drag series
    wl = workloads.ams_ensemble()
    series = torch.from_numpy(workloads.score_series(len(wl.members), wl.steps, 3)).cuda()
    t_win = _timed(lambda: window_mean(series, wl.extra["window"]), 3)
    score = window_mean(series, wl.extra["window"])
    t_sel = _timed(lambda: ams_score_kill_branch(score, 26, 1, 0), 3)
    out["ams_selection"] = {"workload": wl.name, "ms_window_mean": round(t_win, 3), "ms_kill_branch": round(t_sel, 3)}
    # learned score: one training step (forward + backward + Adam) on a batch of 256 pictures
    p = workloads.cnn_params(1)
    flat = np.concatenate([np.ravel(p[k]) for k in ("w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4")])
    net = ScoreNet(torch.from_numpy(flat.astype(np.float32)), 256)
    xb, lb = workloads.cnn_batch(256, 2)
    xt = torch.from_numpy(xb.astype(np.float32)).cuda()
    lt = torch.from_numpy(lb.astype(np.float32)).cuda()
    net.train_step(xt, lt)
    t_train = _timed(lambda: net.train_step(xt, lt), 10)
    t_fwd = _timed(lambda: net.forward(xt), 10)
    flop_fwd = 256 * 32 * 2 * (27 + 288 + 288)            # per picture, convolutions only
    flop_train = flop_fwd + 256 * 32 * 2 * (288 + 288) + 256 * 32 * 2 * (27 + 288 + 288)
    out["score_net"] = {"batch": 256, "ms_train_step": round(t_train, 4), "ms_forward": round(t_fwd, 4),
                        "pictures_per_s_train": round(256 / (t_train / 1e3), 1),
                        "mfma_TFLOPs_train": round(256 * flop_train / (t_train / 1e3) / 1e12, 3),
                        "mfma_TFLOPs_forward": round(256 * flop_fwd / (t_fwd / 1e3) / 1e12, 3)}
    del net, xt, lt
    # uneven sizes in one launch: 64 members each of 256x64, 512x128 and 1024x256
    wl = workloads.mixed_sizes()
    ens = Ensemble(wl.members, series_capacity=300)
    ens.init(wl.seed, wl.noise_amp)
    ens.step(20)
    torch.cuda.synchronize()
    t_mixed = _timed(lambda: ens.step(256)) / 256
    fluid = sum(m.fluid_cells for m in wl.members)
    out["mixed_sizes"] = {"workload": wl.name, "steps_per_launch": ens.launch_steps(),
                          "ms_per_step": round(t_mixed, 4), "MLUPS": round(wl.cells / t_mixed / 1e3, 1),
                          "GBs_72B_per_update": round(BYTES_PER_LUP * fluid / t_mixed / 1e6, 1),
                          "nonfinite_members": int(ens.flags().sum().item())}
    ens.close()
    del ens
    torch.cuda.empty_cache()
    # the same batch with its launch shape tuned, and a row range per lattice size
    ens = Ensemble(wl.members, series_capacity=300)
    tile = ens.autotune(16)
    ens.init(wl.seed, wl.noise_amp)
    ens.step(20)
    torch.cuda.synchronize()
    t_tuned = _timed(lambda: ens.step(256)) / 256
    out["mixed_sizes"]["tuned"] = {"tile": tile, "rows_per_workgroup_per_size": ens.run_rows(),
                                   "ms_per_step": round(t_tuned, 4), "MLUPS": round(wl.cells / t_tuned / 1e3, 1)}
    ens.close()
    del ens
    torch.cuda.empty_cache()
    # launch-bound batches (an AMS branch re-simulates a handful of members): full 64-step chunks
    # replayed from a captured HIP graph against launching every kernel of every chunk
    m = workloads.ams_ensemble().members[0]
    small = {}
    for graphs in (True, False):
        ens = Ensemble([m] * 16, series_capacity=1100)
        ens.set_graphs(graphs)
        ens.init(1, 1e-3)
        ens.step(64)
        torch.cuda.synchronize()
        small["graphs" if graphs else "launches"] = _timed(lambda: ens.step(1024)) / 1024
        ens.close()
    out["small_batch"] = {"workload": "16 x 512x128 (AMS branch size)", "ms_per_step_graphs": round(small["graphs"], 5),
                          "ms_per_step_launches": round(small["launches"], 5),
                          "MLUPS_graphs": round(16 * m.cells / small["graphs"] / 1e3, 1),
                          "MLUPS_launches": round(16 * m.cells / small["launches"] / 1e3, 1)}
    # the paper's open channel (inlet, grid, sponge, outlet ghost column), central moments:
    # one step per launch plus the small ghost-column launch
    wl = workloads.open_channel()
    op = wl.extra["open"]
    ens = Ensemble(wl.members, series_capacity=301)
    ens.set_collision("central", *wl.extra["rates"])
    ens.set_open_channel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau)
    ens.init(wl.seed, wl.noise_amp)
    ens.step(20)
    torch.cuda.synchronize()
    t_open = _timed(lambda: ens.step(256))
    fluid = sum(m.fluid_cells for m in wl.members) - len(wl.members) * _grid_cells(wl.members[0], op)
    gbs = BYTES_PER_LUP * fluid * 256 / (t_open / 1e3) / 1e9
    out["open_channel"] = {"workload": wl.name, "collision": "central", "steps": 256,
                           "ms_per_step": round(t_open / 256, 4),
                           "MLUPS": round(wl.cells * 256 / (t_open / 1e3) / 1e6, 1),
                           "GBs_per_step_72B": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                           "nonfinite_members": int(ens.flags().sum().item())}
    ens.close()
    return out


def _grid_cells(m, op) -> int:
    """Solid cells of an open channel's entrance grid (bars of op.bar rows and columns)."""
    b = op.bar
    return b * sum(1 for y in range(b // 2, m.ny) if (y - b // 2) % (2 * b) < b) if b > 0 else 0


def score_scaling(batches) -> None:
    """Score network forward and training step (forward, backward, reduction, Adam) against the
    batch size: one JSON line per batch, BF16 matrix-core TFLOP/s of the convolutions."""
    import numpy as np
    import torch

    import workloads
    from paper_2005_09323_amd.ensemble import ScoreNet

    torch.cuda.set_device(0)
    p = workloads.cnn_params(1)
    flat = np.concatenate([np.ravel(p[k]) for k in ("w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4")])
    flop_fwd = 256 * 32 * 2 * (27 + 288 + 288)            # per picture, convolutions only
    flop_train = flop_fwd + 256 * 32 * 2 * (288 + 288) + 256 * 32 * 2 * (27 + 288 + 288)
    for b in batches:
        net = ScoreNet(torch.from_numpy(flat.astype(np.float32)), b)
        xb, lb = workloads.cnn_batch(b, 2)
        xt = torch.from_numpy(xb.astype(np.float32)).cuda()
        lt = torch.from_numpy(lb.astype(np.float32)).cuda()
        net.train_step(xt, lt)
        t_fwd = _timed(lambda: net.forward(xt), 20)
        t_train = _timed(lambda: net.train_step(xt, lt), 20)
        print(json.dumps({"batch": b, "ms_forward": round(t_fwd, 4), "ms_train_step": round(t_train, 4),
                          "mfma_TFLOPs_forward": round(b * flop_fwd / (t_fwd / 1e3) / 1e12, 1),
                          "mfma_TFLOPs_train": round(b * flop_train / (t_train / 1e3) / 1e12, 1),
                          "frac_of_bf16_peak_forward": round(b * flop_fwd / (t_fwd / 1e3) / 2.5e15, 4)}),
              flush=True)
        del net, xt, lt
        torch.cuda.empty_cache()


def open_parts(steps: int = 256) -> None:
    """Where the open channel's time goes: 1024 members of 512 x 128 with the square R = 16
    at the centre, the two-step kernel, with parts of the open channel (entrance grid, sponge)
    taken away and against periodic x.  One JSON line per variant, ms per lattice step."""
    import torch

    import workloads
    from paper_2005_09323_amd.ensemble import Ensemble

    torch.cuda.set_device(0)
    sq = workloads.centred_square(256, 64, 16)
    with_sq = workloads.Member(512, 128, 0.501, 0.0, sq)
    no_sq = workloads.Member(512, 128, 0.501, 0.0, None)
    full = (0.05, 32, 8, 447, 1.0)
    variants = [("open, central moments", with_sq, full, True),
                ("open, central moments, no grid", with_sq, (0.05, 32, 0, 447, 1.0), True),
                ("open, central moments, no sponge", with_sq, (0.05, 32, 8, 1 << 30, 1.0), True),
                ("open, BGK", with_sq, full, False),
                ("periodic, central moments", with_sq, None, True),
                ("periodic, central moments, no square", no_sq, None, True),
                ("periodic, BGK", with_sq, None, False),
                ("periodic, BGK, no square", no_sq, None, False)]
    for name, m, op, central in variants:
        ens = Ensemble([m] * 1024, series_capacity=2 * steps + 2)
        ens.set_tile(20)
        if central:
            ens.set_collision("central", 1.0, 1.0, 1.0)
        if op is not None:
            ens.set_open_channel(*op)
        ens.init(300, 1e-3)
        ens.step(128)
        ms = _timed(lambda: ens.step(steps)) / steps
        print(json.dumps({"variant": name, "ms_per_step": round(ms, 4),
                          "MLUPS_all_cells": round(1024 * m.nx * m.ny / (ms / 1e3) / 1e6),
                          "nonfinite_members": int(ens.flags().sum())}), flush=True)
        ens.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--settle-s", type=float, default=0.5,
                    help="untimed clock-settling run before the timed region, at least this many seconds")
    ap.add_argument("--settle-steps", type=int, default=640,
                    help="... and at least this many lattice steps (320 two-step launches)")
    ap.add_argument("--workload", default="ensemble", choices=["ensemble", "mixed", "single", "open"])
    ap.add_argument("--tile", type=int, default=16,
                    help="lattice launch shape (-1: autotune; 16, two steps per launch, is the profiled default)")
    ap.add_argument("--cpu-steps", type=int, default=800, help="oracle steps for the CPU baseline (0: skip)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "step2_kernel_ensemble1024_traffic.json"))
    ap.add_argument("--mode", default="bench", choices=["bench", "copy", "score-scaling", "open-parts"],
                    help="copy: time a plain device copy of --copy-mib MiB (counter calibration); "
                         "score-scaling: the score network against the batch size; "
                         "open-parts: the open channel with parts taken away")
    ap.add_argument("--copy-mib", type=int, default=2048)
    ap.add_argument("--no-legs", action="store_true", help="skip the GKTL / AMS / score-network legs")
    ap.add_argument("--collision", default="bgk", choices=["bgk", "central"],
                    help="collision operator (central: central moments, unit bulk / higher-order rates)")
    args = ap.parse_args()
    if args.mode == "copy":
        return copy_calibration(args.copy_mib, max(args.steps, 1))
    if args.mode == "score-scaling":
        return score_scaling([256, 1024, 4096, 16384, 65536])
    if args.mode == "open-parts":
        return open_parts()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the library has no multi-GPU path"}))
        sys.exit(2)

    import torch

    from paper_2005_09323_amd.ensemble import Ensemble

    wl = _workload(args.workload)
    torch.cuda.set_device(0)
    chunk = 128
    ens = Ensemble(wl.members, series_capacity=max(args.warmup, args.steps, chunk) + 1)
    tile = ens.autotune(8) if args.tile < 0 else args.tile
    ens.set_tile(tile)
    if args.collision == "central":
        ens.set_collision("central", 1.0, 1.0, 1.0)
    op = wl.extra.get("open")
    if op is not None:
        ens.set_open_channel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau)
    ens.init(wl.seed, wl.noise_amp)
    ens.step(args.warmup)
    torch.cuda.synchronize()
    # Clock settling, untimed and independent of --warmup: the first few hundred launches of
    # a freshly started device run slower while its clocks come up, so the timed region only
    # starts after at least settle_s seconds and settle_steps steps of the same workload.  The
    # drag columns are reused (the series cursor is rewound before every chunk).
    t_settle = time.perf_counter()
    settled = 0
    while settled < args.settle_steps or time.perf_counter() - t_settle < args.settle_s:
        ens.set_time(1)
        ens.step(chunk)
        torch.cuda.synchronize()
        settled += chunk
    settle = {"steps": settled, "seconds": round(time.perf_counter() - t_settle, 3)}
    ens.set_time(1)

    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record(stream)
    ens.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1)
    sec = ms / 1e3

    cells = wl.cells
    fluid = sum(m.fluid_cells for m in wl.members)
    if op is not None:
        fluid -= len(wl.members) * _grid_cells(wl.members[0], op)
    mlups = cells * args.steps / sec / 1e6
    # the dominant kernel moves the state through HBM once per launch (72 B per
    # fluid cell) and makes `per_launch` lattice steps doing so
    per_launch = ens.launch_steps()
    launch_s = sec / args.steps * per_launch           # per launch, chunk reductions (0.15 %) included
    achieved = BYTES_PER_LUP * fluid / launch_s / 1e9  # GB/s
    equiv = BYTES_PER_LUP * fluid * args.steps / sec / 1e9
    flags = int(ens.flags().sum().item())

    # HBM bytes per launch from the committed counter run, valid only while the
    # kernel source is the one the counters were taken on
    traffic = None
    if os.path.exists(args.traffic_json):
        tj = json.load(open(args.traffic_json))
        same_kernel = kernel_sources_sha256().startswith(tj.get("kernel_sources_sha256_prefix", "-"))
        if (tj.get("workload") == wl.name and same_kernel and tile == tj.get("tile_id")
                and args.collision == tj.get("collision", "bgk")):
            traffic = tj.get("bytes_per_launch")

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp64 update, fp32 storage",
        "data": "synthetic: seeded Philox density noise +-1e-3 on equilibrium "
                + ("at rest" if op is None else "with the inlet profile"),
        "config": {"workload": wl.name, "members": len(wl.members),
                   "cells_per_step": cells, "fluid_cells_per_step": fluid,
                   "tile_id": tile, "collision": args.collision, "nonfinite_members": flags,
                   "wall_s": round(wall, 3)},
        "settle": settle,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        # the same throughput priced at one HBM round trip per lattice step (72 B per fluid-cell update)
        "lup_equivalent": {"steps_per_launch": per_launch, "bytes_per_lup": BYTES_PER_LUP,
                           "GBs": round(equiv, 1), "frac_of_peak": round(equiv / HBM_PEAK_GBS, 4)},
    }
    diag_ms = None
    if not args.no_legs:
        ens.face_diagnostics()
        torch.cuda.synchronize()
        diag_ms = _timed(lambda: ens.face_diagnostics(), 10)
    ens.close()
    del ens
    torch.cuda.empty_cache()
    # the same launch priced against a plain copy on this machine (its practical HBM ceiling)
    cbw = copy_bandwidth()
    out["copy_reference"] = {"GBs": round(cbw, 1), "frac_of_copy": round(achieved / cbw, 4),
                             "what": "torch copy_ of 1 GiB FP32, read + write bytes"}
    if not args.no_legs:
        out["legs"] = legs()
        out["legs"]["face_diagnostics"] = {"workload": wl.name, "ms_per_call": round(diag_ms, 4)}
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
