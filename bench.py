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
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(wl, steps: int):
    """Time the FP64 oracle on member 0 of the workload (single thread)."""
    from threadpoolctl import threadpool_limits

    from oracle import lbm as olbm
    m = wl.members[0]
    ch = olbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square)
    f = olbm.init_populations(ch, olbm.init_density(ch, wl.seed, 0, wl.noise_amp))
    with threadpool_limits(limits=1):
        olbm.run(ch, f, 2)  # warm caches of the geometry tables
        t0 = time.perf_counter()
        olbm.run(ch, f, steps)
        dt = time.perf_counter() - t0
    return {"value": round(m.cells * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"member 0 ({m.nx}x{m.ny}) of the same workload, {steps} steps, FP64 numpy, 1 thread; "
                      f"host {platform.processor() or platform.machine()}, os.cpu_count()={os.cpu_count()}"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ensemble", choices=["ensemble", "mixed", "single"])
    ap.add_argument("--tile", type=int, default=-1, help="step-kernel tile id (-1: autotune)")
    ap.add_argument("--cpu-steps", type=int, default=120, help="oracle steps for the CPU baseline (0: skip)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "step_kernel_traffic.json"))
    ap.add_argument("--mode", default="bench", choices=["bench", "copy"],
                    help="copy: time a plain device copy of --copy-mib MiB (counter calibration)")
    ap.add_argument("--copy-mib", type=int, default=2048)
    args = ap.parse_args()
    if args.mode == "copy":
        return copy_calibration(args.copy_mib, max(args.steps, 1))
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not part of this build"}))
        sys.exit(2)

    import torch

    from paper_2005_09323_amd.ensemble import Ensemble

    wl = _workload(args.workload)
    torch.cuda.set_device(0)
    total = args.warmup + args.steps
    ens = Ensemble(wl.members, series_capacity=total + 1)
    tile = ens.autotune(8) if args.tile < 0 else args.tile
    ens.set_tile(tile)
    ens.init(wl.seed, wl.noise_amp)
    ens.step(args.warmup)
    torch.cuda.synchronize()

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
    mlups = cells * args.steps / sec / 1e6
    achieved = BYTES_PER_LUP * fluid / (sec / args.steps) / 1e9  # GB/s per step (kernel + reduction)
    flags = int(ens.flags().sum().item())

    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json))
            if tj.get("workload") == wl.name:
                traffic = tj.get("bytes_per_launch")
        except Exception:
            traffic = None

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
        "dtype": "f32",
        "data": "synthetic: seeded Philox density noise +-1e-3 on equilibrium at rest",
        "config": {"workload": wl.name, "members": len(wl.members),
                   "cells_per_step": cells, "fluid_cells_per_step": fluid,
                   "tile_id": tile, "nonfinite_members": flags, "wall_s": round(wall, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
    }
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    ens.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
