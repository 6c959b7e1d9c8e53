"""Write the stored expected drag series used by the full-size parity tests.

Calls only ``oracle/`` (and the workload tables in ``workloads.py``).  Each
fixture is the FP64 oracle drag series f_d(t), t = 0..n-1, of one member of
one workload, started from the seeded equilibrium of the initial-density
Philox stream.  Run from the repository root:

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import lbm  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))

FIXTURES = [
    # (file, workload factory, member index, steps)
    ("ensemble1024_m0_drag1000.txt", workloads.ensemble_1024, 0, 1000),
    ("ensemble1024_m127_drag1000.txt", workloads.ensemble_1024, 127, 1000),
    ("mixed_m0_drag1000.txt", workloads.mixed_sizes, 0, 1000),
    ("mixed_m64_drag1000.txt", workloads.mixed_sizes, 64, 1000),
    ("mixed_m191_drag1000.txt", workloads.mixed_sizes, 191, 1000),
    # the paper's open channel (inlet, grid, sponge, outlet), central moments
    ("open1024_m0_drag2000.txt", workloads.open_channel, 0, 2000),
    ("open1024_m777_drag2000.txt", workloads.open_channel, 777, 2000),
    ("open1024_m1023_drag2000.txt", workloads.open_channel, 1023, 2000),
]


def channel(wl, m):
    op = wl.extra.get("open")
    if op is None:
        return lbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square)
    from oracle.open_channel import OpenChannel
    return lbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square, wl.extra.get("rates"),
                       open=OpenChannel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau, op.outlet_rho))


def start(ch, rho):
    """Step-0 input: equilibrium at rest (periodic) or on the inlet profile (open channel)."""
    if ch.open is None:
        return lbm.init_populations(ch, rho)
    from oracle.open_channel import inlet_velocity
    u = np.repeat(inlet_velocity(ch)[:, None], ch.nx, axis=1)
    f0 = lbm.equilibrium(rho, u, np.zeros_like(u))
    f0[:, lbm.solid_mask(ch)] = 0.0
    return f0


def main(only=None):
    for name, factory, idx, steps in FIXTURES:
        if only and name not in only:
            continue
        wl = factory()
        m = wl.members[idx]
        ch = channel(wl, m)
        rho = lbm.init_density(ch, wl.seed, idx, wl.noise_amp)
        _, drags = lbm.run(ch, start(ch, rho), steps)
        extra = "" if ch.open is None else f"; open channel {wl.extra['open']}, central-moment rates {wl.extra['rates']}"
        header = (f"oracle FP64 drag series f_d(t), t=0..{steps - 1}\n"
                  f"workload: {wl.name}; member {idx}: nx={m.nx} ny={m.ny} tau={m.tau!r} "
                  f"force_x={m.force_x!r} square={m.square}; seed={wl.seed} noise_amp={wl.noise_amp}{extra}\n"
                  f"written by tests/golden/make_golden.py")
        np.savetxt(os.path.join(OUT, name), drags, fmt="%.17g", header=header)
        print("wrote", name, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
