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
]


def channel(m):
    return lbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square)


def main(only=None):
    for name, factory, idx, steps in FIXTURES:
        if only and name not in only:
            continue
        wl = factory()
        m = wl.members[idx]
        ch = channel(m)
        rho = lbm.init_density(ch, wl.seed, idx, wl.noise_amp)
        _, drags = lbm.run(ch, lbm.init_populations(ch, rho), steps)
        header = (f"oracle FP64 drag series f_d(t), t=0..{steps - 1}\n"
                  f"workload: {wl.name}; member {idx}: nx={m.nx} ny={m.ny} tau={m.tau!r} "
                  f"force_x={m.force_x!r} square={m.square}; seed={wl.seed} noise_amp={wl.noise_amp}\n"
                  f"written by tests/golden/make_golden.py")
        np.savetxt(os.path.join(OUT, name), drags, fmt="%.17g", header=header)
        print("wrote", name, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
