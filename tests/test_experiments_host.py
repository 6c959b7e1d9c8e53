"""Host-side helpers of the return-time experiment driver (no GPU)."""
import math

import numpy as np
import torch

from paper_2005_09323_amd import experiments


def test_distinct_roots_traces_lineages():
    # 4 slots, 3 periods: ancestors[i][m] = slot of period i-1... traced from the last period back
    anc = torch.tensor([[0, 0, 2, 3],    # period 0: slots 0,1 <- 0; 2 <- 2; 3 <- 3
                        [1, 1, 2, 2],    # period 1
                        [0, 3, 3, 3]],   # period 2
                       dtype=torch.int32)
    # final slot m -> period-2 ancestor -> period-1 ancestor -> period-0 ancestor
    # m=0: 0 -> 1 -> 0 ; m=1..3: 3 -> 2 -> 2
    assert experiments._distinct_roots(anc) == 2
    assert experiments._distinct_roots(torch.arange(5, dtype=torch.int32).repeat(3, 1)) == 5


def test_rel_scatter():
    v = np.array([[1.0, 2.0, math.inf], [3.0, 2.0, 1.0]])
    out = experiments._rel_scatter(v)
    assert abs(out[0] - np.std([1.0, 3.0], ddof=1) / 2.0) < 1e-15
    assert out[1] == 0.0
    assert math.isinf(out[2])


def test_autocorrelation_first_zero_of_a_sine():
    """A sine of period P decorrelates at lag P/4 (the autocorrelation of a long sine is cos)."""
    import numpy as np
    from paper_2005_09323_amd.experiments import _autocorrelation, _first_zero
    P = 400
    t = np.arange(40 * P)
    d = np.stack([np.sin(2 * np.pi * t / P + ph) for ph in (0.0, 1.0, 2.0)])
    acf = _autocorrelation(d)
    assert abs(acf[0] - 1) < 1e-12
    assert abs(_first_zero(acf) - P / 4) <= 1


def test_return_time_flows_follow_their_workloads():
    """The GKTL and AMS experiment flows keep their workloads' lattice, square and tau (only the
    force density and the collision are the experiments' own, for stability)."""
    import workloads
    from paper_2005_09323_amd import experiments
    for flow, wl in ((experiments.gktl_flow(), workloads.gktl_ensemble()),
                     (experiments.ams_flow(), workloads.ams_ensemble())):
        m = wl.members[0]
        assert (flow.nx, flow.ny, flow.tau, tuple(flow.square)) == (m.nx, m.ny, m.tau, tuple(m.square))
        assert flow.collision == "central" and callable(flow.start) and callable(flow.ensemble)
