"""Captured chunks (HIP graphs) in lbm_step_batch against launching every kernel.

Every replay is compared with an ensemble that launches each kernel itself,
on the same inputs, with the library's own eager work (state copies,
perturbations, mask and observable changes) and synchronisations between the
replays.  Results must be bit-identical.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import lbm as olbm
from oracle.open_channel import OpenChannel

pytestmark = pytest.mark.gpu


def _pair(members, cap, open_params=None, collision=None):
    from paper_2005_09323_amd.ensemble import Ensemble
    out = []
    for graphs in (True, False):
        ens = Ensemble(members, series_capacity=cap)
        ens.pop_a.zero_()  # solid cells are never written: give both ensembles the same zeros there
        ens.pop_b.zero_()
        ens.set_graphs(graphs)
        if collision is not None:
            ens.set_collision("central", *collision)
        if open_params is not None:
            op = open_params
            ens.set_open_channel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau)
        out.append(ens)
    return out


def _same(g, e, n):
    torch.cuda.synchronize()
    assert np.array_equal(g.drag(0, g.time(0)).cpu().numpy(), e.drag(0, e.time(0)).cpu().numpy())
    assert torch.equal(g.accum, e.accum)
    for i in range(n):
        assert g.time(i) == e.time(i)
        assert torch.equal(g.state(i), e.state(i)), i


@pytest.mark.parametrize("case", ["two_step", "one_step_ragged", "open_central"])
def test_graph_replays_match_eager_launches(case):
    if case == "two_step":
        members = [workloads.Member(512, 40, 0.55, 2e-5, (100, 14, 8))] * 6
        pair = _pair(members, 1200)
    elif case == "one_step_ragged":
        members = [workloads.Member(130, 21, 0.56, 3e-5, (40, 6, 5))] * 3 + [workloads.Member(64, 16, 0.7, 4e-5, None)] * 2
        pair = _pair(members, 1200)
    else:
        members = [workloads.Member(192, 48, 0.56, 0.0, (70, 19, 8))] * 4
        pair = _pair(members, 1200, workloads.OpenParams(0.05, 12, 6, 110, 0.95), (1.2, 1.0, 1.0))
    g, e = pair
    n = len(members)
    snaps = torch.stack([torch.zeros_like(g.state(0)) for _ in range(2)])
    for ens in pair:
        ens.init(3, 1e-3)
        ens.set_observable(0.01, 0.02, 1.0 / 64)
    for ens in pair:
        ens.step(200)                 # three replays of one capture and an eager remainder
    _same(g, e, n)
    for ens in pair:
        ens.step(128)                 # two more replays
    _same(g, e, n)
    mask = [1 if i % 2 == 0 else 0 for i in range(n)]
    for ens in pair:                  # fewer active members: a new capture
        ens.set_active(mask)
        ens.step(64)
    _same(g, e, n)
    for ens in pair:                  # eager work between replays, then all members again
        ens.copy_state_in(1, ens.state(0).clone(), ens.time(1))
        if case != "one_step_ragged":  # (perturbation needs one lattice shape)
            snaps[0].copy_(ens.state(2))
            snaps[1].copy_(ens.state(0))
            ens.perturb([0, 1] + [0] * (n - 2), 5, 1, 1e-3, snaps)
        ens.set_active(None)
        ens.set_observable(0.0, 0.05, 1.0 / 32)  # a changed observable: a new capture
        ens.step(192)
    _same(g, e, n)
    for ens in pair:
        ens.close()


def test_reconfiguring_after_replays_matches_a_fresh_ensemble():
    """Replays, then a new open-channel configuration (a new ghost block), a collision change and
    back to periodic: each phase equals a fresh ensemble set up that way from the start."""
    from paper_2005_09323_amd.ensemble import Ensemble
    members = [workloads.Member(256, 33, 0.58, 0.0, (100, 12, 8))] * 3
    op1 = workloads.OpenParams(0.04, 30, 4, 200, 0.8)
    op2 = workloads.OpenParams(0.05, 20, 6, 180, 0.9)

    def fresh(op, collision, steps):
        ens = Ensemble(members, series_capacity=300)
        ens.pop_a.zero_()
        ens.pop_b.zero_()
        if collision is not None:
            ens.set_collision("central", *collision)
        if op is not None:
            ens.set_open_channel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau)
        ens.init(5, 1e-3)
        ens.step(steps)
        torch.cuda.synchronize()
        out = [ens.state(i).clone() for i in range(len(members))], ens.drag(0, steps + 1).clone()
        ens.close()
        return out

    ens = Ensemble(members, series_capacity=300)
    ens.pop_a.zero_()
    ens.pop_b.zero_()
    phases = [(op1, None), (op2, None), (op2, (1.1, 1.0, 1.0)), (None, (1.1, 1.0, 1.0)), (None, None)]
    for op, collision in phases:
        ens.set_collision("central", *collision) if collision is not None else ens.set_collision("bgk")
        if op is not None:
            ens.set_open_channel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau)
        else:
            ens.set_open_channel(None)
        ens.init(5, 1e-3)
        ens.step(192)
        torch.cuda.synchronize()
        ref_states, ref_drag = fresh(op, collision, 192)
        assert torch.equal(ens.drag(0, 193), ref_drag), (op, collision)
        # solid cells may hold what an earlier geometry left there: compare the fluid cells
        m = members[0]
        oc = None if op is None else OpenChannel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau)
        fluid = torch.from_numpy(~olbm.solid_mask(olbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square,
                                                               open=oc))).cuda()
        for i in range(len(members)):
            assert torch.equal(ens.state(i)[:, fluid], ref_states[i][:, fluid]), (op, collision, i)
    ens.close()
