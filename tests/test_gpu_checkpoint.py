"""Checkpoint and resume: 2n steps in one go against n steps, save, load into a new
ensemble, n more steps.  Every result must be bit-identical: states, drag series,
FP64 observable integrals, times, non-finite flags, and for a GKTL run the
ancestors, normalisers and period integrals of every selection.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import lbm as olbm
from oracle.open_channel import OpenChannel

pytestmark = pytest.mark.gpu

OPEN = workloads.OpenParams(0.05, 12, 6, 110, 0.95)


def _bits(t):
    return t.contiguous().view(torch.int32 if t.dtype == torch.float32 else torch.int64)


def _configure(ens, case):
    if case == "open_central":
        ens.set_collision("central", 1.2, 1.0, 1.0)
        ens.set_open_channel(OPEN.u_c, OPEN.grid_x0, OPEN.bar, OPEN.sponge_x0, OPEN.sponge_tau)


def _fluid(m, case):
    """Fluid cells of member m: solid cells are never written and hold whatever their memory held."""
    oc = OpenChannel(OPEN.u_c, OPEN.grid_x0, OPEN.bar, OPEN.sponge_x0, OPEN.sponge_tau) if case == "open_central" else None
    return torch.from_numpy(~olbm.solid_mask(olbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square, open=oc))).cuda()


def _members(case):
    if case == "open_central":
        return [workloads.Member(192, 48, 0.56, 0.0, (70, 19, 8))] * 3
    return ([workloads.Member(256, 24, 0.58, 3e-5, (60, 8, 6))] * 2 + [workloads.Member(130, 21, 0.6, 2e-5, (40, 6, 5))]
            + [workloads.Member(64, 16, 0.7, 4e-5, None)])


def _same_ensembles(a, b, case="periodic"):
    torch.cuda.synchronize()
    assert a.n == b.n
    for m in range(a.n):
        assert a.time(m) == b.time(m)
        fluid = _fluid(a.members[m], case)
        assert torch.equal(_bits(a.state(m))[:, fluid], _bits(b.state(m))[:, fluid]), m
    assert torch.equal(_bits(a.series), _bits(b.series))
    assert torch.equal(_bits(a.accum), _bits(b.accum))
    assert torch.equal(a.flags(), b.flags())


@pytest.mark.parametrize("case", ["periodic_mixed", "open_central"])
def test_save_load_resume_is_bit_exact(case, tmp_path):
    from paper_2005_09323_amd.ensemble import Ensemble
    members = _members(case)
    n_first, n_second, cap = 147, 154, 400
    straight = Ensemble(members, series_capacity=cap)
    split = Ensemble(members, series_capacity=cap)
    for ens in (straight, split):
        _configure(ens, case)
        ens.init(11, 1e-3)
        ens.set_observable(0.01, 0.02, 1.0 / 64)
        if case == "periodic_mixed":
            ens.state(1)[3, 5, 7] = float("nan")  # a member that blows up: its flag must survive the resume
            ens.set_active([1, 1, 0, 1])           # and a frozen one
    straight.step(n_first)
    straight.step(n_second)
    split.step(n_first)
    path = str(tmp_path / "ensemble.pt")
    split.save(path)
    split.close()
    resumed = Ensemble.load(path)
    assert resumed.members == [type(resumed.members[0])(m.nx, m.ny, m.tau, m.force_x, m.square) for m in members]
    resumed.step(n_second)
    _same_ensembles(straight, resumed, case)
    if case == "periodic_mixed":
        assert resumed.flags().cpu().tolist() == [0, 1, 0, 0]
        assert resumed.time(2) == 1 and resumed.time(0) == 1 + n_first + n_second
    straight.close()
    resumed.close()


def test_gktl_run_resumed_from_a_checkpoint_is_bit_exact(tmp_path):
    from paper_2005_09323_amd import rare
    from paper_2005_09323_amd.ensemble import Ensemble
    m = workloads.Member(256, 32, 0.57, 2e-5, (60, 12, 8))
    n, tau, k, key, eps = 16, 24, 0.8, 5, 2e-3
    cap = 6 * tau + 1

    def fresh():
        ens = Ensemble([m] * n, series_capacity=cap)
        ens.init(23, 1e-2)
        ens.set_observable(0.0, 1e-4, 1.0 / 32)
        return ens

    straight = fresh()
    snaps = torch.stack([straight.state(i).clone() for i in (1, 4, 9)])
    whole = rare.run_gktl(straight, k, 6, tau, key, eps, snaps)

    split = fresh()
    first = rare.run_gktl(split, k, 4, tau, key, eps, snaps)
    path = str(tmp_path / "gktl.pt")
    split.save(path)
    split.close()
    resumed = Ensemble.load(path)
    second = rare.run_gktl(resumed, k, 2, tau, key, eps, snaps, first_period=4)
    joined = first.then(second)

    assert torch.equal(whole.ancestors, joined.ancestors)
    assert torch.equal(_bits(whole.ln_r), _bits(joined.ln_r))
    assert torch.equal(_bits(whole.integrals), _bits(joined.integrals))
    assert len(np.unique(whole.ancestors[-1].cpu().numpy())) < n  # selection really cloned
    _same_ensembles(straight, resumed)
    tr_a = rare.rebuild(whole, straight)
    tr_b = rare.rebuild(joined, resumed)
    assert torch.equal(_bits(tr_a.series), _bits(tr_b.series))
    assert torch.equal(_bits(tr_a.log_weight), _bits(tr_b.log_weight))
    with pytest.raises(ValueError):
        first.then(first)
    straight.close()
    resumed.close()
